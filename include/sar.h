/*
 * sar.h -- C ABI of the MI355X (gfx950) near-field MIMO-SAR image-formation
 * library for irregular (multi-planar, multistatic) scanning geometries.
 *
 * Method: J. W. Smith and M. Torlak, "Efficient 3-D Near-Field MIMO-SAR
 * Imaging for Irregular Scanning Geometries", IEEE Access (2022).
 * Equation numbers below count the paper's displayed equations in order
 * ((1) far-field criterion ... (17) spatial resolution).
 *
 * Pipeline of one scan (Sec. III, Fig. 3):
 *   a0  virtual elements x' = (x_T + x_R)/2, y' likewise, d = x_R - x_T,
 *       d^z = z_l - Z_0 (Eqs. (3)-(4)); residual path
 *       beta = 2 sign(Z_0 - z_c) d^z + (d_x^2 + d_y^2) / (4 |z_c - Z_0|)
 *       (Eqs. (7), (12) written in the array frame);
 *   a1  compensation s_hat = s exp(+j k beta), k = 2 pi f / c (Eq. (11));
 *   a2  Kaiser-Bessel gridding of the irregular (x', y') samples onto an
 *       oversampled uniform grid (type-1 NUFFT spreading, the FT_2D of
 *       Eq. (16) evaluated with a NUFFT as in Sec. III);
 *   a3  2-D FFT, deapodisation and crop to the image's (k_x, k_y) modes:
 *       S(p,q,f) ~ sum_n s_hat_n(f) exp(-j[k_x,p (x'_n - x_c) + k_y,q (y'_n - y_c)]),
 *       k_x,p = 2 pi p / (nx dx), p = -nx/2 .. nx/2-1, x_c = x0 + (nx/2) dx;
 *   a4  filter k_z exp(-j k_z Z_0) / P(f), P = 1, k_z^2 = 4k^2 - k_x^2 - k_y^2,
 *       evanescent modes dropped (Eqs. (14)-(15));
 *   a5  Stolt map onto uniform k_z and the z transform, evaluated as a 1-D
 *       type-1 NUFFT per (k_x, k_y) column of
 *       Z(p,q,z_w) = sum_f F(p,q,f) exp(+j k_z z_w), z_w = z0 + w dz;
 *   a6  inverse 2-D transform to the image (rest of IFT_3D, Eq. (16)):
 *       o(u,v,w) = sum_{p,q} Z(p,q,w) exp(+j[k_x,p (x_u - x_c) + k_y,q (y_v - y_c)]),
 *       unnormalised.
 *
 * Conventions
 *   - Units: metres, hertz.  c = 299 792 458 m/s.
 *   - Layouts (all row-major, last index fastest):
 *       positions  double [n_pos][3]                      (x, y, z of the device origin per shot)
 *       echo       [n_pos][n_tx*n_rx][n_freq]  pair = t*n_rx + r
 *                  SAR_ECHO_C64: float2 (re, im);  SAR_ECHO_F16X2: two IEEE halves (re, im),
 *                  value = half * echo_scale
 *       spectrum   float2 [ny][nx][n_freq]   mode index j = p + nx/2 (centred)
 *       image      float2 [nx][ny][nz]       voxel (u,v,w) at (x0+u dx, y0+v dy, z0+w dz)
 *   - Device pointers ("d_") are HIP device memory on the plan's device and are
 *     owned by the caller.  Host arrays passed to sar_plan_create are copied;
 *     the caller may free them on return.
 *   - Every call returns a status; nothing aborts or throws across the ABI.
 *     On failure sar_last_error() describes the cause (thread-local string,
 *     valid until the next call on the same thread).
 *   - Compute calls are asynchronous and ordered on the given HIP stream
 *     (NULL = the null stream); they do not allocate and do not synchronise.
 */
#ifndef SAR_H_
#define SAR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sar_plan_s* sar_plan;
typedef struct sar_server_s* sar_server;
typedef struct sar_batch_s* sar_batch;
typedef void* sar_stream_t; /* a hipStream_t */

typedef enum {
  SAR_OK = 0,
  SAR_ERR_INVALID = 1,     /* bad argument or descriptor */
  SAR_ERR_NOMEM = 2,       /* device allocation failed */
  SAR_ERR_DEVICE = 3,      /* HIP runtime / launch error */
  SAR_ERR_BUSY = 4,        /* resource has work in flight */
  SAR_ERR_NOT_FOUND = 5,   /* unknown handle or ticket */
  SAR_ERR_UNSUPPORTED = 6  /* valid request the library does not implement */
} sar_status;

typedef enum { SAR_ECHO_C64 = 0, SAR_ECHO_F16X2 = 1 } sar_echo_type;

/* flags */
#define SAR_NO_COMPENSATION 0x1u /* beta = 0: plain RMA on raw multi-planar data (Sec. III ablation) */
/* Precision diagnostic: the phase arguments (k beta of the compensation, the
 * Stolt pre-phase k_z (z - Z_0) and grid position) and the position-to-grid
 * offsets in float32 instead of float64.  Not for production: it exists to
 * measure what the float64 arguments buy.  Needs complex64 echo and a 4-tap
 * lateral kernel (SAR_ERR_UNSUPPORTED otherwise). */
#define SAR_FP32_ARGS 0x2u
/* Stolt density compensation: the filter of Eq. (15) is further multiplied by
 * the Jacobian of the change of variables from k to k_z, dk_z/dk = 4k / k_z
 * (from Eq. (14) at fixed k_x, k_y), so the sum over frequency of step a5
 * weights each sample by the k_z interval it covers.  The paper states only
 * the k_z factor; off by default. */
#define SAR_STOLT_DCF 0x4u
/* Amplitude half of the compensation: besides exp(+j k beta) of Eq. (11),
 * each sample is scaled by R^T R^R / R_0^2, the ratio between the multistatic
 * amplitude of Eq. (9) and the planar monostatic one of Eq. (10), for a
 * scatterer straight ahead of the sample's virtual element at the reference
 * depth z_c (z_focus, or the z-centre of a depth slab):
 *     ((d_x^2 + d_y^2) / 4 + (z_c - z_l)^2) / (z_c - Z_0)^2,
 * with d the pair's Rx - Tx offset and z_l the shot's height.  The paper's
 * compensation is phase only; off by default.  Independent of
 * SAR_NO_COMPENSATION (which zeroes beta only). */
#define SAR_AMPLITUDE 0x8u

/* Plan descriptor: array geometry, frequency sweep and image grid.
 * Constraints (SAR_ERR_INVALID otherwise):
 *   n_tx, n_rx >= 1, n_tx * n_rx <= 4096; n_freq >= 1, freq_hz finite,
 *   strictly increasing, > 0;
 *   nx, ny in [8, 2048], each a product 2^a 3^b 5^c (odd sides included);
 *   nz 1 or a power of two in [2, 512]
 *   (nz = 1: one x-y plane at z0, the paper's 2-D image at a known depth,
 *   Sec. V-A; steps a4-a5 become one exact sum over frequency per column);
 *   dx, dy, dz > 0; the scene reference depth and the image volume in front
 *   of the projection plane (z_focus > z_ref, z0 > z_ref);
 *   0 <= max_pos and max_pos * n_tx * n_rx < 2^31;
 *   tol 0 or in (0, 0.1]: target relative L2 error of the lateral NUFFT
 *   (0 selects 1e-3); the kernel width is the smallest whose calibrated
 *   error 5 exp(-pi W sqrt(1 - 1/sigma)) meets it;
 *   upsample 0 (automatic: what sar_plan_autotune stored for the plan's size
 *   bucket, see below, else per axis a power of two between 1.5 n and 2 n if
 *   there is one, else the grid of upsample 2) or in [1.25, 4]
 *   (SAR_ERR_UNSUPPORTED otherwise): the lateral grid has the smallest
 *   multiple of 8 cells of the form 2^a 3^b 5^c at or above upsample * n along
 *   each axis (the next power of two instead when it is at most 1/8 larger),
 *   at most 4096 cells (SAR_ERR_UNSUPPORTED beyond; sar_plan_info reports the
 *   effective ratio);
 *   kernel_width 0 (from tol) or 3..8 taps;
 *   n_slabs 0 or 1 (one reference depth z_focus for the whole volume) or a
 *   power of two that divides nz: depth slabs, see below.
 *
 * Depth slabs (n_slabs > 1).  The residual path of the compensation (Eqs. (7),
 * (12)) uses one reference range R_c = |z_focus - z_ref| in its multistatic
 * term, so targets far from z_focus keep a residual phase that grows with the
 * Tx/Rx separation; the paper notes the resulting aberrations in depth
 * (Sec. V-A).  With n_slabs = S > 1 the volume is cut along z into S
 * slabs of nz / S planes; slab j is reconstructed with its own reference
 * depth, the z-centre of its planes, z0 + (j nz/S + (nz/S - 1)/2) dz, and
 * writes only its planes of the image.  z_focus is then unused (it must still
 * satisfy z_focus > z_ref).  Each slab repeats steps a0-a3, so a call costs
 * about S single-depth front ends plus one back end; sar_spectrum and
 * sar_image_from_spectrum (one spectrum per depth) return
 * SAR_ERR_UNSUPPORTED, and per-stage timing (sar_plan_set_timing) records
 * nothing for such plans. */
typedef struct {
  int32_t n_tx;
  int32_t n_rx;
  const double* tx_xy; /* [n_tx][2] Tx offsets from the device origin; z offset 0 */
  const double* rx_xy; /* [n_rx][2] Rx offsets from the device origin; z offset 0 */
  int32_t n_freq;
  const double* freq_hz; /* [n_freq] stepped frequencies */
  double z_ref;          /* Z_0: plane the samples are projected on (Eqs. (4), (10)) */
  double z_focus;        /* z_c: scene reference depth for beta's multistatic term */
  int32_t nx, ny, nz;
  double x0, y0, z0; /* first voxel centre */
  double dx, dy, dz; /* voxel pitch */
  int64_t max_pos;   /* largest n_pos a workspace from this plan must serve */
  int32_t echo_type; /* sar_echo_type */
  double tol;
  double upsample;
  int32_t kernel_width;
  uint32_t flags;
  int32_t n_slabs;   /* depth slabs with their own reference depth (0 or 1: none) */
} sar_plan_desc;

/* What a plan chose (read-only). */
typedef struct {
  int32_t mx, my;        /* oversampled lateral grid (cells) */
  int32_t width;         /* lateral Kaiser-Bessel kernel width (taps) */
  double kb_beta;        /* its shape parameter */
  int32_t mz;            /* oversampled Stolt grid (cells) */
  int32_t width_z;       /* Stolt kernel width (taps) */
  double es_beta_z;      /* its shape parameter */
  int32_t n_pair;        /* n_tx * n_rx */
  int32_t n_stages;      /* entries returned by sar_plan_stage_times */
  size_t workspace_bytes_max; /* workspace for n_pos = max_pos */
  int32_t grid_tile;     /* gridding tile configuration in use (see sar_plan_autotune) */
  int32_t grid_tile_x, grid_tile_y;  /* its cells per wave along x and y */
  int32_t grid_freqs_per_lane;       /* its frequencies per lane (64 lanes per wave) */
  int32_t n_slabs;       /* depth slabs (1: one reference depth) */
  /* the descriptor's sizes as the plan keeps them */
  int32_t nx, ny, nz;
  int32_t n_freq;
  int32_t echo_type;     /* sar_echo_type */
  uint32_t flags;
  int64_t max_pos;
  double sigma_x, sigma_y;  /* effective lateral oversampling mx / nx, my / ny */
} sar_plan_info;

/* Create a plan on HIP device `device`: validates the descriptor, chooses the
 * NUFFT parameters, and uploads its tables (wavenumbers, deapodisation,
 * twiddles, pair offsets) to the device, where they stay until
 * sar_plan_destroy.  Geometry: Sec. II-B; sweep: Sec. II-C; grid: Sec. III.
 * Errors: SAR_ERR_INVALID (descriptor), SAR_ERR_NOMEM, SAR_ERR_DEVICE. */
sar_status sar_plan_create(const sar_plan_desc* desc, int device, sar_plan* out);

/* Release the plan's device tables.  NULL is accepted.  SAR_ERR_BUSY (and
 * nothing released) while a server request submitted with the plan has not
 * finished or a batch built from it has not been destroyed.  Work queued on
 * streams by the caller's own sar_reconstruct / sar_spectrum calls is not
 * tracked: the caller must ensure it has finished. */
sar_status sar_plan_destroy(sar_plan plan);

/* Bytes of device workspace sar_reconstruct / sar_spectrum /
 * sar_image_from_spectrum need for a scan of n_pos shots (0 <= n_pos <= max_pos). */
sar_status sar_plan_workspace_bytes(sar_plan plan, int64_t n_pos, size_t* bytes);

sar_status sar_plan_get_info(sar_plan plan, sar_plan_info* info);

/* Steps a0-a6: image of one scan.
 *   d_pos       device double [n_pos][3]
 *   n_pos       shots in this scan, 0 <= n_pos <= max_pos (0 gives a zero image)
 *   d_echo      device echo [n_pos][n_pair][n_freq] of the plan's echo type
 *   echo_scale  multiplies every echo value (use 1 for SAR_ECHO_C64)
 *   d_image     device float2 [nx][ny][nz], written
 *   d_workspace device scratch of sar_plan_workspace_bytes(plan, n_pos) bytes,
 *               256-byte aligned; contents undefined afterwards
 *   stream      HIP stream the work is queued on
 * Asynchronous; errors reported here are argument errors and launch errors. */
sar_status sar_reconstruct(sar_plan plan, const double* d_pos, int64_t n_pos, const void* d_echo,
                           float echo_scale, void* d_image, void* d_workspace, sar_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * pipeline as sar_reconstruct with no workspace argument.  Its workspace is a
 * fixed array of SAR_NOALLOC_SCRATCH_BYTES in the library's device memory, one
 * per device, held until the process ends; the call allocates nothing.
 * Scans whose workspace (sar_plan_workspace_bytes) exceeds it return
 * SAR_ERR_UNSUPPORTED with nothing queued.  Calls that overlap on one device
 * (several streams or host threads) share the array and race; serialise them.
 * Other arguments, ordering and errors as sar_reconstruct. */
#define SAR_NOALLOC_SCRATCH_BYTES (64u << 20)
sar_status sar_reconstruct_noalloc(sar_plan plan, const double* d_pos, int64_t n_pos, const void* d_echo,
                                   float echo_scale, void* d_image, sar_stream_t stream);

/* Steps a0-a3 only: the compensated spatial spectrum S, written to
 * d_spectrum (device float2 [ny][nx][n_freq], centred mode order). */
sar_status sar_spectrum(sar_plan plan, const double* d_pos, int64_t n_pos, const void* d_echo,
                        float echo_scale, void* d_spectrum, void* d_workspace, sar_stream_t stream);

/* Steps a4-a6 only: image of a given spectrum (layout as sar_spectrum's
 * output).  d_workspace needs sar_plan_workspace_bytes(plan, 0) bytes. */
sar_status sar_image_from_spectrum(sar_plan plan, const void* d_spectrum, void* d_image, void* d_workspace,
                                   sar_stream_t stream);

/* Direct back-projection with exact ranges, the paper's gold standard
 * (Sec. III, Sec. V; ranges of Eq. (2)):
 *   o_B(u,v,w) = sum_n sum_i s_n(f_i) exp(+j k_i (R_T,n + R_R,n)(x_u, y_v, z_w)),
 * unit amplitude weight, on the plan's image grid (layouts and arguments as
 * sar_reconstruct; no workspace).  Cost n_pos * n_pair * n_freq * nx*ny*nz:
 * meant for small scans, to compare the fast method's images and times.
 * Asynchronous on `stream`.  SAR_ERR_UNSUPPORTED (nothing queued) when
 * n_pos * n_pair * n_freq * nx * ny * nz exceeds 1e12 terms (about a second of
 * one MI355X): a single dispatch that long would look like a hang. */
sar_status sar_backproject(sar_plan plan, const double* d_pos, int64_t n_pos, const void* d_echo, float echo_scale,
                           void* d_image, sar_stream_t stream);

/* Autotuner: times the whole pipeline on the given scan (which should be
 * representative of the plan's workload) for every candidate and keeps the
 * fastest for every later call of this plan.  Candidates: the lateral
 * oversampling (the automatic choice, 1.25, 1.5 and 2 when the plan was
 * created with upsample = 0, else only the requested one; the kernel width
 * follows the plan's tolerance at each) times every gridding tile
 * configuration compiled for that width:
 *   0: 4 x 4 cells per wave, 2 frequencies per lane (kernels of 3 to 8 taps);
 *   1: 8 x 8 cells per wave, 1 frequency per lane (3 to 5 taps);
 *   2: 8 x 4 cells per wave, 2 frequencies per lane (5 and 6 taps);
 *   3: 8 x 8 cells per 4-wave workgroup, 2 frequencies per lane (3 to 5 taps).
 * Candidates whose workspace would exceed the plan's current
 * sar_plan_workspace_bytes(plan, n_pos) are skipped, so d_workspace as sized
 * before the call stays large enough.  Runs each candidate a few times on
 * `stream` and waits for them (synchronous).  The default before tuning:
 * the automatic oversampling (see upsample), tile 1 when the
 * sweep has at most 64 frequencies (and the width allows it), else tile 3 for
 * kernels of up to 5 taps, else tile 0.  If the environment variable
 * SAR_AUTOTUNE_FILE names a file, the choice is also stored there for the
 * plan's size bucket (image and sweep sizes, pairs, echo type, flags,
 * tolerance, n_pos rounded up to a power of two), and plans created later
 * with upsample = 0 and a max_pos in the same bucket start from it.
 * SAR_ERR_BUSY while batches or server requests use the plan; tune before
 * creating batches from it and not while other calls use it.  tile_out (may
 * be NULL) receives the chosen tile; sar_plan_get_info reports the rest.
 * Arguments as sar_reconstruct. */
sar_status sar_plan_autotune(sar_plan plan, const double* d_pos, int64_t n_pos, const void* d_echo,
                             float echo_scale, void* d_workspace, sar_stream_t stream, int32_t* tile_out);

/* Select a gridding tile configuration directly (0 to 3, as listed for
 * sar_plan_autotune).  SAR_ERR_UNSUPPORTED if it is not compiled for the
 * plan's kernel width; same restrictions as sar_plan_autotune. */
sar_status sar_plan_set_grid_tile(sar_plan plan, int32_t tile);

/* Per-stage timing with HIP events recorded on the call's stream around each
 * kernel group (stage order: 0 geometry+sort, 1 gridding, 2 FFT along x,
 * 3 FFT along y, 4 Stolt, 5 inverse FFT along y, 6 inverse FFT along x).
 * enable != 0 starts recording (and clears earlier records);
 * sar_plan_stage_times waits for the recorded events, returns the summed
 * milliseconds per stage over all recorded calls and their count, and clears
 * the records.  ms must hold sar_plan_info.n_stages doubles. */
sar_status sar_plan_set_timing(sar_plan plan, int enable);
sar_status sar_plan_stage_times(sar_plan plan, double* ms, int32_t n, int64_t* n_calls);

/* ---- Fused batches of uneven scans ----
 * A batch runs the per-scan pipeline (Sec. III) of several scans, each with
 * its own plan (sizes may differ), in one fused launch per pipeline step:
 * every kernel grid holds the blocks of all scans that use the same kernel
 * at that step, each scan reading its arguments from a device table.  The
 * launch sequence depends only on the plans (per-sample grids are sized for
 * each plan's max_pos), so it is captured once into a HIP graph and replayed
 * by every later call.
 *
 * sar_batch_create: plans[0..n-1], all on one device, one per item (a plan
 *   may appear several times); the plans must outlive the batch.  flags:
 *   SAR_BATCH_NO_GRAPH issues the fused launches directly instead of
 *   replaying a graph.  Errors: SAR_ERR_INVALID, SAR_ERR_NOMEM.
 * sar_batch_workspace_bytes: device workspace for one call (sum over items of
 *   the plan's workspace at its max_pos, each 256-byte aligned).
 * sar_batch_reconstruct: host arrays of n entries: d_pos[i], n_pos[i]
 *   (<= the plan's max_pos), d_echo[i], echo_scale[i] (NULL = all 1),
 *   d_image[i] (device buffers, layouts as sar_reconstruct).  Asynchronous on
 *   `stream`; calls on one batch are ordered even across streams (the device
 *   argument tables are shared).  The first call captures the graph.
 *   Errors: SAR_ERR_INVALID (arguments, per item), SAR_ERR_DEVICE.
 * sar_batch_destroy: waits for the batch's last call, then releases it. */
#define SAR_BATCH_NO_GRAPH 0x1u
sar_status sar_batch_create(const sar_plan* plans, int32_t n, uint32_t flags, sar_batch* out);
sar_status sar_batch_workspace_bytes(sar_batch batch, size_t* bytes);
sar_status sar_batch_reconstruct(sar_batch batch, const double* const* d_pos, const int64_t* n_pos,
                                 const void* const* d_echo, const float* echo_scale, void* const* d_image,
                                 void* d_workspace, sar_stream_t stream);
sar_status sar_batch_destroy(sar_batch batch);

/* ---- Serving: continuous admission of scans under a device-memory budget ----
 * The paper forms one image per scan (Sec. III); a server runs that same
 * per-scan pipeline for a stream of independent scans of different sizes,
 * overlapping them on one device.
 *
 * sar_server_create: a server on HIP device `device` owning one arena of
 *   hbm_budget_bytes of device memory (rounded down to 256 bytes), four HIP
 *   streams, a worker thread and 8 MiB each of pinned host and device memory
 *   for argument tables.  Errors: SAR_ERR_INVALID (no such device, budget <
 *   256 bytes), SAR_ERR_NOMEM (an allocation failed).
 *
 * sar_submit: queue one scan; returns at once with a ticket.
 *   plan           a plan created on the server's device; it must outlive the request
 *   pos_xyz, echo  positions [n_pos][3] (double) and echo [n_pos][n_pair][n_freq]
 *                  of the plan's echo type: device memory if echo_on_device != 0,
 *                  else host memory (pinned for full copy speed) that the server
 *                  uploads into its arena on the scan's stream
 *   image_dst      device float2 [nx][ny][nz], written
 *   The caller must keep every buffer unchanged until sar_poll reports the
 *   ticket done.  Requests are admitted in arrival order as soon as their
 *   memory (sar_plan_workspace_bytes, plus the uploaded inputs for host
 *   inputs) fits in the arena, with at most 32 scans in flight.  The scans
 *   admitted together (up to 16) form one unit: one scan runs its own
 *   kernels, several run in fused launches as in a batch; each unit goes to
 *   the least-loaded stream, so units overlap on the device.
 *   Errors: SAR_ERR_INVALID (arguments, plan on another device),
 *   SAR_ERR_NOMEM (the request alone exceeds the whole budget; a request
 *   that merely does not fit yet waits), SAR_ERR_BUSY (server shutting down).
 *
 * sar_poll: non-blocking.  *done = 0 while the scan is queued or running.
 *   When it has finished, *done = 1, *latency_s (if not NULL) = seconds from
 *   sar_submit to the completion of the scan's last kernel, the ticket is
 *   released (a later poll of it gives SAR_ERR_NOT_FOUND), and the return
 *   value is the scan's own status (SAR_OK, or the error it failed with,
 *   described by sar_last_error()).
 *
 * sar_server_destroy: waits until every submitted scan has finished, then
 *   releases the arena, streams and thread.  NULL is accepted. */
sar_status sar_server_create(int device, size_t hbm_budget_bytes, sar_server* out);
sar_status sar_submit(sar_server server, sar_plan plan, const double* pos_xyz, int64_t n_pos, const void* echo,
                      int echo_on_device, float echo_scale, void* image_dst, uint64_t* ticket);
sar_status sar_poll(sar_server server, uint64_t ticket, int* done, double* latency_s);
sar_status sar_server_destroy(sar_server server);

/* Thread-local description of the last failure on this thread. */
const char* sar_last_error(void);

/* Library version string. */
const char* sar_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SAR_H_ */
