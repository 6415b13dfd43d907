"""Benchmark of the per-scan image formation on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --copy-calibration BYTES

Workload: one large freehand scan -- 2Tx x 4Rx array, 256 frequencies over
77-81 GHz, 512 x 256 shots along a smooth seeded random-walk trajectory
(1 048 576 virtual samples), image 512 x 256 x 256 voxels (complex64).  A step
is one sar_reconstruct call: geometry + sort, compensation + gridding, 2-D
FFT, k_z filter + Stolt, inverse 2-D FFT, with inputs already resident in
HBM.  Prints one JSON line.

--copy-calibration runs only a plain device copy (y = -x over float32) of
BYTES bytes, three times: the reference for scaling the HBM byte counters
(FETCH_SIZE, WRITE_SIZE) of a profiled run to bytes.
"""

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxels/s + scans/s & p99 latency (served vs plain GPU) at ≤1e-3 rel-L2 vs FP64"
HBM_PEAK_GBS = 8000.0
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_gridding_freehand-512x256x256.md")
GRID_SOURCES = ["k_grid_impl.hpp", "k_grid_union.hpp", "device_common.hpp", "sar_internal.hpp"]


def grid_kernel_hash():
    h = hashlib.sha256()
    for f in GRID_SOURCES:
        with open(os.path.join(ROOT, "paper_2305_02064_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic():
    """HBM bytes per gridding launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    if not os.path.exists(PMC_FILE):
        return None
    txt = open(PMC_FILE).read()
    m_h = re.search(r"kernel_source_sha:\s*([0-9a-f]+)", txt)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_h or not m_b or m_h.group(1) != grid_kernel_hash():
        return None
    return float(m_b.group(1))


def cpu_model():
    """The host CPU's model name with its family, model, clock and cache
    (first processor entry of /proc/cpuinfo; virtual machines often report a
    bare vendor name, which the family and model numbers then identify)."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not line.strip():
                    break  # end of the first processor entry
                k, _, v = line.partition(":")
                info.setdefault(k.strip(), v.strip())
    except OSError:
        return "unknown"
    name = info.get("model name", "unknown")
    extra = [f"{k} {info[k]}" for k in ("cpu family", "model", "cpu MHz", "cache size") if k in info]
    return f"{name} ({', '.join(extra)})" if extra else name


def tiny_oracle_single_core():
    """The FP64 oracle on the tiny scan with one BLAS thread, median of 3 (s)."""
    import numpy as np
    import oracle
    from sarsynth import config1_scan
    from threadpoolctl import threadpool_limits
    scan = config1_scan(0)
    ts = []
    with threadpool_limits(limits=1):
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, scan.grid)
            ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def tiny_bpa_oracle(planes=1):
    """The FP64 oracle's direct back-projection (exact ranges) of the tiny
    scan on the host, timed on `planes` of its z planes and extrapolated to
    the whole image (s)."""
    import dataclasses
    import oracle
    from sarsynth import config1_scan
    scan = config1_scan(0)
    g = scan.grid
    sub = dataclasses.replace(g, nz=planes)
    t0 = time.perf_counter()
    oracle.bpa(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, sub)
    t = time.perf_counter() - t0
    return t * g.nz / planes, f"{planes} of {g.nz} z planes ({t:.1f} s), extrapolated"


def cpu_baseline(scan, echo_host_fn):
    """The FP64 oracle (direct sums) timed on a bounded sample of the same scan:
    the 2-D non-uniform DFT for one of the N_f frequencies, the direct Stolt
    sum for 4 of the N_y k_y rows, and the exact inverse DFT in full; the total
    is extrapolated to the whole scan."""
    import numpy as np
    import oracle
    g = scan.grid
    nf = scan.n_freq
    k_sample = 1
    rows = 4
    echo_s = echo_host_fn(k_sample)                      # [n_pos, n_pair, k]
    k = oracle.wavenumber(scan.freq)
    t0 = time.perf_counter()
    xv, yv, dxx, dyy, dzz = oracle.virtual_samples(scan.pos, scan.tx_xy, scan.rx_xy, g.z_ref)
    beta = oracle.residual_path(dxx, dyy, dzz, g.z_ref, g.z_focus).ravel()
    shat = oracle.compensate(echo_s.reshape(-1, k_sample), k[:k_sample], beta)
    kx, ky, xc, yc = oracle.mode_axes(g.nx, g.ny, g.x0, g.y0, g.dx, g.dy)
    spec_part = oracle.nudft2(shat, xv.ravel(), yv.ravel(), kx, ky, xc, yc, block=32768)
    t_nudft = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    spec_rows = (rng.standard_normal((rows, g.nx, nf)) + 1j * rng.standard_normal((rows, g.nx, nf)))
    t0 = time.perf_counter()
    kz, mask = oracle.axial_wavenumber(k, kx, ky[:rows])
    filt = oracle.rma_filter(spec_rows, kz, mask, g.z_ref)
    zc = oracle.stolt_direct(filt, kz, mask, g.z0 + g.dz * np.arange(g.nz))
    t_stolt = time.perf_counter() - t0
    zfull = np.zeros((g.ny, g.nx, g.nz), np.complex128)
    zfull[:rows] = zc
    t0 = time.perf_counter()
    oracle.idft2(zfull)
    t_idft = time.perf_counter() - t0
    del spec_part
    total = t_nudft * nf / k_sample + t_stolt * g.ny / rows + t_idft
    threads = int(os.environ.get("OPENBLAS_NUM_THREADS", os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0)))))
    t_single = tiny_oracle_single_core()
    t_bpa, bpa_how = tiny_bpa_oracle()
    return {
        "value": g.n_voxels / total,
        "unit": "voxels/s",
        "cores": threads,
        "cpu_model": cpu_model(),
        "host_cores_available": len(os.sched_getaffinity(0)),
        "tiny_scan_oracle_single_core_ms": t_single * 1e3,
        "tiny_scan_bpa_oracle_s": t_bpa,
        "tiny_scan_bpa_oracle_sample": bpa_how,
        "kind": "oracle",
        "sample": (f"direct 2-D NUDFT of all {scan.n_pos * scan.n_pair} virtual samples for {k_sample} of {nf} "
                   f"frequencies ({t_nudft:.1f} s), direct Stolt sum for {rows} of {g.ny} k_y rows "
                   f"({t_stolt:.1f} s), exact inverse DFT in full ({t_idft:.1f} s); extrapolated to "
                   f"{total:.0f} s per scan; BLAS threads {threads}, exp single-threaded"),
        "seconds_per_scan_extrapolated": total,
    }


def oracle_uneven(n_small=8, n_random=4, full_macs=1.2e11, seed=0):
    """The FP64 oracle beside the GPU on scans of the uneven batch: the n_small
    cheapest of the 64 (by direct-NUDFT size N_v x S^2 x N_f) and n_random others
    drawn with a fixed seed.  A scan whose NUDFT exceeds full_macs complex
    multiply-adds is timed on a sample (the NUDFT for enough frequencies to
    reach about full_macs, the Stolt sum for 4 k_y rows, the inverse DFT in full)
    and extrapolated; the others run the whole oracle.  Echoes are seeded random
    values (the oracle's work does not depend on them)."""
    import numpy as np
    import torch
    import oracle
    from paper_2305_02064_amd import sar
    from sarsynth import config4_scan
    scans = [config4_scan(sd, with_echo=False) for sd in range(64)]
    cost = [sc.n_pos * sc.n_pair * sc.grid.nx * sc.grid.ny * sc.n_freq for sc in scans]
    order = sorted(range(64), key=lambda i: cost[i])
    rng = np.random.default_rng(seed)
    pick = order[:n_small] + sorted(rng.choice(order[n_small:], n_random, replace=False).tolist())
    rows_out = []
    dev = torch.device("cuda", 0)
    for i in pick:
        sc = scans[i]
        g = sc.grid
        er = np.random.default_rng(100 + i)
        echo = (er.standard_normal((sc.n_pos, sc.n_pair, sc.n_freq))
                + 1j * er.standard_normal((sc.n_pos, sc.n_pair, sc.n_freq)))
        plan = sar.Plan(sc.tx_xy, sc.rx_xy, sc.freq, g, sc.n_pos)
        pos_d = torch.from_numpy(np.ascontiguousarray(sc.pos)).to(dev)
        echo_d = torch.from_numpy(echo.astype(np.complex64)).to(dev)
        img = plan.new_image()
        plan.reconstruct(pos_d, echo_d, img)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            plan.reconstruct(pos_d, echo_d, img)
        torch.cuda.synchronize()
        gpu_ms = (time.perf_counter() - t0) / 5 * 1e3
        plan.close()
        if cost[i] <= full_macs:
            t0 = time.perf_counter()
            oracle.reconstruct_direct(sc.pos, sc.tx_xy, sc.rx_xy, sc.freq, echo, g)
            cpu_s = time.perf_counter() - t0
            how = "full"
        else:
            kf = max(1, int(full_macs // (sc.n_pos * sc.n_pair * g.nx * g.ny)))
            k = oracle.wavenumber(sc.freq)
            t0 = time.perf_counter()
            xv, yv, dxx, dyy, dzz = oracle.virtual_samples(sc.pos, sc.tx_xy, sc.rx_xy, g.z_ref)
            beta = oracle.residual_path(dxx, dyy, dzz, g.z_ref, g.z_focus).ravel()
            shat = oracle.compensate(echo[:, :, :kf].reshape(-1, kf), k[:kf], beta)
            kx, ky, xc, yc = oracle.mode_axes(g.nx, g.ny, g.x0, g.y0, g.dx, g.dy)
            oracle.nudft2(shat, xv.ravel(), yv.ravel(), kx, ky, xc, yc, block=32768)
            t_nu = time.perf_counter() - t0
            rows = 4
            spec_rows = er.standard_normal((rows, g.nx, sc.n_freq)) + 1j * er.standard_normal((rows, g.nx, sc.n_freq))
            t0 = time.perf_counter()
            kz, mask = oracle.axial_wavenumber(k, kx, ky[:rows])
            zc = oracle.stolt_direct(oracle.rma_filter(spec_rows, kz, mask, g.z_ref), kz, mask,
                                     g.z0 + g.dz * np.arange(g.nz))
            t_st = time.perf_counter() - t0
            zfull = np.zeros((g.ny, g.nx, g.nz), np.complex128)
            zfull[:rows] = zc
            t0 = time.perf_counter()
            oracle.idft2(zfull)
            t_id = time.perf_counter() - t0
            cpu_s = t_nu * sc.n_freq / kf + t_st * g.ny / rows + t_id
            how = f"extrapolated ({kf} of {sc.n_freq} frequencies, {rows} of {g.ny} rows)"
        rows_out.append({"seed": i, "side": int(round(np.sqrt(sc.n_pos))), "n_freq": sc.n_freq,
                         "image": [g.nx, g.ny, g.nz], "gpu_ms": gpu_ms, "oracle_s": cpu_s, "oracle": how,
                         "speedup": cpu_s * 1e3 / gpu_ms})
        print(f"oracle on uneven scan {i}: {cpu_s:.2f} s ({how}), GPU {gpu_ms:.3f} ms", file=sys.stderr, flush=True)
    threads = int(os.environ.get("OPENBLAS_NUM_THREADS", os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0)))))
    return {"scans": rows_out, "cores": threads,
            "selection": f"{n_small} cheapest of the 64 uneven-batch scans plus {n_random} others (seed {seed})"}


def serving_bench(big_scan, big_pos, big_plan, n_requests, rates, host_rates=(), seed=0):
    """Served vs plain per-scan path on a stream of scans shaped like the
    serving workload: 95% scans of the uneven batch (64 distinct scans, side
    64-256 positions, 64-256 frequencies), 5% scans of the large freehand size.
    Echoes are seeded random device tensors (the kernels' work does not depend
    on the values; accuracy is covered by the parity tests).

    plain:  one sar_reconstruct per scan in arrival order on one stream;
    served: sar_submit of every scan to one server (continuous admission under
            an HBM budget, scans overlapping on four streams).
    Saturation: all requests present at t=0.  Poisson: arrivals at each rate,
    latency = arrival to completion of the scan's last kernel."""
    import numpy as np
    import torch
    from paper_2305_02064_amd import sar
    from sarsynth import config4_scan

    dev = torch.device("cuda", 0)
    distinct = []
    for sd in range(64):
        sc = config4_scan(sd, with_echo=False)
        g = torch.Generator(device=dev)
        g.manual_seed(10_000 + sd)
        shape = (sc.n_pos, sc.n_pair, sc.n_freq)
        echo = torch.complex(torch.randn(shape, generator=g, device=dev), torch.randn(shape, generator=g, device=dev))
        pos = torch.from_numpy(np.ascontiguousarray(sc.pos)).to(dev)
        plan = sar.Plan(sc.tx_xy, sc.rx_xy, sc.freq, sc.grid, sc.n_pos, workspace=False)
        distinct.append((plan, pos, echo, sc.grid.n_voxels))
    distinct.append((big_plan, big_pos, big_scan.echo, big_scan.grid.n_voxels))
    rng = np.random.default_rng(seed)
    seq = [64 if rng.random() < 0.05 else int(rng.integers(64)) for _ in range(n_requests)]
    ws_max = max(sar.sar_plan_workspace_bytes(distinct[i][0].handle, distinct[i][1].shape[0]) for i in set(seq))
    ws = torch.empty(ws_max + 256, dtype=torch.uint8, device=dev)
    ws = ws[(-ws.data_ptr()) % 256:][:ws_max]
    images = {i: distinct[i][0].new_image() for i in set(seq)}
    stream = torch.cuda.current_stream()
    voxels = sum(distinct[i][3] for i in seq)

    def plain_one(i):
        plan, pos, echo, _ = distinct[i]
        sar.sar_reconstruct(plan.handle, pos, pos.shape[0], echo, 1.0, images[i], ws, stream)

    # warm both paths on every distinct scan of the sequence
    for i in set(seq):
        plain_one(i)
    torch.cuda.synchronize()
    budget = max(24 << 30, 4 * ws_max)
    srv = sar.Server(budget)
    for t in [srv.submit(distinct[i][0], distinct[i][1], distinct[i][2], images[i]) for i in set(seq)]:
        srv.wait(t)

    # saturation throughput
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in seq:
        plain_one(i)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    tickets = [srv.submit(distinct[i][0], distinct[i][1], distinct[i][2], images[i]) for i in seq]
    lat_sat = [srv.wait(t)[0] for t in tickets]
    t_served = time.perf_counter() - t0

    def pct(v):
        return {"p50_ms": float(np.percentile(v, 50) * 1e3), "p99_ms": float(np.percentile(v, 99) * 1e3)}

    # fused batch of the 64 distinct uneven scans (one captured graph) vs the
    # same 64 scans through the plain path
    uneven = list(range(64))
    vox64 = sum(distinct[i][3] for i in uneven)
    for i in uneven:
        images.setdefault(i, distinct[i][0].new_image())
    batch = sar.Batch([distinct[i][0] for i in uneven])
    bpos = [distinct[i][1] for i in uneven]
    bech = [distinct[i][2] for i in uneven]
    bimg = [images[i] for i in uneven]
    for _ in range(2):
        batch.reconstruct(bpos, bech, bimg)
        for i in uneven:
            plain_one(i)
    reps = 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        batch.reconstruct(bpos, bech, bimg)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        for i in uneven:
            plain_one(i)
    torch.cuda.synchronize()
    t_plain64 = (time.perf_counter() - t0) / reps
    batched = {
        "workload": "64 distinct uneven scans (64-256 side, 64-256 freq) as one fused batch, captured graph",
        "plain": {"scans_per_s": 64 / t_plain64, "voxels_per_s": vox64 / t_plain64, "ms_per_64": t_plain64 * 1e3},
        "batched": {"scans_per_s": 64 / t_batch, "voxels_per_s": vox64 / t_batch, "ms_per_64": t_batch * 1e3},
        "speedup": t_plain64 / t_batch,
    }
    batch.close()

    out = {
        "workload": (f"{n_requests} requests: 95% uneven-batch scans (64 distinct, 64-256 side, 64-256 freq), "
                     f"5% 512x256-shot freehand scans; {len(set(seq))} distinct scans, random device echoes"),
        "voxels_per_request_mean": voxels / n_requests,
        "saturation": {
            "plain": {"scans_per_s": n_requests / t_plain, "voxels_per_s": voxels / t_plain},
            "served": {"scans_per_s": n_requests / t_served, "voxels_per_s": voxels / t_served, **pct(lat_sat)},
            "speedup": t_plain / t_served,
        },
        "poisson": [],
        "batched_uneven": batched,
        "hbm_budget_bytes": budget,
    }
    for rate in rates:
        arr = np.cumsum(rng.exponential(1.0 / rate, n_requests))
        # plain: each arrival launches its scan on the one stream; completion
        # seen by polling an event recorded behind it
        pending = []
        lat_p = []

        def retire(t0):
            keep = []
            for a, e in pending:
                if e.query():
                    lat_p.append(time.perf_counter() - t0 - a)
                else:
                    keep.append((a, e))
            pending[:] = keep

        t0 = time.perf_counter()
        for k, i in enumerate(seq):
            while time.perf_counter() - t0 < arr[k]:
                retire(t0)
            plain_one(i)
            e = torch.cuda.Event()
            e.record(stream)
            pending.append((arr[k], e))
            if k % 500 == 499:
                print(f"poisson {rate}/s plain: {k + 1} of {n_requests} submitted", file=sys.stderr, flush=True)
        while pending:
            retire(t0)
        t_p = time.perf_counter() - t0
        # served
        lat_s = []
        live = []
        t0 = time.perf_counter()
        for k, i in enumerate(seq):
            while time.perf_counter() - t0 < arr[k]:
                still = []
                for t in live:
                    done, lat, _ = srv.poll(t)
                    if done:
                        lat_s.append(lat)
                    else:
                        still.append(t)
                live = still
            live.append(srv.submit(distinct[i][0], distinct[i][1], distinct[i][2], images[i]))
            if k % 500 == 499:
                print(f"poisson {rate}/s served: {k + 1} of {n_requests} submitted", file=sys.stderr, flush=True)
        for t in live:
            lat_s.append(srv.wait(t)[0])
        t_s = time.perf_counter() - t0
        out["poisson"].append({"rate_per_s": rate, "plain": {"scans_per_s": n_requests / t_p, **pct(lat_p)},
                               "served": {"scans_per_s": n_requests / t_s, **pct(lat_s)}})
    # the same Poisson streams with every request's positions and echo starting
    # in pinned host memory (uploads counted in the latency).  Plain: each
    # arrival copies its inputs to the device on the one stream, then
    # reconstructs; served: the host tensors go to sar_submit, which stages the
    # uploads itself.
    if host_rates:
        hin = {i: (distinct[i][1].cpu().pin_memory(), distinct[i][2].cpu().pin_memory()) for i in set(seq)}
        mean_up = sum(hin[i][0].numel() * 8 + hin[i][1].numel() * 8 for i in seq) / n_requests
        out["poisson_host_input"] = {"mean_upload_bytes": mean_up, "rates": []}
        for rate in host_rates:
            arr = np.cumsum(rng.exponential(1.0 / rate, n_requests))
            pending = []
            lat_p = []

            def retire_h(t0):
                keep = []
                for a, e in pending:
                    if e.query():
                        lat_p.append(time.perf_counter() - t0 - a)
                    else:
                        keep.append((a, e))
                pending[:] = keep

            t0 = time.perf_counter()
            for k, i in enumerate(seq):
                while time.perf_counter() - t0 < arr[k]:
                    retire_h(t0)
                distinct[i][1].copy_(hin[i][0], non_blocking=True)
                distinct[i][2].copy_(hin[i][1], non_blocking=True)
                plain_one(i)
                e = torch.cuda.Event()
                e.record(stream)
                pending.append((arr[k], e))
                if k % 500 == 499:
                    print(f"poisson host-fed {rate}/s plain: {k + 1} of {n_requests} submitted", file=sys.stderr,
                          flush=True)
            while pending:
                retire_h(t0)
            t_p = time.perf_counter() - t0
            lat_s = []
            live = []
            t0 = time.perf_counter()
            for k, i in enumerate(seq):
                while time.perf_counter() - t0 < arr[k]:
                    still = []
                    for t in live:
                        done, lat, _ = srv.poll(t)
                        if done:
                            lat_s.append(lat)
                        else:
                            still.append(t)
                    live = still
                live.append(srv.submit(distinct[i][0], hin[i][0], hin[i][1], images[i]))
                if k % 500 == 499:
                    print(f"poisson host-fed {rate}/s served: {k + 1} of {n_requests} submitted", file=sys.stderr,
                          flush=True)
            for t in live:
                lat_s.append(srv.wait(t)[0])
            t_s = time.perf_counter() - t0
            out["poisson_host_input"]["rates"].append({
                "rate_per_s": rate, "offered_GB_per_s": rate * mean_up / 1e9,
                "plain": {"scans_per_s": n_requests / t_p, **pct(lat_p)},
                "served": {"scans_per_s": n_requests / t_s, **pct(lat_s)}})
        del hin

    # echoes starting in pinned host memory (uploads counted): the 16 smallest
    # uneven scans, 64 requests, all submitted at once
    small = sorted(range(64), key=lambda i: distinct[i][2].numel())[:16]
    host = {i: (distinct[i][1].cpu().pin_memory(), distinct[i][2].cpu().pin_memory()) for i in small}
    hseq = [small[j % 16] for j in range(64)]
    up_bytes = sum(host[i][0].numel() * 8 + host[i][1].numel() * 8 for i in hseq)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat_h = [srv.wait(t)[0] for t in [srv.submit(distinct[i][0], host[i][0], host[i][1], images[i]) for i in hseq]]
    t_h = time.perf_counter() - t0
    t0 = time.perf_counter()
    lat_d = [srv.wait(t)[0] for t in [srv.submit(distinct[i][0], distinct[i][1], distinct[i][2], images[i])
                                     for i in hseq]]
    t_d = time.perf_counter() - t0
    out["host_input"] = {
        "workload": "64 requests over the 16 smallest uneven scans, echo and positions in pinned host memory",
        "scans_per_s": 64 / t_h, "upload_GB_per_s": up_bytes / t_h / 1e9, **pct(lat_h),
        "pre_resident": {"scans_per_s": 64 / t_d, **pct(lat_d)},
    }
    srv.close()
    for plan, _, _, _ in distinct[:64]:
        plan.close()
    return out


def comparison_tiny(reps=20):
    """The paper's comparison (Table I) on the tiny scan, all on the GPU: the
    proposed method, the same range-migration pipeline without compensation,
    and direct back-projection with exact ranges; milliseconds per image."""
    import numpy as np
    import torch
    from paper_2305_02064_amd import sar
    from sarsynth import config1_scan
    scan = config1_scan(0)
    pos = torch.from_numpy(np.ascontiguousarray(scan.pos)).cuda()
    echo = torch.from_numpy(np.ascontiguousarray(scan.echo)).cuda()
    plan = sar.Plan(scan.tx_xy, scan.rx_xy, scan.freq, scan.grid, scan.n_pos)
    raw = sar.Plan(scan.tx_xy, scan.rx_xy, scan.freq, scan.grid, scan.n_pos, flags=sar.SAR_NO_COMPENSATION)
    # the same scan as a one-item fused batch: one captured HIP graph replayed
    # per call instead of 14 separate launches
    one = sar.Batch([plan])
    img1 = [plan.new_image()]
    out = {}
    for name, fn in (("proposed", lambda: plan.reconstruct(pos, echo)),
                     ("proposed_graph", lambda: one.reconstruct([pos], [echo], img1)),
                     ("rma_uncompensated", lambda: raw.reconstruct(pos, echo)),
                     ("bpa", lambda: plan.backproject(pos, echo))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        out[name + "_ms"] = (time.perf_counter() - t0) * 1e3 / reps
    out["workload"] = "tiny scan: 32x16 shots x 8 pairs x 32 freq -> 32x32x16 voxels"
    # the FP64 oracle on the same scan (host cores), median of 3
    import oracle
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.reconstruct_direct(scan.pos, scan.tx_xy, scan.rx_xy, scan.freq, scan.echo, scan.grid)
        ts.append(time.perf_counter() - t0)
    out["oracle_cpu_ms"] = float(np.median(ts)) * 1e3
    out["oracle_cpu_threads"] = int(os.environ.get("OPENBLAS_NUM_THREADS", os.environ.get(
        "OMP_NUM_THREADS", len(os.sched_getaffinity(0)))))
    one.close()
    plan.close()
    raw.close()
    return out


def clustered_bench(plan, pos, echo, image, stream, reps=10):
    """The large scan with its middle quarter of shots (32 768) moved to one
    position: eight cells of the gridding grid then hold 32 768 samples each.
    Same echo values (the kernels' work does not depend on them); per-stage
    milliseconds, mean of reps calls."""
    import torch
    from paper_2305_02064_amd import sar
    n = pos.shape[0]
    p2 = pos.clone()
    q0 = 3 * n // 8
    p2[q0:q0 + n // 4] = pos[n // 2]
    plan.reconstruct(p2, echo, image)
    torch.cuda.synchronize()
    sar.sar_plan_set_timing(plan.handle, True)
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.reconstruct(p2, echo, image)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    stage_ms, n_calls = sar.sar_plan_stage_times(plan.handle)
    sar.sar_plan_set_timing(plan.handle, False)
    return {"workload": f"large scan, shots {q0}..{q0 + n // 4 - 1} at one position", "ms_per_scan": ms,
            "stage_ms": {k: v / max(n_calls, 1) for k, v in stage_ms.items()}}


def slab_bench(scan, pos, echo, n_slabs=4, reps=5):
    """The large scan with a reference depth per depth slab (n_slabs sub-plans:
    one front end per slab, each slab's back end on its planes); milliseconds
    per scan, mean of reps calls."""
    import torch
    from paper_2305_02064_amd import sar
    plan = sar.Plan(scan.tx_xy, scan.rx_xy, scan.freq, scan.grid, scan.n_pos, n_slabs=n_slabs)
    image = plan.new_image()
    plan.reconstruct(pos, echo, image)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.reconstruct(pos, echo, image)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    plan.close()
    return {"workload": f"large scan, {n_slabs} depth slabs", "n_slabs": n_slabs, "ms_per_scan": ms}


def copy_calibration(nbytes, launches=3):
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(launches):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": x.numel() * 4, "bytes_written": y.numel() * 4,
                                           "launches": launches}}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES")
    ap.add_argument("--no-serving", action="store_true", help="skip the tiny-scan comparison and the serving runs")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-rates", type=str, default="50,200,500")
    ap.add_argument("--serve-host-rates", type=str, default="",
                    help="Poisson rates for a sweep with every request's inputs in pinned host memory (opt-in)")
    ap.add_argument("--oracle-uneven", action="store_true",
                    help="also time the FP64 oracle beside the GPU on 12 scans of the uneven batch (minutes of CPU)")
    ap.add_argument("--no-slabs", action="store_true", help="skip the depth-slab timing of the large scan")
    ap.add_argument("--clustered", action="store_true",
                    help="also time the large scan with a quarter of its shots at one position (a dwelling hand)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library forms each image on a single device (got --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    import numpy as np
    import torch
    from paper_2305_02064_amd import sar
    from sarsynth import config2_scan

    dev = torch.device("cuda", 0)
    t_gen = time.perf_counter()
    scan = config2_scan(args.seed, device=dev)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    g = scan.grid
    pos = torch.from_numpy(np.ascontiguousarray(scan.pos)).to(dev)
    echo = scan.echo
    plan = sar.Plan(scan.tx_xy, scan.rx_xy, scan.freq, g, scan.n_pos)
    info = plan.info
    image = plan.new_image()
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        plan.reconstruct(pos, echo, image)
    torch.cuda.synchronize()

    sar.sar_plan_set_timing(plan.handle, True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        plan.reconstruct(pos, echo, image)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stage_ms, n_calls = sar.sar_plan_stage_times(plan.handle)
    sar.sar_plan_set_timing(plan.handle, False)
    step_ms = np.array([a.elapsed_time(b) for a, b in ev])

    ms_per_step = elapsed * 1e3 / args.steps
    voxels = g.n_voxels
    n_v = scan.n_pos * scan.n_pair
    nf = scan.n_freq
    grid_avg_ms = stage_ms["gridding"] / max(n_calls, 1)
    rec_bytes = {3: 48, 4: 48, 5: 64, 6: 64, 7: 80, 8: 80}[info["width"]]
    alg_bytes = n_v * nf * 8 + info["mx"] * info["my"] * nf * 8 + n_v * rec_bytes
    achieved = alg_bytes / (grid_avg_ms * 1e-3) / 1e9
    traffic = recorded_traffic()
    # a plain device copy of 1 GiB for context: what the memory system gives a
    # perfectly streaming kernel (read + write bytes over time)
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(10):
        dst.copy_(src)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbps = 10 * 2 * src.numel() * 4 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst
    out = {
        "metric": METRIC,
        "value": voxels / (ms_per_step * 1e-3),
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "freehand scan 512x256 shots x 2Tx4Rx x 256 freq (77-81 GHz) -> 512x256x256 voxels",
            "n_virtual_samples": n_v, "n_freq": nf, "image": [g.nx, g.ny, g.nz],
            "grid": [info["mx"], info["my"]], "kernel_width": info["width"], "stolt_grid": info["mz"],
            "echo": "complex64", "path": "plain per-scan sar_reconstruct, one stream",
        },
        "scans_per_s": 1e3 / ms_per_step,
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "stage_ms": {k: v / max(n_calls, 1) for k, v in stage_ms.items()},
        "roofline": {
            "bound": "hbm",
            "kernel": "gridding (compensation + Kaiser-Bessel spreading)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "timer": ("HIP events recorded on the launch stream around the gridding stage of every timed step "
                      "(split planning, spreading and combining kernels), mean over the steps"),
            "algorithmic_bytes_per_launch": alg_bytes,
            "measured_copy_GB_per_s": copy_gbps,
        },
        "input_generation_s": t_gen,
    }
    if not args.no_serving:
        out["comparison_tiny"] = comparison_tiny()
        out["serving"] = serving_bench(scan, pos, plan, args.serve_requests,
                                       [float(r) for r in args.serve_rates.split(",") if r],
                                       [float(r) for r in args.serve_host_rates.split(",") if r])
    if not args.no_cpu_baseline:
        def echo_host(kk):
            return echo[:, :, :kk].cpu().numpy().astype(np.complex128)
        out["cpu_baseline"] = cpu_baseline(scan, echo_host)
    if args.oracle_uneven:
        out["oracle_uneven"] = oracle_uneven()
    if args.clustered:
        out["clustered"] = clustered_bench(plan, pos, echo, image, stream)
    if not args.no_slabs:
        out["slabs"] = slab_bench(scan, pos, echo)
    print(json.dumps(out))
    plan.close()


if __name__ == "__main__":
    main()
