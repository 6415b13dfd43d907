// Dispatch of the gridding kernel over the compiled kernel widths.
#include "sar_internal.hpp"

namespace sar {

#define SAR_DECLARE_GRID(W)                                                                      \
  sar_status launch_gridding_w##W(const Plan& p, const void* d_echo, float echo_scale,           \
                                  const Workspace& ws, float2* grid, LaunchSink& sink);
SAR_DECLARE_GRID(3)
SAR_DECLARE_GRID(4)
SAR_DECLARE_GRID(5)
SAR_DECLARE_GRID(6)
SAR_DECLARE_GRID(7)
SAR_DECLARE_GRID(8)

sar_status launch_gridding(const Plan& p, const void* d_echo, float echo_scale, const Workspace& ws, float2* grid,
                           LaunchSink& sink) {
  switch (p.w) {
    case 3: return launch_gridding_w3(p, d_echo, echo_scale, ws, grid, sink);
    case 4: return launch_gridding_w4(p, d_echo, echo_scale, ws, grid, sink);
    case 5: return launch_gridding_w5(p, d_echo, echo_scale, ws, grid, sink);
    case 6: return launch_gridding_w6(p, d_echo, echo_scale, ws, grid, sink);
    case 7: return launch_gridding_w7(p, d_echo, echo_scale, ws, grid, sink);
    case 8: return launch_gridding_w8(p, d_echo, echo_scale, ws, grid, sink);
    default: return fail(SAR_ERR_UNSUPPORTED, "kernel width not compiled");
  }
}

}  // namespace sar
