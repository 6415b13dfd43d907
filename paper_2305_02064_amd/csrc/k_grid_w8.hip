// Gridding kernel instantiation for a 8-tap Kaiser-Bessel kernel.
#include "k_grid_impl.hpp"

namespace sar {
SAR_INSTANTIATE_GRID(8)
}  // namespace sar
