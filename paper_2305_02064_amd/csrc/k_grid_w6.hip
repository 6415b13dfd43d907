// Gridding kernel instantiation for a 6-tap Kaiser-Bessel kernel.
#include "k_grid_impl.hpp"

namespace sar {
SAR_INSTANTIATE_GRID(6)
}  // namespace sar
