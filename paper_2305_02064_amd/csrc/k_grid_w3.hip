// Gridding kernel instantiation for a 3-tap Kaiser-Bessel kernel.
#include "k_grid_impl.hpp"

namespace sar {
SAR_INSTANTIATE_GRID(3)
}  // namespace sar
