// Gridding kernel instantiation for a 4-tap Kaiser-Bessel kernel.
#include "k_grid_impl.hpp"

namespace sar {
SAR_INSTANTIATE_GRID(4)
}  // namespace sar
