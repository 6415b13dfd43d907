// Gridding kernel instantiation for a 7-tap Kaiser-Bessel kernel.
#include "k_grid_impl.hpp"

namespace sar {
SAR_INSTANTIATE_GRID(7)
}  // namespace sar
