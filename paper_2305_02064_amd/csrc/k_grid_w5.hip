// Gridding kernel instantiation for a 5-tap Kaiser-Bessel kernel.
#include "k_grid_impl.hpp"

namespace sar {
SAR_INSTANTIATE_GRID(5)
}  // namespace sar
