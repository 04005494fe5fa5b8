// Fused tiled G apply / residual instantiated for d = 2 (see tile_impl.h).
#include "tile_impl.h"

namespace hpg {
namespace dev {
HPG_TILE_INST(double, 2, MODE_APPLY)
HPG_TILE_INST(double, 2, MODE_RES)
HPG_TILE_INST(float, 2, MODE_APPLY)
HPG_TILE_INST(float, 2, MODE_RES)
}  // namespace dev
}  // namespace hpg
