// Instantiations of the two-sweep (temporally blocked) FP64 pass.
#include "sweep2.h"

namespace j3d {
namespace sweep_detail {

namespace {

template <int BY, int VAR, unsigned FL>
hipError_t go2(const Launch& L) {
  constexpr int TR = BY * rows_per_thread(VAR);
  if constexpr (TR < 4 || TR > 32) {
    return hipErrorInvalidValue;
  } else {
  const GridArgs& g = *L.one;
  int grid = virtual_tiles(g.tiles_x * g.tiles_y * g.tiles_z, g.order, g.chunk);
  if (L.c->persistent) {
    static int cap = 0;
    if (cap == 0) cap = resident_blocks(k_sweep2_one<BY, VAR, FL>, WAVE * BY);
    grid = min(grid, cap);
  }
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_sweep2_one<BY, VAR, FL>), dim3(grid), dim3(WAVE, BY), 0, L.st, g, L.partials,
                     L.done);
  return hipGetLastError();
  }
}

// Supported (rows, rows per thread): block heights 4 to 32 rows.
template <int BY, unsigned FL>
hipError_t by_variant2(const Launch& L) {
  switch (L.c->variant) {
    case 0: return go2<BY, 0, FL>(L);
    case 4: return go2<BY, 4, FL>(L);
    case 2: return go2<BY, 2, FL>(L);
    case 6: return go2<BY, 6, FL>(L);
    case 16: return go2<BY, 16, FL>(L);
    case 20: return go2<BY, 20, FL>(L);
    default: return hipErrorInvalidValue;
  }
}

template <unsigned FL>
hipError_t by_rows2(const Launch& L) {
  switch (L.c->rows) {
    case 1: return by_variant2<1, FL>(L);
    case 2: return by_variant2<2, FL>(L);
    case 4: return by_variant2<4, FL>(L);
    case 8: return by_variant2<8, FL>(L);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t dispatch_sweep2(unsigned flags, const Launch& L) {
  if (L.batch) return hipErrorInvalidValue;
  switch (flags) {
    case F_WRITE: return by_rows2<F_WRITE>(L);
    case F_WRITE | F_RES: return by_rows2<F_WRITE | F_RES>(L);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sweep_detail
}  // namespace j3d
