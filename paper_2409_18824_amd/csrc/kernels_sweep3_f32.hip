// Instantiations of the FP32 three-sweep pass, single-grid and batched: the
// correction sweeps of the mixed-precision solve and of the server (first
// pass from a zero iterate, middle passes, last pass added into the FP64
// field).
#include "sweep3.h"

namespace j3d {
namespace sweep_detail {

hipError_t dispatch_sweep3_f32(unsigned flags, const TileCfg& c, const GridArgs& g, double* partials,
                               const int* done, hipStream_t st) {
  switch (flags) {
    case F_WRITE: return by_shape3<float, F_WRITE>(c, g, partials, done, st);
    case F_WRITE | F_FIRST: return by_shape3<float, F_WRITE | F_FIRST>(c, g, partials, done, st);
    case F_LAST: return by_shape3<float, F_LAST>(c, g, partials, done, st);
    case F_LAST | F_FIRST: return by_shape3<float, F_LAST | F_FIRST>(c, g, partials, done, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t dispatch_sweep3_batch_f32(unsigned flags, const TileCfg& c, const GridArgs* table, int ngrids,
                                     int ntiles, const TileSlot* slots, int nslots, double* partials,
                                     const int* done, hipStream_t st) {
  switch (flags) {
    case F_WRITE: return by_shape3_batch<float, F_WRITE>(c, table, ngrids, ntiles, slots, nslots, partials, done, st);
    case F_WRITE | F_FIRST:
      return by_shape3_batch<float, F_WRITE | F_FIRST>(c, table, ngrids, ntiles, slots, nslots, partials, done, st);
    case F_LAST: return by_shape3_batch<float, F_LAST>(c, table, ngrids, ntiles, slots, nslots, partials, done, st);
    case F_LAST | F_FIRST:
      return by_shape3_batch<float, F_LAST | F_FIRST>(c, table, ngrids, ntiles, slots, nslots, partials, done, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sweep_detail
}  // namespace j3d
