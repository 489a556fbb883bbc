// Instantiations of the FP64 three-sweep pass: plain sweeps, optionally
// with the fused residual of the input iterate or of either intermediate
// iterate.
#include "sweep3.h"

namespace j3d {
namespace sweep_detail {

hipError_t dispatch_sweep3_f64(unsigned flags, const TileCfg& c, const GridArgs& g, double* partials,
                               const int* done, hipStream_t st) {
  switch (flags) {
    case F_WRITE: return by_shape3<double, F_WRITE>(c, g, partials, done, st);
    case F_WRITE | F_RES: return by_shape3<double, F_WRITE | F_RES>(c, g, partials, done, st);
    case F_WRITE | F_RES1: return by_shape3<double, F_WRITE | F_RES1>(c, g, partials, done, st);
    case F_WRITE | F_RES2: return by_shape3<double, F_WRITE | F_RES2>(c, g, partials, done, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t dispatch_sweep3_batch_f64(unsigned flags, const TileCfg& c, const GridArgs* table, int ngrids,
                                     int ntiles, const TileSlot* slots, int nslots, double* partials,
                                     const int* done, hipStream_t st) {
  switch (flags) {
    case F_WRITE: return by_shape3_batch<double, F_WRITE>(c, table, ngrids, ntiles, slots, nslots, partials, done, st);
    case F_WRITE | F_RES:
      return by_shape3_batch<double, F_WRITE | F_RES>(c, table, ngrids, ntiles, slots, nslots, partials, done, st);
    case F_WRITE | F_RES1:
      return by_shape3_batch<double, F_WRITE | F_RES1>(c, table, ngrids, ntiles, slots, nslots, partials, done, st);
    case F_WRITE | F_RES2:
      return by_shape3_batch<double, F_WRITE | F_RES2>(c, table, ngrids, ntiles, slots, nslots, partials, done, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sweep_detail
}  // namespace j3d
