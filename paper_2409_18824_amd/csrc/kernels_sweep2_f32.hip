// Instantiations of the FP32 two-sweep pass: the correction sweeps of the
// mixed-precision solve (first pair from a zero iterate, middle pairs, last
// pair added into the FP64 field).
#include "sweep2.h"

namespace j3d {
namespace sweep_detail {

hipError_t dispatch_sweep2_f32(unsigned flags, const Launch& L) {
  switch (flags) {
    case F_WRITE: return by_rows2<float, F_WRITE>(L);
    case F_WRITE | F_FIRST: return by_rows2<float, F_WRITE | F_FIRST>(L);
    case F_LAST: return by_rows2<float, F_LAST>(L);
    case F_LAST | F_FIRST: return by_rows2<float, F_LAST | F_FIRST>(L);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sweep_detail
}  // namespace j3d
