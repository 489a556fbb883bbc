// jacobi3d_sweep3_noalloc: the three-sweep pass with its fused residual,
// for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, hosts that forbid hipMalloc).
//
// jacobi3d_sweep3 keeps the per-tile partial sums of the residual in library
// scratch that it allocates on first use.  This entry point keeps them in a
// fixed array in device global memory instead, sized for kNoAllocTiles
// tiles: the code object places one copy of it on every GPU the library
// runs on, where it stays until the process ends.  Host code never uses the
// array's name as an address (on the host that name is a stand-in, not a
// device pointer): the device copy's address is looked up once per device
// with hipGetSymbolAddress and kept in g_scratch_ptr.
//
// The kernels are those of jacobi3d_sweep3 with the same tile shape, so the
// output and the norm are bit-identical to it.  Every slot the reduction
// reads is written by the pass just before it, so nothing needs clearing
// between calls.  Calls that overlap in time on one GPU (concurrent streams
// or threads) share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "runtime.h"

namespace {

constexpr int kNoAllocTiles = 65536;  // 512 KiB of FP64 partials per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kNoAllocTiles];

std::mutex g_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up on the first
// call with the device current.
int scratch_address(double** out) {
  int dev = 0;
  J3D_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return j3d::fail(J3D_EINVAL, "device ordinal %d beyond the %d this entry point supports", dev,
                     kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return j3d::hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (p == nullptr) return j3d::fail(J3D_EHIP, "hipGetSymbolAddress(scratch) returned null");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return J3D_OK;
}

}  // namespace

using namespace j3d;

extern "C" int jacobi3d_sweep3_noalloc(const j3d_array* u_in, j3d_array* u_out, const j3d_array* f,
                                       double h, uint32_t flags, double* resid_out, void* stream) {
  if (resid_out == nullptr) return fail(J3D_EINVAL, "resid_out: null pointer");
  if ((flags & J3D_HOST_RESULT) != 0)
    return fail(J3D_EINVAL, "J3D_HOST_RESULT is not accepted: resid_out must be a device address");
  Sweep3Call k;
  J3D_TRY(check_sweep3_call(u_in, u_out, f, h, flags, resid_out, &k));
  const long long nt = (long long)k.g.tiles_x * k.g.tiles_y * k.g.tiles_z;
  if (nt > kNoAllocTiles)
    return fail(J3D_EINVAL, "grid %d x %d x %d needs %lld tile partials, more than the %d of the static scratch",
                k.a.nx(), k.a.ny(), k.a.nz(), nt, kNoAllocTiles);
  double* partials = nullptr;
  J3D_TRY(scratch_address(&partials));
  hipStream_t st = static_cast<hipStream_t>(stream);
  J3D_HIP(launch_sweep3_one(J3D_F64, F_WRITE | k.res_flag, k.cfg, k.g, partials, nullptr, st));
  J3D_HIP(launch_reduce_one(partials, 0, (int)nt, resid_out, nullptr, 0.0, 0, nullptr, nullptr, nullptr, st));
  return J3D_OK;
}
