// The paper's 2D jacobi benchmark on gfx950: Jacobi iteration for Laplace's
// equation on a 2D grid u(0:nx+1, 0:ny+1) with the boundary values in the
// halo (Sec. "Flang performance comparison": 1024 x 1024, 100000
// iterations),
//   u'(i,j) = (((u(i-1,j) + u(i+1,j)) + u(i,j-1)) + u(i,j+1)) / 4,
// T sweeps per launch.
//
// The grid is small (8 MB per FP64 array at 1024^2) and stays in the caches,
// so a sweep costs little more than a launch: the kernel does T sweeps per
// launch, each wavefront on an independent tile held in registers.  Lane l,
// register r of a wavefront holds cell (x0 - T + l, y0 - T + r) of a 64 x R
// tile.  A sweep updates the tile's interior cells in place, rolling down the
// rows (the old value of the row above is kept in a temporary): x-neighbours
// come from the adjacent lanes (DPP wave shifts), y-neighbours from the
// registers of the rows above and below.  A cell whose neighbour lies outside
// the tile takes a wrong value, and a wrong value travels one cell per sweep,
// so after T sweeps the inner (64 - 2T) x (R - 2T) cells are exact: those are
// stored.  Tiles overlap by 2T columns and rows; there is no LDS and no
// barrier.  Halo cells, and the clamped cells beyond the halo, are never
// updated.  Each cell is computed with exactly the arithmetic above, so T
// sweeps per launch equal T single sweeps bit for bit.
#include <cstdlib>

#include "sweep.h"

namespace j3d {
namespace {

using sweep_detail::from_left;
using sweep_detail::from_right;
using sweep_detail::WAVE;

constexpr int kWavesPerBlock = 4;

template <int T, int R>
__global__ void __launch_bounds__(WAVE * kWavesPerBlock)
    k_jacobi2d(const double* __restrict__ in, double* __restrict__ out, int nx, int ny, int si, int so,
               int tiles_x, int ntiles, const int* __restrict__ done) {
  static_assert(2 * T < WAVE && 2 * T < R, "a tile needs inner cells");
  constexpr int W = WAVE - 2 * T;
  constexpr int H = R - 2 * T;
  if (done != nullptr && *done != 0) return;
  const int lane = threadIdx.x & (WAVE - 1);
  const int tile = blockIdx.x * kWavesPerBlock + (threadIdx.x / WAVE);
  if (tile >= ntiles) return;  // the whole wavefront leaves together
  const int tx = tile % tiles_x;
  const int ty = tile / tiles_x;
  const int x = tx * W + 1 - T + lane;  // column of this lane
  const int y0 = ty * H + 1 - T;        // row of register 0
  const int xc = min(max(x, 0), nx + 1);
  const bool x_in = x >= 1 && x <= nx;
  double v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int yc = min(max(y0 + r, 0), ny + 1);
    v[r] = in[xc + si * yc];
  }
#pragma unroll
  for (int s = 0; s < T; ++s) {
    double above = v[0];  // old value of the row above (row 0: none in the tile)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double left = from_left(v[r]);
      const double right = from_right(v[r]);
      const double below = r + 1 < R ? v[r + 1] : v[r];
      double t = left + right;
      t = t + above;
      t = t + below;
      const double nv = t / 4.0;
      const int y = y0 + r;
      above = v[r];
      v[r] = (x_in && y >= 1 && y <= ny) ? nv : v[r];
    }
  }
  const bool lane_out = lane >= T && lane < T + W && x_in;
#pragma unroll
  for (int r = T; r < T + H; ++r) {
    const int y = y0 + r;
    if (lane_out && y >= 1 && y <= ny) out[x + so * y] = v[r];
  }
}

// T sweeps per launch by a workgroup of BY wavefronts stacked in y, each
// holding R rows of a 64-column tile in registers (lane l, register r is
// cell (x0 - T + l, y0 - T + wy*R + r)).  Before every sweep each wavefront
// publishes its first and last row in LDS (two parity slots, one barrier
// per sweep), and the rows just outside its own are the neighbours' values
// of the previous sweep, so only the workgroup's outer T rows and the
// wavefront's outer T columns hold wrong values after T sweeps: the inner
// (64 - 2T) x (BY*R - 2T) cells are stored.  Same arithmetic per cell as
// k_jacobi2d.
template <int T, int R, int BY>
__global__ void __launch_bounds__(WAVE * BY)
    k_jacobi2d_wg(const double* __restrict__ in, double* __restrict__ out, int nx, int ny, int si, int so,
                  int tiles_x, const int* __restrict__ done) {
  constexpr int W = WAVE - 2 * T;
  constexpr int H = BY * R - 2 * T;
  static_assert(2 * T < WAVE && H > 0, "a tile needs inner cells");
  __shared__ double edge[2][BY][2][WAVE];
  if (done != nullptr && *done != 0) return;  // uniform over the launch
  const int lane = threadIdx.x & (WAVE - 1);
  const int wy = threadIdx.x / WAVE;
  const int tx = blockIdx.x % tiles_x;
  const int ty = blockIdx.x / tiles_x;
  const int x = tx * W + 1 - T + lane;
  const int y0 = ty * H + 1 - T + wy * R;  // row of register 0
  const int xc = min(max(x, 0), nx + 1);
  const bool x_in = x >= 1 && x <= nx;
  double v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = in[xc + si * min(max(y0 + r, 0), ny + 1)];
#pragma unroll
  for (int s = 0; s < T; ++s) {
    edge[s & 1][wy][0][lane] = v[0];
    edge[s & 1][wy][1][lane] = v[R - 1];
    __syncthreads();
    const double lo = wy > 0 ? edge[s & 1][wy - 1][1][lane] : v[0];      // row y0 - 1, old
    const double hi = wy < BY - 1 ? edge[s & 1][wy + 1][0][lane] : v[R - 1];  // row y0 + R, old
    double above = lo;  // old value of the row below index r (y - 1)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double left = from_left(v[r]);
      const double right = from_right(v[r]);
      const double below = r + 1 < R ? v[r + 1] : hi;
      double t = left + right;
      t = t + above;
      t = t + below;
      const double nv = t / 4.0;
      const int y = y0 + r;
      above = v[r];
      v[r] = (x_in && y >= 1 && y <= ny) ? nv : v[r];
    }
  }
  const bool lane_out = lane >= T && lane < T + W && x_in;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int br = wy * R + r;
    const int y = y0 + r;
    if (lane_out && br >= T && br < T + H && y >= 1 && y <= ny) out[x + so * y] = v[r];
  }
}

template <int T, int R, int BY>
hipError_t go2d_wg(const double* in, double* out, int nx, int ny, int si, int so, const int* done,
                   hipStream_t st) {
  constexpr int W = WAVE - 2 * T;
  constexpr int H = BY * R - 2 * T;
  const int tx = (nx + W - 1) / W;
  const int ty = (ny + H - 1) / H;
  hipLaunchKernelGGL((k_jacobi2d_wg<T, R, BY>), dim3(tx * ty), dim3(WAVE * BY), 0, st, in, out, nx, ny, si, so,
                     tx, done);
  return hipGetLastError();
}

// Sum of r^2 with r = (S - 4 u) / h^2 over one block of rows: thread q of
// the block takes columns q, q + 256, ... of each row in order; wave
// butterfly, wave-ordered sum, fixed slot per block.
constexpr int kResRows = 8;

__global__ void __launch_bounds__(256)
    k_laplace2d_res(const double* __restrict__ u, int nx, int ny, int su, double h2,
                    double* __restrict__ partials) {
  __shared__ double red[256 / WAVE];
  double acc = 0.0;
  const int j0 = 1 + blockIdx.x * kResRows;
  for (int j = j0; j < min(j0 + kResRows, ny + 1); ++j)
    for (int i = 1 + (int)threadIdx.x; i <= nx; i += 256) {
      const double* p = u + i + su * j;
      double t = p[-1] + p[1];
      t = t + p[-su];
      t = t + p[su];
      const double r = (t - 4.0 * p[0]) / h2;
      acc += r * r;
    }
  acc = sweep_detail::wave_sum(acc);
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = red[0];
#pragma unroll
    for (int w = 1; w < 256 / WAVE; ++w) tot += red[w];
    partials[blockIdx.x] = tot;
  }
}

template <int T, int R>
hipError_t go2d(const double* in, double* out, int nx, int ny, int si, int so, const int* done,
                hipStream_t st) {
  constexpr int W = WAVE - 2 * T;
  constexpr int H = R - 2 * T;
  const int tx = (nx + W - 1) / W;
  const int ty = (ny + H - 1) / H;
  const int ntiles = tx * ty;
  const int blocks = (ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL((k_jacobi2d<T, R>), dim3(blocks), dim3(WAVE * kWavesPerBlock), 0, st, in, out, nx, ny,
                     si, so, tx, ntiles, done);
  return hipGetLastError();
}

}  // namespace

// Shape of the 8-sweep launches: 0 one wavefront per 64 x 32 tile; 1..8
// workgroups of wavefronts stacked in y exchanging edge rows through LDS
// (wavefronts x rows each: 1: 4 x 16, 2: 8 x 8, 3: 8 x 16, 4: 4 x 12,
// 5: 8 x 10, 6: 16 x 6, 7: 16 x 8, 8: 16 x 4).  J3D_JACOBI2D_SHAPE overrides the
// default (shape sweeps).
static int jacobi2d_shape() {
  int shape = 2;  // 8 wavefronts x 8 rows: 151 ms for 100000 sweeps of 1024^2 (229 with shape 0)
  if (const char* e = std::getenv("J3D_JACOBI2D_SHAPE")) {
    const int v = std::atoi(e);
    if (v >= 0 && v <= 8) shape = v;
  }
  return shape;
}

hipError_t launch_jacobi2d(int sweeps, const double* in, double* out, int nx, int ny, int si, int so,
                           const int* done, hipStream_t st) {
  const int shape = sweeps == 8 ? jacobi2d_shape() : 0;
  switch (sweeps) {
    case 1: return go2d<1, 16>(in, out, nx, ny, si, so, done, st);
    case 2: return go2d<2, 16>(in, out, nx, ny, si, so, done, st);
    case 4: return go2d<4, 24>(in, out, nx, ny, si, so, done, st);
    case 8:
      switch (shape) {
        case 1: return go2d_wg<8, 16, 4>(in, out, nx, ny, si, so, done, st);
        case 2: return go2d_wg<8, 8, 8>(in, out, nx, ny, si, so, done, st);
        case 3: return go2d_wg<8, 16, 8>(in, out, nx, ny, si, so, done, st);
        case 4: return go2d_wg<8, 12, 4>(in, out, nx, ny, si, so, done, st);
        case 5: return go2d_wg<8, 10, 8>(in, out, nx, ny, si, so, done, st);
        case 6: return go2d_wg<8, 6, 16>(in, out, nx, ny, si, so, done, st);
        case 7: return go2d_wg<8, 8, 16>(in, out, nx, ny, si, so, done, st);
        case 8: return go2d_wg<8, 4, 16>(in, out, nx, ny, si, so, done, st);
        default: return go2d<8, 32>(in, out, nx, ny, si, so, done, st);
      }
    default: return hipErrorInvalidValue;
  }
}

int laplace2d_res_blocks(int ny) { return (ny + kResRows - 1) / kResRows; }

hipError_t launch_laplace2d_res(const double* u, int nx, int ny, int su, double h, double* partials,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_laplace2d_res, dim3(laplace2d_res_blocks(ny)), dim3(256), 0, st, u, nx, ny, su, h * h,
                     partials);
  return hipGetLastError();
}

}  // namespace j3d
