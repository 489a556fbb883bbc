// Multi-field 3D stencils on gfx950: the momentum advection standing in for
// the paper's pw-advection benchmark (three velocity fields in, three
// tendencies out) and the tracer advection standing in for tra-adv (six
// fields, iterated); Sec. "Flang performance comparison" gives their field
// counts and grid sizes.
//
// Both are streaming stencils with a few flops per byte: HBM-bound, no dense
// contraction, no MFMA.  The kernels follow the z-marching design of the
// Jacobi sweep.  A wavefront owns a tile of 64 x-points (one 128-byte-aligned
// 512-byte row segment per field and row, so every load and store covers
// whole cache lines) by RY y-rows (one thread holds all RY rows of its
// column, plus one row above and below) and a chunk of z-planes, and keeps a
// rolling window of the planes k-1, k, k+1 in registers: every plane of every
// field is read once per tile.  x-neighbours come from the adjacent lanes by
// DPP wave shifts; the two halo columns left and right of the tile come from
// one gather load per field and plane (lane q < RY+2 reads the left column
// of row q, lane 32+q the right one) and reach lanes 0 and 63 by readlane.
// y- and z-neighbours come from registers.  Four wavefronts of a workgroup
// take neighbouring rows, so the rows they share hit in the vector cache.
// Offsets within a plane are 32-bit; plane offsets are 64-bit, so one field
// may exceed 2^31 elements (the pw-advection grid does).
//
// Arithmetic order is fixed and the library is built with contraction off,
// so the results equal the definitions below bit for bit.
//
// Momentum advection (centred flux form of Piacsek and Williams on a
// staggered grid: u on east faces, v on north faces, w on top faces):
//   flux difference  D(am, bm, ap, bp, c) = (am * bm - ap * bp) * c,
//   c = 0.25 / spacing, am / bm the two-point sums of the advecting velocity
//   and of the advected component at the lower face, ap / bp at the upper;
//   tendency = (Dx + Dy) + Dz.
// Tracer advection (donor cell):
//   F = q+ * t(below) + q- * t(above), q+ = q > 0 ? q : 0, q- = q < 0 ? q : 0,
//   t' = t - r * (((Fe - Fw) + (Fn - Fs)) + (Ft - Fb)).
#include "advect.h"
#include "sweep.h"

namespace j3d {
namespace {

using sweep_detail::from_left;
using sweep_detail::from_right;
using sweep_detail::lane_value;
using sweep_detail::put;
using sweep_detail::WAVE;
using sweep_detail::xcd_remap;

constexpr int kWaves = 4;  // wavefronts per workgroup (stacked in y)

struct TileMap {
  int lane;
  int x;      // column of this lane
  int xc;     // column clamped into the array
  int j0;     // first output row
  int k0, k1; // planes k0 .. k1-1
  int goff;   // in-plane offset of this lane's halo-column element
  bool gat;   // this lane takes part in the halo gather
  bool valid;
};

__device__ __forceinline__ TileMap tile_of(const AdvArgs& a, int ry) {
  TileMap m;
  m.lane = threadIdx.x & (WAVE - 1);
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = b % a.tiles_x;
  const int rest = b / a.tiles_x;
  const int yb = rest % a.yblocks;
  const int kc = rest / a.yblocks;
  const int ty = yb * kWaves + (int)(threadIdx.x / WAVE);
  m.valid = ty < a.tiles_y;
  const int x0 = 1 + tx * WAVE;
  m.x = x0 + m.lane;
  m.xc = min(m.x, a.nx + 1);
  m.j0 = 1 + ty * ry;
  m.k0 = 1 + kc * a.planes;
  m.k1 = min(m.k0 + a.planes, a.nz + 1);
  // lane q < ry+2: column x0-1 of row j0-1+q; lane 32+q: column x0+64
  // (clamped onto the halo column) of the same row
  const int q = m.lane < 32 ? m.lane : m.lane - 32;
  m.gat = q < ry + 2;
  const int gx = m.lane < 32 ? x0 - 1 : min(x0 + WAVE, a.nx + 1);
  m.goff = gx + a.siy * min(m.j0 - 1 + min(q, ry + 1), a.ny + 1);
  return m;
}

// Left / right x-neighbour of value v of row r, whose halo columns are in
// the gathered vector g (lane r: left, lane 32+r: right).
__device__ __forceinline__ double nb_left(double v, double g, int r, int lane) {
  const double h = lane_value(g, r);
  const double s = from_left(v);
  return lane == 0 ? h : s;
}
__device__ __forceinline__ double nb_right(double v, double g, int r, int lane) {
  const double h = lane_value(g, 32 + r);
  const double s = from_right(v);
  return lane == WAVE - 1 ? h : s;
}

__device__ __forceinline__ double flux_diff(double am, double bm, double ap, double bp, double c) {
  return (am * bm - ap * bp) * c;
}

template <int RY, bool NT>
__global__ void __launch_bounds__(WAVE * kWaves) k_pw_advect(AdvArgs a) {
  const TileMap m = tile_of(a, RY);
  if (!m.valid) return;  // the whole wavefront leaves together
  const int lane = m.lane;
  int roff[RY + 2];  // in-plane offsets of rows j0-1 .. j0+RY (clamped)
#pragma unroll
  for (int r = 0; r < RY + 2; ++r) roff[r] = m.xc + a.siy * min(m.j0 - 1 + r, a.ny + 1);
  const double* __restrict__ pu = a.in[0];
  const double* __restrict__ pv = a.in[1];
  const double* __restrict__ pw = a.in[2];
  // planes k-1, k, k+1 of each field, and their gathered halo columns
  double U[3][RY + 2], V[3][RY + 2], W[3][RY + 2], GU[3], GV[3], GW[3];
  auto load = [&](int s, int k) {
    const long long pz = (long long)k * a.siz;
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
      U[s][r] = pu[pz + roff[r]];
      V[s][r] = pv[pz + roff[r]];
      W[s][r] = pw[pz + roff[r]];
    }
    GU[s] = m.gat ? pu[pz + m.goff] : 0.0;
    GV[s] = m.gat ? pv[pz + m.goff] : 0.0;
    GW[s] = m.gat ? pw[pz + m.goff] : 0.0;
  };
  load(0, m.k0 - 1);
  load(1, m.k0);
  const bool lane_out = m.x <= a.nx;
  const double cx = a.cx, cy = a.cy, cz = a.cz;
  for (int k = m.k0; k < m.k1; ++k) {
    load(2, k + 1);
    const long long oz = (long long)k * a.soz;
#pragma unroll
    for (int r = 1; r <= RY; ++r) {
      const double u = U[1][r], v = V[1][r], w = W[1][r];
      const double uL = nb_left(u, GU[1], r, lane), uR = nb_right(u, GU[1], r, lane);
      const double vL = nb_left(v, GV[1], r, lane), vR = nb_right(v, GV[1], r, lane);
      const double wL = nb_left(w, GW[1], r, lane), wR = nb_right(w, GW[1], r, lane);
      // u at the east face (i+1/2, j, k)
      const double sxm = uL + u, sxp = u + uR;
      double tx = flux_diff(sxm, sxm, sxp, sxp, cx);
      const double vs = V[1][r - 1];
      double ty = flux_diff(vs + nb_right(vs, GV[1], r - 1, lane), U[1][r - 1] + u, v + vR, u + U[1][r + 1], cy);
      const double wb = W[0][r];
      double tz = flux_diff(wb + nb_right(wb, GW[0], r, lane), U[0][r] + u, w + wR, u + U[2][r], cz);
      const double su = (tx + ty) + tz;
      // v at the north face (i, j+1/2, k)
      const double un = U[1][r + 1];
      tx = flux_diff(uL + nb_left(un, GU[1], r + 1, lane), vL + v, u + un, v + vR, cx);
      const double syn = vs + v, syp = v + V[1][r + 1];
      ty = flux_diff(syn, syn, syp, syp, cy);
      tz = flux_diff(wb + W[0][r + 1], V[0][r] + v, w + W[1][r + 1], v + V[2][r], cz);
      const double sv = (tx + ty) + tz;
      // w at the top face (i, j, k+1/2)
      const double ut = U[2][r];
      tx = flux_diff(uL + nb_left(ut, GU[2], r, lane), wL + w, u + ut, w + wR, cx);
      const double vt = V[2][r - 1];
      ty = flux_diff(vs + vt, W[1][r - 1] + w, v + V[2][r], w + W[1][r + 1], cy);
      const double szm = wb + w, szp = w + W[2][r];
      tz = flux_diff(szm, szm, szp, szp, cz);
      const double sw = (tx + ty) + tz;
      const int j = m.j0 + r - 1;
      if (lane_out && j <= a.ny) {
        const long long o = oz + m.x + (long long)a.soy * j;
        put<double, NT>(a.out[0] + o, su);
        put<double, NT>(a.out[1] + o, sv);
        put<double, NT>(a.out[2] + o, sw);
      }
    }
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
      U[0][r] = U[1][r]; U[1][r] = U[2][r];
      V[0][r] = V[1][r]; V[1][r] = V[2][r];
      W[0][r] = W[1][r]; W[1][r] = W[2][r];
    }
    GU[0] = GU[1]; GU[1] = GU[2];
    GV[0] = GV[1]; GV[1] = GV[2];
    GW[0] = GW[1]; GW[1] = GW[2];
  }
}

// The momentum advection with the loads of plane k+2 issued at the start of
// step k (one plane ahead of the three-plane window the step uses), the
// results of step k stored at the start of step k+1, and every plane
// addressed through a scalar buffer resource with 32-bit per-lane offsets:
// no branch surrounds a memory operation (lanes and rows outside the
// interior store with an out-of-range offset, which the hardware drops),
// so the compiler's waits cover exactly the loads a step consumes.  Needs
// every plane of the six fields under 2^31 bytes (AdvArgs::buffer_ok).
// Same arithmetic and order as k_pw_advect.
template <int RY, bool NT>
__global__ void __launch_bounds__(WAVE * kWaves) k_pw_advect_pf(AdvArgs a) {
  using sweep_detail::bload;
  using sweep_detail::bstore;
  using sweep_detail::kDropOffset;
  using sweep_detail::plane_rsrc_n;
  constexpr int R = RY + 2;
  const TileMap m = tile_of(a, RY);
  if (!m.valid) return;  // the whole wavefront leaves together
  const int lane = m.lane;
  uint32_t roff[R];  // byte offsets of rows j0-1 .. j0+RY (clamped)
#pragma unroll
  for (int r = 0; r < R; ++r) roff[r] = (uint32_t)(m.xc + a.siy * min(m.j0 - 1 + r, a.ny + 1)) * 8u;
  const uint32_t goff = (uint32_t)m.goff * 8u;  // every lane loads; only the gather lanes' values are used
  const bool lane_out = m.x <= a.nx;
  uint32_t oo[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int j = m.j0 + r;
    oo[r] = (lane_out && j <= a.ny) ? (uint32_t)(m.x + a.soy * j) * 8u : kDropOffset;
  }
  const uint32_t rin = ((uint32_t)(a.nx + 1) + (uint32_t)a.siy * (uint32_t)(a.ny + 1) + 1u) * 8u;
  const uint32_t rout = ((uint32_t)(a.nx + 1) + (uint32_t)a.soy * (uint32_t)(a.ny + 1) + 1u) * 8u;
  const uint64_t zin = (uint64_t)a.siz * 8u, zout = (uint64_t)a.soz * 8u;
  struct Plane {
    double u[R], v[R], w[R], gu, gv, gw;
  };
  auto load = [&](Plane& p, int k) {
    const auto ru = plane_rsrc_n(a.in[0], zin, k, rin);
    const auto rv = plane_rsrc_n(a.in[1], zin, k, rin);
    const auto rw = plane_rsrc_n(a.in[2], zin, k, rin);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      p.u[r] = bload<double>(ru, roff[r]);
      p.v[r] = bload<double>(rv, roff[r]);
      p.w[r] = bload<double>(rw, roff[r]);
    }
    p.gu = bload<double>(ru, goff);
    p.gv = bload<double>(rv, goff);
    p.gw = bload<double>(rw, goff);
  };
  // tendencies of the previous step, stored at the start of the next one
  double ts[3][RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) ts[0][r] = ts[1][r] = ts[2][r] = 0.0;
  auto flush = [&](int kk, bool any) {
    const auto o0 = plane_rsrc_n(a.out[0], zout, kk, rout);
    const auto o1 = plane_rsrc_n(a.out[1], zout, kk, rout);
    const auto o2 = plane_rsrc_n(a.out[2], zout, kk, rout);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const uint32_t off = any ? oo[r] : kDropOffset;
      bstore<double, NT>(ts[0][r], o0, off);
      bstore<double, NT>(ts[1][r], o1, off);
      bstore<double, NT>(ts[2][r], o2, off);
    }
  };
  // planes k-1, k, k+1 of the step, and the next plane in flight
  Plane P0, P1, P2, N;
  load(P0, m.k0 - 1);
  load(P1, m.k0);
  load(N, m.k0 + 1);
  const double cx = a.cx, cy = a.cy, cz = a.cz;
  for (int k = m.k0; k < m.k1; ++k) {
    P2 = N;
    load(N, min(k + 2, a.nz + 1));
    flush(max(k - 1, 0), k > m.k0);
#pragma unroll
    for (int r = 1; r <= RY; ++r) {
      const double u = P1.u[r], v = P1.v[r], w = P1.w[r];
      const double uL = nb_left(u, P1.gu, r, lane), uR = nb_right(u, P1.gu, r, lane);
      const double vL = nb_left(v, P1.gv, r, lane), vR = nb_right(v, P1.gv, r, lane);
      const double wL = nb_left(w, P1.gw, r, lane), wR = nb_right(w, P1.gw, r, lane);
      // u at the east face (i+1/2, j, k)
      const double sxm = uL + u, sxp = u + uR;
      double tx = flux_diff(sxm, sxm, sxp, sxp, cx);
      const double vs = P1.v[r - 1];
      double ty = flux_diff(vs + nb_right(vs, P1.gv, r - 1, lane), P1.u[r - 1] + u, v + vR, u + P1.u[r + 1], cy);
      const double wb = P0.w[r];
      double tz = flux_diff(wb + nb_right(wb, P0.gw, r, lane), P0.u[r] + u, w + wR, u + P2.u[r], cz);
      const double su = (tx + ty) + tz;
      // v at the north face (i, j+1/2, k)
      const double un = P1.u[r + 1];
      tx = flux_diff(uL + nb_left(un, P1.gu, r + 1, lane), vL + v, u + un, v + vR, cx);
      const double syn = vs + v, syp = v + P1.v[r + 1];
      ty = flux_diff(syn, syn, syp, syp, cy);
      tz = flux_diff(wb + P0.w[r + 1], P0.v[r] + v, w + P1.w[r + 1], v + P2.v[r], cz);
      const double sv = (tx + ty) + tz;
      // w at the top face (i, j, k+1/2)
      const double ut = P2.u[r];
      tx = flux_diff(uL + nb_left(ut, P2.gu, r, lane), wL + w, u + ut, w + wR, cx);
      const double vt = P2.v[r - 1];
      ty = flux_diff(vs + vt, P1.w[r - 1] + w, v + P2.v[r], w + P1.w[r + 1], cy);
      const double szm = wb + w, szp = w + P2.w[r];
      tz = flux_diff(szm, szm, szp, szp, cz);
      const double sw = (tx + ty) + tz;
      ts[0][r - 1] = su;
      ts[1][r - 1] = sv;
      ts[2][r - 1] = sw;
    }
    P0 = P1;
    P1 = P2;
  }
  flush(m.k1 - 1, true);
}

__device__ __forceinline__ double upwind(double q, double below, double above) {
  const double qp = q > 0.0 ? q : 0.0;
  const double qm = q < 0.0 ? q : 0.0;
  return qp * below + qm * above;
}

// in[0..3] = u, v, w, r; t = input iterate; out[0] = output iterate.
template <int RY, bool NT>
__global__ void __launch_bounds__(WAVE * kWaves) k_tracer_advect(AdvArgs a) {
  const TileMap m = tile_of(a, RY);
  if (!m.valid) return;
  const int lane = m.lane;
  int roff[RY + 2];
#pragma unroll
  for (int r = 0; r < RY + 2; ++r) roff[r] = m.xc + a.siy * min(m.j0 - 1 + r, a.ny + 1);
  const double* __restrict__ pt = a.t;
  const double* __restrict__ pu = a.in[0];
  const double* __restrict__ pv = a.in[1];
  const double* __restrict__ pw = a.in[2];
  const double* __restrict__ pr = a.in[3];
  double T[3][RY + 2], Wb[RY + 2];
  double GT1, GT2;  // halo columns of planes k and k+1 of t
  {
    const long long z0 = (long long)(m.k0 - 1) * a.siz, z1 = (long long)m.k0 * a.siz;
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
      T[0][r] = pt[z0 + roff[r]];
      T[1][r] = pt[z1 + roff[r]];
      Wb[r] = pw[z0 + roff[r]];
    }
    GT1 = m.gat ? pt[z1 + m.goff] : 0.0;
  }
  const bool lane_out = m.x <= a.nx;
  for (int k = m.k0; k < m.k1; ++k) {
    const long long pz = (long long)k * a.siz;
    const long long nz = pz + a.siz;
    double U[RY + 2], V[RY + 2], W[RY + 2], R[RY + 2];
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
      T[2][r] = pt[nz + roff[r]];
      if (r >= 1 && r <= RY) {
        U[r] = pu[pz + roff[r]];
        W[r] = pw[pz + roff[r]];
        R[r] = pr[pz + roff[r]];
      }
      if (r <= RY) V[r] = pv[pz + roff[r]];
    }
    GT2 = m.gat ? pt[nz + m.goff] : 0.0;
    const double GU = m.gat ? pu[pz + m.goff] : 0.0;
#pragma unroll
    for (int r = 1; r <= RY; ++r) {
      const double tc = T[1][r];
      const double tl = nb_left(tc, GT1, r, lane), tr = nb_right(tc, GT1, r, lane);
      const double fe = upwind(U[r], tc, tr);
      const double fw = upwind(nb_left(U[r], GU, r, lane), tl, tc);
      const double fn = upwind(V[r], tc, T[1][r + 1]);
      const double fs = upwind(V[r - 1], T[1][r - 1], tc);
      const double ft = upwind(W[r], tc, T[2][r]);
      const double fb = upwind(Wb[r], T[0][r], tc);
      const double div = ((fe - fw) + (fn - fs)) + (ft - fb);
      const double tn = tc - R[r] * div;
      const int j = m.j0 + r - 1;
      if (lane_out && j <= a.ny) put<double, NT>(a.out[0] + (pz + m.x + (long long)a.siy * j), tn);
    }
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
      T[0][r] = T[1][r];
      T[1][r] = T[2][r];
      if (r >= 1 && r <= RY) Wb[r] = W[r];
    }
    GT1 = GT2;
  }
}

// Two tracer steps in one pass: t2 = S(S(t0)), u, v, w, r read once for
// both.  Lane l of a wavefront is column x0 - 2 + l (tiles 60 wide, x0 =
// 1 + 60 tx, overlapping by four columns): the intermediate t1 is valid on
// lanes 1..62, t2 on lanes 2..61, which are stored.  A workgroup of four
// wavefronts, each owning RY consecutive rows, covers 4 RY rows; the first
// and last of them form a ring around the 4 RY - 2 output rows (the
// neighbouring workgroups output them).  Marching through z, step k
// computes t1 at plane k on every row of the workgroup and t2 at plane k-1
// on the output rows.  A wavefront loads its own rows of every field, one
// row of t0 beyond each end of them and one row of v below; the t1 rows just
// outside its own come from the neighbouring wavefronts through LDS (three
// plane slots, one barrier per plane).  t1 at a halo cell (outside the
// interior in any axis) is t0 there, the fixed boundary value.  Each point
// of t1 and t2 has exactly the arithmetic of one step.
constexpr int kOut2 = WAVE - 4;  // outputs per wavefront along x

template <int RY, bool NT>
__global__ void __launch_bounds__(WAVE * kWaves) k_tracer2_advect(AdvArgs a) {
  constexpr int TR = kWaves * RY;  // workgroup rows
  constexpr int H = TR - 2;        // output rows
  __shared__ double edge[3][kWaves][2][WAVE];  // t1: plane slot, wavefront, first/last row
  const int lane = threadIdx.x & (WAVE - 1);
  const int wy = threadIdx.x / WAVE;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = b % a.tiles_x;
  const int rest = b / a.tiles_x;
  const int ty = rest % a.tiles_y;  // workgroup-uniform
  const int kc = rest / a.tiles_y;
  const int x = tx * kOut2 - 1 + lane;  // x0 - 2 + lane
  const int xc = min(max(x, 0), a.nx + 1);
  const bool x_in = x >= 1 && x <= a.nx;
  const bool lane_out = lane >= 2 && lane <= kOut2 + 1 && x_in;
  const int y0 = ty * H + wy * RY;  // row of this wavefront's first own row
  const int k0 = 1 + kc * a.planes;
  const int k1 = min(k0 + a.planes, a.nz + 1);
  // t0 window rows i = 0 .. RY+1 are rows y0 - 1 + i (own rows at i = 1..RY);
  // v rows i = 0 .. RY are rows y0 - 1 + i
  int roff[RY + 2];
  bool row_in[RY], row_out[RY];
#pragma unroll
  for (int i = 0; i < RY + 2; ++i) roff[i] = xc + a.siy * min(max(y0 - 1 + i, 0), a.ny + 1);
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int y = y0 + r;
    const int br = wy * RY + r;
    row_in[r] = y >= 1 && y <= a.ny;
    row_out[r] = lane_out && br >= 1 && br <= H && y <= a.ny;
  }
  const double* __restrict__ pt = a.t;
  const double* __restrict__ pu = a.in[0];
  const double* __restrict__ pv = a.in[1];
  const double* __restrict__ pw = a.in[2];
  const double* __restrict__ pr = a.in[3];
  double T0[3][RY + 2];            // t0 at planes k-1, k, k+1
  double T1[3][RY];                // t1 at planes k-2, k-1, k (own rows)
  double W[3][RY];                 // w at planes k-2, k-1, k
  double U[2][RY], R[2][RY], V[2][RY + 1];  // planes k-1, k
  auto zoff = [&](int k) { return (long long)min(max(k, 0), a.nz + 1) * a.siz; };
  {
    const long long za = zoff(k0 - 2), zb = zoff(k0 - 1);
#pragma unroll
    for (int i = 0; i < RY + 2; ++i) {
      T0[0][i] = pt[za + roff[i]];
      T0[1][i] = pt[zb + roff[i]];
    }
    // w at plane k0-2 goes to the newest slot: the first shift moves it to
    // plane k-1 of step k0-1
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      W[2][r] = pw[za + roff[r + 1]];
      W[1][r] = 0.0;
      T1[1][r] = 0.0;
      T1[2][r] = 0.0;
      U[1][r] = R[1][r] = 0.0;
    }
#pragma unroll
    for (int i = 0; i < RY + 1; ++i) V[1][i] = 0.0;
  }
  for (int k = k0 - 1; k <= k1; ++k) {
    // shift the windows: plane k becomes the newest
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      T1[0][r] = T1[1][r];
      T1[1][r] = T1[2][r];
      W[0][r] = W[1][r];
      W[1][r] = W[2][r];
      U[0][r] = U[1][r];
      R[0][r] = R[1][r];
    }
#pragma unroll
    for (int i = 0; i < RY + 1; ++i) V[0][i] = V[1][i];
    const long long zk = zoff(k), zn = zoff(k + 1);
#pragma unroll
    for (int i = 0; i < RY + 2; ++i) T0[2][i] = pt[zn + roff[i]];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      U[1][r] = pu[zk + roff[r + 1]];
      W[2][r] = pw[zk + roff[r + 1]];
      R[1][r] = pr[zk + roff[r + 1]];
    }
#pragma unroll
    for (int i = 0; i < RY + 1; ++i) V[1][i] = pv[zk + roff[i]];
    // stage 1: t1 at plane k on the own rows
    const bool k_in = k >= 1 && k <= a.nz;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const double tc = T0[1][r + 1];
      const double tl = from_left(tc), tr = from_right(tc);
      const double fe = upwind(U[1][r], tc, tr);
      const double fw = upwind(from_left(U[1][r]), tl, tc);
      const double fn = upwind(V[1][r + 1], tc, T0[1][r + 2]);
      const double fs = upwind(V[1][r], T0[1][r], tc);
      const double ft = upwind(W[2][r], tc, T0[2][r + 1]);
      const double fb = upwind(W[1][r], T0[0][r + 1], tc);
      const double div = ((fe - fw) + (fn - fs)) + (ft - fb);
      const double t1 = tc - R[1][r] * div;
      T1[2][r] = (x_in && row_in[r] && k_in) ? t1 : tc;
    }
    edge[k % 3][wy][0][lane] = T1[2][0];
    edge[k % 3][wy][1][lane] = T1[2][RY - 1];
    __syncthreads();
    // stage 2: t2 at plane k-1 on the output rows
    if (k - 1 >= k0) {
      const int sl = (k + 2) % 3;  // slot of plane k-1
      const double below = wy > 0 ? edge[sl][wy - 1][1][lane] : 0.0;
      const double above = wy < kWaves - 1 ? edge[sl][wy + 1][0][lane] : 0.0;
      const long long zo = (long long)(k - 1) * a.soz;
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        const double tc = T1[1][r];
        const double tl = from_left(tc), tr = from_right(tc);
        const double ts = r == 0 ? below : T1[1][r - 1];
        const double tn = r == RY - 1 ? above : T1[1][r + 1];
        const double fe = upwind(U[0][r], tc, tr);
        const double fw = upwind(from_left(U[0][r]), tl, tc);
        const double fn = upwind(V[0][r + 1], tc, tn);
        const double fs = upwind(V[0][r], ts, tc);
        const double ft = upwind(W[1][r], tc, T1[2][r]);
        const double fb = upwind(W[0][r], T1[0][r], tc);
        const double div = ((fe - fw) + (fn - fs)) + (ft - fb);
        const double t2 = tc - R[0][r] * div;
        if (row_out[r]) put<double, NT>(a.out[0] + (zo + x + (long long)a.soy * (y0 + r)), t2);
      }
    }
#pragma unroll
    for (int i = 0; i < RY + 2; ++i) {
      T0[0][i] = T0[1][i];
      T0[1][i] = T0[2][i];
    }
  }
}

template <typename Kernel>
hipError_t go2(Kernel kern, AdvArgs a, int ry, hipStream_t st) {
  const int h = kWaves * ry - 2;  // output rows per workgroup
  a.tiles_x = (a.nx + kOut2 - 1) / kOut2;
  a.tiles_y = (a.ny + h - 1) / h;
  a.yblocks = a.tiles_y;
  const int zchunks = (a.nz + a.planes - 1) / a.planes;
  const long long blocks = (long long)a.tiles_x * a.tiles_y * zchunks;
  if (blocks <= 0) return hipSuccess;
  if (blocks >= (1LL << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(WAVE * kWaves), 0, st, a);
  return hipGetLastError();
}

template <typename Kernel>
hipError_t go(Kernel kern, AdvArgs a, int ry, hipStream_t st) {
  a.tiles_x = (a.nx + WAVE - 1) / WAVE;
  a.tiles_y = (a.ny + ry - 1) / ry;
  a.yblocks = (a.tiles_y + kWaves - 1) / kWaves;
  const int zchunks = (a.nz + a.planes - 1) / a.planes;
  const long long blocks = (long long)a.tiles_x * a.yblocks * zchunks;
  if (blocks <= 0) return hipSuccess;
  if (blocks >= (1LL << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(WAVE * kWaves), 0, st, a);
  return hipGetLastError();
}

}  // namespace

bool advect_cfg_supported(const AdvectCfg& c) {
  return (c.ry == 2 || c.ry == 4 || c.ry == 8) && c.planes >= 1 && (c.nt == 0 || c.nt == 1) &&
         (c.pf == 0 || c.pf == 1);
}

hipError_t launch_pw_advect(const AdvArgs& a, const AdvectCfg& c, hipStream_t st) {
  if (!advect_cfg_supported(c)) return hipErrorInvalidValue;
  AdvArgs g = a;
  g.planes = c.planes;
  if (c.pf && a.buffer_ok) {
    switch (c.ry * 2 + c.nt) {
      case 4: return go(k_pw_advect_pf<2, false>, g, 2, st);
      case 5: return go(k_pw_advect_pf<2, true>, g, 2, st);
      case 8: return go(k_pw_advect_pf<4, false>, g, 4, st);
      case 9: return go(k_pw_advect_pf<4, true>, g, 4, st);
      default: break;  // 8 rows: the kernel without the prefetch
    }
  }
  switch (c.ry * 2 + c.nt) {
    case 4: return go(k_pw_advect<2, false>, g, 2, st);
    case 5: return go(k_pw_advect<2, true>, g, 2, st);
    case 8: return go(k_pw_advect<4, false>, g, 4, st);
    case 9: return go(k_pw_advect<4, true>, g, 4, st);
    case 16: return go(k_pw_advect<8, false>, g, 8, st);
    default: return go(k_pw_advect<8, true>, g, 8, st);
  }
}

hipError_t launch_tracer_advect(const AdvArgs& a, const AdvectCfg& c, hipStream_t st) {
  if (!advect_cfg_supported(c)) return hipErrorInvalidValue;
  AdvArgs g = a;
  g.planes = c.planes;
  switch (c.ry * 2 + c.nt) {
    case 4: return go(k_tracer_advect<2, false>, g, 2, st);
    case 5: return go(k_tracer_advect<2, true>, g, 2, st);
    case 8: return go(k_tracer_advect<4, false>, g, 4, st);
    case 9: return go(k_tracer_advect<4, true>, g, 4, st);
    case 16: return go(k_tracer_advect<8, false>, g, 8, st);
    default: return go(k_tracer_advect<8, true>, g, 8, st);
  }
}

bool tracer2_cfg_supported(const AdvectCfg& c) {
  return (c.ry == 2 || c.ry == 4 || c.ry == 6) && c.planes >= 1 && (c.nt == 0 || c.nt == 1);
}

hipError_t launch_tracer2_advect(const AdvArgs& a, const AdvectCfg& c, hipStream_t st) {
  if (!tracer2_cfg_supported(c)) return hipErrorInvalidValue;
  AdvArgs g = a;
  g.planes = c.planes;
  switch (c.ry * 2 + c.nt) {
    case 4: return go2(k_tracer2_advect<2, false>, g, 2, st);
    case 5: return go2(k_tracer2_advect<2, true>, g, 2, st);
    case 8: return go2(k_tracer2_advect<4, false>, g, 4, st);
    case 9: return go2(k_tracer2_advect<4, true>, g, 4, st);
    case 12: return go2(k_tracer2_advect<6, false>, g, 6, st);
    default: return go2(k_tracer2_advect<6, true>, g, 6, st);
  }
}

}  // namespace j3d
