// Internal interface between the host runtime and the gfx950 kernels of libj3d.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "j3d.h"

namespace j3d {

// Per-grid launch descriptor.  Every pointer addresses the array element at
// Fortran index (lbound0, lbound1, lbound2), i.e. the corner of the halo, so
// that interior point (i,j,k), 1 <= i <= nx etc., is at i + sy*j + sz*k.
struct GridArgs {
  const void* u;    // input iterate (T)
  void* o;          // output iterate (T), written with F_WRITE
  const void* f;    // right-hand side (T); for FP32 correction sweeps: r32
  double* u64;      // FP64 field the update is added to, with F_LAST
  float* r32;       // FP32 copy of the residual, written with F_R32
  int nx, ny, nz;
  int su_y, su_z;   // strides of u
  int so_y, so_z;   // strides of o
  int sf_y, sf_z;   // strides of f
  int s64_y, s64_z; // strides of u64
  int sr_y, sr_z;   // strides of r32
  int tiles_x, tiles_y, tiles_z;
  int tile0;        // first tile of this grid in the batch's tile numbering
  int planes;       // z-planes per tile
  int id;           // index of this grid's flags and norms in per-grid arrays
  double h2;        // h*h in FP64
  float h2f;        // (float)(h*h)
  int order;        // tile order: 0 XCD-blocked, 1 as launched, 2 chunked per XCD
  int chunk;        // order 2: tiles per XCD chunk
  int wide_planes;  // some plane of an array spans 2^31 bytes or more: the one-sweep
                    // pass takes its pointer-addressed path
};

// Kernel pass flags (compile-time).
enum : unsigned {
  F_WRITE = 1u,   // write the Jacobi update to o
  F_RES = 2u,     // accumulate sum of r^2 of the input iterate (FP64)
  F_R32 = 4u,     // store (float) r to r32
  F_FIRST = 8u,   // the input iterate is identically zero (not read)
  F_LAST = 16u,   // add (double) update to u64 instead of writing o
  F_NORM = 32u,   // accumulate sum of f^2 only
  F_RES1 = 64u,   // three-sweep pass: sum of r^2 of the iterate after its first sweep (FP64)
  F_RES2 = 128u,  // three-sweep pass: sum of r^2 of the iterate after its second sweep (FP64)
};

// One dispatch slot of a batched pass launched from a slot list: the tile
// (in the batch's flat tile numbering, -1 for none) and the grid owning it.
struct alignas(8) TileSlot {
  int tile;
  int grid;
};

// Tile order of batched three-sweep passes launched from a slot list (the
// slots carry the order; see build_slots3).
constexpr int kOrderSlots = 3;

struct TileCfg {
  int rows;       // wavefronts per workgroup
  int planes;     // z-planes per tile
  int variant;    // bit set: 1 LDS plane; 2, 16 rows per thread; 4 nontemporal stores
  int persistent; // 1: fixed grid striding over tiles
  int order;      // 0 XCD-blocked, 1 as launched, 2 chunked per XCD within each slab
  int cols;       // wavefronts side by side along x (1, 2 or 4)
};

// Supported rows values and variants (kernels are instantiated for these).
bool tile_cfg_supported(const TileCfg& c);

// Number of tiles of one grid under a tile shape.
void tile_counts(int nx, int ny, int nz, const TileCfg& c, int* tx, int* ty, int* tz);

// Tile shapes of the two-sweep pass of element type dtype (cols = 1): a block
// of 64 x (rows x rows-per-thread) columns with 60 x (rows x rows-per-thread
// - 2) outputs.
bool tile2_cfg_supported(int dtype, const TileCfg& c);
void tile2_counts(int nx, int ny, int nz, const TileCfg& c, int* tx, int* ty, int* tz);

// Two sweeps in one pass: g.o = J(J(g.u)).  FP64 flags: F_WRITE, optionally
// with F_RES (residual of g.u into partials, one slot per tile).  FP32
// flags: F_WRITE or F_LAST (add to g.u64), optionally with F_FIRST (g.u is
// zero and not read).
hipError_t launch_sweep2_one(int dtype, unsigned flags, const TileCfg& c, const GridArgs& g,
                             double* partials, const int* done, hipStream_t st);
// The same over a table of grids (as launch_pass_batch; tile counts from
// tile2_counts).
hipError_t launch_sweep2_batch(int dtype, unsigned flags, const TileCfg& c, const GridArgs* table,
                               int ngrids, int ntiles, double* partials, const int* done,
                               hipStream_t st);

// Three sweeps in one pass: g.o = J(J(J(g.u))), tile shapes of rows 2, 4, 8
// or 16 wavefronts of 2 or 4 rows per thread (variants 6 and 20), cols 1, not
// persistent; 58 x (rows x rows-per-thread - 4) outputs per block.  Flags as
// for the two-sweep pass.
bool tile3_cfg_supported(int dtype, const TileCfg& c);
void tile3_counts(int nx, int ny, int nz, const TileCfg& c, int* tx, int* ty, int* tz);
hipError_t launch_sweep3_one(int dtype, unsigned flags, const TileCfg& c, const GridArgs& g,
                             double* partials, const int* done, hipStream_t st);
// The three-sweep pass over a table of grids: FP64 with F_WRITE and at
// most one of F_RES, F_RES1, F_RES2; FP32 with the flags of the correction
// cycles (F_WRITE or F_LAST, each with or without F_FIRST).
// With slots, workgroup b runs tile slots[b].tile of grid slots[b].grid
// (nslots workgroups; tile -1: none) and c.order may be kOrderSlots.
hipError_t launch_sweep3_batch(int dtype, unsigned flags, const TileCfg& c, const GridArgs* table, int ngrids,
                               int ntiles, double* partials, const int* done, hipStream_t st,
                               const TileSlot* slots = nullptr, int nslots = 0);

// Number of resident workgroups used for persistent launches.
int persistent_grid(const TileCfg& c);

// Launch one pass over one grid (args by value).  partials receives one
// double per tile (slot = tile index) when flags include F_RES or F_NORM.
// done, if not null, is a flag: when *done != 0 the launch does nothing.
hipError_t launch_pass_one(int dtype, unsigned flags, const TileCfg& c, const GridArgs& g,
                           double* partials, const int* done, hipStream_t st);

// The check of the previous pass, reduced by one extra workgroup of a
// one-sweep pass instead of by a kernel of its own: the sum of
// partials[0 .. n) in the order of the reduction kernels (launch_reduce_*:
// 1024 threads, thread q adding slots q, q + 1024, ... in turn, then each
// wavefront's butterfly, then the 16 wavefront sums in order), then what
// launch_reduce_count does with it: hist[*qnext] = sqrt(sum), *done and
// *conv_at set when it is not finite or at most rtol * *normf (*nonfinite
// too when not finite), *qnext advanced.  partials == nullptr: no check.
struct PreReduce {
  const double* partials;
  int n;
  double* hist;
  const double* normf;
  double rtol;
  int* done;
  long long* conv_at;
  int* nonfinite;
  long long* qnext;
};

// launch_pass_one with the previous pass's check reduced by an extra
// workgroup of the same launch (which then must not run when *pr.done is
// set: pass done == pr.done).  pr.partials must not be the partials this
// pass writes.
hipError_t launch_pass_one_pre(int dtype, unsigned flags, const TileCfg& c, const GridArgs& g,
                               double* partials, const int* done, const PreReduce& pr, hipStream_t st);

// Launch one pass over a table of grids in device memory (tile0 ascending,
// tiles of grid g are [tile0[g], tile0[g] + tx*ty*tz)).  done, if not
// null, is a flag array indexed by GridArgs::id; tiles of done grids are
// skipped.
hipError_t launch_pass_batch(int dtype, unsigned flags, const TileCfg& c, const GridArgs* table,
                             int ngrids, int ntiles, double* partials, const int* done,
                             hipStream_t st);

// Deterministic sum of partials[part0 .. part0+n) -> sqrt -> *out.
// If test_normf is not null: when sqrt(sum) <= rtol * (*test_normf) or is not
// finite, set *done = 1 and *conv_at = s; a non-finite value also sets
// *nonfinite = 1.  When done is not null and *done != 0 on entry, nothing is
// written.
hipError_t launch_reduce_one(const double* partials, int part0, int n, double* out,
                             const double* test_normf, double rtol, long long s, int* done,
                             long long* conv_at, int* nonfinite, hipStream_t st);

// The solve drivers' check: sum of partials[0 .. n) -> sqrt -> hist[*qnext];
// convergence test against rtol * (*normf) as launch_reduce_one with
// s = *qnext; then *qnext += 1.  Nothing happens once *done != 0.
hipError_t launch_reduce_count(const double* partials, int n, double* hist, const double* normf,
                               double rtol, int* done, long long* conv_at, int* nonfinite,
                               long long* qnext, hipStream_t st);

// Batched reduce: one workgroup per table entry; entry g (id = table[g].id)
// sums its own tile slots and writes sqrt to out[id*ostride + q].  Grids
// flagged done[id] are skipped.  With normf (indexed by id) the convergence
// test of launch_reduce_one is applied per grid (done, conv_at, nonfinite,
// rtol all indexed by id).
hipError_t launch_reduce_batch(const double* partials, const GridArgs* table, int ngrids,
                               double* out, int ostride, int q, const double* normf,
                               const double* rtol, long long s, int* done, long long* conv_at,
                               int* nonfinite, hipStream_t st);

// sum / dot_product of FP64 vectors (y null: sum of x).  Blocks of the
// fixed partition of n (sum_blocks(n) partial slots, at most kSumMaxBlocks),
// then the fixed-pattern sum of the partials into *out (device).
constexpr int kSumMaxBlocks = 65536;
long long sum_chunk(long long n);
int sum_blocks(long long n);
hipError_t launch_sum(const double* x, const double* y, long long n, double* partials, double* out,
                      hipStream_t st);

// The 2D Laplace jacobi benchmark: `sweeps` (1, 2, 4 or 8) Jacobi sweeps of
// the interior nx x ny of `in` (row stride si) written to `out` (row stride
// so); in and out hold the same halo.  Skipped when *done != 0.
hipError_t launch_jacobi2d(int sweeps, const double* in, double* out, int nx, int ny, int si, int so,
                           const int* done, hipStream_t st);
// Per-block sums of r^2, r = (S - 4 u) / h^2, over the interior of a 2D
// array (laplace2d_res_blocks(ny) slots).
int laplace2d_res_blocks(int ny);
hipError_t launch_laplace2d_res(const double* u, int nx, int ny, int su, double h, double* partials,
                                hipStream_t st);

hipError_t launch_fill_uniform(double* a, int ex, int ey, int ez, long long sy, long long sz,
                               unsigned long long key, double lo, double hi, double halo,
                               hipStream_t st);
hipError_t launch_fill_const(void* a, int dtype, int ex, int ey, int ez, long long sy,
                             long long sz, double v, hipStream_t st);
hipError_t launch_copy(const double* src, double* dst, long long n, hipStream_t st);
// Copy kernels of the bandwidth probe: 0 the library's copy (grid-stride
// over 16-byte elements), 1 one 16-byte element per thread, 2 the same
// with nontemporal loads and stores, 3 four per thread, 4 four per thread
// nontemporal.
constexpr int kCopyVariants = 5;
hipError_t launch_copy_variant(int v, const double* src, double* dst, long long n, hipStream_t st);
// Kernels of the two-reads-one-write probe (dst = a + b): 0 one 16-byte
// element per thread with nontemporal stores, 1 the same with plain
// stores, 2 four per thread with nontemporal stores.
constexpr int kTriadVariants = 3;
hipError_t launch_triad_variant(int v, const double* a, const double* b, double* dst, long long n,
                                hipStream_t st);
hipError_t launch_copy_interior(const double* src, double* dst, int nx, int ny, int nz,
                                long long ssy, long long ssz, long long dsy, long long dsz,
                                hipStream_t st);
hipError_t launch_set_int(int* p, int n, int v, hipStream_t st);

}  // namespace j3d
