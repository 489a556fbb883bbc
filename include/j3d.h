/*
 * j3d.h -- C ABI of libj3d: 3D 7-point Jacobi / Poisson kernels for AMD
 * Instinct MI355X (gfx950), with Fortran array semantics.
 *
 * The computation is the Fortran loop nest that the paper's jacobi
 * benchmark runs (Sec. "Flang performance comparison"), taken to three
 * dimensions as a Poisson problem -Lap(u) = f on a grid with spacing h:
 *
 *   sweep:     u'(i,j,k) = (u(i-1,j,k) + u(i+1,j,k) + u(i,j-1,k) + u(i,j+1,k)
 *                           + u(i,j,k-1) + u(i,j,k+1) + h^2 f(i,j,k)) / 6
 *   residual:  r(i,j,k)  = f(i,j,k) - (6 u(i,j,k) - [same six-neighbour sum]) / h^2
 *   norm:      ||r||_2   = sqrt(sum of r^2 over the interior)
 *
 * The norm is a sum reduction initialised at zero, the pattern the paper
 * lowers Fortran's sum/dot_product intrinsics to (Sec. "Handling of other
 * constructs", Listing 8).  Sums of neighbours are formed in the order
 * x-, x+, y-, y+, z-, z+ and no multiply-add is contracted, so results are
 * reproducible bit for bit.
 *
 * ARRAYS.  Every field is a Fortran array with explicit bounds, described by
 * a j3d_array in the manner of an MLIR memref (base, sizes, strides; Sec.
 * "Handling of memory"): element (i,j,k) lives at
 *     base + (i-lbound[0])*stride[0] + (j-lbound[1])*stride[1] + (k-lbound[2])*stride[2]
 * elements, which is Fortran's lower-bound subtraction.  The outermost
 * layer on every side is a one-cell halo holding Dirichlet boundary values;
 * the interior is lbound+1 .. ubound-1 on each axis and must be at least one
 * cell wide.  x is the unit-stride (column-major) axis.  Strided subviews
 * are accepted as they are, without a copy.  Kernels read the halo of their
 * input and never write any halo.
 *
 * INTENT.  A pointer argument is const exactly when the call only reads
 * what it points to (intent(in)).  An array descriptor, or a table of
 * descriptors, is not const when the call writes the array it describes,
 * whether it overwrites it (intent(out)) or reads and then overwrites it
 * (intent(inout)); the descriptor struct itself is never modified.
 * Scalars are passed by value (the paper lowers intent(in) scalars to
 * values, Sec. "Handling of control structures").  Inputs and outputs of one call must not
 * overlap in memory (Fortran's rule for modified dummy arguments; an
 * in-place Jacobi sweep would turn into an order-dependent Gauss-Seidel
 * sweep): overlap is rejected with J3D_EALIAS.
 *
 * OWNERSHIP.  Array memory belongs to the caller: the library never
 * allocates, reallocates or frees it.  It must stay valid until the stream
 * has passed the call.  Scratch memory (per-tile partial sums, flags,
 * solver work arrays, captured graphs) belongs to the library, is cached per
 * device and stream, and is released by j3d_release_cache().
 *
 * STREAMS.  `stream` is a hipStream_t passed as void* (NULL: the null
 * stream).  Calls are asynchronous and stream-ordered unless stated.
 *
 * ERRORS.  Every call returns J3D_OK (0) or a negative J3D_E* code; no
 * exception crosses the ABI.  j3d_last_error() returns a message for the
 * last failure on the calling thread.  Argument checks happen before any
 * device work is queued: a call that fails validation has no effect.
 * Device faults of asynchronous work surface as J3D_EHIP at a later
 * synchronising call.
 */
#ifndef J3D_H
#define J3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define J3D_ABI_VERSION 2

/* dtype codes */
#define J3D_F64 0
#define J3D_F32 1

/* status codes */
#define J3D_OK 0
#define J3D_EINVAL (-1)     /* null pointer, bad bounds/strides, n < 1, h <= 0 or not finite */
#define J3D_EDTYPE (-2)     /* wrong element type for the argument */
#define J3D_EALIAS (-3)     /* inputs and outputs overlap */
#define J3D_ENOMEM (-4)     /* library scratch allocation failed */
#define J3D_EBUDGET (-5)    /* a served request can never fit the memory budget */
#define J3D_EHIP (-6)       /* HIP runtime error (message in j3d_last_error) */
#define J3D_ENONFINITE (-7) /* residual is NaN or Inf */
#define J3D_EAGAIN (-8)     /* serve queue full; try again later */
#define J3D_ESTATE (-9)     /* call not valid in the object's current state */

/* flags for jacobi3d_sweep */
#define J3D_HOST_RESULT 1u  /* resid_out is a host pointer; the call waits for the stream */
/* flags for jacobi3d_sweep3: the fused residual is that of the iterate after
 * the pass's first sweep, J(u_in), or after its second, J(J(u_in)), instead
 * of u_in's (at most one of the two) */
#define J3D_RESID_AFTER_1 2u
#define J3D_RESID_AFTER_2 4u

/*
 * A Fortran array u(lbound[0]:ubound[0], lbound[1]:ubound[1], lbound[2]:ubound[2]).
 * base points at element (lbound[0], lbound[1], lbound[2]) in device memory.
 * Bounds are inclusive and include the one-cell halo.  Strides are in
 * elements: stride[0] must be 1, stride[1] >= extent[0], stride[2] >=
 * stride[1]*extent[1], where extent[d] = ubound[d]-lbound[d]+1 >= 3.  The
 * largest element offset must be below 2^31, except for the advection
 * entry points and the fills, which only need the offsets within one
 * z-plane below 2^31 (and the whole array below 2^46 elements).
 */
typedef struct j3d_array {
  void* base;
  int32_t dtype;      /* J3D_F64 or J3D_F32 */
  int32_t reserved;   /* must be 0 */
  int64_t lbound[3];
  int64_t ubound[3];
  int64_t stride[3];
} j3d_array;

/* Library version (J3D_ABI_VERSION) and the last error text of this thread. */
int j3d_abi_version(void);
const char* j3d_last_error(void);

/*
 * Host-only: the element offset of Fortran index (i,j,k) in `a`, computed by
 * lower-bound subtraction (Sec. "Handling of memory", Listings 6-7).  Returns
 * J3D_EINVAL if `a` is not a valid descriptor or (i,j,k) lies outside its
 * bounds.  Touches no device.
 */
int j3d_element_offset(const j3d_array* a, int64_t i, int64_t j, int64_t k, int64_t* offset);

/*
 * Host-only: validate a descriptor for use as a field of the given dtype.
 * Returns J3D_OK, J3D_EINVAL or J3D_EDTYPE.  Touches no device.
 */
int j3d_check_array(const j3d_array* a, int32_t dtype);

/*
 * One Jacobi sweep u_out = J(u_in; f, h) over the interior (the update
 * formula above).  All three arrays have the same dtype (FP64 or FP32) and
 * the same interior extents; each may have its own bounds and strides.
 * u_out's halo is not written (give both ping-pong arrays the same halo).
 * If resid_out is not NULL, the L2 norm of the residual of u_in,
 * ||f - A u_in||_2, is computed in FP64 in the same pass (from the values
 * the sweep loads, so it costs no extra memory traffic) and stored to
 * *resid_out: a device address, or a host address with J3D_HOST_RESULT
 * (then the call synchronises the stream).  The fused residual needs FP64
 * arrays (J3D_EDTYPE otherwise).  FP32 sweeps use h^2 = (float)(h*h).
 */
int jacobi3d_sweep(const j3d_array* u_in, j3d_array* u_out, const j3d_array* f,
                   double h, uint32_t flags, double* resid_out, void* stream);

/*
 * Two Jacobi sweeps in one pass over memory: u_out = J(J(u_in; f, h)), all
 * three arrays FP64 or all FP32.  The intermediate iterate stays on chip
 * (temporal blocking in z), so the pass streams u_in and f once and writes
 * u_out once for two sweeps' worth of updates; every point is computed
 * exactly as two jacobi3d_sweep calls would (bit-identical).  resid_out and
 * flags are as in jacobi3d_sweep: the fused residual is that of u_in and
 * needs FP64 arrays.
 */
int jacobi3d_sweep2(const j3d_array* u_in, j3d_array* u_out, const j3d_array* f,
                    double h, uint32_t flags, double* resid_out, void* stream);

/*
 * Three Jacobi sweeps in one pass over memory: u_out = J(J(J(u_in; f, h))),
 * as jacobi3d_sweep2 with a third sweep (bit-identical to three
 * jacobi3d_sweep calls).  The two intermediate iterates stay on chip, so the
 * pass streams u_in and f once and writes u_out once for three sweeps' worth
 * of updates.  resid_out and flags as in jacobi3d_sweep (the residual of
 * u_in; FP64 only), and with J3D_RESID_AFTER_1 or J3D_RESID_AFTER_2 the
 * residual of the first or second intermediate iterate, formed on chip from
 * the same neighbour sum that produces the next sweep (so a fixed-length
 * run of three-sweep passes can report the residual of any iterate it
 * passes through; EINVAL if both are set or without resid_out).
 */
int jacobi3d_sweep3(const j3d_array* u_in, j3d_array* u_out, const j3d_array* f,
                    double h, uint32_t flags, double* resid_out, void* stream);

/*
 * jacobi3d_sweep3 with its fused residual, allocating nothing: for callers
 * that cannot allocate device memory (code being captured into a HIP graph,
 * serving loops that must not call hipMalloc, hosts that forbid it).
 * Arguments, flags and results as in jacobi3d_sweep3, with the same tile
 * shape and kernels (u_out and *resid_out are bit-identical to it), except:
 * u_in, u_out, f are FP64 and resid_out is a non-null device address
 * (J3D_HOST_RESULT is rejected).  The per-tile partial sums live in a
 * static device array of 65536 doubles (512 KiB) that every GPU the library
 * runs on holds until the process ends; a grid whose three-sweep tiling
 * needs more tiles than that returns J3D_EINVAL before any device work
 * (with the default tile shapes every cube within the 2^31-element limit
 * fits; a smaller pinned or autotuned tile shape can exceed it).  Every call on
 * one GPU uses that GPU's one array, so calls that may overlap in time on
 * the same GPU (other streams, other threads) race and must be ordered by
 * the caller.  Errors: as jacobi3d_sweep3, and J3D_EINVAL for the cases
 * above.
 */
int jacobi3d_sweep3_noalloc(const j3d_array* u_in, j3d_array* u_out, const j3d_array* f,
                            double h, uint32_t flags, double* resid_out, void* stream);

/*
 * ||f - A u||_2 over the interior, in FP64 (u and f FP64).  `out` is a
 * device address, or a host address with J3D_HOST_RESULT in flags (then
 * the call synchronises the stream).  The flags argument is the same one
 * jacobi3d_sweep takes for its resid_out: without it a caller that wants
 * the number on the host would need a device buffer and a copy of its own.
 */
int residual_l2(const j3d_array* u, const j3d_array* f, double h, uint32_t flags,
                double* out, void* stream);

/*
 * Fortran's sum and dot_product intrinsics over contiguous FP64 vectors
 * (a whole contiguous array of any rank is the vector of its elements).
 * The paper lowers both to a reduction initialised at zero that adds every
 * element, or every elementwise product, into the accumulator (Sec.
 * "Handling of other constructs"); its intrinsics table runs them on a
 * 32768 x 32768 FP64 array (sum) and on FP64 vectors of 134 million
 * elements (dot_product).
 *
 * x, y: device arrays of n doubles (borrowed, 8-byte aligned, read only; x
 * and y may be the same array).  n >= 0 (n = 0 gives 0).  *out: a device
 * address (must not overlap x or y), or a host address with
 * J3D_HOST_RESULT in flags (then the call synchronises the stream).
 * Products are rounded to FP64 before they are added (no fused
 * multiply-add).  The additions follow a fixed partition of n into blocks
 * and a fixed tree within and across blocks, so the result depends only on
 * the inputs and n, bit for bit; its error is within the recursive-summation
 * bound of that tree.  Errors: J3D_EINVAL (null or misaligned pointer,
 * n < 0, unknown flags), J3D_EALIAS, J3D_EHIP.
 */
int j3d_sum(const double* x, int64_t n, uint32_t flags, double* out, void* stream);
int j3d_dot(const double* x, const double* y, int64_t n, uint32_t flags, double* out, void* stream);

/*
 * The paper's jacobi benchmark (Sec. "Flang performance comparison": Jacobi
 * iteration for Laplace's equation on a 1024 x 1024 grid, 100000
 * iterations): nsweeps sweeps of
 *   u'(i,j) = (((u(i-1,j) + u(i+1,j)) + u(i,j-1)) + u(i,j+1)) / 4
 * over the interior of rank-2 FP64 arrays (j3d_array with lbound[2] ==
 * ubound[2]; the halo holds the boundary values, the same in both arrays).
 * Sweeps alternate u_a -> u_b -> u_a ...: the result is in u_a when nsweeps
 * is even, else in u_b; both arrays are written.  If resid_out is not NULL,
 * ||r||_2 of the result, r = (S - 4 u) / h^2 over the interior (Laplace's
 * equation, right-hand side zero), goes to *resid_out (device; host with
 * J3D_HOST_RESULT).  Every sweep has exactly the arithmetic above (bit for
 * bit the same as one sweep at a time).  Errors: J3D_EINVAL (bounds, rank,
 * nsweeps < 0, h with resid_out), J3D_EDTYPE, J3D_EALIAS, J3D_EHIP.
 */
int jacobi2d_sweeps(j3d_array* u_a, j3d_array* u_b, int64_t nsweeps, double h,
                    uint32_t flags, double* resid_out, void* stream);

/*
 * Multi-field stencils.  The paper compares compilers on two stencil codes
 * it does not list, pw-advection (three fields on a 2048 x 1024 x 1024
 * grid) and tra-adv (six fields on 1024 x 512 x 512, 20 iterations), Sec.
 * "Flang performance comparison"; these two calls are documented stencils
 * with those field counts and shapes.
 *
 * pw_advection: momentum advection in the centred flux form of Piacsek and
 * Williams (1970) on a staggered grid.  u(i,j,k) is the x-velocity on the
 * east face of cell (i,j,k), v on its north face, w on its top face.  The
 * tendency of each component at its own point is minus the divergence of
 * its momentum flux; the flux through a face is the advecting velocity
 * averaged onto the face times the advected component averaged onto it,
 * each the mean of two neighbours.  With c = 0.25 / spacing and, per
 * direction, am, bm (ap, bp) the two-point sums of advecting velocity and
 * advected component at the lower (upper) face,
 *   D = (am * bm - ap * bp) * c,   tendency = (Dx + Dy) + Dz,
 * which is exact for the arithmetic written (no fused multiply-add).
 * u, v, w: FP64 inputs (0:nx+1, 0:ny+1, 0:nz+1) with equal bounds and
 * strides, halo = boundary values.  su, sv, sw: FP64 outputs with the same
 * bounds (their own common strides); only the interior is written.
 * dx, dy, dz > 0 and finite.  Outputs may not overlap each other or the
 * inputs.  Asynchronous on `stream`.  Errors: J3D_EINVAL (bounds, strides,
 * spacing), J3D_EDTYPE, J3D_EALIAS, J3D_EHIP.
 */
int pw_advection(const j3d_array* u, const j3d_array* v, const j3d_array* w,
                 j3d_array* su, j3d_array* sv, j3d_array* sw,
                 double dx, double dy, double dz, void* stream);

/*
 * tracer_advection: niter explicit donor-cell (first-order upwind) steps of
 * a tracer t carried by volume transports u, v, w through the east, north
 * and top faces of each cell:
 *   F = q+ * t(cell below the face) + q- * t(cell above the face),
 *   q+ = q if q > 0 else 0, q- = q if q < 0 else 0,
 *   t' = t - r * (((Fe - Fw) + (Fn - Fs)) + (Ft - Fb)),
 * r = time step / cell volume.  Six FP64 arrays (0:nx+1, 0:ny+1, 0:nz+1)
 * with equal bounds and strides: t_a holds the initial tracer, its halo the
 * boundary values, which t_b must hold too; u(0,..), v(..,0,..), w(..,0)
 * are the transports through the lower domain faces.  Steps alternate
 * t_a -> t_b -> t_a ...: the result is in t_a when niter is even, else in
 * t_b; the interiors of both are written (for niter >= 2).  niter >= 0.
 * Steps run two per pass over memory where the parity allows (each point of
 * either step has exactly the arithmetic above).
 * t_a and t_b may not overlap each other or u, v, w, r.  Asynchronous on
 * `stream`.  Errors: J3D_EINVAL, J3D_EDTYPE, J3D_EALIAS, J3D_EHIP.
 */
int tracer_advection(j3d_array* t_a, j3d_array* t_b, const j3d_array* u,
                     const j3d_array* v, const j3d_array* w, const j3d_array* r,
                     int64_t niter, void* stream);

/* Solver modes */
#define J3D_MODE_FP64 0  /* FP64 Jacobi sweeps */
#define J3D_MODE_MIXED 1 /* FP32 correction sweeps with FP64 defect correction */

typedef struct j3d_solve_opts {
  int32_t mode;          /* J3D_MODE_FP64 or J3D_MODE_MIXED */
  int32_t check_every;   /* FP64 mode: sweeps between residual checks (>= 1) */
  int32_t inner_sweeps;  /* MIXED mode: FP32 sweeps per defect step (>= 1) */
  int32_t reserved;      /* must be 0 */
  int64_t max_sweeps;    /* sweep cap (>= 0); MIXED counts FP32 sweeps */
  double rtol;           /* stop at the first check with ||r||_2 <= rtol * ||f||_2 */
  double* history;       /* host array for ||r||_2 at every check, in order (nullable) */
  int64_t history_cap;   /* capacity of history */
} j3d_solve_opts;

typedef struct j3d_solve_result {
  int64_t sweeps;        /* sweeps performed up to the returned iterate */
  double resid;          /* ||f - A u||_2 of the returned u (FP64) */
  double resid0;         /* ||f - A u0||_2 of the initial guess */
  double norm_f;         /* ||f||_2 */
  int32_t converged;     /* 1 if resid <= rtol * norm_f */
  int32_t status;        /* J3D_OK or J3D_ENONFINITE */
  int64_t history_len;   /* entries written to opts->history */
} j3d_solve_result;

/*
 * Solve A u = f by Jacobi iteration from the initial guess in u; the result
 * overwrites u's interior (u, f FP64; halo of u = Dirichlet data).
 *
 * FP64 mode: the residual of the iterate after sweep s is checked at
 * s = 0, c, 2c, ... (c = check_every), fused into sweep s+1; the solve stops
 * at the first check with ||r|| <= rtol*||f|| or after max_sweeps sweeps.
 * This is an early-exit loop (cf. the paper's lowering of iterate_while,
 * Sec. "Handling of control structures"); the test runs on the device.
 *
 * MIXED mode (defect correction): each cycle does an FP64 defect step
 * (u += e from the previous cycle, r = f - A u, ||r||, convergence test)
 * then min(inner_sweeps, sweeps left) FP32 Jacobi sweeps on A e = (float) r
 * from e = 0 with h^2 = (float)(h*h).  The last cycle ends with a defect
 * step, so u includes every correction and `resid` is its residual.
 *
 * Sweeps run two or three per pass over memory (as jacobi3d_sweep2 and
 * jacobi3d_sweep3), three when the arrays of a pass exceed 512 MB, i.e.
 * overflow the last-level cache; J3D_SOLVE_SWEEPS_PER_PASS=1, 2 or 3 fixes
 * the pass length.  Every schedule gives the same iterate bit for bit.
 *
 * Not converging is not an error (converged = 0).  A NaN/Inf residual stops
 * the solve with status and return value J3D_ENONFINITE.  The call blocks
 * until the solve has finished.  Work arrays (one FP64 array in FP64 mode,
 * three FP32 arrays in MIXED mode) are allocated by the library and cached.
 */
int poisson_solve(j3d_array* u, const j3d_array* f, double h,
                  const j3d_solve_opts* opts, j3d_solve_result* result, void* stream);

/* One grid of a batch: two ping-pong arrays with equal halos, and f (all FP64). */
typedef struct j3d_grid {
  j3d_array u_a;   /* initial iterate; holds the result if nsweeps is even */
  j3d_array u_b;   /* second buffer; holds the result if nsweeps is odd */
  j3d_array f;
  double h;
} j3d_grid;

/*
 * Tile shape of the sweep kernels.  A workgroup of rows x cols 64-lane
 * wavefronts sweeps 64*cols x-points x (rows x rows-per-thread) y-rows x
 * `planes` z-planes,
 * marching through z with the previous, current and next plane in
 * registers.  variant is a bit set: 1 stages each plane in LDS (else x/y
 * neighbours are read through the cache); 2 and 16 give each thread
 * 2^(bit 2 + 2 x bit 16) consecutive rows (register blocking in y); 4 writes
 * outputs with nontemporal stores (8 is not used).  persistent = 1 launches a
 * fixed grid of workgroups that stride over the tile list, 0 one workgroup
 * per tile.  order maps dispatch order to tiles: 0 gives each of the 8 XCDs
 * one contiguous block of tiles, 1 keeps the launch order, 2 cuts each z-slab
 * into 8 contiguous chunks, one per XCD.  cols is the number of wavefronts
 * side by side along x (1, 2 or 4): a tile is 64 x cols points wide.
 */
typedef struct j3d_tune {
  int32_t rows;
  int32_t planes;
  int32_t variant;
  int32_t persistent;
  int32_t order;
  int32_t cols;
} j3d_tune;

/* Number of supported tile shapes, and the i-th one (host-only). */
int j3d_tune_count(void);
int j3d_tune_get(int32_t index, j3d_tune* out);

/*
 * Sweep `ngrids` independent grids of uneven sizes `nsweeps` times each,
 * all grids in one kernel per sweep over a packed tile list, the sweeps
 * captured in one HIP graph (cached per argument set and stream, replayed on
 * later identical calls).  The result of grid g lands in u_a if nsweeps is
 * even, else in u_b.  If resid_out is not NULL it is a device array of
 * ngrids * (nsweeps/resid_every + 1) doubles: row g holds ||f - A u||_2 of
 * grid g after sweeps 0, e, 2e, ... (e = resid_every), fused into the
 * following sweep where there is one.  Each grid's numbers equal those of
 * the same grid swept alone with the same tile shapes and pass kind (one,
 * two or up to three sweeps per pass, below), bit for bit; the iterates are
 * the same bit for bit in every case, the residual norms agree to rounding.
 * tune = NULL selects the tile shape with the autotuner (timed once per
 * batch shape class and cached; J3D_TUNE_CACHE names an optional file).
 * When nsweeps >= 2 and resid_every is even (or resid_out is NULL), sweeps
 * run two per pass over memory (as jacobi3d_sweep2) if that is faster on
 * this batch shape class, timed once per process; the environment variable
 * J3D_BATCH_PAIRS=0 or =1 forces one-sweep or two-sweep passes.  When
 * nsweeps >= 3 and the three-sweep pass (as jacobi3d_sweep3) is faster per
 * sweep than those, the call runs three-sweep passes straight through, for
 * any resid_every: each residual is fused into the pass that forms its
 * iterate, at that stage of the pass (a shorter pass covers the rest, and
 * one pass is split when needed to keep the u_a/u_b placement above);
 * J3D_BATCH_TRIPLES=0 or =1 forces this off or on.  The three-sweep shape
 * is timed on the batch among the jacobi3d_sweep3 shapes in the XCD-blocked
 * tile order (order 0) and in a balanced order (order 3, batches only: the
 * tile list cut into one run of about equal work per XCD, each run longest
 * tile first); J3D_BATCH_TILE3="rows,planes,variant,order" fixes it
 * (J3D_EINVAL for a shape the three-sweep pass does not have).
 */
int jacobi3d_sweep_batch(int32_t ngrids, j3d_grid* grids, int32_t nsweeps,
                         int32_t resid_every, double* resid_out, const j3d_tune* tune,
                         void* stream);

/* Autotune: time each supported tile shape on these grids (one sweep each,
 * after a warm-up) and write the fastest to *best.  Writes to u_b only.
 * Blocks until done. */
int j3d_autotune(int32_t ngrids, j3d_grid* grids, j3d_tune* best, void* stream);

/* The plan of this thread's most recent jacobi3d_sweep_batch call that
 * launched work: *sweeps_per_pass = 3, 2 or 1 for three-, two- or one-sweep
 * passes (the kind its passes of full length had), *shape = the tile shape
 * of those passes (order 3: the balanced slot order of three-sweep passes).
 * Both written by the call (intent(out)).  Host-only; J3D_EINVAL for a null
 * pointer, J3D_ESTATE when this thread has made no such call. */
int j3d_batch_last_plan(int32_t* sweeps_per_pass, j3d_tune* shape);

/* Kernel kinds for the single-grid tuning calls: J3D_F64 and J3D_F32 name
 * the one-sweep passes of that element type, J3D_KIND_F64X2 and
 * J3D_KIND_F32X2 the two-sweep passes of jacobi3d_sweep2 (the FP32 one also
 * runs the correction sweeps of the mixed solve).  Two-sweep shapes have one
 * wavefront along x (cols = 1) and rows x rows-per-thread between 4 and 32
 * (a block of that many rows has that many minus 2 output rows, and 60
 * output columns); variant bits 2, 4, 16 as above, no LDS bit. */
#define J3D_KIND_F64X2 2
#define J3D_KIND_F32X2 3
/* The three-sweep passes of jacobi3d_sweep3 (the FP32 one also runs the
 * correction sweeps of the mixed solve): one wavefront along x, not
 * persistent, rows 2, 4, 8 or 16 wavefronts of 2 or 4 rows per thread
 * (variants 6 and 20) with rows x rows-per-thread between 8 and 32; a block
 * has that many rows minus 4 output rows and 58 output columns. */
#define J3D_KIND_F64X3 4
#define J3D_KIND_F32X3 5

/* Autotune the single-grid pass of this kind and interior shape on
 * library-allocated scratch arrays; the choice is used by jacobi3d_sweep,
 * jacobi3d_sweep2, jacobi3d_sweep3, residual_l2 and poisson_solve for this
 * shape from then on.  Blocks. */
int j3d_autotune_single(int32_t kind, int32_t nx, int32_t ny, int32_t nz, j3d_tune* best,
                        void* stream);

/* Pin the tile shape used for single-grid calls of this kind and shape. */
int j3d_tune_set_single(int32_t kind, int32_t nx, int32_t ny, int32_t nz, const j3d_tune* t);

/* The tile shape single-grid calls of this kind and interior shape use now:
 * the pinned or autotuned one, else the library default (host-only). */
int j3d_tune_query_single(int32_t kind, int32_t nx, int32_t ny, int32_t nz, j3d_tune* out);

/* ------------------------------------------------------------------ */
/* Serving: continuous batching of Poisson solves under a memory budget */
/* ------------------------------------------------------------------ */

typedef struct j3d_server j3d_server;

/* Precision of a server's solves */
#define J3D_SERVE_MIXED 0 /* FP32 correction sweeps with FP64 defect correction */
#define J3D_SERVE_FP64 1  /* plain FP64 Jacobi sweeps (the reference form) */

typedef struct j3d_serve_opts {
  uint64_t hbm_budget_bytes;  /* device memory the server may hold for request state */
  int32_t max_slots;          /* maximum concurrently active requests */
  int32_t cycle_sweeps;       /* sweeps per cycle (e.g. 50): FP32 sweeps per defect-correction
                                 cycle, or FP64 sweeps between residual checks */
  int32_t device;             /* HIP device ordinal */
  int32_t queue_cap;          /* maximum queued (not yet admitted) requests */
  uint64_t max_active_points; /* admit while active interior points stay at or below
                                 this (a request is admitted regardless when nothing is
                                 active); 0: no limit */
  int32_t precision;          /* J3D_SERVE_MIXED or J3D_SERVE_FP64 */
  int32_t reserved;           /* must be 0 */
} j3d_serve_opts;

typedef struct j3d_request {
  int32_t nx, ny, nz;         /* interior extents (>= 1) */
  int32_t reserved;           /* must be 0 */
  double h;                   /* grid spacing (> 0) */
  const double* f_host;       /* padded right-hand side, (nz+2)(ny+2)(nx+2) doubles
                                 with x fastest; NULL: draw f ~ U[-1,1) from `seed` */
  uint64_t seed;              /* used when f_host is NULL */
  double rtol;                /* target ||r||_2 / ||f||_2 */
  int64_t max_sweeps;         /* FP32 sweep cap */
  double* u_host;             /* nullable: receives the padded solution when done */
} j3d_request;

typedef struct j3d_result {
  uint64_t ticket;
  int32_t status;             /* J3D_OK or J3D_ENONFINITE */
  int32_t converged;
  int64_t sweeps;
  double resid;               /* FP64 ||r||_2 of the returned solution */
  double norm_f;
  double t_submit, t_admit, t_done;  /* seconds on the server's monotonic clock */
} j3d_result;

/* Bytes of device state one request of this size holds while active on a
 * mixed-precision server (u, f FP64; r, two corrections FP32: about 28 bytes
 * per padded point), and on a server of either precision (FP64: u, f and a
 * second iterate, about 24 bytes per padded point); 0 for bad arguments. */
uint64_t j3d_request_bytes(int32_t nx, int32_t ny, int32_t nz);
uint64_t j3d_request_state_bytes(int32_t precision, int32_t nx, int32_t ny, int32_t nz);

/*
 * Create a server with its own worker thread and HIP stream on opts->device.
 * Requests are admitted in arrival order while their state fits the budget,
 * a slot is free and the active points stay within max_active_points (enough
 * to fill the GPU: more only delays every request); every active request is
 * a slot in one batched
 * mixed-precision cycle (FP64 defect step + cycle_sweeps FP32 sweeps over
 * all slots' tiles).  At every cycle boundary converged or capped requests
 * retire and waiting ones are admitted (continuous batching).  A request's
 * result does not depend on which others share its cycles.  The FP32 sweeps
 * of a cycle run two per pass over memory, or three when the cycle's FP32
 * state exceeds 512 MB (J3D_SERVE_TRIPLES=0 or =1 forces one or the other);
 * the iterates are the same bit for bit either way.  A request's result is
 * that of poisson_solve in MIXED mode with inner_sweeps = cycle_sweeps and
 * max_sweeps rounded up to whole cycles.
 * With precision J3D_SERVE_FP64 a cycle is instead the FP64 residual check
 * of each slot's current iterate followed by cycle_sweeps FP64 Jacobi sweeps
 * (two or three per pass over memory, three when the cycle's FP64 state
 * exceeds 512 MB), so a request's result is that of poisson_solve in FP64
 * mode with check_every = cycle_sweeps: the plain form the mixed one is
 * measured against, under the same admission and batching.  Errors:
 * J3D_EINVAL (bad options, precision or reserved), J3D_EHIP.
 */
int poisson_serve_create(const j3d_serve_opts* opts, j3d_server** out);
/* Queue a request.  J3D_EBUDGET if it can never fit; J3D_EAGAIN if the queue
 * is full.  f_host is copied before the call returns; u_host must stay valid
 * until the ticket's result has been polled. */
int poisson_serve_submit(j3d_server* s, const j3d_request* req, uint64_t* ticket);
/* Move up to cap finished results into out[0..*n). Non-blocking. */
int poisson_serve_poll(j3d_server* s, j3d_result* out, int32_t cap, int32_t* n);
/* Block until every submitted request has finished (or timeout_s elapses;
 * returns J3D_EAGAIN on timeout).  timeout_s <= 0 waits forever. */
int poisson_serve_drain(j3d_server* s, double timeout_s);
/* Current server clock (seconds) and counters: active, queued, finished. */
int poisson_serve_stats(j3d_server* s, double* now, int32_t* active, int32_t* queued,
                        int64_t* finished);
/* Stop the worker (after finishing the cycle in flight) and free all state. */
int poisson_serve_destroy(j3d_server* s);

/* ------------------------------------------------------------------ */
/* Utilities                                                           */
/* ------------------------------------------------------------------ */

/*
 * Fill the interior of an FP64 array with U[lo,hi) draws, counter-based:
 * point (i,j,k) takes counter (i-1) + nx*((j-1) + ny*(k-1)) of SplitMix64
 * (Steele, Lea, Flood 2014) seeded with seed XOR (stream_id << 40); value
 * lo + (hi-lo) * ((bits >> 11) * 2^-53).  The halo is set to `halo`.
 */
int j3d_fill_uniform(j3d_array* a, uint64_t seed, uint32_t stream_id, double lo,
                     double hi, double halo, void* stream);

/* Set every element (halo included) of an FP64 or FP32 array to `value`. */
int j3d_fill_const(j3d_array* a, double value, void* stream);

/*
 * Streaming probe for the achievable memory bandwidth: copies n doubles from
 * src to dst (device) `reps` times with each of several copy kernels (a
 * grid-stride loop over 16-byte elements; one or four 16-byte elements per
 * thread, each with plain or nontemporal loads and stores) and returns the
 * best rate in GB/s (bytes read + written per second).  Blocks.
 */
int j3d_bandwidth_probe(const double* src, double* dst, int64_t n, int32_t reps,
                        double* gbps, void* stream);

/*
 * The same for the traffic mix of the sweep passes (two streams read, one
 * written, in equal lengths): dst[i] = a[i] + b[i] over n doubles (device),
 * `reps` times with each of three kernels (one or four 16-byte elements per
 * thread, nontemporal or plain stores); returns the best rate in GB/s
 * (bytes read + written per second).  dst may not overlap a or b; a and b
 * may coincide.  Buffers 16-byte aligned, n >= 2.  Blocks.
 */
int j3d_bandwidth_probe_triad(const double* a, const double* b, double* dst, int64_t n,
                              int32_t reps, double* gbps, void* stream);

/* Free every cached scratch buffer and graph of the calling process. */
int j3d_release_cache(void);

#ifdef __cplusplus
}
#endif

#endif /* J3D_H */
