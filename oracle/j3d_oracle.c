/*
 * Plain CPU oracle for the 3D 7-point Jacobi / Poisson hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the HIP path is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg load it; the product
 * library never links, loads or calls it, and it shares no code, header or
 * constant with the product.
 *
 * What it computes (each a direct transcription of a definition, no blocking
 * or fusion):
 *   - the Jacobi sweep of the 7-point Poisson operator,
 *       u'(i,j,k) = (sum of the 6 neighbours + h^2 f(i,j,k)) / 6,
 *     over the interior of a Fortran array u(0:nx+1,0:ny+1,0:nz+1) whose
 *     one-cell halo holds the Dirichlet data.  This is the loop nest the
 *     paper's jacobi benchmark runs (Sec. "Flang performance comparison",
 *     generalised from its 2D Laplace grid to 3D Poisson);
 *   - the residual r = f - A u with A u = (6 u - sum of neighbours) / h^2,
 *     and its Euclidean norm over the interior, a sum reduction initialised
 *     at zero as the paper lowers Fortran's sum intrinsic (Sec. "Handling of
 *     other constructs", Listing 8);
 *   - the plain FP64 solve (sweep until ||r||/||f|| <= tol, tested every
 *     check_every sweeps, an early-exit loop like the paper's iterate_while
 *     lowering, Sec. "Handling of control structures");
 *   - the mixed-precision solve: FP32 Jacobi sweeps on a correction e with
 *     FP64 defect correction u += e, r = f - A u.
 *
 * Arithmetic order is fixed and contraction is off (-ffp-contract=off):
 *   S  = ((((u[i-1] + u[i+1]) + u[j-1]) + u[j+1]) + u[k-1]) + u[k+1]
 *   u' = (S + h2 * f) / 6,          h2 = h * h
 *   r  = f - (6 * u - S) / h2
 * Norms use Neumaier-compensated summation, per z-plane and then over planes
 * in plane order, so the result does not depend on the thread count.
 *
 * Addressing follows Fortran's lbound subtraction (Sec. "Handling of
 * memory"): element (i,j,k), counted from the array's lower bounds, sits at
 * a[i + sy*j + sz*k] with unit stride in x.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef int64_t idx_t;

#define AT(i, j, k) ((i) + sy * (j) + sz * (k))

/* Number of threads the loops below run on. */
int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Compensated summation                                               */
/* ------------------------------------------------------------------ */

typedef struct { double s, c; } nsum;

static void nsum_add(nsum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

/* ------------------------------------------------------------------ */
/* FP64 sweep                                                          */
/* ------------------------------------------------------------------ */

void oracle_sweep_f64(const double* u, double* un, const double* f,
                      idx_t nx, idx_t ny, idx_t nz, idx_t sy, idx_t sz,
                      double h) {
  const double h2 = h * h;
#pragma omp parallel for schedule(static)
  for (idx_t k = 1; k <= nz; ++k)
    for (idx_t j = 1; j <= ny; ++j)
      for (idx_t i = 1; i <= nx; ++i) {
        double s = u[AT(i - 1, j, k)] + u[AT(i + 1, j, k)];
        s = s + u[AT(i, j - 1, k)];
        s = s + u[AT(i, j + 1, k)];
        s = s + u[AT(i, j, k - 1)];
        s = s + u[AT(i, j, k + 1)];
        un[AT(i, j, k)] = (s + h2 * f[AT(i, j, k)]) / 6.0;
      }
}

/* Per-point residual r = f - A u (interior only; r's halo untouched). */
void oracle_residual_field_f64(const double* u, const double* f, double* r,
                               idx_t nx, idx_t ny, idx_t nz, idx_t sy, idx_t sz,
                               double h) {
  const double h2 = h * h;
#pragma omp parallel for schedule(static)
  for (idx_t k = 1; k <= nz; ++k)
    for (idx_t j = 1; j <= ny; ++j)
      for (idx_t i = 1; i <= nx; ++i) {
        double s = u[AT(i - 1, j, k)] + u[AT(i + 1, j, k)];
        s = s + u[AT(i, j - 1, k)];
        s = s + u[AT(i, j + 1, k)];
        s = s + u[AT(i, j, k - 1)];
        s = s + u[AT(i, j, k + 1)];
        r[AT(i, j, k)] = f[AT(i, j, k)] - (6.0 * u[AT(i, j, k)] - s) / h2;
      }
}

/* Sum of squares over the interior of a FP64 array, plane by plane. */
static double sumsq_planes(const double* a, idx_t nx, idx_t ny, idx_t nz,
                           idx_t sy, idx_t sz) {
  nsum* part = (nsum*)calloc((size_t)nz, sizeof(nsum));
#pragma omp parallel for schedule(static)
  for (idx_t k = 1; k <= nz; ++k) {
    nsum acc = {0.0, 0.0};
    for (idx_t j = 1; j <= ny; ++j)
      for (idx_t i = 1; i <= nx; ++i) {
        double v = a[AT(i, j, k)];
        nsum_add(&acc, v * v);
      }
    part[k - 1] = acc;
  }
  nsum tot = {0.0, 0.0};
  for (idx_t k = 0; k < nz; ++k) {
    nsum_add(&tot, part[k].s);
    nsum_add(&tot, part[k].c);
  }
  free(part);
  return tot.s + tot.c;
}

/* ||a||_2 over the interior. */
double oracle_norm2_f64(const double* a, idx_t nx, idx_t ny, idx_t nz,
                        idx_t sy, idx_t sz) {
  return sqrt(sumsq_planes(a, nx, ny, nz, sy, sz));
}

/* ||f - A u||_2 over the interior. */
double oracle_residual_l2_f64(const double* u, const double* f,
                              idx_t nx, idx_t ny, idx_t nz, idx_t sy, idx_t sz,
                              double h) {
  const double h2 = h * h;
  nsum* part = (nsum*)calloc((size_t)nz, sizeof(nsum));
#pragma omp parallel for schedule(static)
  for (idx_t k = 1; k <= nz; ++k) {
    nsum acc = {0.0, 0.0};
    for (idx_t j = 1; j <= ny; ++j)
      for (idx_t i = 1; i <= nx; ++i) {
        double s = u[AT(i - 1, j, k)] + u[AT(i + 1, j, k)];
        s = s + u[AT(i, j - 1, k)];
        s = s + u[AT(i, j + 1, k)];
        s = s + u[AT(i, j, k - 1)];
        s = s + u[AT(i, j, k + 1)];
        double r = f[AT(i, j, k)] - (6.0 * u[AT(i, j, k)] - s) / h2;
        nsum_add(&acc, r * r);
      }
    part[k - 1] = acc;
  }
  nsum tot = {0.0, 0.0};
  for (idx_t k = 0; k < nz; ++k) {
    nsum_add(&tot, part[k].s);
    nsum_add(&tot, part[k].c);
  }
  free(part);
  return sqrt(tot.s + tot.c);
}

/* ------------------------------------------------------------------ */
/* FP32 sweep (inner sweeps of the mixed-precision solve)              */
/* ------------------------------------------------------------------ */

void oracle_sweep_f32(const float* e, float* en, const float* r,
                      idx_t nx, idx_t ny, idx_t nz, idx_t sy, idx_t sz,
                      float h2) {
#pragma omp parallel for schedule(static)
  for (idx_t k = 1; k <= nz; ++k)
    for (idx_t j = 1; j <= ny; ++j)
      for (idx_t i = 1; i <= nx; ++i) {
        float s = e[AT(i - 1, j, k)] + e[AT(i + 1, j, k)];
        s = s + e[AT(i, j - 1, k)];
        s = s + e[AT(i, j + 1, k)];
        s = s + e[AT(i, j, k - 1)];
        s = s + e[AT(i, j, k + 1)];
        en[AT(i, j, k)] = (s + h2 * r[AT(i, j, k)]) / 6.0f;
      }
}

/*
 * FP64 defect step of the mixed solve: if e != NULL, u += (double) e over the
 * interior; then r = f - A u in FP64, r32 = (float) r, and return ||r||_2.
 * The update is finished over the whole grid before any residual is formed.
 */
double oracle_defect(double* u, const float* e, const double* f, float* r32,
                     idx_t nx, idx_t ny, idx_t nz,
                     idx_t sy, idx_t sz,     /* strides of u and f (FP64) */
                     idx_t sy4, idx_t sz4,   /* strides of e and r32 (FP32) */
                     double h) {
  const double h2 = h * h;
  if (e) {
#pragma omp parallel for schedule(static)
    for (idx_t k = 1; k <= nz; ++k)
      for (idx_t j = 1; j <= ny; ++j)
        for (idx_t i = 1; i <= nx; ++i)
          u[AT(i, j, k)] = u[AT(i, j, k)] + (double)e[i + sy4 * j + sz4 * k];
  }
  nsum* part = (nsum*)calloc((size_t)nz, sizeof(nsum));
#pragma omp parallel for schedule(static)
  for (idx_t k = 1; k <= nz; ++k) {
    nsum acc = {0.0, 0.0};
    for (idx_t j = 1; j <= ny; ++j)
      for (idx_t i = 1; i <= nx; ++i) {
        double s = u[AT(i - 1, j, k)] + u[AT(i + 1, j, k)];
        s = s + u[AT(i, j - 1, k)];
        s = s + u[AT(i, j + 1, k)];
        s = s + u[AT(i, j, k - 1)];
        s = s + u[AT(i, j, k + 1)];
        double r = f[AT(i, j, k)] - (6.0 * u[AT(i, j, k)] - s) / h2;
        r32[i + sy4 * j + sz4 * k] = (float)r;
        nsum_add(&acc, r * r);
      }
    part[k - 1] = acc;
  }
  nsum tot = {0.0, 0.0};
  for (idx_t k = 0; k < nz; ++k) {
    nsum_add(&tot, part[k].s);
    nsum_add(&tot, part[k].c);
  }
  free(part);
  return sqrt(tot.s + tot.c);
}

/* ------------------------------------------------------------------ */
/* Solves                                                              */
/* ------------------------------------------------------------------ */

/*
 * Result record shared by both solves (filled on return):
 *   out[0] sweeps performed
 *   out[1] final ||r||_2 of the returned iterate
 *   out[2] ||r_0||_2 of the initial guess
 *   out[3] ||f||_2
 *   out[4] 1 if converged, else 0
 *   out[5] number of history entries written
 */

/*
 * Plain FP64 Jacobi solve.  The residual r_s of the iterate after sweep s is
 * taken at s = 0, c, 2c, ... (c = check_every); the loop stops at the first
 * check with ||r_s|| <= rtol * ||f||, or after max_sweeps sweeps.  The
 * returned iterate is left in u (work is a second array of the same layout
 * whose halo equals u's).  hist receives ||r_s|| for every check, in order.
 */
void oracle_solve_plain(double* u, double* work, const double* f,
                        idx_t nx, idx_t ny, idx_t nz, idx_t sy, idx_t sz,
                        double h, double rtol, int64_t check_every,
                        int64_t max_sweeps, double* hist, int64_t hist_cap,
                        double* out) {
  const double normf = oracle_norm2_f64(f, nx, ny, nz, sy, sz);
  double* cur = u;
  double* nxt = work;
  int64_t nh = 0, s = 0, converged = 0;
  double rn = oracle_residual_l2_f64(cur, f, nx, ny, nz, sy, sz, h);
  const double r0 = rn;
  if (nh < hist_cap) hist[nh] = rn;
  ++nh;
  if (rn <= rtol * normf) converged = 1;
  while (!converged && s < max_sweeps) {
    oracle_sweep_f64(cur, nxt, f, nx, ny, nz, sy, sz, h);
    double* t = cur; cur = nxt; nxt = t;
    ++s;
    if (s % check_every == 0 || s == max_sweeps) {
      rn = oracle_residual_l2_f64(cur, f, nx, ny, nz, sy, sz, h);
      if (s % check_every == 0) {
        if (nh < hist_cap) hist[nh] = rn;
        ++nh;
        if (rn <= rtol * normf) converged = 1;
      }
    }
  }
  if (cur != u) {
    for (idx_t k = 1; k <= nz; ++k)
      for (idx_t j = 1; j <= ny; ++j)
        memcpy(&u[AT(1, j, k)], &cur[AT(1, j, k)], (size_t)nx * sizeof(double));
  }
  out[0] = (double)s; out[1] = rn; out[2] = r0; out[3] = normf;
  out[4] = (double)converged; out[5] = (double)(nh < hist_cap ? nh : hist_cap);
}

/*
 * Mixed-precision solve (FP32 correction sweeps, FP64 defect correction).
 * Each cycle: defect step (u += e from the previous cycle, r = f - A u,
 * r32 = (float) r, ||r|| in FP64), convergence test ||r|| <= rtol ||f||,
 * then e := 0 and min(inner, max_sweeps - sweeps) FP32 Jacobi sweeps on
 * A e = r32 with h2_32 = (float)(h*h).  The first cycle has no e to add.
 * The last cycle always ends with a defect step, so u includes every
 * correction and the reported residual is that of the returned u.
 * e_a, e_b are FP32 arrays whose halo is zero; r32 is FP32 (halo unused).
 */
void oracle_solve_mixed(double* u, const double* f, float* r32, float* e_a,
                        float* e_b, idx_t nx, idx_t ny, idx_t nz,
                        idx_t sy, idx_t sz, idx_t sy4, idx_t sz4, double h,
                        double rtol, int64_t inner, int64_t max_sweeps,
                        double* hist, int64_t hist_cap, double* out) {
  const double normf = oracle_norm2_f64(f, nx, ny, nz, sy, sz);
  const float h2f = (float)(h * h);
  const float* e_last = NULL;
  int64_t s = 0, nh = 0, converged = 0;
  double rn = 0.0, r0 = 0.0;
  for (;;) {
    rn = oracle_defect(u, e_last, f, r32, nx, ny, nz, sy, sz, sy4, sz4, h);
    if (nh == 0) r0 = rn;
    if (nh < hist_cap) hist[nh] = rn;
    ++nh;
    if (rn <= rtol * normf) { converged = 1; break; }
    if (s >= max_sweeps) break;
    int64_t m = inner < max_sweeps - s ? inner : max_sweeps - s;
    /* e := 0 (interior; the halo is zero already) */
    for (idx_t k = 1; k <= nz; ++k)
      for (idx_t j = 1; j <= ny; ++j)
        for (idx_t i = 1; i <= nx; ++i) e_a[i + sy4 * j + sz4 * k] = 0.0f;
    float* ec = e_a;
    float* en = e_b;
    for (int64_t q = 0; q < m; ++q) {
      oracle_sweep_f32(ec, en, r32, nx, ny, nz, sy4, sz4, h2f);
      float* t = ec; ec = en; en = t;
    }
    e_last = ec;
    s += m;
  }
  out[0] = (double)s; out[1] = rn; out[2] = r0; out[3] = normf;
  out[4] = (double)converged; out[5] = (double)(nh < hist_cap ? nh : hist_cap);
}

/* ------------------------------------------------------------------ */
/* The paper's 2D jacobi benchmark                                     */
/* ------------------------------------------------------------------ */

/*
 * The jacobi benchmark the paper compares compilers on (Sec. "Flang
 * performance comparison"): Jacobi iteration for Laplace's equation on a 2D
 * grid u(0:nx+1, 0:ny+1) whose one-cell halo holds the boundary values,
 *   u'(i,j) = (((u(i-1,j) + u(i+1,j)) + u(i,j-1)) + u(i,j+1)) / 4
 * over the interior.  nsweeps sweeps alternate a -> b -> a ...; the result is
 * in a when nsweeps is even, else in b (both must hold the same halo).
 * Element (i,j) sits at a[i + sy*j].
 */
void oracle_jacobi2d(double* a, double* b, idx_t nx, idx_t ny, idx_t sy, idx_t nsweeps) {
  for (idx_t s = 0; s < nsweeps; ++s) {
    const double* u = (s % 2 == 0) ? a : b;
    double* un = (s % 2 == 0) ? b : a;
#pragma omp parallel for schedule(static)
    for (idx_t j = 1; j <= ny; ++j)
      for (idx_t i = 1; i <= nx; ++i) {
        double t = u[(i - 1) + sy * j] + u[(i + 1) + sy * j];
        t = t + u[i + sy * (j - 1)];
        t = t + u[i + sy * (j + 1)];
        un[i + sy * j] = t / 4.0;
      }
  }
}

/*
 * ||r||_2 over the interior for Laplace's equation (right-hand side zero):
 * r(i,j) = (S - 4 u(i,j)) / h^2 with S the four-neighbour sum in the order
 * above; compensated sum of squares, row by row in order.
 */
double oracle_laplace2d_resid_l2(const double* u, idx_t nx, idx_t ny, idx_t sy, double h) {
  const double h2 = h * h;
  nsum acc = {0.0, 0.0};
  for (idx_t j = 1; j <= ny; ++j)
    for (idx_t i = 1; i <= nx; ++i) {
      double t = u[(i - 1) + sy * j] + u[(i + 1) + sy * j];
      t = t + u[i + sy * (j - 1)];
      t = t + u[i + sy * (j + 1)];
      const double r = (t - 4.0 * u[i + sy * j]) / h2;
      nsum_add(&acc, r * r);
    }
  return sqrt(acc.s + acc.c);
}

/* ------------------------------------------------------------------ */
/* Multi-field stencils at the shapes of pw-advection and tra-adv      */
/* ------------------------------------------------------------------ */

/*
 * The paper names two more stencil benchmarks, pw-advection (three fields
 * on a 2048 x 1024 x 1024 grid) and tra-adv (six fields on 1024 x 512 x 512,
 * 20 iterations), Sec. "Flang performance comparison", without their
 * sources.  The two functions below are the documented synthetic stencils
 * that stand in for them.
 *
 * Momentum advection (pw-advection): the centred flux form of Piacsek and
 * Williams (J. Comput. Phys. 6, 1970) on a staggered grid.  u(i,j,k) sits on
 * the east face of cell (i,j,k), v(i,j,k) on its north face, w(i,j,k) on its
 * top face.  The tendency of each component is minus the divergence of its
 * momentum flux; a flux through a face is the product of the advecting
 * velocity averaged onto that face and the advected component averaged onto
 * it, each average of two neighbours.  With c = 0.25 / spacing, for the
 * x-flux of a component q through the faces on either side of its point,
 *   ((a_- * b_-) - (a_+ * b_+)) * cx,
 * where a_-, b_- are the two-point sums of the advecting velocity and of q at
 * the lower face and a_+, b_+ at the upper face.  The three directions add
 * as (x + y) + z.  All six arrays are (0:nx+1, 0:ny+1, 0:nz+1) with the
 * same strides; su, sv, sw are written on the interior only.
 */
static double flux_diff(double am, double bm, double ap, double bp, double c) {
  return (am * bm - ap * bp) * c;
}

void oracle_pw_advection(const double* u, const double* v, const double* w,
                         double* su, double* sv, double* sw,
                         idx_t nx, idx_t ny, idx_t nz, idx_t sy, idx_t sz,
                         double dx, double dy, double dz) {
  const double cx = 0.25 / dx, cy = 0.25 / dy, cz = 0.25 / dz;
#pragma omp parallel for schedule(static)
  for (idx_t k = 1; k <= nz; ++k)
    for (idx_t j = 1; j <= ny; ++j)
      for (idx_t i = 1; i <= nx; ++i) {
#define UU(a, b, c) u[AT(i + (a), j + (b), k + (c))]
#define VV(a, b, c) v[AT(i + (a), j + (b), k + (c))]
#define WW(a, b, c) w[AT(i + (a), j + (b), k + (c))]
        /* u at the east face (i+1/2, j, k) */
        double tx = flux_diff(UU(-1, 0, 0) + UU(0, 0, 0), UU(-1, 0, 0) + UU(0, 0, 0),
                              UU(0, 0, 0) + UU(1, 0, 0), UU(0, 0, 0) + UU(1, 0, 0), cx);
        double ty = flux_diff(VV(0, -1, 0) + VV(1, -1, 0), UU(0, -1, 0) + UU(0, 0, 0),
                              VV(0, 0, 0) + VV(1, 0, 0), UU(0, 0, 0) + UU(0, 1, 0), cy);
        double tz = flux_diff(WW(0, 0, -1) + WW(1, 0, -1), UU(0, 0, -1) + UU(0, 0, 0),
                              WW(0, 0, 0) + WW(1, 0, 0), UU(0, 0, 0) + UU(0, 0, 1), cz);
        su[AT(i, j, k)] = (tx + ty) + tz;
        /* v at the north face (i, j+1/2, k) */
        tx = flux_diff(UU(-1, 0, 0) + UU(-1, 1, 0), VV(-1, 0, 0) + VV(0, 0, 0),
                       UU(0, 0, 0) + UU(0, 1, 0), VV(0, 0, 0) + VV(1, 0, 0), cx);
        ty = flux_diff(VV(0, -1, 0) + VV(0, 0, 0), VV(0, -1, 0) + VV(0, 0, 0),
                       VV(0, 0, 0) + VV(0, 1, 0), VV(0, 0, 0) + VV(0, 1, 0), cy);
        tz = flux_diff(WW(0, 0, -1) + WW(0, 1, -1), VV(0, 0, -1) + VV(0, 0, 0),
                       WW(0, 0, 0) + WW(0, 1, 0), VV(0, 0, 0) + VV(0, 0, 1), cz);
        sv[AT(i, j, k)] = (tx + ty) + tz;
        /* w at the top face (i, j, k+1/2) */
        tx = flux_diff(UU(-1, 0, 0) + UU(-1, 0, 1), WW(-1, 0, 0) + WW(0, 0, 0),
                       UU(0, 0, 0) + UU(0, 0, 1), WW(0, 0, 0) + WW(1, 0, 0), cx);
        ty = flux_diff(VV(0, -1, 0) + VV(0, -1, 1), WW(0, -1, 0) + WW(0, 0, 0),
                       VV(0, 0, 0) + VV(0, 0, 1), WW(0, 0, 0) + WW(0, 1, 0), cy);
        tz = flux_diff(WW(0, 0, -1) + WW(0, 0, 0), WW(0, 0, -1) + WW(0, 0, 0),
                       WW(0, 0, 0) + WW(0, 0, 1), WW(0, 0, 0) + WW(0, 0, 1), cz);
        sw[AT(i, j, k)] = (tx + ty) + tz;
#undef UU
#undef VV
#undef WW
      }
}

/*
 * Tracer advection (tra-adv): a tracer t carried by the volume transports
 * u, v, w through the east, north and top faces of each cell, donor-cell
 * (first-order upwind) fluxes, explicit in time:
 *   F(face) = q+ * t(cell below the face) + q- * t(cell above the face),
 *   q+ = q if q > 0 else 0,  q- = q if q < 0 else 0,
 *   t'(i,j,k) = t - r * (((Fe - Fw) + (Fn - Fs)) + (Ft - Fb)),
 * with r = time step / cell volume.  Six fields: t_a, t_b (the iterate, in
 * turn), u, v, w, r, all (0:nx+1, 0:ny+1, 0:nz+1) with the same strides; the
 * halo of t holds the boundary values (the same in t_a and t_b), u(0,..),
 * v(..,0,..), w(..,0) are the transports through the lower domain faces.
 * niter iterations alternate t_a -> t_b -> t_a ...: the result is in t_a when
 * niter is even, else in t_b.
 */
static double upwind(double q, double below, double above) {
  const double qp = q > 0.0 ? q : 0.0;
  const double qm = q < 0.0 ? q : 0.0;
  return qp * below + qm * above;
}

void oracle_tracer_advection(double* ta, double* tb, const double* u, const double* v,
                             const double* w, const double* r, idx_t nx, idx_t ny, idx_t nz,
                             idx_t sy, idx_t sz, int64_t niter) {
  for (int64_t s = 0; s < niter; ++s) {
    const double* t = (s % 2 == 0) ? ta : tb;
    double* tn = (s % 2 == 0) ? tb : ta;
#pragma omp parallel for schedule(static)
    for (idx_t k = 1; k <= nz; ++k)
      for (idx_t j = 1; j <= ny; ++j)
        for (idx_t i = 1; i <= nx; ++i) {
          const idx_t c = AT(i, j, k);
          const double fe = upwind(u[c], t[c], t[c + 1]);
          const double fw = upwind(u[c - 1], t[c - 1], t[c]);
          const double fn = upwind(v[c], t[c], t[c + sy]);
          const double fs = upwind(v[c - sy], t[c - sy], t[c]);
          const double ft = upwind(w[c], t[c], t[c + sz]);
          const double fb = upwind(w[c - sz], t[c - sz], t[c]);
          const double div = ((fe - fw) + (fn - fs)) + (ft - fb);
          tn[c] = t[c] - r[c] * div;
        }
  }
}
