// poisson_solve: plain FP64 Jacobi and FP32-sweep / FP64-defect-correction
// mixed-precision solves, with the convergence test on the device.
//
// The host enqueues kernels in chunks of a few milliseconds and, between
// chunks, reads a pinned copy of the device's `done` flag.  Every kernel
// queued after the flag is raised returns at once, so overshooting the
// convergence point costs only empty launches.  This is the early-exit loop
// of the paper's iterate_while lowering (Sec. "Handling of control
// structures") with the exit test evaluated where the data lives.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "runtime.h"

namespace j3d {
namespace {

// Chunk length (in sweeps) that keeps the device busy for about 2 ms.
long long chunk_sweeps(long long points, double bytes_per_point, long long multiple) {
  const double t = std::max(3e-6, bytes_per_point * (double)points / 5e12);
  long long n = (long long)std::ceil(2e-3 / t);
  n = std::max<long long>(n, 1);
  n = std::min<long long>(n, 1 << 16);
  n = ((n + multiple - 1) / multiple) * multiple;
  return n;
}

// Three-sweep passes pay off once the arrays a pass touches overflow the
// 256 MB last-level cache: measured on cubes, they save 20-27% per sweep at
// 384^3 and 512^3, but at 256^3 the cache holds most of the arrays and the
// three-sweep tile's wider halo cancels the saving (two-sweep passes are
// as fast or faster there).
bool three_sweep_passes_pay(double pass_bytes) { return pass_bytes > 512e6; }

// J3D_SOLVE_SWEEPS_PER_PASS=1, 2 or 3 fixes the pass length of both modes
// (the schedules above, with that step); unset or other values choose it
// from the grid size.
int forced_step() {
  const char* e = std::getenv("J3D_SOLVE_SWEEPS_PER_PASS");
  const int v = e != nullptr ? std::atoi(e) : 0;
  return (v >= 1 && v <= 3) ? v : 0;
}

int publish_done(Scratch* s, int slot, hipStream_t st) {
  J3D_HIP(hipMemcpyAsync(&s->ctl_host->done, &s->ctl->done, sizeof(int), hipMemcpyDeviceToHost, st));
  J3D_HIP(hipEventRecord(s->ev[slot & 1], st));
  return J3D_OK;
}

// Waits for the event of an earlier chunk and returns the flag it published.
int poll_done(Scratch* s, int slot, bool* done) {
  J3D_HIP(hipEventSynchronize(s->ev[slot & 1]));
  *done = __atomic_load_n(&s->ctl_host->done, __ATOMIC_ACQUIRE) != 0;
  return J3D_OK;
}

int read_control(Scratch* s, Control* out, hipStream_t st) {
  J3D_HIP(hipMemcpyAsync(s->ctl_host, s->ctl, sizeof(Control), hipMemcpyDeviceToHost, st));
  J3D_HIP(hipStreamSynchronize(st));
  std::memcpy(out, s->ctl_host, sizeof(Control));
  return J3D_OK;
}

int read_history(Scratch* s, long long nh, std::vector<double>* h, hipStream_t st) {
  h->assign((size_t)nh, 0.0);
  if (nh > 0)
    J3D_HIP(hipMemcpyAsync(h->data(), s->hist, (size_t)nh * sizeof(double), hipMemcpyDeviceToHost, st));
  J3D_HIP(hipStreamSynchronize(st));
  return J3D_OK;
}

int norm_f(const Field& f, const TileCfg& c, Scratch* s, hipStream_t st) {
  GridArgs g = make_args(nullptr, nullptr, &f, nullptr, nullptr, 1.0, c, 0);
  const int nt = g.tiles_x * g.tiles_y * g.tiles_z;
  J3D_TRY(ensure_partials(s, nt));
  J3D_HIP(launch_pass_one(J3D_F64, F_NORM, c, g, s->partials, nullptr, st));
  J3D_HIP(launch_reduce_one(s->partials, 0, nt, &s->ctl->normf, nullptr, 0.0, 0, nullptr, nullptr,
                            nullptr, st));
  return J3D_OK;
}

void fill_result(j3d_solve_result* r, long long sweeps, double resid, const std::vector<double>& hist,
                 double normf, bool converged, bool nonfinite, const j3d_solve_opts& o) {
  r->sweeps = sweeps;
  r->resid = resid;
  r->resid0 = hist.empty() ? resid : hist[0];
  r->norm_f = normf;
  r->converged = (converged && !nonfinite) ? 1 : 0;
  r->status = nonfinite ? J3D_ENONFINITE : J3D_OK;
  long long n = 0;
  if (o.history != nullptr && o.history_cap > 0) {
    n = std::min<long long>((long long)hist.size(), o.history_cap);
    std::memcpy(o.history, hist.data(), (size_t)n * sizeof(double));
  }
  r->history_len = n;
}

// ---------------------------------------------------------------------
// FP64 mode
// ---------------------------------------------------------------------

// Solves that check after every sweep on grids of at most 2^24 points,
// where a check's reduction kernel costs about half a sweep: each pass's
// check is reduced by an extra workgroup of the next pass
// (launch_pass_one_pre).  That pass runs before the check's verdict is
// known, so the iterates rotate through three arrays (the pass after a
// converged check writes the array of the iterate before it, never the
// converged one) and the per-tile partials through two.  Same kernels,
// same reduction order, same results as the schedule with a reduction
// kernel per check.  J3D_SOLVE_FUSED_CHECKS=0 turns it off.
bool fused_checks_apply(long long c, long long points) {
  const char* e = std::getenv("J3D_SOLVE_FUSED_CHECKS");
  if (e != nullptr && std::atoi(e) == 0) return false;
  return c == 1 && points <= (1LL << 24);
}

int solve_fp64_fused_checks(const Field& u, const Field& f, double h, const j3d_solve_opts& o,
                            j3d_solve_result* res, hipStream_t st) {
  Scratch* s = nullptr;
  J3D_TRY(get_scratch(st, &s));
  const TileCfg cfg = default_cfg(J3D_F64, u.nx(), u.ny(), u.nz());
  const long long S = o.max_sweeps;
  const long long points = (long long)u.nx() * u.ny() * u.nz();

  // u, and two arrays of u's layout in the work buffer, all with u's halo
  const size_t span = (u.span_bytes() + 255) / 256 * 256;
  J3D_TRY(ensure_work(s, 2 * span));
  Field buf3[3] = {u, u, u};
  buf3[1].base = static_cast<char*>(s->work);
  buf3[2].base = static_cast<char*>(s->work) + span;
  J3D_HIP(hipMemcpyAsync(buf3[1].base, u.base, u.span_bytes(), hipMemcpyDeviceToDevice, st));
  J3D_HIP(hipMemcpyAsync(buf3[2].base, u.base, u.span_bytes(), hipMemcpyDeviceToDevice, st));

  GridArgs one[3], resid[3];
  for (int b = 0; b < 3; ++b) {
    one[b] = make_args(&buf3[b], &buf3[(b + 1) % 3], &f, nullptr, nullptr, h, cfg, 0);
    resid[b] = make_args(&buf3[b], nullptr, &f, nullptr, nullptr, h, cfg, 0);
  }
  const int nt = one[0].tiles_x * one[0].tiles_y * one[0].tiles_z;
  const size_t ntp = ((size_t)nt + 31) / 32 * 32;
  J3D_TRY(ensure_partials(s, 2 * ntp));
  double* part[2] = {s->partials, s->partials + ntp};
  J3D_TRY(ensure_hist(s, (size_t)S + 1));
  J3D_HIP(hipMemsetAsync(s->ctl, 0, sizeof(Control), st));
  J3D_TRY(norm_f(f, cfg, s, st));
  int* done = &s->ctl->done;
  auto pre_of = [&](long long q) {  // the reduction of check q (the partials of pass q)
    PreReduce pr{part[q & 1], nt, s->hist, &s->ctl->normf, o.rtol, done, &s->ctl->conv_at,
                 &s->ctl->nonfinite, &s->ctl->qnext};
    return pr;
  };
  // pass p: iterate p (array p % 3) -> p + 1, residual of iterate p into
  // part[p % 2], the check of pass p - 1 reduced on the side
  auto pass = [&](long long p, hipStream_t q) -> int {
    const int b = (int)(p % 3);
    if (p == 0) {
      J3D_HIP(launch_pass_one(J3D_F64, F_WRITE | F_RES, cfg, one[b], part[0], done, q));
    } else {
      J3D_HIP(launch_pass_one_pre(J3D_F64, F_WRITE | F_RES, cfg, one[b], part[p & 1], done, pre_of(p - 1), q));
    }
    return J3D_OK;
  };
  const long long chunk = chunk_sweeps(points, 24.0, 6);  // a multiple of the 3 x 2 rotation
  long long p = 0;
  int slot = 0;
  bool seen = false;
  if (S > 0) {
    J3D_TRY(pass(0, st));
    p = 1;
  }
  // whole chunks starting at passes 1, 1 + M, ... replayed from one graph
  const long long M = std::min(chunk, (S - 1) / 2 / 6 * 6);
  if (S > 0 && M > 0) {
    std::string key = "fp64-fused";
    auto add = [&key](const void* x, size_t n) { key.append(static_cast<const char*>(x), n); };
    add(one, sizeof one);
    add(&cfg, sizeof cfg);
    const long long meta[3] = {M, nt, (long long)ntp};
    add(meta, sizeof meta);
    const void* ptrs[3] = {s->partials, s->hist, s->ctl};
    add(ptrs, sizeof ptrs);
    add(&o.rtol, sizeof o.rtol);
    hipGraphExec_t exec = nullptr;
    J3D_TRY(solve_graph(s, key, [&](hipStream_t q) -> int {
      for (long long i = 1; i <= M; ++i) J3D_TRY(pass(i, q));
      return J3D_OK;
    }, &exec));
    while (p + M <= S && !seen) {
      J3D_HIP(hipGraphLaunch(exec, st));
      p += M;
      J3D_TRY(publish_done(s, slot, st));
      if (slot > 0) J3D_TRY(poll_done(s, slot - 1, &seen));
      ++slot;
    }
  }
  while (p < S && !seen) {
    const long long end = std::min(S, p + chunk);
    for (; p < end; ++p) J3D_TRY(pass(p, st));
    J3D_TRY(publish_done(s, slot, st));
    if (slot > 0) J3D_TRY(poll_done(s, slot - 1, &seen));
    ++slot;
  }
  // the residual of the last iterate (check S), which also reduces check
  // S - 1; skipped, like every kernel after it, once a check converged
  const int bl = (int)(S % 3);
  if (S > 0)
    J3D_HIP(launch_pass_one_pre(J3D_F64, F_RES, cfg, resid[bl], part[S & 1], done, pre_of(S - 1), st));
  else
    J3D_HIP(launch_pass_one(J3D_F64, F_RES, cfg, resid[bl], part[0], done, st));
  J3D_HIP(launch_reduce_count(part[S & 1], nt, s->hist, &s->ctl->normf, o.rtol, done, &s->ctl->conv_at,
                              &s->ctl->nonfinite, &s->ctl->qnext, st));
  Control ctl;
  J3D_TRY(read_control(s, &ctl, st));
  long long sweeps, nh;
  int at;
  if (ctl.done) {
    sweeps = ctl.conv_at;
    nh = ctl.conv_at + 1;
    at = (int)(ctl.conv_at % 3);
  } else {
    sweeps = S;
    nh = S + 1;
    at = bl;
  }
  std::vector<double> hist;
  J3D_TRY(read_history(s, nh, &hist, st));
  if (at != 0) {
    J3D_HIP(launch_copy_interior(reinterpret_cast<const double*>(buf3[at].base), reinterpret_cast<double*>(u.base),
                                 u.nx(), u.ny(), u.nz(), u.sy, u.sz, u.sy, u.sz, st));
    J3D_HIP(hipStreamSynchronize(st));
  }
  fill_result(res, sweeps, hist[(size_t)nh - 1], hist, ctl.normf, ctl.done != 0, ctl.nonfinite != 0, o);
  return ctl.nonfinite ? fail(J3D_ENONFINITE, "residual became non-finite") : J3D_OK;
}

int solve_fp64(const Field& u, const Field& f, double h, const j3d_solve_opts& o,
               j3d_solve_result* res, hipStream_t st) {
  if (forced_step() == 0 && fused_checks_apply(o.check_every, (long long)u.nx() * u.ny() * u.nz()))
    return solve_fp64_fused_checks(u, f, h, o, res, st);
  Scratch* s = nullptr;
  J3D_TRY(get_scratch(st, &s));
  const TileCfg cfg = default_cfg(J3D_F64, u.nx(), u.ny(), u.nz());
  const TileCfg cfg2 = default_cfg2(J3D_F64, u.nx(), u.ny(), u.nz());
  const TileCfg cfg3 = default_cfg3(J3D_F64, u.nx(), u.ny(), u.nz());
  const long long S = o.max_sweeps;
  const long long c = o.check_every;
  const long long points = (long long)u.nx() * u.ny() * u.nz();
  // Passes of `step` sweeps: three on grids whose arrays overflow the
  // cache, else two when every check falls on an even sweep count, else
  // one.  A check group of c sweeps opens with one pass of c mod step
  // sweeps (none when step divides c), which carries the check's residual,
  // and continues in passes of step sweeps; with three-sweep passes and
  // c mod 3 = 1 it opens with two two-sweep passes instead, since the
  // residual of a single sweep leaves many more per-tile partials to
  // reduce.  A pass ends at the next check and at the end of the range it
  // belongs to.
  // (w has u's layout; a three-sweep pass needs planes below 4 GiB)
  const bool fit3 = plane_fits_u32(u) && plane_fits_u32(f);
  long long step = forced_step() != 0 ? forced_step()
                   : three_sweep_passes_pay(24.0 * (double)points) ? 3 : ((c % 2) == 0 ? 2 : 1);
  if (step == 3 && !fit3) step = 2;
  const long long lead = c % step;
  const bool two_pairs = step == 3 && lead == 1 && c >= 4;
  auto pass_len = [&](long long sw, long long to) -> int {
    const long long p = sw % c;
    const long long len = two_pairs ? ((p == 0 || p == 2) ? 2 : 3) : ((p == 0 && lead != 0) ? lead : step);
    return (int)std::min(std::min(len, c - p), to - sw);
  };
  const long long group_passes = (lead != 0 ? 1 : 0) + c / step;

  // The second ping-pong array has u's layout and starts as a copy of u
  // (which gives it the same halo).
  Field w = u;
  J3D_TRY(ensure_work(s, u.span_bytes()));
  w.base = static_cast<char*>(s->work);
  J3D_HIP(hipMemcpyAsync(w.base, u.base, u.span_bytes(), hipMemcpyDeviceToDevice, st));

  const Field* buf[2] = {&u, &w};
  GridArgs one[2], two[2], three[2], resid[2];
  for (int b = 0; b < 2; ++b) {
    one[b] = make_args(buf[b], buf[1 - b], &f, nullptr, nullptr, h, cfg, 0);
    two[b] = make_args2(buf[b], buf[1 - b], &f, nullptr, h, cfg2, 0);
    three[b] = make_args3(buf[b], buf[1 - b], &f, nullptr, h, cfg3, 0);
    resid[b] = make_args(buf[b], nullptr, &f, nullptr, nullptr, h, cfg, 0);
  }
  const int nt1 = one[0].tiles_x * one[0].tiles_y * one[0].tiles_z;
  const int nt2 = two[0].tiles_x * two[0].tiles_y * two[0].tiles_z;
  const int nt3 = three[0].tiles_x * three[0].tiles_y * three[0].tiles_z;
  J3D_TRY(ensure_partials(s, std::max(nt1, std::max(nt2, nt3))));
  const long long nchecks = S / c + 1;
  J3D_TRY(ensure_hist(s, (size_t)nchecks));

  J3D_HIP(hipMemsetAsync(s->ctl, 0, sizeof(Control), st));
  J3D_TRY(norm_f(f, cfg, s, st));
  int* done = &s->ctl->done;

  // which_at[q]: buffer holding the iterate whose residual is check q
  std::vector<unsigned char> which_at((size_t)nchecks, 0);
  // The passes for sweeps [from, to) starting from buffer b (chunk ends are
  // multiples of c, so chunking never changes the schedule).  Checks take
  // their index from the device counter, so a chunk is the same kernel
  // sequence wherever it starts and can be replayed.
  auto passes = [&](long long from, long long to, int b, hipStream_t q) -> int {
    for (long long sw = from; sw < to;) {
      const bool check = (sw % c) == 0;
      const unsigned fl = F_WRITE | (check ? F_RES : 0u);
      const int len = pass_len(sw, to);
      int nt;
      if (len == 3) {
        J3D_HIP(launch_sweep3_one(J3D_F64, fl, cfg3, three[b], s->partials, done, q));
        nt = nt3;
      } else if (len == 2) {
        J3D_HIP(launch_sweep2_one(J3D_F64, fl, cfg2, two[b], s->partials, done, q));
        nt = nt2;
      } else {
        J3D_HIP(launch_pass_one(J3D_F64, fl, cfg, one[b], s->partials, done, q));
        nt = nt1;
      }
      sw += len;
      if (check)
        J3D_HIP(launch_reduce_count(s->partials, nt, s->hist, &s->ctl->normf, o.rtol, done, &s->ctl->conv_at,
                                    &s->ctl->nonfinite, &s->ctl->qnext, q));
      b = 1 - b;
    }
    return J3D_OK;
  };
  // Host mirror of the schedule: the buffer of every check, and at the end.
  auto track = [&](long long from, long long to, int b) -> int {
    for (long long sw = from; sw < to;) {
      if (sw % c == 0) which_at[(size_t)(sw / c)] = (unsigned char)b;
      sw += pass_len(sw, to);
      b = 1 - b;
    }
    return b;
  };
  const long long unit = group_passes % 2 == 0 ? c : 2 * c;  // an even number of passes
  const long long chunk = chunk_sweeps(points, 24.0 * group_passes / c, unit);
  long long sw = 0;
  int cur = 0;
  int slot = 0;
  bool seen = false;
  // Whole chunks from one captured graph, replayed (each leaves the iterate
  // in u again), when there are at least two of them.
  const long long M = std::min(chunk, S / 2 / unit * unit);
  if (M > 0) {
    std::string key = "fp64";
    auto add = [&key](const void* p, size_t n) { key.append(static_cast<const char*>(p), n); };
    add(one, sizeof one);
    add(two, sizeof two);
    add(three, sizeof three);
    add(&cfg, sizeof cfg);
    add(&cfg2, sizeof cfg2);
    add(&cfg3, sizeof cfg3);
    const long long meta[6] = {c, M, nt1, nt2, nt3, step};
    add(meta, sizeof meta);
    const void* ptrs[3] = {s->partials, s->hist, s->ctl};
    add(ptrs, sizeof ptrs);
    add(&o.rtol, sizeof o.rtol);
    hipGraphExec_t exec = nullptr;
    J3D_TRY(solve_graph(s, key, [&](hipStream_t q) { return passes(0, M, 0, q); }, &exec));
    for (long long r = 0; r < S / M && !seen; ++r) {
      J3D_HIP(hipGraphLaunch(exec, st));
      (void)track(sw, sw + M, 0);
      sw += M;
      J3D_TRY(publish_done(s, slot, st));
      if (slot > 0) J3D_TRY(poll_done(s, slot - 1, &seen));
      ++slot;
    }
  }
  while (sw < S && !seen) {
    const long long end = std::min(S, sw + chunk);
    J3D_TRY(passes(sw, end, cur, st));
    cur = track(sw, end, cur);
    sw = end;
    J3D_TRY(publish_done(s, slot, st));
    if (slot > 0) J3D_TRY(poll_done(s, slot - 1, &seen));
    ++slot;
  }
  // Residual of the iterate after the last sweep (a check when S % c == 0).
  // When the loop stopped early (converged), every kernel below is skipped.
  {
    if (S % c == 0) which_at[(size_t)(S / c)] = (unsigned char)cur;
    J3D_HIP(launch_pass_one(J3D_F64, F_RES, cfg, resid[cur], s->partials, done, st));
    if (S % c == 0)  // check S / c: the counter holds exactly that index here
      J3D_HIP(launch_reduce_count(s->partials, nt1, s->hist, &s->ctl->normf, o.rtol, done, &s->ctl->conv_at,
                                  &s->ctl->nonfinite, &s->ctl->qnext, st));
    else
      J3D_HIP(launch_reduce_one(s->partials, 0, nt1, &s->ctl->value, nullptr, 0.0, 0, done, nullptr,
                                nullptr, st));
  }
  Control ctl;
  J3D_TRY(read_control(s, &ctl, st));
  long long sweeps, nh;
  int at;
  if (ctl.done) {
    sweeps = ctl.conv_at * c;
    nh = ctl.conv_at + 1;
    at = which_at[(size_t)ctl.conv_at];
  } else {
    sweeps = S;
    nh = S / c + 1;
    at = cur;
  }
  std::vector<double> hist;
  J3D_TRY(read_history(s, nh, &hist, st));
  const double resid_v = (ctl.done || S % c == 0) ? hist[(size_t)nh - 1] : ctl.value;
  if (at == 1) {
    J3D_HIP(launch_copy_interior(reinterpret_cast<const double*>(w.base), reinterpret_cast<double*>(u.base),
                                 u.nx(), u.ny(), u.nz(), w.sy, w.sz, u.sy, u.sz, st));
    J3D_HIP(hipStreamSynchronize(st));
  }
  fill_result(res, sweeps, resid_v, hist, ctl.normf, ctl.done != 0, ctl.nonfinite != 0, o);
  return ctl.nonfinite ? fail(J3D_ENONFINITE, "residual became non-finite") : J3D_OK;
}

// ---------------------------------------------------------------------
// Mixed mode
// ---------------------------------------------------------------------

// A compact FP32 array with the interior extents of `like`, rows padded to
// 128 bytes and element (1, j, k) 128-byte aligned, carved from `mem`.
Field f32_field(const Field& like, char* mem, size_t* bytes) {
  Field a;
  a.dtype = J3D_F32;
  a.esize = 4;
  a.ex = like.ex;
  a.ey = like.ey;
  a.ez = like.ez;
  const long long ld = ((long long)like.ex + 31) / 32 * 32;
  a.sy = ld;
  a.sz = ld * like.ey;
  a.base = mem + 31 * 4;
  *bytes = (size_t)(a.sz * a.ez + 32) * 4;
  *bytes = (*bytes + 255) / 256 * 256;
  return a;
}

int solve_mixed(const Field& u, const Field& f, double h, const j3d_solve_opts& o,
                j3d_solve_result* res, hipStream_t st) {
  Scratch* s = nullptr;
  J3D_TRY(get_scratch(st, &s));
  const TileCfg cd = default_cfg(J3D_F64, u.nx(), u.ny(), u.nz());
  const TileCfg cs = default_cfg(J3D_F32, u.nx(), u.ny(), u.nz());
  const long long S = o.max_sweeps;
  const long long m_in = o.inner_sweeps;

  size_t b1 = 0;
  (void)f32_field(u, nullptr, &b1);
  J3D_TRY(ensure_work(s, 3 * b1));
  char* mem = static_cast<char*>(s->work);
  size_t tmp;
  const Field r32 = f32_field(u, mem, &tmp);
  const Field e0 = f32_field(u, mem + b1, &tmp);
  const Field e1 = f32_field(u, mem + 2 * b1, &tmp);
  J3D_HIP(hipMemsetAsync(mem, 0, 3 * b1, st));  // zero halos of the correction

  // A cycle of m correction sweeps e_1 = J(0), e_{p+1} = J(e_p), u += e_m
  // runs as passes of `step` sweeps (three on grids whose arrays overflow
  // the cache, else two): the first pass starts from zero without reading
  // it (m mod step sweeps, step when step divides m), the middle passes
  // ping-pong between e0 and e1, and the last pass adds its result to u.
  const long long points = (long long)u.nx() * u.ny() * u.nz();
  int step = forced_step() != 0 ? forced_step() : three_sweep_passes_pay(12.0 * (double)points) ? 3 : 2;
  if (step == 3 && !(plane_fits_u32(u) && plane_fits_u32(r32))) step = 2;
  const TileCfg cs2 = default_cfg2(J3D_F32, u.nx(), u.ny(), u.nz());
  const TileCfg cs3 = default_cfg3(J3D_F32, u.nx(), u.ny(), u.nz());
  const GridArgs defect = make_args(&u, nullptr, &f, nullptr, &r32, h, cd, 0);
  auto pass_args = [&](int len, const Field* in, const Field* out, const Field* add_to) -> GridArgs {
    if (len == 3) return make_args3(in, out, &r32, add_to, h, cs3, 0);
    if (len == 2) return make_args2(in, out, &r32, add_to, h, cs2, 0);
    return make_args(in, out, &r32, add_to, nullptr, h, cs, 0);
  };
  GridArgs first[4] = {}, first_last[4] = {};  // indexed by the pass length
  for (int len = 1; len <= 3; ++len) {
    first[len] = pass_args(len, nullptr, &e0, nullptr);
    first_last[len] = pass_args(len, nullptr, nullptr, &u);
  }
  const GridArgs mid[2] = {pass_args(step, &e0, &e1, nullptr), pass_args(step, &e1, &e0, nullptr)};
  const GridArgs last[2] = {pass_args(step, &e0, nullptr, &u), pass_args(step, &e1, nullptr, &u)};
  const int nt = defect.tiles_x * defect.tiles_y * defect.tiles_z;
  J3D_TRY(ensure_partials(s, nt));
  const long long ncyc = (S + m_in - 1) / m_in + 1;  // defect steps at most
  J3D_TRY(ensure_hist(s, (size_t)ncyc));

  J3D_HIP(hipMemsetAsync(s->ctl, 0, sizeof(Control), st));
  J3D_TRY(norm_f(f, cd, s, st));
  int* done = &s->ctl->done;

  auto correction_pass = [&](int len, unsigned fl, const GridArgs& g, hipStream_t q) -> hipError_t {
    if (len == 3) return launch_sweep3_one(J3D_F32, fl, cs3, g, nullptr, done, q);
    if (len == 2) return launch_sweep2_one(J3D_F32, fl, cs2, g, nullptr, done, q);
    return launch_pass_one(J3D_F32, fl, cs, g, nullptr, done, q);
  };
  // One unit: the defect step with its check (index from the device
  // counter), then a correction cycle of m sweeps (none for the final
  // defect step).  Units with the same m are the same kernel sequence.
  auto unit = [&](long long m, hipStream_t q) -> int {
    J3D_HIP(launch_pass_one(J3D_F64, F_RES | F_R32, cd, defect, s->partials, done, q));
    J3D_HIP(launch_reduce_count(s->partials, nt, s->hist, &s->ctl->normf, o.rtol, done, &s->ctl->conv_at,
                                &s->ctl->nonfinite, &s->ctl->qnext, q));
    if (m == 0) return J3D_OK;
    if (m <= step) {
      J3D_HIP(correction_pass((int)m, F_LAST | F_FIRST, first_last[m], q));
    } else {
      const long long lead = m % step == 0 ? step : m % step;
      J3D_HIP(correction_pass((int)lead, F_WRITE | F_FIRST, first[lead], q));
      const long long rest = (m - lead) / step;  // passes after the first, >= 1
      int cur = 0;                               // e0 holds the iterate
      for (long long p = 1; p < rest; ++p) {
        J3D_HIP(correction_pass(step, F_WRITE, mid[cur], q));
        cur = 1 - cur;
      }
      J3D_HIP(correction_pass(step, F_LAST, last[cur], q));
    }
    return J3D_OK;
  };

  const long long chunk = chunk_sweeps(points, 6.6, m_in);
  const long long full = S / m_in;                            // units with a whole cycle
  const long long K = std::max<long long>(1, chunk / m_in);   // units per replayed graph
  long long sw = 0, q = 0;
  int slot = 0;
  bool seen = false;
  auto poll = [&]() -> int {
    J3D_TRY(publish_done(s, slot, st));
    if (slot > 0) J3D_TRY(poll_done(s, slot - 1, &seen));
    ++slot;
    return J3D_OK;
  };
  if (full / K >= 2) {
    std::string key = "mixed";
    auto add = [&key](const void* p, size_t n) { key.append(static_cast<const char*>(p), n); };
    add(&defect, sizeof defect);
    add(first, sizeof first);
    add(first_last, sizeof first_last);
    add(mid, sizeof mid);
    add(last, sizeof last);
    add(&cd, sizeof cd);
    add(&cs, sizeof cs);
    add(&cs2, sizeof cs2);
    add(&cs3, sizeof cs3);
    const long long meta[4] = {m_in, K, nt, step};
    add(meta, sizeof meta);
    const void* ptrs[3] = {s->partials, s->hist, s->ctl};
    add(ptrs, sizeof ptrs);
    add(&o.rtol, sizeof o.rtol);
    hipGraphExec_t exec = nullptr;
    J3D_TRY(solve_graph(s, key, [&](hipStream_t qs) {
      for (long long k = 0; k < K; ++k) J3D_TRY(unit(m_in, qs));
      return J3D_OK;
    }, &exec));
    for (long long r = 0; r < full / K && !seen; ++r) {
      J3D_HIP(hipGraphLaunch(exec, st));
      sw += K * m_in;
      q += K;
      J3D_TRY(poll());
    }
  }
  long long since = 0;
  while (!seen) {
    const long long m = std::min(m_in, S - sw);  // 0: the final defect step
    J3D_TRY(unit(m, st));
    if (m == 0) break;
    sw += m;
    ++q;
    since += m;
    if (since >= chunk) {
      since = 0;
      J3D_TRY(poll());
    }
  }
  Control ctl;
  J3D_TRY(read_control(s, &ctl, st));
  long long nh, sweeps;
  if (ctl.done) {
    nh = ctl.conv_at + 1;
    sweeps = std::min(ctl.conv_at * m_in, S);
  } else {
    nh = q + 1;
    sweeps = S;
  }
  std::vector<double> hist;
  J3D_TRY(read_history(s, nh, &hist, st));
  fill_result(res, sweeps, hist[(size_t)nh - 1], hist, ctl.normf, ctl.done != 0, ctl.nonfinite != 0, o);
  return ctl.nonfinite ? fail(J3D_ENONFINITE, "residual became non-finite") : J3D_OK;
}

}  // namespace
}  // namespace j3d

using namespace j3d;

extern "C" int poisson_solve(j3d_array* u, const j3d_array* f, double h,
                             const j3d_solve_opts* opts, j3d_solve_result* result, void* stream) {
  Field a, b;
  J3D_TRY(check_field(u, J3D_F64, &a, "u"));
  J3D_TRY(check_field(f, J3D_F64, &b, "f"));
  J3D_TRY(check_same_interior(a, b, "u", "f"));
  J3D_TRY(check_h(h));
  if (opts == nullptr || result == nullptr) return fail(J3D_EINVAL, "opts/result: null pointer");
  if (opts->reserved != 0) return fail(J3D_EINVAL, "opts: reserved field must be 0");
  if (fields_overlap(a, b)) return fail(J3D_EALIAS, "u and f overlap");
  if (opts->max_sweeps < 0) return fail(J3D_EINVAL, "max_sweeps must be >= 0");
  if (!(opts->rtol >= 0.0) || !std::isfinite(opts->rtol)) return fail(J3D_EINVAL, "rtol must be finite and >= 0");
  if (opts->history_cap < 0 || (opts->history_cap > 0 && opts->history == nullptr))
    return fail(J3D_EINVAL, "history buffer missing");
  std::memset(result, 0, sizeof(*result));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (opts->mode == J3D_MODE_FP64) {
    if (opts->check_every < 1) return fail(J3D_EINVAL, "check_every must be >= 1");
    return solve_fp64(a, b, h, *opts, result, st);
  }
  if (opts->mode == J3D_MODE_MIXED) {
    if (opts->inner_sweeps < 1) return fail(J3D_EINVAL, "inner_sweeps must be >= 1");
    return solve_mixed(a, b, h, *opts, result, st);
  }
  return fail(J3D_EINVAL, "unknown solve mode %d", opts->mode);
}
