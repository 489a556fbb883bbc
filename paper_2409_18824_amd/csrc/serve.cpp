// Continuous-batching Poisson server.
//
// Each admitted request is a slot holding its device state (u, f in FP64;
// r32, e0, e1 in FP32).  One worker thread runs cycles over all active slots:
//   1. FP64 defect step of every slot in one batched kernel (r = f - A u,
//      r32 = (float) r, per-tile sums of r^2), one batched reduce that writes
//      each slot's ||r|| and raises its done flag when ||r|| <= rtol ||f||;
//   2. cycle_sweeps batched FP32 correction sweeps over the slots that still
//      have sweeps left (done slots are skipped by flag), two sweeps per pass
//      over memory where the count allows; the last pass adds the correction
//      to u.
// With J3D_SERVE_FP64 precision a slot holds u, f and a second FP64 iterate
// w instead, and a cycle is the residual check of the current iterate
// (batched residual pass and reduce, as above) followed by cycle_sweeps
// batched FP64 Jacobi sweeps ping-ponging between u and w: the plain FP64
// solve with a check every cycle_sweeps sweeps, served the same way.
// While a cycle runs on the GPU the worker admits queued requests (in
// arrival order, while their state fits the memory budget and a slot is
// free): it allocates their state and queues their set-up behind the cycle.
// At the cycle boundary it retires converged and capped slots, copies their
// results out, and the admitted requests join the next cycle.
//
// Every slot sees the same sequence of operations as a solo mixed solve
// with inner_sweeps = cycle_sweeps, so its result does not depend on which
// other requests share its cycles.  A request's max_sweeps is rounded up to a
// whole number of cycles.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "runtime.h"

namespace j3d {
TileCfg default_cfg(int dtype, int nx, int ny, int nz);
const char* last_error_text();
}

using namespace j3d;

namespace {

struct Layout {
  Field u, f, r32, e0, e1;  // mixed precision
  Field w;                  // FP64: the second iterate
  size_t bytes = 0;
};

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Carve the arrays of a request out of one allocation (mixed: u, f, r32, e0,
// e1; FP64: u, f, w).  Rows are padded to 128 bytes and element (1, j, k) of
// every row is 128-byte aligned.
Layout make_layout(int nx, int ny, int nz, char* mem, int precision) {
  Layout L;
  size_t off = 0;
  auto place = [&](Field& a, int dtype) {
    const int es = dtype == J3D_F64 ? 8 : 4;
    const int al = 128 / es;
    a.dtype = dtype;
    a.esize = es;
    a.ex = nx + 2;
    a.ey = ny + 2;
    a.ez = nz + 2;
    a.sy = ((long long)a.ex + al - 1) / al * al;
    a.sz = a.sy * a.ey;
    a.base = mem ? mem + off + (size_t)(al - 1) * es : nullptr;
    off += round256((size_t)(a.sz * a.ez + al) * es);
  };
  place(L.u, J3D_F64);
  place(L.f, J3D_F64);
  if (precision == J3D_SERVE_FP64) {
    place(L.w, J3D_F64);
  } else {
    place(L.r32, J3D_F32);
    place(L.e0, J3D_F32);
    place(L.e1, J3D_F32);
  }
  L.bytes = off;
  return L;
}

struct Request {
  uint64_t ticket = 0;
  j3d_request r{};
  std::vector<double> f;  // copy of f_host (empty: draw from seed)
  double t_submit = 0, t_admit = 0;
  int64_t max_sweeps = 0;
  size_t bytes = 0;
  uint64_t points = 0;
};

struct Slot {
  Request* req = nullptr;
  int id = -1;
  char* mem = nullptr;
  Layout L;
  int64_t sweeps = 0;
  bool ready = false;  // set-up queued before the current cycle
  int cur = 0;         // FP64 precision: the iterate is in u (0) or w (1)
};

}  // namespace

struct j3d_server {
  j3d_serve_opts o{};
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work;
  std::condition_variable cv_done;
  std::deque<Request*> queue;
  std::vector<j3d_result> finished;
  std::vector<Slot*> active;
  std::vector<int> free_ids;
  bool stop = false;
  uint64_t next_ticket = 1;
  int64_t n_submitted = 0;
  int64_t n_finished = 0;
  size_t used_bytes = 0;
  uint64_t active_points = 0;
  double t0 = 0;
  int error = J3D_OK;
  std::string error_text;

  // device state (owned by the worker)
  hipStream_t st = nullptr;
  double* d_normf = nullptr;  // [max_slots]
  double* d_rtol = nullptr;
  double* d_resid = nullptr;
  int* d_done = nullptr;
  int* d_nonfinite = nullptr;
  long long* d_conv = nullptr;
  GridArgs* d_tab = nullptr;  // 6 kinds * max_slots
  double* d_part = nullptr;
  size_t part_cap = 0;
  GridArgs* h_tab = nullptr;  // pinned staging
  double* h_rtol = nullptr;
  double* h_out = nullptr;    // pinned: resid[max_slots]
  int* h_flags = nullptr;     // pinned: done[max_slots], nonfinite[max_slots]
  hipEvent_t ev = nullptr;
  TileCfg cd{}, cs{}, cs2{}, cs3{};  // defect, one-, two- and three-sweep FP32 passes
  TileCfg cs_one64{}, c64_2{}, c64_3{};  // FP64 precision: one-, two- and three-sweep passes
  int passes_in_cycle = 0;           // FP64 precision: passes the last cycle queued

  double now() const { return now_seconds() - t0; }
};

namespace {

// Launch tables of a cycle: the defect step, the one-sweep FP32 passes
// (first sweep into e0; first and last sweep at once), the two-sweep FP32
// passes (first pair into e0; first and last pair at once; middle pairs
// e0 -> e1 and e1 -> e0; last pairs from e0 and from e1) and the three-sweep
// FP32 passes (the same six kinds).
enum Kind {
  K_DEF = 0,
  K_FIRST1,
  K_FL1,
  K_FIRST2,
  K_FL2,
  K_MID2A,
  K_MID2B,
  K_LAST2A,
  K_LAST2B,
  K_FIRST3,
  K_FL3,
  K_MID3A,
  K_MID3B,
  K_LAST3A,
  K_LAST3B,
  K_NKINDS
};

// FP64 precision uses the same table storage: K_DEF is the residual check
// of each slot's current iterate; pass tables of one, two or three sweeps
// from the current iterate to the other (parity 0) or back (parity 1).
constexpr int kP64[3][2] = {{K_FIRST1, K_FL1}, {K_FIRST2, K_FL2}, {K_FIRST3, K_FL3}};

// Three-sweep correction passes when the FP32 state the cycle sweeps (r,
// e0, e1 of every slot) exceeds 512 MB, twice the last-level cache, as in
// the solver; J3D_SERVE_TRIPLES=0 or =1 forces two-sweep or three-sweep
// passes.  Every schedule gives the same iterates bit for bit.
bool serve_triples(long long points) {
  const char* e = std::getenv("J3D_SERVE_TRIPLES");
  if (e != nullptr && *e == '0') return false;
  if (e != nullptr && *e == '1') return true;
  return 12.0 * (double)points > 512e6;
}

// The same rule for FP64 sweeps (24 bytes per point of u, w and f).
bool serve_triples64(long long points) {
  const char* e = std::getenv("J3D_SERVE_TRIPLES");
  if (e != nullptr && *e == '0') return false;
  if (e != nullptr && *e == '1') return true;
  return 24.0 * (double)points > 512e6;
}

int serve_fail(j3d_server* s, int code, const char* what) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->error == J3D_OK) {
    s->error = code;
    s->error_text = what;
  }
  s->stop = true;
  s->cv_done.notify_all();
  return code;
}

// A three-sweep tile shape from the environment ("rows,planes,variant,
// persistent,order,cols"), if set and supported.
void tile3_from_env(const char* name, int dtype, TileCfg* c) {
  const char* e = std::getenv(name);
  if (e == nullptr) return;
  TileCfg t{};
  if (std::sscanf(e, "%d,%d,%d,%d,%d,%d", &t.rows, &t.planes, &t.variant, &t.persistent, &t.order, &t.cols) == 6 &&
      tile3_cfg_supported(dtype, t))
    *c = t;
}

int setup_device(j3d_server* s) {
  const int n = s->o.max_slots;
  J3D_HIP(hipSetDevice(s->o.device));
  J3D_HIP(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
  J3D_HIP(hipEventCreateWithFlags(&s->ev, hipEventDisableTiming));
  void* p = nullptr;
  J3D_TRY(dev_alloc(&p, n * sizeof(double), "serve normf")); s->d_normf = (double*)p;
  J3D_TRY(dev_alloc(&p, n * sizeof(double), "serve rtol")); s->d_rtol = (double*)p;
  J3D_TRY(dev_alloc(&p, n * sizeof(double), "serve resid")); s->d_resid = (double*)p;
  J3D_TRY(dev_alloc(&p, 2 * n * sizeof(int), "serve flags")); s->d_done = (int*)p;
  s->d_nonfinite = s->d_done + n;
  J3D_TRY(dev_alloc(&p, n * sizeof(long long), "serve conv")); s->d_conv = (long long*)p;
  J3D_TRY(dev_alloc(&p, (size_t)K_NKINDS * n * sizeof(GridArgs), "serve tables")); s->d_tab = (GridArgs*)p;
  J3D_HIP(hipHostMalloc((void**)&s->h_tab, (size_t)K_NKINDS * n * sizeof(GridArgs), hipHostMallocDefault));
  J3D_HIP(hipHostMalloc((void**)&s->h_rtol, n * sizeof(double), hipHostMallocDefault));
  J3D_HIP(hipHostMalloc((void**)&s->h_out, n * sizeof(double), hipHostMallocDefault));
  J3D_HIP(hipHostMalloc((void**)&s->h_flags, 2 * n * sizeof(int), hipHostMallocDefault));
  J3D_HIP(hipMemsetAsync(s->d_done, 0, 2 * n * sizeof(int), s->st));
  s->cd = default_cfg(J3D_F64, 128, 128, 128);
  s->cs = default_cfg(J3D_F32, 128, 128, 128);
  s->cs2 = default_cfg2(J3D_F32, 128, 128, 128);
  // the batched three-sweep passes run over up to 2e8 active points of
  // grids of 32^3 to 384^3; shapes measured on the served stream (see
  // below), J3D_SERVE_TILE3 / J3D_SERVE_TILE3_FP64 override them
  s->cs3 = TileCfg{4, 24, 20, 0, 2, 1};
  tile3_from_env("J3D_SERVE_TILE3", J3D_F32, &s->cs3);
  s->cs_one64 = default_cfg(J3D_F64, 128, 128, 128);
  s->cs_one64.persistent = 0;
  s->c64_2 = default_cfg2(J3D_F64, 128, 128, 128);
  s->c64_3 = TileCfg{4, 48, 20, 0, 1, 1};
  tile3_from_env("J3D_SERVE_TILE3_FP64", J3D_F64, &s->c64_3);
  s->cd.persistent = 0;
  s->cs.persistent = 0;
  s->cs2.persistent = 0;
  return J3D_OK;
}

void teardown_device(j3d_server* s) {
  if (s->st) (void)hipStreamSynchronize(s->st);
  for (Slot* sl : s->active) {
    if (sl->mem) (void)hipFree(sl->mem);
    delete sl->req;
    delete sl;
  }
  s->active.clear();
  (void)hipFree(s->d_normf);
  (void)hipFree(s->d_rtol);
  (void)hipFree(s->d_resid);
  (void)hipFree(s->d_done);
  (void)hipFree(s->d_conv);
  (void)hipFree(s->d_tab);
  if (s->d_part) (void)hipFree(s->d_part);
  if (s->h_tab) (void)hipHostFree(s->h_tab);
  if (s->h_rtol) (void)hipHostFree(s->h_rtol);
  if (s->h_out) (void)hipHostFree(s->h_out);
  if (s->h_flags) (void)hipHostFree(s->h_flags);
  if (s->ev) (void)hipEventDestroy(s->ev);
  if (s->st) (void)hipStreamDestroy(s->st);
}

// Queue the set-up of an admitted slot on the server stream: zero state
// (zero initial guess and zero Dirichlet halo), f from the host copy or the
// seed, ||f|| into d_normf[id], flags cleared.
int queue_setup(j3d_server* s, Slot* sl) {
  const Request& q = *sl->req;
  J3D_HIP(hipMemsetAsync(sl->mem, 0, sl->L.bytes, s->st));
  const Field& f = sl->L.f;
  if (!q.f.empty()) {
    J3D_HIP(hipMemcpy2DAsync(f.base, (size_t)f.sy * 8, q.f.data(), (size_t)f.ex * 8, (size_t)f.ex * 8,
                             (size_t)f.ey * f.ez, hipMemcpyHostToDevice, s->st));
  } else {
    const unsigned long long key = q.r.seed ^ (2ull << 40);  // stream 2: right-hand sides
    J3D_HIP(launch_fill_uniform(reinterpret_cast<double*>(f.base), f.ex, f.ey, f.ez, f.sy, f.sz, key,
                                -1.0, 1.0, 0.0, s->st));
  }
  GridArgs g = make_args(nullptr, nullptr, &f, nullptr, nullptr, q.r.h, s->cd, 0);
  const int nt = g.tiles_x * g.tiles_y * g.tiles_z;
  if ((size_t)nt > s->part_cap) {
    // Growing the partials buffer: wait for users of the old one.
    J3D_HIP(hipStreamSynchronize(s->st));
    if (s->d_part) J3D_HIP(hipFree(s->d_part));
    s->d_part = nullptr;
    void* p = nullptr;
    J3D_TRY(dev_alloc(&p, (size_t)nt * 2 * sizeof(double), "serve partials"));
    s->d_part = (double*)p;
    s->part_cap = (size_t)nt * 2;
  }
  J3D_HIP(launch_pass_one(J3D_F64, F_NORM, s->cd, g, s->d_part, nullptr, s->st));
  J3D_HIP(launch_reduce_one(s->d_part, 0, nt, s->d_normf + sl->id, nullptr, 0.0, 0, nullptr, nullptr,
                            nullptr, s->st));
  J3D_HIP(launch_set_int(s->d_done + sl->id, 1, 0, s->st));
  J3D_HIP(launch_set_int(s->d_nonfinite + sl->id, 1, 0, s->st));
  sl->ready = true;
  return J3D_OK;
}

// Admit queued requests while budget and slots allow.
int admit(j3d_server* s) {
  for (;;) {
    Request* q = nullptr;
    int id = -1;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->queue.empty() || s->free_ids.empty()) return J3D_OK;
      Request* head = s->queue.front();
      if (s->used_bytes + head->bytes > s->o.hbm_budget_bytes) return J3D_OK;
      if (s->o.max_active_points != 0 && s->active_points != 0 &&
          s->active_points + head->points > s->o.max_active_points)
        return J3D_OK;
      s->queue.pop_front();
      id = s->free_ids.back();
      s->free_ids.pop_back();
      s->used_bytes += head->bytes;
      s->active_points += head->points;
      q = head;
    }
    Slot* sl = new Slot();
    sl->req = q;
    sl->id = id;
    void* mem = nullptr;
    int rc = dev_alloc(&mem, q->bytes, "request state");
    if (rc != J3D_OK) {
      // Could not allocate now: put it back and retry after a retirement.
      std::lock_guard<std::mutex> lk(s->mu);
      s->queue.push_front(q);
      s->free_ids.push_back(id);
      s->used_bytes -= q->bytes;
      s->active_points -= q->points;
      delete sl;
      return s->active.empty() ? rc : J3D_OK;
    }
    sl->mem = static_cast<char*>(mem);
    sl->L = make_layout(q->r.nx, q->r.ny, q->r.nz, sl->mem, s->o.precision);
    q->t_admit = s->now();
    J3D_TRY(queue_setup(s, sl));
    s->active.push_back(sl);
  }
}

// Build the per-kind tables of the active slots and queue one cycle.
int queue_cycle(j3d_server* s, const std::vector<Slot*>& slots) {
  const int n = (int)slots.size();
  const int cyc = s->o.cycle_sweeps;
  GridArgs* T[K_NKINDS];
  for (int k = 0; k < K_NKINDS; ++k) T[k] = s->h_tab + (size_t)k * s->o.max_slots;
  int nt_def = 0, nt_swp = 0, nt_swp2 = 0, nt_swp3 = 0, n_in = 0;
  long long pts_in = 0;
  bool fit3 = true;  // every plane below 4 GiB (needed by three-sweep passes)
  for (int g = 0; g < n; ++g) {
    Slot* sl = slots[g];
    const Layout& L = sl->L;
    const double h = sl->req->r.h;
    GridArgs d = make_args(&L.u, nullptr, &L.f, nullptr, &L.r32, h, s->cd, nt_def);
    d.id = sl->id;
    T[K_DEF][g] = d;
    nt_def += d.tiles_x * d.tiles_y * d.tiles_z;
    s->h_rtol[sl->id] = sl->req->r.rtol;
    if (sl->sweeps >= sl->req->max_sweeps) continue;  // final defect only
    GridArgs a[K_NKINDS];
    a[K_FIRST1] = make_args(nullptr, &L.e0, &L.r32, nullptr, nullptr, h, s->cs, nt_swp);
    a[K_FL1] = make_args(nullptr, nullptr, &L.r32, &L.u, nullptr, h, s->cs, nt_swp);
    a[K_FIRST2] = make_args2(nullptr, &L.e0, &L.r32, nullptr, h, s->cs2, nt_swp2);
    a[K_FL2] = make_args2(nullptr, nullptr, &L.r32, &L.u, h, s->cs2, nt_swp2);
    a[K_MID2A] = make_args2(&L.e0, &L.e1, &L.r32, nullptr, h, s->cs2, nt_swp2);
    a[K_MID2B] = make_args2(&L.e1, &L.e0, &L.r32, nullptr, h, s->cs2, nt_swp2);
    a[K_LAST2A] = make_args2(&L.e0, nullptr, &L.r32, &L.u, h, s->cs2, nt_swp2);
    a[K_LAST2B] = make_args2(&L.e1, nullptr, &L.r32, &L.u, h, s->cs2, nt_swp2);
    a[K_FIRST3] = make_args3(nullptr, &L.e0, &L.r32, nullptr, h, s->cs3, nt_swp3);
    a[K_FL3] = make_args3(nullptr, nullptr, &L.r32, &L.u, h, s->cs3, nt_swp3);
    a[K_MID3A] = make_args3(&L.e0, &L.e1, &L.r32, nullptr, h, s->cs3, nt_swp3);
    a[K_MID3B] = make_args3(&L.e1, &L.e0, &L.r32, nullptr, h, s->cs3, nt_swp3);
    a[K_LAST3A] = make_args3(&L.e0, nullptr, &L.r32, &L.u, h, s->cs3, nt_swp3);
    a[K_LAST3B] = make_args3(&L.e1, nullptr, &L.r32, &L.u, h, s->cs3, nt_swp3);
    for (int k = K_FIRST1; k < K_NKINDS; ++k) {
      a[k].id = sl->id;
      T[k][n_in] = a[k];
    }
    nt_swp += a[K_FIRST1].tiles_x * a[K_FIRST1].tiles_y * a[K_FIRST1].tiles_z;
    nt_swp2 += a[K_FIRST2].tiles_x * a[K_FIRST2].tiles_y * a[K_FIRST2].tiles_z;
    nt_swp3 += a[K_FIRST3].tiles_x * a[K_FIRST3].tiles_y * a[K_FIRST3].tiles_z;
    pts_in += (long long)L.u.nx() * L.u.ny() * L.u.nz();
    fit3 = fit3 && plane_fits_u32(L.u) && plane_fits_u32(L.r32) && plane_fits_u32(L.e0) && plane_fits_u32(L.e1);
    ++n_in;
  }
  if ((size_t)nt_def > s->part_cap) {
    J3D_HIP(hipStreamSynchronize(s->st));
    if (s->d_part) J3D_HIP(hipFree(s->d_part));
    s->d_part = nullptr;
    void* p = nullptr;
    J3D_TRY(dev_alloc(&p, (size_t)nt_def * 2 * sizeof(double), "serve partials"));
    s->d_part = (double*)p;
    s->part_cap = (size_t)nt_def * 2;
  }
  const size_t row = (size_t)s->o.max_slots;
  J3D_HIP(hipMemcpyAsync(s->d_tab, s->h_tab, (size_t)K_NKINDS * row * sizeof(GridArgs),
                         hipMemcpyHostToDevice, s->st));
  J3D_HIP(hipMemcpyAsync(s->d_rtol, s->h_rtol, row * sizeof(double), hipMemcpyHostToDevice, s->st));
  GridArgs* D[K_NKINDS];
  for (int k = 0; k < K_NKINDS; ++k) D[k] = s->d_tab + (size_t)k * row;
  int* done = s->d_done;
  J3D_HIP(launch_pass_batch(J3D_F64, F_RES | F_R32, s->cd, D[K_DEF], n, nt_def, s->d_part, done, s->st));
  J3D_HIP(launch_reduce_batch(s->d_part, D[K_DEF], n, s->d_resid, 1, 0, s->d_normf, s->d_rtol, 0, done,
                              s->d_conv, s->d_nonfinite, s->st));
  // The correction sweeps in passes of `step` sweeps, as in a solo mixed
  // solve: the first pass starts from zero (cyc mod step sweeps, step when
  // step divides cyc), the middle passes ping-pong between e0 and e1, the
  // last adds its result to u.
  if (n_in > 0) {
    const int step = (fit3 && serve_triples(pts_in)) ? 3 : 2;
    auto pass = [&](int len, unsigned fl, Kind k1, Kind k2, Kind k3) -> hipError_t {
      if (len == 3) return launch_sweep3_batch(J3D_F32, fl, s->cs3, D[k3], n_in, nt_swp3, nullptr, done, s->st);
      if (len == 2) return launch_sweep2_batch(J3D_F32, fl, s->cs2, D[k2], n_in, nt_swp2, nullptr, done, s->st);
      return launch_pass_batch(J3D_F32, fl, s->cs, D[k1], n_in, nt_swp, nullptr, done, s->st);
    };
    if (cyc <= step) {
      J3D_HIP(pass(cyc, F_LAST | F_FIRST, K_FL1, K_FL2, K_FL3));
    } else {
      const int lead = cyc % step == 0 ? step : cyc % step;
      J3D_HIP(pass(lead, F_WRITE | F_FIRST, K_FIRST1, K_FIRST2, K_FIRST3));
      const int rest = (cyc - lead) / step;  // passes after the first, >= 1
      bool in_e0 = true;
      for (int p = 1; p < rest; ++p) {
        J3D_HIP(pass(step, F_WRITE, K_FIRST1, in_e0 ? K_MID2A : K_MID2B, in_e0 ? K_MID3A : K_MID3B));
        in_e0 = !in_e0;
      }
      J3D_HIP(pass(step, F_LAST, K_FIRST1, in_e0 ? K_LAST2A : K_LAST2B, in_e0 ? K_LAST3A : K_LAST3B));
    }
  }
  // Residuals and flags of this cycle's defect step, for the host.
  J3D_HIP(hipMemcpyAsync(s->h_out, s->d_resid, row * sizeof(double), hipMemcpyDeviceToHost, s->st));
  J3D_HIP(hipMemcpyAsync(s->h_flags, s->d_done, 2 * row * sizeof(int), hipMemcpyDeviceToHost, s->st));
  J3D_HIP(hipEventRecord(s->ev, s->st));
  return J3D_OK;
}

// FP64 precision: the residual check of every slot's current iterate, then
// cycle_sweeps FP64 sweeps over the slots that still have sweeps left, in
// passes of `step` sweeps (three when the FP64 state of the cycle exceeds
// 512 MB, else two; the first pass takes cycle_sweeps mod step sweeps when
// step does not divide it), alternating between u and w.
int queue_cycle64(j3d_server* s, const std::vector<Slot*>& slots) {
  const int n = (int)slots.size();
  const int cyc = s->o.cycle_sweeps;
  GridArgs* T[K_NKINDS];
  for (int k = 0; k < K_NKINDS; ++k) T[k] = s->h_tab + (size_t)k * s->o.max_slots;
  int nt_def = 0, nt[3] = {0, 0, 0}, n_in = 0;
  long long pts_in = 0;
  bool fit3 = true;
  for (int g = 0; g < n; ++g) {
    Slot* sl = slots[g];
    const Layout& L = sl->L;
    const double h = sl->req->r.h;
    const Field* a = sl->cur ? &L.w : &L.u;  // the current iterate
    const Field* b = sl->cur ? &L.u : &L.w;
    GridArgs d = make_args(a, nullptr, &L.f, nullptr, nullptr, h, s->cd, nt_def);
    d.id = sl->id;
    T[K_DEF][g] = d;
    nt_def += d.tiles_x * d.tiles_y * d.tiles_z;
    s->h_rtol[sl->id] = sl->req->r.rtol;
    if (sl->sweeps >= sl->req->max_sweeps) continue;  // final check only
    for (int par = 0; par < 2; ++par) {
      const Field* src = par ? b : a;
      const Field* dst = par ? a : b;
      GridArgs p1 = make_args(src, dst, &L.f, nullptr, nullptr, h, s->cs_one64, nt[0]);
      GridArgs p2 = make_args2(src, dst, &L.f, nullptr, h, s->c64_2, nt[1]);
      GridArgs p3 = make_args3(src, dst, &L.f, nullptr, h, s->c64_3, nt[2]);
      p1.id = p2.id = p3.id = sl->id;
      T[kP64[0][par]][n_in] = p1;
      T[kP64[1][par]][n_in] = p2;
      T[kP64[2][par]][n_in] = p3;
    }
    {
      const GridArgs& p1 = T[kP64[0][0]][n_in];
      const GridArgs& p2 = T[kP64[1][0]][n_in];
      const GridArgs& p3 = T[kP64[2][0]][n_in];
      nt[0] += p1.tiles_x * p1.tiles_y * p1.tiles_z;
      nt[1] += p2.tiles_x * p2.tiles_y * p2.tiles_z;
      nt[2] += p3.tiles_x * p3.tiles_y * p3.tiles_z;
    }
    pts_in += (long long)L.u.nx() * L.u.ny() * L.u.nz();
    fit3 = fit3 && plane_fits_u32(L.u) && plane_fits_u32(L.w) && plane_fits_u32(L.f);
    ++n_in;
  }
  if ((size_t)nt_def > s->part_cap) {
    J3D_HIP(hipStreamSynchronize(s->st));
    if (s->d_part) J3D_HIP(hipFree(s->d_part));
    s->d_part = nullptr;
    void* p = nullptr;
    J3D_TRY(dev_alloc(&p, (size_t)nt_def * 2 * sizeof(double), "serve partials"));
    s->d_part = (double*)p;
    s->part_cap = (size_t)nt_def * 2;
  }
  const size_t row = (size_t)s->o.max_slots;
  J3D_HIP(hipMemcpyAsync(s->d_tab, s->h_tab, (size_t)K_NKINDS * row * sizeof(GridArgs),
                         hipMemcpyHostToDevice, s->st));
  J3D_HIP(hipMemcpyAsync(s->d_rtol, s->h_rtol, row * sizeof(double), hipMemcpyHostToDevice, s->st));
  GridArgs* D[K_NKINDS];
  for (int k = 0; k < K_NKINDS; ++k) D[k] = s->d_tab + (size_t)k * row;
  int* done = s->d_done;
  J3D_HIP(launch_pass_batch(J3D_F64, F_RES, s->cd, D[K_DEF], n, nt_def, s->d_part, done, s->st));
  J3D_HIP(launch_reduce_batch(s->d_part, D[K_DEF], n, s->d_resid, 1, 0, s->d_normf, s->d_rtol, 0, done,
                              s->d_conv, s->d_nonfinite, s->st));
  s->passes_in_cycle = 0;
  if (n_in > 0) {
    const int step = (fit3 && serve_triples64(pts_in)) ? 3 : 2;
    auto pass = [&](int len, int par) -> hipError_t {
      const GridArgs* t = D[kP64[len - 1][par]];
      if (len == 3) return launch_sweep3_batch(J3D_F64, F_WRITE, s->c64_3, t, n_in, nt[2], nullptr, done, s->st);
      if (len == 2) return launch_sweep2_batch(J3D_F64, F_WRITE, s->c64_2, t, n_in, nt[1], nullptr, done, s->st);
      return launch_pass_batch(J3D_F64, F_WRITE, s->cs_one64, t, n_in, nt[0], nullptr, done, s->st);
    };
    int left = cyc, par = 0;
    const int lead = cyc % step;
    if (lead != 0) {
      J3D_HIP(pass(lead, par));
      left -= lead;
      par ^= 1;
      ++s->passes_in_cycle;
    }
    for (; left > 0; left -= step) {
      J3D_HIP(pass(step, par));
      par ^= 1;
      ++s->passes_in_cycle;
    }
  }
  J3D_HIP(hipMemcpyAsync(s->h_out, s->d_resid, row * sizeof(double), hipMemcpyDeviceToHost, s->st));
  J3D_HIP(hipMemcpyAsync(s->h_flags, s->d_done, 2 * row * sizeof(int), hipMemcpyDeviceToHost, s->st));
  J3D_HIP(hipEventRecord(s->ev, s->st));
  return J3D_OK;
}

int retire(j3d_server* s, Slot* sl, bool converged, bool nonfinite, double resid, double normf) {
  Request* q = sl->req;
  if (q->r.u_host != nullptr) {
    const Field& u = sl->cur ? sl->L.w : sl->L.u;
    J3D_HIP(hipMemcpy2DAsync(q->r.u_host, (size_t)u.ex * 8, u.base, (size_t)u.sy * 8, (size_t)u.ex * 8,
                             (size_t)u.ey * u.ez, hipMemcpyDeviceToHost, s->st));
    J3D_HIP(hipStreamSynchronize(s->st));
  }
  J3D_HIP(hipFree(sl->mem));
  j3d_result r{};
  r.ticket = q->ticket;
  r.status = nonfinite ? J3D_ENONFINITE : J3D_OK;
  r.converged = (converged && !nonfinite) ? 1 : 0;
  r.sweeps = sl->sweeps;
  r.resid = resid;
  r.norm_f = normf;
  r.t_submit = q->t_submit;
  r.t_admit = q->t_admit;
  r.t_done = s->now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->finished.push_back(r);
    s->n_finished++;
    s->used_bytes -= q->bytes;
    s->active_points -= q->points;
    s->free_ids.push_back(sl->id);
  }
  s->cv_done.notify_all();
  delete q;
  delete sl;
  return J3D_OK;
}

int worker_loop(j3d_server* s) {
  J3D_TRY(setup_device(s));
  std::vector<double> normf_h((size_t)s->o.max_slots, 0.0);
  for (;;) {
    J3D_TRY(admit(s));
    if (s->active.empty()) {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
      if (s->stop) return J3D_OK;
      continue;
    }
    std::vector<Slot*> cyc = s->active;  // slots in this cycle
    if (s->o.precision == J3D_SERVE_FP64)
      J3D_TRY(queue_cycle64(s, cyc));
    else
      J3D_TRY(queue_cycle(s, cyc));
    // Overlap: admit arrivals while the cycle runs; their set-up is queued
    // behind it and they join the next cycle.
    J3D_TRY(admit(s));
    J3D_HIP(hipEventSynchronize(s->ev));
    J3D_HIP(hipMemcpy(normf_h.data(), s->d_normf, normf_h.size() * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<Slot*> keep;
    const int ms = s->o.max_slots;
    for (Slot* sl : s->active) {
      const bool in_cycle = std::find(cyc.begin(), cyc.end(), sl) != cyc.end();
      if (!in_cycle) {
        keep.push_back(sl);
        continue;
      }
      const bool done = s->h_flags[sl->id] != 0;
      const bool bad = s->h_flags[ms + sl->id] != 0;
      const double resid = s->h_out[sl->id];
      if (done || bad) {
        J3D_TRY(retire(s, sl, done, bad, resid, normf_h[sl->id]));
      } else if (sl->sweeps >= sl->req->max_sweeps) {
        J3D_TRY(retire(s, sl, false, false, resid, normf_h[sl->id]));
      } else {
        sl->sweeps += s->o.cycle_sweeps;
        if (s->passes_in_cycle & 1) sl->cur ^= 1;  // FP64: the sweeps ended in the other array
        keep.push_back(sl);
      }
    }
    s->active.swap(keep);
    bool stop;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      stop = s->stop;
    }
    if (stop) return J3D_OK;
  }
}

void worker_main(j3d_server* s) {
  int rc = worker_loop(s);
  if (rc != J3D_OK) serve_fail(s, rc, j3d::last_error_text());
  teardown_device(s);
}

}  // namespace

extern "C" {

uint64_t j3d_request_bytes(int32_t nx, int32_t ny, int32_t nz) {
  if (nx < 1 || ny < 1 || nz < 1) return 0;
  return make_layout(nx, ny, nz, nullptr, J3D_SERVE_MIXED).bytes;
}

uint64_t j3d_request_state_bytes(int32_t precision, int32_t nx, int32_t ny, int32_t nz) {
  if (nx < 1 || ny < 1 || nz < 1) return 0;
  if (precision != J3D_SERVE_MIXED && precision != J3D_SERVE_FP64) return 0;
  return make_layout(nx, ny, nz, nullptr, precision).bytes;
}

int poisson_serve_create(const j3d_serve_opts* opts, j3d_server** out) {
  if (opts == nullptr || out == nullptr) return fail(J3D_EINVAL, "opts/out: null pointer");
  if (opts->max_slots < 1 || opts->max_slots > 65536) return fail(J3D_EINVAL, "max_slots out of range");
  if (opts->cycle_sweeps < 1) return fail(J3D_EINVAL, "cycle_sweeps must be >= 1");
  if (opts->queue_cap < 1) return fail(J3D_EINVAL, "queue_cap must be >= 1");
  if (opts->hbm_budget_bytes == 0) return fail(J3D_EINVAL, "hbm_budget_bytes must be > 0");
  if (opts->precision != J3D_SERVE_MIXED && opts->precision != J3D_SERVE_FP64)
    return fail(J3D_EINVAL, "precision must be J3D_SERVE_MIXED or J3D_SERVE_FP64");
  if (opts->reserved != 0) return fail(J3D_EINVAL, "reserved field must be 0");
  int ndev = 0;
  J3D_HIP(hipGetDeviceCount(&ndev));
  if (opts->device < 0 || opts->device >= ndev) return fail(J3D_EINVAL, "no such device");
  j3d_server* s = new j3d_server();
  s->o = *opts;
  s->t0 = now_seconds();
  for (int i = opts->max_slots - 1; i >= 0; --i) s->free_ids.push_back(i);
  s->worker = std::thread(worker_main, s);
  *out = s;
  return J3D_OK;
}

int poisson_serve_submit(j3d_server* s, const j3d_request* req, uint64_t* ticket) {
  if (s == nullptr || req == nullptr || ticket == nullptr) return fail(J3D_EINVAL, "null pointer");
  if (req->nx < 1 || req->ny < 1 || req->nz < 1) return fail(J3D_EINVAL, "extents must be >= 1");
  if (req->reserved != 0) return fail(J3D_EINVAL, "reserved field must be 0");
  J3D_TRY(check_h(req->h));
  if (!(req->rtol >= 0.0) || !std::isfinite(req->rtol)) return fail(J3D_EINVAL, "rtol must be finite and >= 0");
  if (req->max_sweeps < 0) return fail(J3D_EINVAL, "max_sweeps must be >= 0");
  const long long ex = req->nx + 2LL, ey = req->ny + 2LL, ez = req->nz + 2LL;
  if (ey > 65535 || ez > 65535 || ((ex + 31) / 32 * 32) * ey * ez >= (1LL << 31) - 64)
    return fail(J3D_EINVAL, "grid too large");
  const size_t bytes = make_layout(req->nx, req->ny, req->nz, nullptr, s->o.precision).bytes;
  if (bytes > s->o.hbm_budget_bytes)
    return fail(J3D_EBUDGET, "request needs %zu bytes, budget is %llu", bytes,
                (unsigned long long)s->o.hbm_budget_bytes);
  Request* q = new Request();
  q->r = *req;
  q->bytes = bytes;
  q->points = (uint64_t)req->nx * (uint64_t)req->ny * (uint64_t)req->nz;
  const int64_t c = s->o.cycle_sweeps;
  q->max_sweeps = (req->max_sweeps + c - 1) / c * c;
  if (req->f_host != nullptr) q->f.assign(req->f_host, req->f_host + ex * ey * ez);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->error != J3D_OK) {
    delete q;
    return fail(s->error, "server stopped: %s", s->error_text.c_str());
  }
  if ((int)s->queue.size() >= s->o.queue_cap) {
    delete q;
    return fail(J3D_EAGAIN, "queue full");
  }
  q->ticket = s->next_ticket++;
  q->t_submit = s->now();
  s->queue.push_back(q);
  s->n_submitted++;
  *ticket = q->ticket;
  s->cv_work.notify_one();
  return J3D_OK;
}

int poisson_serve_poll(j3d_server* s, j3d_result* out, int32_t cap, int32_t* n) {
  if (s == nullptr || n == nullptr || (cap > 0 && out == nullptr)) return fail(J3D_EINVAL, "null pointer");
  std::lock_guard<std::mutex> lk(s->mu);
  const int m = std::min<int>(cap, (int)s->finished.size());
  for (int i = 0; i < m; ++i) out[i] = s->finished[i];
  s->finished.erase(s->finished.begin(), s->finished.begin() + m);
  *n = m;
  if (s->error != J3D_OK) return fail(s->error, "server stopped: %s", s->error_text.c_str());
  return J3D_OK;
}

int poisson_serve_drain(j3d_server* s, double timeout_s) {
  if (s == nullptr) return fail(J3D_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto pred = [&] { return s->n_finished >= s->n_submitted || s->error != J3D_OK; };
  if (timeout_s <= 0) {
    s->cv_done.wait(lk, pred);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
    return fail(J3D_EAGAIN, "drain timed out");
  }
  if (s->error != J3D_OK) return fail(s->error, "server stopped: %s", s->error_text.c_str());
  return J3D_OK;
}

int poisson_serve_stats(j3d_server* s, double* now, int32_t* active, int32_t* queued, int64_t* finished) {
  if (s == nullptr) return fail(J3D_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  if (now) *now = s->now();
  if (active) *active = (int32_t)(s->o.max_slots - (int)s->free_ids.size());
  if (queued) *queued = (int32_t)s->queue.size();
  if (finished) *finished = s->n_finished;
  return J3D_OK;
}

int poisson_serve_destroy(j3d_server* s) {
  if (s == nullptr) return fail(J3D_EINVAL, "null server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (Request* q : s->queue) delete q;
  s->queue.clear();
  delete s;
  return J3D_OK;
}

}  // extern "C"
