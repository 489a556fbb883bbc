// Batched sweeps over uneven grids, captured in one HIP graph, and the tile
// shape autotuner.
//
// A batch is flattened into one tile list: grid g owns tiles
// [tile0[g], tile0[g] + tiles(g)) and its launch descriptor sits in a table in
// device memory (one structure of arrays per grid, as the paper keeps one
// memref per member of a derived type, Sec. "Handling of other
// constructs").  One kernel per sweep walks the whole list; the sweeps of a
// call are captured once into a graph and replayed.  Tile shapes are
// compile-time template parameters picked by the autotuner, the analogue of
// the paper's static-shape specialisation (Sec. "Performance").
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "runtime.h"

namespace j3d {
TileCfg default_cfg(int dtype, int nx, int ny, int nz);

namespace {

// ---------------------------------------------------------------------
// Tune cache
// ---------------------------------------------------------------------
std::mutex g_tune_mu;
bool g_tune_loaded = false;
std::map<std::string, TileCfg> g_tune;

std::string single_key(int dtype, int nx, int ny, int nz) {
  char b[96];
  snprintf(b, sizeof b, "single:%d:%d:%d:%d", dtype, nx, ny, nz);
  return b;
}

uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

std::string batch_key(int ngrids, const Field* ua) {
  uint64_t h = 1469598103934665603ull;
  for (int g = 0; g < ngrids; ++g) {
    int e[3] = {ua[g].nx(), ua[g].ny(), ua[g].nz()};
    h = fnv1a(e, sizeof e, h);
  }
  char b[64];
  snprintf(b, sizeof b, "batch:%d:%016llx", ngrids, (unsigned long long)h);
  return b;
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = getenv("J3D_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* fp = fopen(path, "r");
  if (!fp) return;
  char key[128];
  TileCfg c;
  while (fscanf(fp, "%127s %d %d %d %d %d %d", key, &c.rows, &c.planes, &c.variant, &c.persistent, &c.order,
                &c.cols) == 7)
    if (tile_cfg_supported(c)) g_tune[key] = c;
  fclose(fp);
}

void tune_store(const std::string& key, const TileCfg& c) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  g_tune[key] = c;
  const char* path = getenv("J3D_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* fp = fopen(path, "w");
  if (!fp) return;
  for (auto& kv : g_tune)
    fprintf(fp, "%s %d %d %d %d %d %d\n", kv.first.c_str(), kv.second.rows, kv.second.planes,
            kv.second.variant, kv.second.persistent, kv.second.order, kv.second.cols);
  fclose(fp);
}

bool tune_lookup(const std::string& key, TileCfg* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  *out = it->second;
  return true;
}

// Two-sweep choice per batch shape class: the shape and whether it beats
// one-sweep passes (kept for the life of the process).
std::map<std::string, std::pair<TileCfg, bool>> g_pair;

bool pair_lookup(const std::string& key, TileCfg* c2, bool* use) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_pair.find(key);
  if (it == g_pair.end()) return false;
  *c2 = it->second.first;
  *use = it->second.second;
  return true;
}

void pair_store(const std::string& key, const TileCfg& c2, bool use) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_pair[key] = std::make_pair(c2, use);
}

// ---------------------------------------------------------------------
// Batch validation and tables
// ---------------------------------------------------------------------
struct BatchFields {
  std::vector<Field> a, b, f;
  std::vector<double> h;
};

int check_batch(int ngrids, const j3d_grid* grids, BatchFields* bf) {
  if (ngrids < 1) return fail(J3D_EINVAL, "ngrids must be >= 1");
  if (grids == nullptr) return fail(J3D_EINVAL, "grids: null pointer");
  bf->a.resize(ngrids);
  bf->b.resize(ngrids);
  bf->f.resize(ngrids);
  bf->h.resize(ngrids);
  struct Iv {
    const char* lo;
    const char* hi;
    int grid;
    bool written;
  };
  std::vector<Iv> iv;
  iv.reserve(3 * (size_t)ngrids);
  for (int g = 0; g < ngrids; ++g) {
    char nm[3][32];
    snprintf(nm[0], 32, "grids[%d].u_a", g);
    snprintf(nm[1], 32, "grids[%d].u_b", g);
    snprintf(nm[2], 32, "grids[%d].f", g);
    J3D_TRY(check_field(&grids[g].u_a, J3D_F64, &bf->a[g], nm[0]));
    J3D_TRY(check_field(&grids[g].u_b, J3D_F64, &bf->b[g], nm[1]));
    J3D_TRY(check_field(&grids[g].f, J3D_F64, &bf->f[g], nm[2]));
    J3D_TRY(check_same_interior(bf->a[g], bf->b[g], nm[0], nm[1]));
    J3D_TRY(check_same_interior(bf->a[g], bf->f[g], nm[0], nm[2]));
    J3D_TRY(check_h(grids[g].h));
    bf->h[g] = grids[g].h;
    const Field* fs[3] = {&bf->a[g], &bf->b[g], &bf->f[g]};
    for (int r = 0; r < 3; ++r)
      iv.push_back({fs[r]->base, fs[r]->base + fs[r]->span_bytes(), g, r < 2});
  }
  // Sweep in address order: a written array may overlap nothing, a read-only
  // array (f) may overlap only other read-only arrays.
  std::sort(iv.begin(), iv.end(), [](const Iv& x, const Iv& y) { return x.lo < y.lo; });
  const char* hi_all = nullptr;
  const char* hi_written = nullptr;
  for (const Iv& v : iv) {
    if ((v.written && hi_all && v.lo < hi_all) || (hi_written && v.lo < hi_written))
      return fail(J3D_EALIAS, "an array of grid %d overlaps another array of the batch", v.grid);
    if (!hi_all || v.hi > hi_all) hi_all = v.hi;
    if (v.written && (!hi_written || v.hi > hi_written)) hi_written = v.hi;
  }
  return J3D_OK;
}

// tab[0]: u_a -> u_b (+residual of u_a); tab[1]: u_b -> u_a; tab[2]/[3]:
// residual-only of u_a / u_b.
void build_tables(const BatchFields& bf, const TileCfg& c, std::vector<GridArgs> tab[4], int* ntiles) {
  const int n = (int)bf.a.size();
  for (int t = 0; t < 4; ++t) tab[t].resize(n);
  int tile0 = 0;
  for (int g = 0; g < n; ++g) {
    tab[0][g] = make_args(&bf.a[g], &bf.b[g], &bf.f[g], nullptr, nullptr, bf.h[g], c, tile0);
    tab[1][g] = make_args(&bf.b[g], &bf.a[g], &bf.f[g], nullptr, nullptr, bf.h[g], c, tile0);
    tab[2][g] = make_args(&bf.a[g], nullptr, &bf.f[g], nullptr, nullptr, bf.h[g], c, tile0);
    tab[3][g] = make_args(&bf.b[g], nullptr, &bf.f[g], nullptr, nullptr, bf.h[g], c, tile0);
    for (int t = 0; t < 4; ++t) tab[t][g].id = g;
    tile0 += tab[0][g].tiles_x * tab[0][g].tiles_y * tab[0][g].tiles_z;
  }
  *ntiles = tile0;
}

// Two-sweep tables (their own tile numbering): tab2[0]: u_a -> u_b,
// tab2[1]: u_b -> u_a.
void build_tables2(const BatchFields& bf, const TileCfg& c2, std::vector<GridArgs> tab2[2], int* ntiles) {
  const int n = (int)bf.a.size();
  for (int t = 0; t < 2; ++t) tab2[t].resize(n);
  int tile0 = 0;
  for (int g = 0; g < n; ++g) {
    tab2[0][g] = make_args2(&bf.a[g], &bf.b[g], &bf.f[g], nullptr, bf.h[g], c2, tile0);
    tab2[1][g] = make_args2(&bf.b[g], &bf.a[g], &bf.f[g], nullptr, bf.h[g], c2, tile0);
    tab2[0][g].id = tab2[1][g].id = g;
    tile0 += tab2[0][g].tiles_x * tab2[0][g].tiles_y * tab2[0][g].tiles_z;
  }
  *ntiles = tile0;
}

// Three-sweep tables (their own tile numbering): tab3[0]: u_a -> u_b,
// tab3[1]: u_b -> u_a.
void build_tables3(const BatchFields& bf, const TileCfg& c3, std::vector<GridArgs> tab3[2], int* ntiles) {
  const int n = (int)bf.a.size();
  for (int t = 0; t < 2; ++t) tab3[t].resize(n);
  int tile0 = 0;
  for (int g = 0; g < n; ++g) {
    tab3[0][g] = make_args3(&bf.a[g], &bf.b[g], &bf.f[g], nullptr, bf.h[g], c3, tile0);
    tab3[1][g] = make_args3(&bf.b[g], &bf.a[g], &bf.f[g], nullptr, bf.h[g], c3, tile0);
    tab3[0][g].id = tab3[1][g].id = g;
    tile0 += tab3[0][g].tiles_x * tab3[0][g].tiles_y * tab3[0][g].tiles_z;
  }
  *ntiles = tile0;
}

// Dispatch slots of the balanced tile order of the batched three-sweep pass
// (kOrderSlots).  The flat tile list is cut into 8 contiguous runs of about
// equal work, run x for XCD x (the hardware hands workgroup b to XCD b mod
// 8, so each XCD's L2 keeps the halo rows its neighbouring tiles share, as
// in order 0, which cuts by tile count), and each run is taken longest
// tile first (a stable sort: tiles of equal length keep their neighbours),
// so that the short tiles of grids' last z-slabs fill the end of the
// launch.  A tile's work is counted as its planes plus 8 (the pipeline's
// fill and drain and the tile's set-up).  slots[8 i + x] is the i-th tile
// of run x, or tile -1 past the run's end.
void build_slots3(const std::vector<GridArgs>& tab, int ntiles, std::vector<TileSlot>* slots) {
  std::vector<int> cost((size_t)ntiles), owner((size_t)ntiles);
  long long total = 0;
  for (int g = 0; g < (int)tab.size(); ++g) {
    const GridArgs& a = tab[g];
    const int slab = a.tiles_x * a.tiles_y;
    for (int tz = 0; tz < a.tiles_z; ++tz) {
      const int k0 = 1 + tz * a.planes;
      const int len = std::min(k0 + a.planes, a.nz + 1) - k0 + 8;
      for (int q = 0; q < slab; ++q) {
        cost[(size_t)a.tile0 + (size_t)tz * slab + q] = len;
        owner[(size_t)a.tile0 + (size_t)tz * slab + q] = g;
      }
      total += (long long)len * slab;
    }
  }
  std::vector<int> run[8];
  long long acc = 0;
  int x = 0;
  for (int t = 0; t < ntiles; ++t) {
    while (x < 7 && acc * 8 >= total * (x + 1)) ++x;  // run x holds its share
    run[x].push_back(t);
    acc += cost[t];
  }
  size_t longest = 0;
  for (std::vector<int>& r : run) {
    std::stable_sort(r.begin(), r.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    longest = std::max(longest, r.size());
  }
  slots->assign(8 * longest, TileSlot{-1, 0});
  for (int q = 0; q < 8; ++q)
    for (size_t i = 0; i < run[q].size(); ++i) (*slots)[8 * i + q] = TileSlot{run[q][i], owner[run[q][i]]};
}

// The passes of a call with three-sweep passes: (sweeps in the pass, stage
// of the residual it carries or -1).  Passes run straight through the call
// (a batch has no early exit); the pass through which iterate q*E passes
// carries its residual at the stage that forms it: 0 for the pass's input,
// 1 or 2 for the iterate after its first or second sweep (three-sweep
// passes form both on chip).  A pass ends at the second residual point it
// would hold, and a shorter pass whose later iterate is a residual point
// stops before it.  When the pass count has the wrong parity (the result
// must land in u_a exactly when S is even) the last pass of two or more
// sweeps is split in two.  E = 0: no residuals.
struct PassStep {
  int m;
  int stage;
};

std::vector<PassStep> triple_schedule(int S, int E) {
  std::vector<PassStep> v;
  for (int s = 0; s < S;) {
    int m = std::min(3, S - s);
    int offs[3];
    int no = 0;
    for (int o = 0; E > 0 && o < m; ++o)
      if ((s + o) % E == 0) offs[no++] = o;
    if (no > 1) {
      m = offs[1];
      no = 1;
    }
    if (no == 1 && offs[0] > 0 && m < 3) {
      m = offs[0];
      no = 0;
    }
    v.push_back(PassStep{m, no == 1 ? offs[0] : -1});
    s += m;
  }
  if ((int)(v.size() & 1) != (S & 1)) {
    for (size_t i = v.size(); i-- > 0;) {
      const PassStep q = v[i];
      if (q.m < 2) continue;
      PassStep a, b;
      if (q.m == 3 && q.stage == 2) {
        a = PassStep{2, -1};
        b = PassStep{1, 0};
      } else if (q.m == 3) {
        a = PassStep{1, q.stage == 0 ? 0 : -1};
        b = PassStep{2, q.stage == 1 ? 0 : -1};
      } else {
        a = PassStep{1, q.stage};
        b = PassStep{1, -1};
      }
      v[i] = a;
      v.insert(v.begin() + (long)i + 1, b);
      break;
    }
  }
  return v;
}

// ---------------------------------------------------------------------
// Plans (device tables + captured graph), cached per call signature
// ---------------------------------------------------------------------
struct Plan {
  std::string key;
  int device = 0;
  int ngrids = 0, ntiles = 0, ntiles2 = 0, ntiles3 = 0;
  bool pairs = false;       // two sweeps per pass where the cadence allows
  bool triples = false;     // passes of up to three sweeps (triple_schedule)
  TileCfg c2{};             // tile shape of the two-sweep passes
  TileCfg c3{};             // tile shape of the three-sweep passes
  GridArgs* tab = nullptr;  // device: 4 * ngrids one-sweep, 2 * ngrids two-sweep, 2 * ngrids three-sweep entries
  TileSlot* slots3 = nullptr;  // device: dispatch slots of the three-sweep passes (c3.order == kOrderSlots)
  int nslots3 = 0;
  double* partials = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t stamp = 0;
};

std::mutex g_plan_mu;
std::vector<Plan*> g_plans;
// The pass kind (sweeps per pass, 0: none yet) and tile shape of this
// thread's most recent jacobi3d_sweep_batch call.
struct LastPlan {
  int kind = 0;
  TileCfg c{};
};
thread_local LastPlan g_last_plan;
uint64_t g_stamp = 0;
constexpr size_t kMaxPlans = 16;
hipStream_t g_cap_stream[64] = {};

void free_plan(Plan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->tab) (void)hipFree(p->tab);
  if (p->slots3) (void)hipFree(p->slots3);
  if (p->partials) (void)hipFree(p->partials);
  delete p;
}

int capture_stream(int dev, hipStream_t* out) {
  if (dev < 0 || dev >= 64) return fail(J3D_EINVAL, "device ordinal out of range");
  if (!g_cap_stream[dev]) J3D_HIP(hipStreamCreateWithFlags(&g_cap_stream[dev], hipStreamNonBlocking));
  *out = g_cap_stream[dev];
  return J3D_OK;
}

// Enqueue the whole batch on `st` (used for capture).  With pairs, sweeps
// run two per pass; when the number of pairs is odd the first pair runs as
// two one-sweep passes, so that the number of passes has the parity of
// nsweeps and the result lands in u_a exactly when nsweeps is even.
int enqueue_batch(const Plan& p, const TileCfg& c, int nsweeps, int every, double* resid_out,
                  hipStream_t st) {
  const int n = p.ngrids;
  const int nres = resid_out ? nsweeps / every + 1 : 0;
  int s = 0;
  int buf = 0;  // 0: the current iterate is in u_a
  auto one = [&]() -> int {
    const bool check = resid_out && (s % every) == 0;
    const GridArgs* t = p.tab + (size_t)buf * n;
    J3D_HIP(launch_pass_batch(J3D_F64, F_WRITE | (check ? F_RES : 0u), c, t, n, p.ntiles, p.partials,
                              nullptr, st));
    if (check)
      J3D_HIP(launch_reduce_batch(p.partials, t, n, resid_out, nres, s / every, nullptr, nullptr, 0,
                                  nullptr, nullptr, nullptr, st));
    s += 1;
    buf ^= 1;
    return J3D_OK;
  };
  auto two = [&]() -> int {
    const bool check = resid_out && (s % every) == 0;
    const GridArgs* t = p.tab + (size_t)(4 + buf) * n;
    J3D_HIP(launch_sweep2_batch(J3D_F64, F_WRITE | (check ? F_RES : 0u), p.c2, t, n, p.ntiles2, p.partials,
                                nullptr, st));
    if (check)
      J3D_HIP(launch_reduce_batch(p.partials, t, n, resid_out, nres, s / every, nullptr, nullptr, 0,
                                  nullptr, nullptr, nullptr, st));
    s += 2;
    buf ^= 1;
    return J3D_OK;
  };
  if (p.triples) {
    for (const PassStep& ps : triple_schedule(nsweeps, resid_out ? every : 0)) {
      const bool check = ps.stage >= 0;
      const GridArgs* t;
      if (ps.m == 3) {
        t = p.tab + (size_t)(6 + buf) * n;
        const unsigned rf = !check ? 0u : ps.stage == 0 ? F_RES : ps.stage == 1 ? F_RES1 : F_RES2;
        J3D_HIP(launch_sweep3_batch(J3D_F64, F_WRITE | rf, p.c3, t, n, p.ntiles3, p.partials, nullptr, st, p.slots3,
                                    p.nslots3));
      } else if (ps.m == 2) {
        t = p.tab + (size_t)(4 + buf) * n;
        J3D_HIP(launch_sweep2_batch(J3D_F64, F_WRITE | (check ? F_RES : 0u), p.c2, t, n, p.ntiles2,
                                    p.partials, nullptr, st));
      } else {
        t = p.tab + (size_t)buf * n;
        J3D_HIP(launch_pass_batch(J3D_F64, F_WRITE | (check ? F_RES : 0u), c, t, n, p.ntiles, p.partials,
                                  nullptr, st));
      }
      if (check)
        J3D_HIP(launch_reduce_batch(p.partials, t, n, resid_out, nres, (s + ps.stage) / every, nullptr, nullptr,
                                    0, nullptr, nullptr, nullptr, st));
      s += ps.m;
      buf ^= 1;
    }
  } else {
    int npairs = p.pairs ? nsweeps / 2 : 0;
    if (npairs & 1) {
      J3D_TRY(one());
      J3D_TRY(one());
      --npairs;
    }
    for (int q = 0; q < npairs; ++q) J3D_TRY(two());
    while (s < nsweeps) J3D_TRY(one());
  }
  if (resid_out && nsweeps % every == 0) {
    const GridArgs* t = p.tab + (size_t)(2 + buf) * n;
    J3D_HIP(launch_pass_batch(J3D_F64, F_RES, c, t, n, p.ntiles, p.partials, nullptr, st));
    J3D_HIP(launch_reduce_batch(p.partials, t, n, resid_out, nres, nsweeps / every, nullptr, nullptr,
                                0, nullptr, nullptr, nullptr, st));
  }
  return J3D_OK;
}

int make_plan(const std::string& key, const BatchFields& bf, const TileCfg& c, bool pairs, const TileCfg& c2,
              bool triples, const TileCfg& c3, int nsweeps, int every, double* resid_out, Plan** out) {
  int dev = 0;
  J3D_HIP(hipGetDevice(&dev));
  Plan* p = new Plan();
  p->key = key;
  p->device = dev;
  p->ngrids = (int)bf.a.size();
  p->pairs = pairs;
  p->c2 = c2;
  p->triples = triples;
  p->c3 = c3;
  std::vector<GridArgs> tab[4], tab2[2], tab3[2];
  build_tables(bf, c, tab, &p->ntiles);
  build_tables2(bf, c2, tab2, &p->ntiles2);
  build_tables3(bf, c3, tab3, &p->ntiles3);
  std::vector<GridArgs> flat;
  for (int t = 0; t < 4; ++t) flat.insert(flat.end(), tab[t].begin(), tab[t].end());
  for (int t = 0; t < 2; ++t) flat.insert(flat.end(), tab2[t].begin(), tab2[t].end());
  for (int t = 0; t < 2; ++t) flat.insert(flat.end(), tab3[t].begin(), tab3[t].end());
  void* mem = nullptr;
  int rc = dev_alloc(&mem, flat.size() * sizeof(GridArgs), "batch table");
  if (rc == J3D_OK) {
    p->tab = static_cast<GridArgs*>(mem);
    rc = dev_alloc(&mem, (size_t)std::max(p->ntiles, std::max(p->ntiles2, p->ntiles3)) * sizeof(double),
                   "batch partials");
  }
  if (rc == J3D_OK) p->partials = static_cast<double*>(mem);
  if (rc != J3D_OK) {
    free_plan(p);
    return rc;
  }
  hipError_t e = hipMemcpy(p->tab, flat.data(), flat.size() * sizeof(GridArgs), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_plan(p);
    return hip_fail(e, "upload batch table");
  }
  if (triples && c3.order == kOrderSlots) {
    std::vector<TileSlot> sl;
    build_slots3(tab3[0], p->ntiles3, &sl);
    rc = dev_alloc(&mem, sl.size() * sizeof(TileSlot), "batch slots");
    if (rc != J3D_OK) {
      free_plan(p);
      return rc;
    }
    p->slots3 = static_cast<TileSlot*>(mem);
    p->nslots3 = (int)sl.size();
    e = hipMemcpy(p->slots3, sl.data(), sl.size() * sizeof(TileSlot), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      free_plan(p);
      return hip_fail(e, "upload batch slots");
    }
  }
  hipStream_t cs;
  rc = capture_stream(dev, &cs);
  if (rc != J3D_OK) {
    free_plan(p);
    return rc;
  }
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    free_plan(p);
    return hip_fail(e, "hipStreamBeginCapture");
  }
  rc = enqueue_batch(*p, c, nsweeps, every, resid_out, cs);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  if (rc != J3D_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    free_plan(p);
    return rc != J3D_OK ? rc : hip_fail(e, "hipStreamEndCapture");
  }
  p->graph = graph;
  e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    free_plan(p);
    return hip_fail(e, "hipGraphInstantiate");
  }
  *out = p;
  return J3D_OK;
}

// ---------------------------------------------------------------------
// Autotuning
// ---------------------------------------------------------------------
std::vector<TileCfg> candidates() {
  std::vector<TileCfg> v;
  const int n = j3d_tune_count();
  for (int i = 0; i < n; ++i) {
    j3d_tune t;
    j3d_tune_get(i, &t);
    v.push_back(TileCfg{t.rows, t.planes, t.variant, t.persistent, t.order, t.cols});
  }
  return v;
}

// Time F_WRITE passes of tile shapes and return the fastest.  The search is
// staged rather than exhaustive: rows x planes with a default variant, then
// every variant x persistence x order at the best rows x planes, then rows x
// planes again at the best of those.  `launch` enqueues one pass for a shape.
template <typename Launcher>
int time_candidates(hipStream_t st, TileCfg* best, Launcher&& launch) {
  hipEvent_t e0, e1;
  J3D_HIP(hipEventCreate(&e0));
  J3D_HIP(hipEventCreate(&e1));
  std::map<std::tuple<int, int, int, int, int, int>, float> seen;
  int rc = J3D_OK;
  auto time_of = [&](const TileCfg& c, float* out) -> int {
    auto key = std::make_tuple(c.rows, c.planes, c.variant, c.persistent, c.order, c.cols);
    auto it = seen.find(key);
    if (it != seen.end()) {
      *out = it->second;
      return J3D_OK;
    }
    J3D_TRY(launch(c));  // warm-up (also builds tables)
    float ms_min = 1e30f;
    for (int r = 0; r < 3; ++r) {
      J3D_HIP(hipEventRecord(e0, st));
      J3D_TRY(launch(c));
      J3D_HIP(hipEventRecord(e1, st));
      J3D_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      J3D_HIP(hipEventElapsedTime(&ms, e0, e1));
      ms_min = std::min(ms_min, ms);
    }
    seen[key] = ms_min;
    *out = ms_min;
    return J3D_OK;
  };
  const std::vector<TileCfg> all = candidates();
  std::vector<int> rows_set, planes_set, var_set;
  for (const TileCfg& c : all) {
    if (std::find(rows_set.begin(), rows_set.end(), c.rows) == rows_set.end()) rows_set.push_back(c.rows);
    if (std::find(planes_set.begin(), planes_set.end(), c.planes) == planes_set.end())
      planes_set.push_back(c.planes);
    if (std::find(var_set.begin(), var_set.end(), c.variant) == var_set.end()) var_set.push_back(c.variant);
  }
  TileCfg b{1, 16, 20, 0, 1, 1};
  float bt = 1e30f;
  auto consider = [&](const TileCfg& c) -> int {
    float t = 0.f;
    J3D_TRY(time_of(c, &t));
    if (t < bt) {
      bt = t;
      b = c;
    }
    return J3D_OK;
  };
  for (int stage = 0; stage < 3 && rc == J3D_OK; ++stage) {
    const TileCfg base = b;
    if (stage == 1) {
      for (int v : var_set)
        for (int p = 0; p < 2; ++p)
          for (int o = 0; o < 3; ++o)
            for (int cx : {1, 2, 4}) {
              if (rc != J3D_OK) break;
              const TileCfg cand{base.rows, base.planes, v, p, o, cx};
              if (tile_cfg_supported(cand)) rc = consider(cand);
            }
    } else {
      for (int r : rows_set)
        for (int pl : planes_set) {
          if (rc != J3D_OK) break;
          const TileCfg cand{r, pl, base.variant, base.persistent, base.order, base.cols};
          if (tile_cfg_supported(cand)) rc = consider(cand);
        }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == J3D_OK) *best = b;
  return rc;
}

// Time F_WRITE passes of every listed tile shape; return the fastest.  Each
// shape gets a warm-up and the best of three launches; the (up to) eight
// fastest are then timed again, best of seven, and the fastest of that
// round wins, so that shapes within the launch-to-launch noise of each
// other are not picked by one lucky launch.
template <typename Launcher>
int time_list(hipStream_t st, TileCfg* best, const std::vector<TileCfg>& list, Launcher&& launch,
              float* best_ms = nullptr) {
  hipEvent_t e0, e1;
  J3D_HIP(hipEventCreate(&e0));
  J3D_HIP(hipEventCreate(&e1));
  int rc = J3D_OK;
  auto time_of = [&](const TileCfg& c, int reps, float* out) -> int {
    J3D_TRY(launch(c));  // warm-up (also builds the tables)
    float ms_min = 1e30f;
    for (int r = 0; r < reps; ++r) {
      if (hipEventRecord(e0, st) != hipSuccess) return fail(J3D_EHIP, "event record");
      J3D_TRY(launch(c));
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return fail(J3D_EHIP, "event sync");
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms_min = std::min(ms_min, ms);
    }
    *out = ms_min;
    return J3D_OK;
  };
  std::vector<std::pair<float, size_t>> first;
  for (size_t q = 0; q < list.size() && rc == J3D_OK; ++q) {
    float t = 0.f;
    rc = time_of(list[q], 3, &t);
    if (rc == J3D_OK) first.emplace_back(t, q);
  }
  float bt = 1e30f;
  if (rc == J3D_OK && !first.empty()) {
    std::stable_sort(first.begin(), first.end(),
                     [](const std::pair<float, size_t>& a, const std::pair<float, size_t>& b) { return a.first < b.first; });
    const size_t top = std::min<size_t>(8, first.size());
    if (top == 1) {
      bt = first[0].first;
      *best = list[first[0].second];
    }
    for (size_t q = 0; q < top && top > 1 && rc == J3D_OK; ++q) {
      float t = 0.f;
      rc = time_of(list[first[q].second], 7, &t);
      if (rc == J3D_OK && t < bt) {
        bt = t;
        *best = list[first[q].second];
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_ms != nullptr) *best_ms = bt;
  return rc;
}

std::vector<TileCfg> sweep3_candidates(int dtype) {
  std::vector<TileCfg> v;
  for (int rows : {2, 4, 8, 16})
    for (int var : {6, 20})
      for (int planes : {16, 24, 32, 48, 64, 96, 128, 144, 192})
        for (int order : {0, 1, 2}) {
          TileCfg c{rows, planes, var, 0, order, 1};
          if (tile3_cfg_supported(dtype, c)) v.push_back(c);
        }
  return v;
}

std::vector<TileCfg> sweep2_candidates(int dtype) {
  std::vector<TileCfg> v;
  for (int rows : {1, 2, 4, 8})
    for (int cols : {1, 2, 4})
      for (int var : {0, 4, 2, 6, 16, 20})
        for (int planes : {16, 32, 64})
          for (int order : {0, 1, 2}) {
            TileCfg c{rows, planes, var, 0, order, cols};
            if (tile2_cfg_supported(dtype, c)) v.push_back(c);
          }
  return v;
}

}  // namespace

bool tune_cache_lookup_single(int dtype, int nx, int ny, int nz, TileCfg* out) {
  return tune_lookup(single_key(dtype, nx, ny, nz), out);
}

void release_batch_cache() {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  for (Plan* p : g_plans) {
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    free_plan(p);
  }
  g_plans.clear();
}

// The batched tuners upload a tile table per shape; the launchers keep the
// last shape they uploaded, so that only the warm-up launch of a shape pays
// for the host-side table build and copy and the timed launches are bare.
struct Prepared {
  int kind = 0;  // passes of the uploaded table (0: none)
  TileCfg c{};
  int nt = 0;
  bool holds(int k, const TileCfg& d) const {
    return kind == k && c.rows == d.rows && c.planes == d.planes && c.variant == d.variant &&
           c.persistent == d.persistent && c.order == d.order && c.cols == d.cols;
  }
};

// Tunes the batched sweep for the batch's shape class (used by serve.cpp too).
int autotune_batch_fields(const BatchFields& bf, TileCfg* best, hipStream_t st);

int autotune_batch_fields(const BatchFields& bf, TileCfg* best, hipStream_t st) {
  const int n = (int)bf.a.size();
  GridArgs* dtab = nullptr;
  double* parts = nullptr;
  size_t tab_cap = 0, part_cap = 0;
  Prepared prep;
  auto launch = [&](const TileCfg& c) -> int {
    if (prep.holds(1, c)) {
      J3D_HIP(launch_pass_batch(J3D_F64, F_WRITE, c, dtab, n, prep.nt, parts, nullptr, st));
      return J3D_OK;
    }
    std::vector<GridArgs> tab[4];
    int nt = 0;
    build_tables(bf, c, tab, &nt);
    if ((size_t)n > tab_cap) {
      if (dtab) (void)hipFree(dtab);
      void* m = nullptr;
      J3D_TRY(dev_alloc(&m, (size_t)n * sizeof(GridArgs), "tune table"));
      dtab = static_cast<GridArgs*>(m);
      tab_cap = n;
    }
    if ((size_t)nt > part_cap) {
      if (parts) (void)hipFree(parts);
      void* m = nullptr;
      J3D_TRY(dev_alloc(&m, (size_t)nt * sizeof(double), "tune partials"));
      parts = static_cast<double*>(m);
      part_cap = nt;
    }
    J3D_HIP(hipMemcpyAsync(dtab, tab[0].data(), (size_t)n * sizeof(GridArgs), hipMemcpyHostToDevice, st));
    J3D_HIP(hipStreamSynchronize(st));
    prep.kind = 1;
    prep.c = c;
    prep.nt = nt;
    J3D_HIP(launch_pass_batch(J3D_F64, F_WRITE, c, dtab, n, nt, parts, nullptr, st));
    return J3D_OK;
  };
  int rc = time_candidates(st, best, launch);
  (void)hipStreamSynchronize(st);
  if (dtab) (void)hipFree(dtab);
  if (parts) (void)hipFree(parts);
  return rc;
}

// Tunes the two-sweep batched pass (or, with keep_c2, times the shape in
// *best2 only) and decides whether it beats two one-sweep passes of shape c
// on these grids.
int autotune_batch2_fields(const BatchFields& bf, const TileCfg& c, bool keep_c2, TileCfg* best2, bool* pairs,
                           hipStream_t st) {
  const int n = (int)bf.a.size();
  GridArgs* dtab = nullptr;
  double* parts = nullptr;
  int part_cap = 0;
  int rc = dev_alloc(reinterpret_cast<void**>(&dtab), (size_t)n * sizeof(GridArgs), "tune table");
  if (rc != J3D_OK) return rc;
  Prepared prep;
  auto upload = [&](const std::vector<GridArgs>& tab, int nt) -> int {
    if (nt > part_cap) {
      if (parts) (void)hipFree(parts);
      parts = nullptr;
      J3D_TRY(dev_alloc(reinterpret_cast<void**>(&parts), (size_t)nt * sizeof(double), "tune partials"));
      part_cap = nt;
    }
    J3D_HIP(hipMemcpyAsync(dtab, tab.data(), (size_t)n * sizeof(GridArgs), hipMemcpyHostToDevice, st));
    J3D_HIP(hipStreamSynchronize(st));
    return J3D_OK;
  };
  auto launch2 = [&](const TileCfg& c2) -> int {
    if (!prep.holds(2, c2)) {
      std::vector<GridArgs> tab2[2];
      int nt = 0;
      build_tables2(bf, c2, tab2, &nt);
      J3D_TRY(upload(tab2[0], nt));
      prep.kind = 2;
      prep.c = c2;
      prep.nt = nt;
    }
    J3D_HIP(launch_sweep2_batch(J3D_F64, F_WRITE, c2, dtab, n, prep.nt, parts, nullptr, st));
    return J3D_OK;
  };
  auto launch1 = [&](const TileCfg& c1) -> int {
    if (!prep.holds(1, c1)) {
      std::vector<GridArgs> tab[4];
      int nt = 0;
      build_tables(bf, c1, tab, &nt);
      J3D_TRY(upload(tab[0], nt));
      prep.kind = 1;
      prep.c = c1;
      prep.nt = nt;
    }
    J3D_HIP(launch_pass_batch(J3D_F64, F_WRITE, c1, dtab, n, prep.nt, parts, nullptr, st));
    return J3D_OK;
  };
  float t2 = 0.f, t1 = 0.f;
  TileCfg one = c;
  const std::vector<TileCfg> cand2 = keep_c2 ? std::vector<TileCfg>{*best2} : sweep2_candidates(J3D_F64);
  rc = time_list(st, best2, cand2, launch2, &t2);
  if (rc == J3D_OK) rc = time_list(st, &one, std::vector<TileCfg>{c}, launch1, &t1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(dtab);
  if (parts) (void)hipFree(parts);
  *pairs = t2 < 2.f * t1;
  return rc;
}

// Tunes the three-sweep batched pass (or, with keep_c3, times the shape in
// *best3 only) and decides whether it beats the passes the batch would run
// otherwise: two-sweep passes of shape c2 when `pairs`, else one-sweep
// passes of shape c, compared per sweep.
int autotune_batch3_fields(const BatchFields& bf, const TileCfg& c, bool pairs, const TileCfg& c2, bool keep_c3,
                           TileCfg* best3, bool* use, hipStream_t st) {
  const int n = (int)bf.a.size();
  GridArgs* dtab = nullptr;
  double* parts = nullptr;
  int part_cap = 0;
  int rc = dev_alloc(reinterpret_cast<void**>(&dtab), (size_t)n * sizeof(GridArgs), "tune table");
  if (rc != J3D_OK) return rc;
  Prepared prep;
  auto upload = [&](const std::vector<GridArgs>& tab, int nt) -> int {
    if (nt > part_cap) {
      if (parts) (void)hipFree(parts);
      parts = nullptr;
      J3D_TRY(dev_alloc(reinterpret_cast<void**>(&parts), (size_t)nt * sizeof(double), "tune partials"));
      part_cap = nt;
    }
    J3D_HIP(hipMemcpyAsync(dtab, tab.data(), (size_t)n * sizeof(GridArgs), hipMemcpyHostToDevice, st));
    J3D_HIP(hipStreamSynchronize(st));
    return J3D_OK;
  };
  TileSlot* dslots = nullptr;
  size_t slot_cap = 0;
  int nslots = 0;
  auto launch3 = [&](const TileCfg& k3) -> int {
    if (!prep.holds(3, k3)) {
      std::vector<GridArgs> tab3[2];
      int nt = 0;
      build_tables3(bf, k3, tab3, &nt);
      J3D_TRY(upload(tab3[0], nt));
      nslots = 0;
      if (k3.order == kOrderSlots) {
        std::vector<TileSlot> sl;
        build_slots3(tab3[0], nt, &sl);
        if (sl.size() > slot_cap) {
          if (dslots) (void)hipFree(dslots);
          dslots = nullptr;
          slot_cap = 0;
          J3D_TRY(dev_alloc(reinterpret_cast<void**>(&dslots), sl.size() * sizeof(TileSlot), "tune slots"));
          slot_cap = sl.size();
        }
        J3D_HIP(hipMemcpyAsync(dslots, sl.data(), sl.size() * sizeof(TileSlot), hipMemcpyHostToDevice, st));
        J3D_HIP(hipStreamSynchronize(st));
        nslots = (int)sl.size();
      }
      prep.kind = 3;
      prep.c = k3;
      prep.nt = nt;
    }
    J3D_HIP(launch_sweep3_batch(J3D_F64, F_WRITE, k3, dtab, n, prep.nt, parts, nullptr, st,
                                k3.order == kOrderSlots ? dslots : nullptr, nslots));
    return J3D_OK;
  };
  auto launch2 = [&](const TileCfg& k2) -> int {
    if (!prep.holds(2, k2)) {
      std::vector<GridArgs> tab2[2];
      int nt = 0;
      build_tables2(bf, k2, tab2, &nt);
      J3D_TRY(upload(tab2[0], nt));
      prep.kind = 2;
      prep.c = k2;
      prep.nt = nt;
    }
    J3D_HIP(launch_sweep2_batch(J3D_F64, F_WRITE, k2, dtab, n, prep.nt, parts, nullptr, st));
    return J3D_OK;
  };
  auto launch1 = [&](const TileCfg& k1) -> int {
    if (!prep.holds(1, k1)) {
      std::vector<GridArgs> tab[4];
      int nt = 0;
      build_tables(bf, k1, tab, &nt);
      J3D_TRY(upload(tab[0], nt));
      prep.kind = 1;
      prep.c = k1;
      prep.nt = nt;
    }
    J3D_HIP(launch_pass_batch(J3D_F64, F_WRITE, k1, dtab, n, prep.nt, parts, nullptr, st));
    return J3D_OK;
  };
  float t3 = 0.f, tother = 0.f;
  std::vector<TileCfg> cand3;
  if (keep_c3) {
    cand3.push_back(*best3);
  } else {
    // every single-grid shape in the XCD-blocked order and in the balanced
    // slot order (orders 1 and 2, which give up the per-XCD locality, lose
    // on batches)
    for (const TileCfg& k : sweep3_candidates(J3D_F64)) {
      if (k.order != 0) continue;
      cand3.push_back(k);
      cand3.push_back(TileCfg{k.rows, k.planes, k.variant, k.persistent, kOrderSlots, k.cols});
    }
  }
  rc = time_list(st, best3, cand3, launch3, &t3);
  TileCfg other = pairs ? c2 : c;
  if (rc == J3D_OK)
    rc = pairs ? time_list(st, &other, std::vector<TileCfg>{c2}, launch2, &tother)
               : time_list(st, &other, std::vector<TileCfg>{c}, launch1, &tother);
  (void)hipStreamSynchronize(st);
  (void)hipFree(dtab);
  if (parts) (void)hipFree(parts);
  if (dslots) (void)hipFree(dslots);
  *use = t3 / 3.f < tother / (pairs ? 2.f : 1.f);
  return rc;
}

}  // namespace j3d

using namespace j3d;

extern "C" int jacobi3d_sweep_batch(int32_t ngrids, j3d_grid* grids, int32_t nsweeps,
                                    int32_t resid_every, double* resid_out, const j3d_tune* tune,
                                    void* stream) {
  BatchFields bf;
  J3D_TRY(check_batch(ngrids, grids, &bf));
  if (nsweeps < 0) return fail(J3D_EINVAL, "nsweeps must be >= 0");
  if (resid_out != nullptr && resid_every < 1) return fail(J3D_EINVAL, "resid_every must be >= 1");
  if (nsweeps > (1 << 20)) return fail(J3D_EINVAL, "nsweeps too large for one graph");
  hipStream_t st = static_cast<hipStream_t>(stream);
  TileCfg c;
  if (tune != nullptr) {
    c = TileCfg{tune->rows, tune->planes, tune->variant, tune->persistent, tune->order, tune->cols};
    if (!tile_cfg_supported(c)) return fail(J3D_EINVAL, "unsupported tile shape");
  } else {
    const std::string bk = batch_key(ngrids, bf.a.data());
    if (!tune_lookup(bk, &c)) {
      J3D_TRY(autotune_batch_fields(bf, &c, st));
      tune_store(bk, c);
    }
  }
  if (nsweeps == 0 && resid_out == nullptr) return J3D_OK;
  // Two sweeps per pass when every residual falls on an even sweep count and
  // the two-sweep pass is the faster one on this batch (decided once per
  // batch shape class).
  // J3D_BATCH_PAIRS=0 / =1 turns the choice off / on regardless of timing.
  // With an explicit tile shape the two-sweep passes use that shape too when
  // the two-sweep kernel has it (else the default two-sweep shape), so that
  // a grid's numbers do not depend on the batch it is in.
  bool pairs = false;
  TileCfg c2 = default_cfg2(J3D_F64, 64, 64, 64);
  if (tune != nullptr && tile2_cfg_supported(J3D_F64, c)) c2 = c;
  const char* force = getenv("J3D_BATCH_PAIRS");
  const int mode = (force && *force == '0') ? 0 : (force && *force == '1') ? 1 : -1;
  if (mode != 0 && nsweeps >= 2 && (resid_out == nullptr || resid_every % 2 == 0)) {
    if (mode == 1 && tune != nullptr) {
      pairs = true;
    } else {
      char sig[64];
      snprintf(sig, sizeof sig, ":x2:%d", tune != nullptr ? 1 : 0);
      const std::string k2 = batch_key(ngrids, bf.a.data()) + sig;
      if (!pair_lookup(k2, &c2, &pairs)) {
        J3D_TRY(autotune_batch2_fields(bf, c, tune != nullptr, &c2, &pairs, st));
        pair_store(k2, c2, pairs);
      }
      if (mode == 1) pairs = true;
    }
  }
  // Passes of up to three sweeps (any residual cadence: residuals are fused
  // at the stage that forms their iterate) when the three-sweep pass beats
  // the passes chosen above, per sweep, on this batch (decided once per
  // batch shape class).  J3D_BATCH_TRIPLES=0 / =1 turns the choice off / on
  // regardless of timing; an explicit tile shape is used for the
  // three-sweep passes when that kernel has it.
  bool triples = false;
  TileCfg c3 = default_cfg3(J3D_F64, 64, 64, 64);
  bool keep_c3 = false;
  if (tune != nullptr && tile3_cfg_supported(J3D_F64, c)) {
    c3 = c;
    keep_c3 = true;
  }
  // J3D_BATCH_TILE3="rows,planes,variant,order" fixes the three-sweep shape
  // (order kOrderSlots: the balanced slot order); the choice of pass kind is
  // still timed unless J3D_BATCH_TRIPLES forces it.
  const char* env3 = getenv("J3D_BATCH_TILE3");
  if (env3 != nullptr) {
    TileCfg t{0, 0, 0, 0, 0, 1};
    if (sscanf(env3, "%d,%d,%d,%d", &t.rows, &t.planes, &t.variant, &t.order) != 4)
      return fail(J3D_EINVAL, "J3D_BATCH_TILE3: expected rows,planes,variant,order");
    TileCfg chk = t;
    if (chk.order == kOrderSlots) chk.order = 0;
    if (!tile3_cfg_supported(J3D_F64, chk)) return fail(J3D_EINVAL, "J3D_BATCH_TILE3: unsupported shape");
    c3 = t;
    keep_c3 = true;
  }
  const char* force3 = getenv("J3D_BATCH_TRIPLES");
  int mode3 = (force3 && *force3 == '0') ? 0 : (force3 && *force3 == '1') ? 1 : -1;
  // the three-sweep pass needs every plane below 4 GiB
  for (int g = 0; g < ngrids && mode3 != 0; ++g)
    if (!plane_fits_u32(bf.a[g]) || !plane_fits_u32(bf.b[g]) || !plane_fits_u32(bf.f[g])) mode3 = 0;
  if (mode3 != 0 && nsweeps >= 3) {
    if (mode3 == 1 && tune != nullptr) {
      triples = true;
    } else {
      char sig[64];
      snprintf(sig, sizeof sig, ":x3:%d:%d:%d,%d,%d,%d", keep_c3 ? 1 : 0, pairs ? 1 : 0, keep_c3 ? c3.rows : 0,
               keep_c3 ? c3.planes : 0, keep_c3 ? c3.variant : 0, keep_c3 ? c3.order : 0);
      const std::string k3 = batch_key(ngrids, bf.a.data()) + sig;
      if (!pair_lookup(k3, &c3, &triples)) {
        J3D_TRY(autotune_batch3_fields(bf, c, pairs, c2, keep_c3, &c3, &triples, st));
        pair_store(k3, c3, triples);
      }
      if (mode3 == 1) triples = true;
    }
  }
  // Plan key: every descriptor, h, counts, output and tile shapes.
  std::string key;
  key.append(reinterpret_cast<const char*>(grids), sizeof(j3d_grid) * (size_t)ngrids);
  int dev = 0;
  J3D_HIP(hipGetDevice(&dev));
  const long long meta[7] = {ngrids, nsweeps, resid_every, (long long)(uintptr_t)resid_out, dev,
                             pairs ? 1 : 0, triples ? 1 : 0};
  key.append(reinterpret_cast<const char*>(meta), sizeof meta);
  // the tile shapes as they are (TileCfg holds ints only, so no padding);
  // a shape a plan does not use is zeroed, keeping equal plans' keys equal
  static_assert(sizeof(TileCfg) == 6 * sizeof(int), "TileCfg must have no padding");
  const TileCfg none{};
  const TileCfg shapes[3] = {c, pairs ? c2 : none, triples ? c3 : none};
  key.append(reinterpret_cast<const char*>(shapes), sizeof shapes);
  Plan* plan = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (Plan* p : g_plans)
      if (p->key == key) {
        plan = p;
        break;
      }
    if (plan == nullptr) {
      J3D_TRY(make_plan(key, bf, c, pairs, c2, triples, c3, nsweeps, resid_every, resid_out, &plan));
      if (g_plans.size() >= kMaxPlans) {
        auto it = std::min_element(g_plans.begin(), g_plans.end(),
                                   [](Plan* x, Plan* y) { return x->stamp < y->stamp; });
        (void)hipDeviceSynchronize();
        free_plan(*it);
        g_plans.erase(it);
      }
      g_plans.push_back(plan);
    }
    plan->stamp = ++g_stamp;
  }
  J3D_HIP(hipGraphLaunch(plan->exec, st));
  g_last_plan.kind = triples ? 3 : pairs ? 2 : 1;
  g_last_plan.c = triples ? c3 : pairs ? c2 : c;
  return J3D_OK;
}

extern "C" int j3d_batch_last_plan(int32_t* sweeps_per_pass, j3d_tune* shape) {
  if (sweeps_per_pass == nullptr || shape == nullptr) return fail(J3D_EINVAL, "null pointer");
  if (g_last_plan.kind == 0) return fail(J3D_ESTATE, "this thread has made no jacobi3d_sweep_batch call");
  *sweeps_per_pass = g_last_plan.kind;
  const TileCfg& c = g_last_plan.c;
  *shape = j3d_tune{c.rows, c.planes, c.variant, c.persistent, c.order, c.cols};
  return J3D_OK;
}

extern "C" int j3d_autotune(int32_t ngrids, j3d_grid* grids, j3d_tune* best, void* stream) {
  BatchFields bf;
  J3D_TRY(check_batch(ngrids, grids, &bf));
  if (best == nullptr) return fail(J3D_EINVAL, "best: null pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  TileCfg c{};
  J3D_TRY(autotune_batch_fields(bf, &c, st));
  tune_store(batch_key(ngrids, bf.a.data()), c);
  if (ngrids == 1) tune_store(single_key(J3D_F64, bf.a[0].nx(), bf.a[0].ny(), bf.a[0].nz()), c);
  best->rows = c.rows;
  best->planes = c.planes;
  best->variant = c.variant;
  best->persistent = c.persistent;
  best->order = c.order;
  best->cols = c.cols;
  return J3D_OK;
}

extern "C" int j3d_autotune_single(int32_t dtype, int32_t nx, int32_t ny, int32_t nz, j3d_tune* best,
                                   void* stream) {
  if (dtype != J3D_F64 && dtype != J3D_F32 && dtype != J3D_KIND_F64X2 && dtype != J3D_KIND_F32X2 &&
      dtype != J3D_KIND_F64X3 && dtype != J3D_KIND_F32X3)
    return fail(J3D_EDTYPE, "kind must be J3D_F64, J3D_F32 or a J3D_KIND_* pass kind");
  if (nx < 1 || ny < 1 || nz < 1) return fail(J3D_EINVAL, "extents must be >= 1");
  if (best == nullptr) return fail(J3D_EINVAL, "best: null pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool pair = dtype == J3D_KIND_F64X2 || dtype == J3D_KIND_F32X2;
  const bool triple = dtype == J3D_KIND_F64X3 || dtype == J3D_KIND_F32X3;
  const int et = (dtype == J3D_F32 || dtype == J3D_KIND_F32X2 || dtype == J3D_KIND_F32X3) ? J3D_F32 : J3D_F64;
  const int es = et == J3D_F32 ? 4 : 8;
  const int align = 128 / es;
  Field a;
  a.dtype = et;
  a.esize = es;
  a.ex = nx + 2;
  a.ey = ny + 2;
  a.ez = nz + 2;
  a.sy = ((long long)a.ex + align - 1) / align * align;
  a.sz = a.sy * a.ey;
  if (a.sz * a.ez >= (1LL << 31) - align) return fail(J3D_EINVAL, "grid too large");
  if (triple && !plane_fits_u32(a))
    return fail(J3D_EINVAL, "a z-plane spans 4 GiB or more: the three-sweep pass needs smaller planes");
  const size_t bytes = ((size_t)(a.sz * a.ez + align) * es + 255) / 256 * 256;
  void* mem = nullptr;
  J3D_TRY(dev_alloc(&mem, 3 * bytes, "autotune arrays"));
  char* m = static_cast<char*>(mem);
  hipError_t e = hipMemsetAsync(m, 0, 3 * bytes, st);
  if (e != hipSuccess) {
    (void)hipFree(mem);
    return hip_fail(e, "autotune memset");
  }
  Field u = a, o = a, f = a;
  u.base = m + (align - 1) * es;
  o.base = m + bytes + (align - 1) * es;
  f.base = m + 2 * bytes + (align - 1) * es;
  auto launch = [&](const TileCfg& c) -> int {
    GridArgs g = make_args(&u, &o, &f, nullptr, nullptr, 0.01, c, 0);
    J3D_HIP(launch_pass_one(et, F_WRITE, c, g, nullptr, nullptr, st));
    return J3D_OK;
  };
  auto launch2 = [&](const TileCfg& c) -> int {
    GridArgs g = make_args2(&u, &o, &f, nullptr, 0.01, c, 0);
    J3D_HIP(launch_sweep2_one(et, F_WRITE, c, g, nullptr, nullptr, st));
    return J3D_OK;
  };
  auto launch3 = [&](const TileCfg& c) -> int {
    GridArgs g = make_args3(&u, &o, &f, nullptr, 0.01, c, 0);
    J3D_HIP(launch_sweep3_one(et, F_WRITE, c, g, nullptr, nullptr, st));
    return J3D_OK;
  };
  TileCfg c{};
  int rc = triple ? time_list(st, &c, sweep3_candidates(et), launch3)
           : pair ? time_list(st, &c, sweep2_candidates(et), launch2)
                  : time_candidates(st, &c, launch);
  (void)hipStreamSynchronize(st);
  (void)hipFree(mem);
  if (rc != J3D_OK) return rc;
  tune_store(single_key(dtype, nx, ny, nz), c);
  best->rows = c.rows;
  best->planes = c.planes;
  best->variant = c.variant;
  best->persistent = c.persistent;
  best->order = c.order;
  best->cols = c.cols;
  return J3D_OK;
}

extern "C" int j3d_tune_set_single(int32_t dtype, int32_t nx, int32_t ny, int32_t nz, const j3d_tune* t) {
  if (t == nullptr) return fail(J3D_EINVAL, "tune: null pointer");
  TileCfg c{t->rows, t->planes, t->variant, t->persistent, t->order, t->cols};
  if (dtype != J3D_F64 && dtype != J3D_F32 && dtype != J3D_KIND_F64X2 && dtype != J3D_KIND_F32X2 &&
      dtype != J3D_KIND_F64X3 && dtype != J3D_KIND_F32X3)
    return fail(J3D_EDTYPE, "kind must be J3D_F64, J3D_F32 or a J3D_KIND_* pass kind");
  const bool ok = dtype == J3D_KIND_F64X2   ? tile2_cfg_supported(J3D_F64, c)
                  : dtype == J3D_KIND_F32X2 ? tile2_cfg_supported(J3D_F32, c)
                  : dtype == J3D_KIND_F64X3 ? tile3_cfg_supported(J3D_F64, c)
                  : dtype == J3D_KIND_F32X3 ? tile3_cfg_supported(J3D_F32, c)
                                            : tile_cfg_supported(c);
  if (!ok) return fail(J3D_EINVAL, "unsupported tile shape");
  tune_store(single_key(dtype, nx, ny, nz), c);
  return J3D_OK;
}
