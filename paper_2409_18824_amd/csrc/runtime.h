// Host runtime shared by the C-ABI entry points of libj3d.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "j3d_internal.h"

namespace j3d {

// Records a message for j3d_last_error() on this thread and returns code.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char* what);

#define J3D_HIP(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return ::j3d::hip_fail(e_, #expr); \
  } while (0)

#define J3D_TRY(expr)            \
  do {                           \
    int rc_ = (expr);            \
    if (rc_ != J3D_OK) return rc_; \
  } while (0)

// A validated Fortran array.
struct Field {
  char* base = nullptr;  // element (lbound0, lbound1, lbound2)
  int dtype = 0;
  int esize = 8;
  int ex = 0, ey = 0, ez = 0;  // extents including the halo
  long long sy = 0, sz = 0;    // strides (elements)
  int nx() const { return ex - 2; }
  int ny() const { return ey - 2; }
  int nz() const { return ez - 2; }
  long long span_elems() const { return (long long)(ez - 1) * sz + (long long)(ey - 1) * sy + ex; }
  size_t span_bytes() const { return (size_t)span_elems() * esize; }
};

// Validate a descriptor; dtype < 0 accepts either element type.
int check_field(const j3d_array* a, int dtype, Field* out, const char* name);
// As check_field, for kernels that address planes with 64-bit offsets: only
// the offsets within one plane must stay below 2^31.
int check_field_wide(const j3d_array* a, int dtype, Field* out, const char* name);
// Validate a rank-2 array: axes 0 and 1 as for check_field, axis 2 of
// extent 1 (lbound[2] == ubound[2]); ez = 1 in the result.
int check_field2d(const j3d_array* a, int dtype, Field* out, const char* name);
bool fields_overlap(const Field& a, const Field& b);
// The three-sweep pass addresses each plane of an array through a buffer
// descriptor with 32-bit byte offsets: true when every offset within one
// plane of `a` is below 2^32 bytes.
bool plane_fits_u32(const Field& a);
int check_same_interior(const Field& a, const Field& b, const char* an, const char* bn);
int check_h(double h);

// Launch arguments for one pass.  `o`, `f`, `u64`, `r32` may be null when the
// pass does not touch them.
GridArgs make_args(const Field* u, const Field* o, const Field* f, const Field* u64,
                   const Field* r32, double h, const TileCfg& c, int tile0);
// Launch arguments of the two-sweep pass (its own tile counts).  u may be
// null (a zero input, F_FIRST); u64 is the FP64 field of F_LAST.
GridArgs make_args2(const Field* u, const Field* o, const Field* f, const Field* u64, double h,
                    const TileCfg& c, int tile0);

// Launch arguments of the three-sweep pass (its own tile counts).
GridArgs make_args3(const Field* u, const Field* o, const Field* f, const Field* u64, double h,
                    const TileCfg& c, int tile0);

// Default tile shape for a grid of this size and element type (the
// autotuner's cached choice when there is one).
TileCfg default_cfg(int dtype, int nx, int ny, int nz);
TileCfg default_cfg2(int dtype, int nx, int ny, int nz);  // two-sweep pass
TileCfg default_cfg3(int dtype, int nx, int ny, int nz);  // three-sweep pass

// A validated jacobi3d_sweep3 call: its fields, the residual flag of the
// pass (F_RES, F_RES1 or F_RES2), the tile shape and the launch arguments.
struct Sweep3Call {
  Field a, b, c;
  unsigned res_flag = 0;
  TileCfg cfg{};
  GridArgs g{};
};
// Checks the arguments of jacobi3d_sweep3 (and of its allocation-free
// variant) without touching a device.
int check_sweep3_call(const j3d_array* u_in, const j3d_array* u_out, const j3d_array* f, double h,
                      uint32_t flags, const double* resid_out, Sweep3Call* k);

// Per-(device, stream) scratch: tile partials, control words, pinned host
// words.  Grows on demand; lives until j3d_release_cache().
struct Control {
  double normf;
  double value;
  double value2;
  double pad;
  long long conv_at;
  long long qnext;  // index of the next check (advanced on the device)
  int done;
  int nonfinite;
};

// An instantiated graph of one chunk of a solve, keyed by everything its
// kernels' arguments depend on.
struct SolveGraph {
  std::string key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  unsigned long long stamp = 0;
};

struct Scratch {
  int device = 0;
  hipStream_t stream = nullptr;
  double* partials = nullptr;
  size_t partials_cap = 0;
  Control* ctl = nullptr;      // device
  Control* ctl_host = nullptr; // pinned host mirror
  double* hist = nullptr;      // device history
  size_t hist_cap = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  // work arrays for poisson_solve
  void* work = nullptr;
  size_t work_bytes = 0;
  // graphs of solve chunks replayed on `stream` (captured on `capture`)
  hipStream_t capture = nullptr;
  std::vector<SolveGraph> graphs;
  unsigned long long graph_stamp = 0;
};

// The cached graph for `key`, or a new one captured by enqueue(capture
// stream) and instantiated; at most a few graphs are kept per scratch.
template <typename Enqueue>
int solve_graph(Scratch* s, const std::string& key, Enqueue&& enqueue, hipGraphExec_t* out);
void free_solve_graph(SolveGraph* g);

int get_scratch(hipStream_t st, Scratch** out);
int ensure_partials(Scratch* s, size_t n);
int ensure_hist(Scratch* s, size_t n);
int ensure_work(Scratch* s, size_t bytes);

// Device memory helpers that report through fail().
int dev_alloc(void** p, size_t bytes, const char* what);

// Cached graphs / batch plans are released by this hook (batch.cpp).
void release_batch_cache();

double now_seconds();

template <typename Enqueue>
int solve_graph(Scratch* s, const std::string& key, Enqueue&& enqueue, hipGraphExec_t* out) {
  for (SolveGraph& g : s->graphs)
    if (g.key == key) {
      g.stamp = ++s->graph_stamp;
      *out = g.exec;
      return J3D_OK;
    }
  if (s->capture == nullptr) J3D_HIP(hipStreamCreateWithFlags(&s->capture, hipStreamNonBlocking));
  J3D_HIP(hipStreamBeginCapture(s->capture, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue(s->capture);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(s->capture, &graph);
  if (rc != J3D_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc != J3D_OK ? rc : hip_fail(e, "hipStreamEndCapture");
  }
  SolveGraph g;
  g.key = key;
  g.graph = graph;
  const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(ei, "hipGraphInstantiate");
  }
  g.stamp = ++s->graph_stamp;
  constexpr size_t kMaxGraphs = 4;
  if (s->graphs.size() >= kMaxGraphs) {
    size_t old = 0;
    for (size_t i = 1; i < s->graphs.size(); ++i)
      if (s->graphs[i].stamp < s->graphs[old].stamp) old = i;
    J3D_HIP(hipStreamSynchronize(s->stream));
    free_solve_graph(&s->graphs[old]);
    s->graphs.erase(s->graphs.begin() + (long)old);
  }
  s->graphs.push_back(g);
  *out = g.exec;
  return J3D_OK;
}

}  // namespace j3d
