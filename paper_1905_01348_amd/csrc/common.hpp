// Shared internals of libfock: status/error plumbing, the device context,
// its HBM-budgeted allocator and per-stream workspaces.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <array>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/fock.h"
#include "../../include/fock_prof.h"
#include "../../include/fock_debug.h"

namespace fx {

// ---- error reporting (thread-local text, returned status) -----------------
void set_error(const char* fmt, ...);
void clear_error();

#define FX_FAIL(code, ...)          \
  do {                              \
    ::fx::set_error(__VA_ARGS__);   \
    return (code);                  \
  } while (0)

#define FX_HIP(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ::fx::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                      __LINE__);                                                     \
      return FX_ERR_DEVICE;                                                          \
    }                                                                                \
  } while (0)

#define FX_TRY(expr)              \
  do {                            \
    fx_status s_ = (expr);        \
    if (s_ != FX_OK) return s_;   \
  } while (0)

// Launch-error check after a kernel launch.
#define FX_LAUNCH_CHECK() FX_HIP(hipGetLastError())

// ---- complex scalars --------------------------------------------------------
template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

// ---- device buffers owned by a context --------------------------------------
struct Ctx;

// A growable device buffer charged to the context budget.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// Named scratch buffers for one stream of work (the context has one set, a
// server has one set per in-flight slot).  With an arena set, buffers are
// carved in order from that fixed device region instead of being allocated
// (fx_apply_vx_noalloc); a request that does not fit is refused.
struct Workspace {
  std::map<std::string, DevBuf> bufs;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  size_t arena_used = 0;
};

// Cached per-grid constant tables (twiddles, fold maps, kernel tables).
struct TableKey {
  int n[3];
  double len[3];
  int kind;
  double omega, scale;
  int prec;  // 0 = fp64 tables, 1 = fp32 tables
  int radix[3][4];  // radix schedule of each axis (the fold maps depend on it)
  bool operator<(const TableKey& o) const;
};

struct GridTables {
  // per axis: twiddles w_n^t = exp(-2 pi i t/n), t < n, in the table precision
  void* tw[3] = {nullptr, nullptr, nullptr};
  // per axis: for each position of the digit-reversed spectrum, the folded
  // frequency index |m| in [0, n/2]
  int* fold[3] = {nullptr, nullptr, nullptr};
  // K(G) * (-scale/Omega) on the folded grid (nx/2+1)*(ny/2+1)*(nz/2+1)
  void* kfold = nullptr;
  size_t bytes = 0;
};

// One timed launch: events recorded before and after it on its stream.
struct ProfRec {
  int id;
  double work;  // algorithmic bytes (memory-bound kernels) or executed flops (GEMMs)
  hipEvent_t a, b;
};

}  // namespace fx

struct fx_ctx {
  int device = 0;
  size_t budget = 0;
  size_t in_use = 0;
  size_t peak = 0;
  hipStream_t stream = nullptr;
  int n_cu = 0;
  std::recursive_mutex mu;
  fx::Workspace ws;  // workspace of the context's own calls
  // generations: bumped whenever a workspace is reallocated or released, or a
  // launch configuration changes -- a cached graph made before is stale
  uint64_t ws_gen = 0, cfg_gen = 0;
  // replay cache of fx_apply_vx / fx_apply_ace calls (fx_graph_cache)
  struct GraphEntry {
    std::vector<unsigned char> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t ws_gen = 0, cfg_gen = 0, last_use = 0;
  };
  int graph_max = 0;
  uint64_t graph_tick = 0;
  int64_t graph_hits = 0, graph_misses = 0;
  std::vector<GraphEntry> graphs;
  std::map<fx::TableKey, fx::GridTables> tables;
  // tuned V_X launch configurations, keyed by (n[3], prec, phi == psi form)
  std::map<std::array<int, 5>, fx_vx_config> vx_tuning;
  // set by each entry point: the call's stream is being captured into a
  // graph, so nothing may be allocated or uploaded synchronously
  bool capturing = false;
  // per-kernel timing (fx_prof_enable)
  bool prof = false;
  std::vector<fx::ProfRec> prof_recs;
  std::vector<hipEvent_t> ev_pool;
  int64_t prof_launches[FX_K_COUNT] = {0};
  double prof_ms[FX_K_COUNT] = {0};
  double prof_work[FX_K_COUNT] = {0};
  // live handles created on this context: fx_finalize releases their device
  // memory and detaches them (afterwards only fx_ace_free / fx_serve_destroy
  // may be called on them, and those just delete the handle)
  std::set<fx_ace*> aces;
  std::set<fx_server*> servers;
};

namespace fx {

// Release the device memory of every live ACE handle / server of the context
// and detach them from it (fx_finalize).
void ace_detach_all(fx_ctx* ctx);
void serve_detach_all(fx_ctx* ctx);

// Allocation charged to the context budget.  Returns FX_ERR_OOM when the
// budget would be exceeded or hipMalloc fails.
fx_status ctx_alloc(fx_ctx* ctx, size_t bytes, void** out);
void ctx_free(fx_ctx* ctx, void* p, size_t bytes);

// Let `kernel` use `bytes` of dynamic LDS on the current device (the
// attribute is set once per device and kernel, never again afterwards).
fx_status allow_dynamic_lds(const void* kernel, size_t bytes);

// Replay cache: run `body` on `st` through a cached graph of the call
// described by `key` (every argument, pointers included).  With the cache
// off, or `st` itself being captured, body(st) runs as is.  On a miss body
// runs eagerly on st (so every workspace exists and the result is made), is
// then captured on the context's own stream, and the graph is kept (least
// recently used entries go first); later calls with the same key replay it
// on st.  Entries made before a workspace was reallocated or a launch
// configuration changed are dropped.
template <typename F>
fx_status graph_call(fx_ctx* ctx, const std::vector<unsigned char>& key, hipStream_t st, F body);
void graph_cache_clear(fx_ctx* ctx);

// Record whether `st` is being captured into a graph (ctx->capturing).
fx_status note_capture(fx_ctx* ctx, hipStream_t st);

// Return workspace buffer `name` with at least `bytes`, growing it if needed
// (growth waits for the device before freeing the old buffer).  Under graph
// capture growth is refused with FX_ERR_INVALID.
fx_status ws_get(fx_ctx* ctx, Workspace* ws, const char* name, size_t bytes, void** out);
void ws_release(fx_ctx* ctx, Workspace* ws);

// Plan of an FFT axis: n = R[0] * R[1] * ... (at most 4 radices from
// {2,3,4,6,8,9,12}); DIF stages run in this order.
struct AxisPlan {
  int n;
  int nst;
  int R[4];
};
// The default plan: one stage if n is a radix, else two stages as balanced
// as possible, else up to four.
bool make_axis_plan(int n, AxisPlan* p);
// Whether p is a valid schedule for its n (radices from the set, product n).
bool valid_axis_plan(const AxisPlan& p);
// Schedules of n with at most three stages, fewest stages and most balanced
// first; returns how many were written (at most max_out).
int enumerate_axis_plans(int n, AxisPlan* out, int max_out);
// Frequency index held at each position after the forward DIF stages.
void plan_positions(const AxisPlan& p, std::vector<int>* freq_of_pos);

// The schedules of the three axes of one grid.
struct PlanSet {
  AxisPlan ax[3];
};
void default_plans(const fx_cell* cell, PlanSet* ps);
bool same_plans(const PlanSet& a, const PlanSet& b);

// Device tables for one grid/kernel/precision (built on the host in FP64),
// for the given radix schedules (nullptr: the default ones).
fx_status grid_tables(fx_ctx* ctx, const fx_cell* cell, const fx_kernel* kern, int prec, const PlanSet* plans,
                      const GridTables** out);

// Host copies of the tables (FP64), used to upload and by the host check.
struct HostTables {
  AxisPlan plan[3];
  std::vector<cpx<double>> tw[3];
  std::vector<int> fold[3];
  std::vector<double> kfold;
};
void host_tables(const fx_cell* cell, const fx_kernel* kern, HostTables* h, const PlanSet* plans = nullptr);

bool supported_edge(int n);
fx_status check_cell(const fx_cell* cell);
// Kernel kind used inside the library only: the symbol |G|^2/(2 N_r) of the
// kinetic operator, so that the pair path with the constant orbital 1 applies
// -(1/2) Laplacian.  Public calls reject it.
constexpr int kKineticKind = 100;
fx_status check_kernel(const fx_kernel* k, bool allow_internal = false);

// Bracket a launch with events when timing is on (no-ops otherwise).
fx_status prof_begin(fx_ctx* ctx, hipStream_t st, int id, double work, int* slot);
fx_status prof_end(fx_ctx* ctx, hipStream_t st, int slot);

inline size_t dtype_size(fx_dtype d) { return d == FX_C128 ? 16 : 8; }

// Bytes of a call's arguments, for graph_call keys.
struct KeyBytes {
  std::vector<unsigned char> b;
  template <typename V>
  KeyBytes& add(const V& v) {
    const unsigned char* p = reinterpret_cast<const unsigned char*>(&v);
    b.insert(b.end(), p, p + sizeof(V));
    return *this;
  }
};

template <typename F>
fx_status graph_call(fx_ctx* ctx, const std::vector<unsigned char>& key, hipStream_t st, F body) {
  if (ctx->graph_max <= 0 || ctx->capturing) return body(st);
  auto& G = ctx->graphs;
  for (size_t i = 0; i < G.size(); ++i) {
    if (G[i].key != key) continue;
    if (G[i].ws_gen == ctx->ws_gen && G[i].cfg_gen == ctx->cfg_gen) {
      G[i].last_use = ++ctx->graph_tick;
      ++ctx->graph_hits;
      FX_HIP(hipGraphLaunch(G[i].exec, st));
      return FX_OK;
    }
    (void)hipGraphExecDestroy(G[i].exec);
    (void)hipGraphDestroy(G[i].graph);
    G.erase(G.begin() + i);
    break;
  }
  ++ctx->graph_misses;
  FX_TRY(body(st));
  // capture the same call on the context's stream; workspaces and tables now
  // exist, so the body allocates nothing and waits for nothing
  hipGraph_t g = nullptr;
  FX_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  ctx->capturing = true;
  const fx_status s = body(ctx->stream);
  ctx->capturing = false;
  const hipError_t e = hipStreamEndCapture(ctx->stream, &g);
  if (s != FX_OK || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    clear_error();
    return FX_OK;  // the eager result stands; this call is just not cached
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return FX_OK;
  }
  if ((int)G.size() >= ctx->graph_max) {
    size_t lru = 0;
    for (size_t i = 1; i < G.size(); ++i)
      if (G[i].last_use < G[lru].last_use) lru = i;
    (void)hipGraphExecDestroy(G[lru].exec);
    (void)hipGraphDestroy(G[lru].graph);
    G.erase(G.begin() + lru);
  }
  fx_ctx::GraphEntry en;
  en.key = key;
  en.graph = g;
  en.exec = x;
  en.ws_gen = ctx->ws_gen;
  en.cfg_gen = ctx->cfg_gen;
  en.last_use = ++ctx->graph_tick;
  G.push_back(std::move(en));
  return FX_OK;
}

// Allocation-free form (noalloc.hip): look up, once per device and with that
// device current, the device address of the file-scope scratch region.
fx_status scratch_setup(int device);

// Tuned launch configurations from / to a file (tune.hip).
fx_status load_configs_impl(fx_ctx* ctx, const char* path, int* n_loaded);
fx_status save_configs_impl(fx_ctx* ctx, const char* path);

}  // namespace fx
