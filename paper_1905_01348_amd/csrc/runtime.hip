// libfock runtime: errors, contexts, the HBM-budgeted allocator, workspaces
// and the host-built constant tables (FFT plans, twiddles, kernel K(G)).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "common.hpp"
#include "fft.hpp"

namespace fx {

static thread_local char g_err[1024] = {0};

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  if (getenv("FX_LOG")) fprintf(stderr, "[libfock] %s\n", g_err);
}

void clear_error() { g_err[0] = 0; }

bool TableKey::operator<(const TableKey& o) const {
  for (int a = 0; a < 3; ++a) {
    if (n[a] != o.n[a]) return n[a] < o.n[a];
    if (len[a] != o.len[a]) return len[a] < o.len[a];
  }
  if (kind != o.kind) return kind < o.kind;
  if (omega != o.omega) return omega < o.omega;
  if (scale != o.scale) return scale < o.scale;
  if (prec != o.prec) return prec < o.prec;
  for (int a = 0; a < 3; ++a)
    for (int i = 0; i < 4; ++i)
      if (radix[a][i] != o.radix[a][i]) return radix[a][i] < o.radix[a][i];
  return false;
}

// Optional fault injection for error-path tests: FX_FAULT_INJECT=<k> makes the
// k-th allocation of the process (1-based) fail with FX_ERR_OOM, and
// fx_debug_fail_alloc(k) the k-th allocation after that call (once).
static long g_alloc_count = 0;
static long g_fail_at = 0;  // allocation count that fails (0: none)

fx_status ctx_alloc(fx_ctx* ctx, size_t bytes, void** out) {
  *out = nullptr;
  if (bytes == 0) return FX_OK;
  const char* fi = getenv("FX_FAULT_INJECT");
  long n = __atomic_add_fetch(&g_alloc_count, 1, __ATOMIC_SEQ_CST);
  if (fi && atol(fi) == n) FX_FAIL(FX_ERR_OOM, "injected allocation failure (FX_FAULT_INJECT=%s)", fi);
  long at = n;
  if (__atomic_compare_exchange_n(&g_fail_at, &at, 0L, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST))
    FX_FAIL(FX_ERR_OOM, "injected allocation failure (allocation %ld)", n);
  if (ctx->capturing)
    FX_FAIL(FX_ERR_INVALID,
            "%zu bytes must be allocated while the stream is being captured; run the same call once outside "
            "capture first",
            bytes);
  if (ctx->in_use + bytes > ctx->budget)
    FX_FAIL(FX_ERR_OOM, "HBM budget exceeded: %zu in use + %zu requested > %zu budget", ctx->in_use, bytes,
            ctx->budget);
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) {
    *out = nullptr;
    FX_FAIL(FX_ERR_OOM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  ctx->in_use += bytes;
  if (ctx->in_use > ctx->peak) ctx->peak = ctx->in_use;
  return FX_OK;
}

void ctx_free(fx_ctx* ctx, void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  ctx->in_use -= bytes;
}

fx_status allow_dynamic_lds(const void* kernel, size_t bytes) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, size_t> done;
  if (bytes <= 65536) return FX_OK;
  int dev = 0;
  FX_HIP(hipGetDevice(&dev));
  const std::pair<int, const void*> key(dev, kernel);
  std::lock_guard<std::mutex> lk(mu);
  auto it = done.find(key);
  if (it != done.end() && it->second >= bytes) return FX_OK;
  FX_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  done[key] = bytes;
  return FX_OK;
}

fx_status note_capture(fx_ctx* ctx, hipStream_t st) {
  ctx->capturing = false;
  if (!st) return FX_OK;  // the null stream is never captured
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  FX_HIP(hipStreamIsCapturing(st, &cs));
  ctx->capturing = cs != hipStreamCaptureStatusNone;
  return FX_OK;
}

fx_status ws_get(fx_ctx* ctx, Workspace* ws, const char* name, size_t bytes, void** out) {
  DevBuf& b = ws->bufs[name];
  if (b.bytes >= bytes && b.ptr) {
    *out = b.ptr;
    return FX_OK;
  }
  if (ws->arena) {
    const size_t off = (ws->arena_used + 255) & ~(size_t)255;
    if (off > ws->arena_bytes || bytes > ws->arena_bytes - off)
      FX_FAIL(FX_ERR_INVALID,
              "workspace '%s' needs %zu bytes at offset %zu of a %zu-byte scratch region; the call is too large "
              "for the allocation-free form",
              name, bytes, off, ws->arena_bytes);
    b.ptr = ws->arena + off;
    b.bytes = bytes;
    ws->arena_used = off + bytes;
    *out = b.ptr;
    return FX_OK;
  }
  if (ctx->capturing)
    FX_FAIL(FX_ERR_INVALID,
            "workspace '%s' must grow to %zu bytes while the stream is being captured; "
            "run the same call once outside capture first",
            name, bytes);
  if (b.ptr) {
    // the old buffer may still be in use by queued work
    FX_HIP(hipDeviceSynchronize());
    ctx_free(ctx, b.ptr, b.bytes);
    b.ptr = nullptr;
    b.bytes = 0;
  }
  FX_TRY(ctx_alloc(ctx, bytes, &b.ptr));
  b.bytes = bytes;
  *out = b.ptr;
  ctx->ws_gen++;
  return FX_OK;
}

void ws_release(fx_ctx* ctx, Workspace* ws) {
  if (!ws->arena)
    for (auto& kv : ws->bufs) ctx_free(ctx, kv.second.ptr, kv.second.bytes);
  ws->bufs.clear();
  ws->arena_used = 0;
  if (ctx) ctx->ws_gen++;
}

void graph_cache_clear(fx_ctx* ctx) {
  for (auto& g : ctx->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  ctx->graphs.clear();
}

// ---- per-kernel timing ------------------------------------------------------
static fx_status take_event(fx_ctx* ctx, hipEvent_t* e) {
  if (!ctx->ev_pool.empty()) {
    *e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return FX_OK;
  }
  FX_HIP(hipEventCreate(e));
  return FX_OK;
}

fx_status prof_begin(fx_ctx* ctx, hipStream_t st, int id, double work, int* slot) {
  *slot = -1;
  if (!ctx || !ctx->prof || ctx->capturing) return FX_OK;
  ProfRec r;
  r.id = id;
  r.work = work;
  FX_TRY(take_event(ctx, &r.a));
  FX_TRY(take_event(ctx, &r.b));
  FX_HIP(hipEventRecord(r.a, st));
  ctx->prof_recs.push_back(r);
  *slot = (int)ctx->prof_recs.size() - 1;
  return FX_OK;
}

fx_status prof_end(fx_ctx* ctx, hipStream_t st, int slot) {
  if (!ctx || slot < 0) return FX_OK;
  FX_HIP(hipEventRecord(ctx->prof_recs[slot].b, st));
  return FX_OK;
}

static fx_status prof_drain(fx_ctx* ctx) {
  for (auto& r : ctx->prof_recs) {
    FX_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    FX_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    if (r.id >= 0 && r.id < FX_K_COUNT) {
      ctx->prof_launches[r.id] += 1;
      ctx->prof_ms[r.id] += ms;
      ctx->prof_work[r.id] += r.work;
    }
    ctx->ev_pool.push_back(r.a);
    ctx->ev_pool.push_back(r.b);
  }
  ctx->prof_recs.clear();
  return FX_OK;
}

// ---- FFT plans -------------------------------------------------------------
bool supported_edge(int n) {
  if (n < 2 || n > 96) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

static bool is_radix(int r) {
  return r == 2 || r == 3 || r == 4 || r == 6 || r == 8 || r == 9 || r == 12;
}

bool make_axis_plan(int n, AxisPlan* p) {
  p->n = n;
  p->nst = 0;
  for (int& r : p->R) r = 1;
  if (!supported_edge(n)) return false;
  if (is_radix(n)) {
    p->nst = 1;
    p->R[0] = n;
    return true;
  }
  // two stages, as balanced as possible, larger radix first on ties
  int best = -1, bestmax = 1 << 30;
  const int cand[] = {12, 9, 8, 6, 4, 3, 2};
  for (int r : cand) {
    if (n % r || !is_radix(n / r)) continue;
    int mx = r > n / r ? r : n / r;
    if (mx < bestmax || (mx == bestmax && r > best)) {
      best = r;
      bestmax = mx;
    }
  }
  if (best > 0) {
    p->nst = 2;
    p->R[0] = best;
    p->R[1] = n / best;
    return true;
  }
  // fall back to up to four stages
  int rem = n;
  for (int st = 0; st < 4 && rem > 1; ++st) {
    for (int r : cand) {
      if (rem % r == 0) {
        p->R[p->nst++] = r;
        rem /= r;
        break;
      }
    }
  }
  return rem == 1;
}

// After the forward DIF stages, position pos = k1*(n/R0) + pos' holds the
// frequency k1 + R0*freq'(pos'), freq' being the positions map of the
// remaining stages on n/R0 points.
static void positions_rec(const int* R, int nst, int n, std::vector<int>& f) {
  f.assign(n, 0);
  if (nst == 0 || n == 1) return;
  const int r = R[0], span = n / r;
  std::vector<int> sub;
  positions_rec(R + 1, nst - 1, span, sub);
  for (int k1 = 0; k1 < r; ++k1)
    for (int q = 0; q < span; ++q) f[k1 * span + q] = k1 + r * sub[q];
}

bool valid_axis_plan(const AxisPlan& p) {
  if (p.nst < 1 || p.nst > 4 || !supported_edge(p.n)) return false;
  int prod = 1;
  for (int i = 0; i < p.nst; ++i) {
    if (!is_radix(p.R[i])) return false;
    prod *= p.R[i];
  }
  for (int i = p.nst; i < 4; ++i)
    if (p.R[i] != 1) return false;
  return prod == p.n;
}

int enumerate_axis_plans(int n, AxisPlan* out, int max_out) {
  std::vector<AxisPlan> all;
  const int rad[] = {2, 3, 4, 6, 8, 9, 12};
  auto push = [&](int nst, int a, int b, int c) {
    AxisPlan p;
    p.n = n;
    p.nst = nst;
    p.R[0] = a;
    p.R[1] = b;
    p.R[2] = c;
    p.R[3] = 1;
    if (valid_axis_plan(p)) all.push_back(p);
  };
  if (is_radix(n)) push(1, n, 1, 1);
  for (int a : rad)
    if (n % a == 0 && is_radix(n / a)) push(2, a, n / a, 1);
  for (int a : rad)
    for (int b : rad)
      if (n % (a * b) == 0 && is_radix(n / (a * b))) push(3, a, b, n / (a * b));
  auto maxr = [](const AxisPlan& p) {
    int m = 0;
    for (int i = 0; i < p.nst; ++i) m = p.R[i] > m ? p.R[i] : m;
    return m;
  };
  std::stable_sort(all.begin(), all.end(), [&](const AxisPlan& x, const AxisPlan& y) {
    if (x.nst != y.nst) return x.nst < y.nst;
    return maxr(x) < maxr(y);
  });
  // the default plan first
  AxisPlan d;
  int k = 0;
  if (make_axis_plan(n, &d) && max_out > 0) out[k++] = d;
  for (const AxisPlan& p : all) {
    if (k >= max_out) break;
    bool dup = false;
    for (int i = 0; i < k; ++i) {
      bool eq = out[i].nst == p.nst;
      for (int r = 0; eq && r < p.nst; ++r) eq = out[i].R[r] == p.R[r];
      dup = dup || eq;
    }
    if (!dup) out[k++] = p;
  }
  return k;
}

void default_plans(const fx_cell* cell, PlanSet* ps) {
  for (int a = 0; a < 3; ++a) make_axis_plan(cell->n[a], &ps->ax[a]);
}

bool same_plans(const PlanSet& a, const PlanSet& b) {
  for (int x = 0; x < 3; ++x) {
    if (a.ax[x].n != b.ax[x].n || a.ax[x].nst != b.ax[x].nst) return false;
    for (int i = 0; i < a.ax[x].nst; ++i)
      if (a.ax[x].R[i] != b.ax[x].R[i]) return false;
  }
  return true;
}

void plan_positions(const AxisPlan& p, std::vector<int>* freq_of_pos) {
  positions_rec(p.R, p.nst, p.n, *freq_of_pos);
}

fx_status check_cell(const fx_cell* cell) {
  if (!cell) FX_FAIL(FX_ERR_INVALID, "cell is NULL");
  for (int a = 0; a < 3; ++a) {
    if (!supported_edge(cell->n[a]))
      FX_FAIL(FX_ERR_UNSUPPORTED, "grid edge n[%d] = %d is not 2^a 3^b in [2, 96]", a, cell->n[a]);
    if (!(cell->len[a] > 0.0) || !std::isfinite(cell->len[a]))
      FX_FAIL(FX_ERR_INVALID, "cell length len[%d] = %g must be positive and finite", a, cell->len[a]);
  }
  return FX_OK;
}

fx_status check_kernel(const fx_kernel* k, bool allow_internal) {
  if (!k) FX_FAIL(FX_ERR_INVALID, "kernel is NULL");
  if (k->kind != FX_COULOMB && k->kind != FX_HSE && !(allow_internal && k->kind == kKineticKind))
    FX_FAIL(FX_ERR_UNSUPPORTED, "unknown kernel kind %d", k->kind);
  if (k->kind == FX_HSE && !(k->omega > 0.0)) FX_FAIL(FX_ERR_INVALID, "HSE omega = %g must be positive", k->omega);
  if (!std::isfinite(k->scale)) FX_FAIL(FX_ERR_INVALID, "kernel scale is not finite");
  return FX_OK;
}

// ---- constant tables, built on the host in FP64 ---------------------------
static double kernel_value(int kind, double omega, double g2) {
  const double pi = 3.14159265358979323846264338327950288;
  if (g2 == 0.0) return kind == FX_COULOMB ? 0.0 : pi / (omega * omega);
  double v = 4.0 * pi / g2;
  if (kind == FX_HSE) v *= -std::expm1(-g2 / (4.0 * omega * omega));
  return v;
}

template <typename T>
static fx_status upload(fx_ctx* ctx, const std::vector<T>& h, void** d, size_t* acc) {
  size_t b = h.size() * sizeof(T);
  FX_TRY(ctx_alloc(ctx, b, d));
  FX_HIP(hipMemcpy(*d, h.data(), b, hipMemcpyHostToDevice));
  *acc += b;
  return FX_OK;
}

void host_tables(const fx_cell* cell, const fx_kernel* kern, HostTables* h, const PlanSet* plans) {
  const double pi = 3.14159265358979323846264338327950288;
  for (int a = 0; a < 3; ++a) {
    const int n = cell->n[a];
    AxisPlan p;
    if (plans)
      p = plans->ax[a];
    else
      make_axis_plan(n, &p);
    h->plan[a] = p;
    std::vector<int> fp;
    plan_positions(p, &fp);
    h->fold[a].resize(n);
    for (int i = 0; i < n; ++i) h->fold[a][i] = fp[i] <= n - fp[i] ? fp[i] : n - fp[i];
    h->tw[a].resize(n);
    for (int i = 0; i < n; ++i) h->tw[a][i] = {std::cos(2 * pi * i / n), -std::sin(2 * pi * i / n)};
  }
  const int hx = cell->n[0] / 2 + 1, hy = cell->n[1] / 2 + 1, hz = cell->n[2] / 2 + 1;
  const double vol = cell->len[0] * cell->len[1] * cell->len[2];
  const double nr = (double)cell->n[0] * cell->n[1] * cell->n[2];
  h->kfold.assign((size_t)hx * hy * hz, 0.0);
  for (int z = 0; z < hz; ++z)
    for (int y = 0; y < hy; ++y)
      for (int x = 0; x < hx; ++x) {
        const double gx = 2 * pi * x / cell->len[0], gy = 2 * pi * y / cell->len[1], gz = 2 * pi * z / cell->len[2];
        const double g2 = gx * gx + gy * gy + gz * gz;
        h->kfold[((size_t)z * hy + y) * hx + x] = kern->kind == kKineticKind
                                                      ? 0.5 * g2 / nr
                                                      : -kern->scale / vol * kernel_value(kern->kind, kern->omega, g2);
      }
}

fx_status grid_tables(fx_ctx* ctx, const fx_cell* cell, const fx_kernel* kern, int prec, const PlanSet* plans,
                      const GridTables** out) {
  PlanSet ps;
  if (plans)
    ps = *plans;
  else
    default_plans(cell, &ps);
  TableKey key;
  for (int a = 0; a < 3; ++a) {
    key.n[a] = cell->n[a];
    key.len[a] = cell->len[a];
    for (int i = 0; i < 4; ++i) key.radix[a][i] = i < ps.ax[a].nst ? ps.ax[a].R[i] : 0;
  }
  key.kind = kern->kind;
  key.omega = kern->kind == FX_HSE ? kern->omega : 0.0;
  key.scale = kern->scale;
  key.prec = prec;
  auto it = ctx->tables.find(key);
  if (it != ctx->tables.end()) {
    *out = &it->second;
    return FX_OK;
  }
  if (ctx->capturing)
    FX_FAIL(FX_ERR_INVALID,
            "grid tables for this cell and kernel are not on the device yet and the stream is being captured; "
            "run the same call once outside capture first");
  HostTables h;
  host_tables(cell, kern, &h, &ps);
  GridTables t;
  for (int a = 0; a < 3; ++a) {
    if (prec == 0) {
      FX_TRY(upload(ctx, h.tw[a], &t.tw[a], &t.bytes));
    } else {
      std::vector<cpx<float>> tw(h.tw[a].size());
      for (size_t i = 0; i < tw.size(); ++i) tw[i] = {(float)h.tw[a][i].x, (float)h.tw[a][i].y};
      FX_TRY(upload(ctx, tw, &t.tw[a], &t.bytes));
    }
    void* fd = nullptr;
    FX_TRY(upload(ctx, h.fold[a], &fd, &t.bytes));
    t.fold[a] = (int*)fd;
  }
  if (prec == 0) {
    FX_TRY(upload(ctx, h.kfold, &t.kfold, &t.bytes));
  } else {
    std::vector<float> k32(h.kfold.begin(), h.kfold.end());
    FX_TRY(upload(ctx, k32, &t.kfold, &t.bytes));
  }
  auto ins = ctx->tables.emplace(key, t);
  *out = &ins.first->second;
  return FX_OK;
}

}  // namespace fx

using namespace fx;

extern "C" {

const char* fx_last_error(void) { return g_err; }

fx_status fx_debug_fail_alloc(int64_t k) {
  clear_error();
  if (k < 0) FX_FAIL(FX_ERR_INVALID, "k = %lld must be >= 0", (long long)k);
  const long base = __atomic_load_n(&g_alloc_count, __ATOMIC_SEQ_CST);
  __atomic_store_n(&g_fail_at, k ? base + (long)k : 0L, __ATOMIC_SEQ_CST);
  return FX_OK;
}

const char* fx_version(void) { return "libfock 0.1 (gfx950)"; }

fx_status fx_init(int device, size_t hbm_budget_bytes, fx_ctx** ctx) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  *ctx = nullptr;
  int ndev = 0;
  FX_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) FX_FAIL(FX_ERR_INVALID, "device %d out of range (%d devices)", device, ndev);
  FX_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  FX_HIP(hipGetDeviceProperties(&prop, device));
  size_t free_b = 0, total_b = 0;
  FX_HIP(hipMemGetInfo(&free_b, &total_b));
  fx_ctx* c = new (std::nothrow) fx_ctx();
  if (!c) FX_FAIL(FX_ERR_OOM, "host allocation of the context failed");
  c->device = device;
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)free_b);
  c->n_cu = prop.multiProcessorCount;
  hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete c;
    FX_FAIL(FX_ERR_DEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
  }
  // device address of this device's copy of the allocation-free entry
  // point's scratch region (looked up once per device)
  const fx_status ss = scratch_setup(device);
  if (ss != FX_OK) {
    (void)hipStreamDestroy(c->stream);
    delete c;
    return ss;
  }
  // FX_TUNE_CACHE: tuned launch configurations kept in a file (a missing
  // file is not an error; an unreadable one is)
  if (const char* e = getenv("FX_TUNE_CACHE")) {
    if (*e) {
      if (FILE* f = fopen(e, "r")) {
        fclose(f);
        const fx_status ls = load_configs_impl(c, e, nullptr);
        if (ls != FX_OK) {
          (void)hipStreamDestroy(c->stream);
          delete c;
          return ls;
        }
      }
    }
  }
  *ctx = c;
  return FX_OK;
}

fx_status fx_finalize(fx_ctx* ctx) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  FX_HIP(hipSetDevice(ctx->device));
  FX_HIP(hipDeviceSynchronize());
  // servers and ACE handles still alive give their device memory back here;
  // they stay valid for fx_serve_destroy / fx_ace_free only
  serve_detach_all(ctx);
  ace_detach_all(ctx);
  graph_cache_clear(ctx);
  ws_release(ctx, &ctx->ws);
  for (auto& kv : ctx->tables) {
    GridTables& t = kv.second;
    for (int a = 0; a < 3; ++a) {
      (void)hipFree(t.tw[a]);
      (void)hipFree(t.fold[a]);
    }
    (void)hipFree(t.kfold);
  }
  ctx->tables.clear();
  (void)prof_drain(ctx);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  ctx->ev_pool.clear();
  (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return FX_OK;
}

fx_status fx_graph_cache(fx_ctx* ctx, int32_t max_entries) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  if (max_entries < 0 || max_entries > 4096) FX_FAIL(FX_ERR_INVALID, "max_entries = %d not in [0, 4096]", max_entries);
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  FX_HIP(hipSetDevice(ctx->device));
  FX_HIP(hipDeviceSynchronize());
  graph_cache_clear(ctx);
  ctx->graph_max = max_entries;
  ctx->graph_hits = ctx->graph_misses = 0;
  return FX_OK;
}

fx_status fx_graph_cache_stats(fx_ctx* ctx, int64_t* hits, int64_t* misses, int32_t* entries) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (hits) *hits = ctx->graph_hits;
  if (misses) *misses = ctx->graph_misses;
  if (entries) *entries = (int32_t)ctx->graphs.size();
  return FX_OK;
}

fx_status fx_prof_enable(fx_ctx* ctx, int on) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  FX_TRY(prof_drain(ctx));
  for (int i = 0; i < FX_K_COUNT; ++i) {
    ctx->prof_launches[i] = 0;
    ctx->prof_ms[i] = 0.0;
    ctx->prof_work[i] = 0.0;
  }
  ctx->prof = on != 0;
  return FX_OK;
}

fx_status fx_prof_read(fx_ctx* ctx, int id, int64_t* launches, double* total_ms, double* work) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  if (id < 0 || id >= FX_K_COUNT) FX_FAIL(FX_ERR_INVALID, "kernel id %d out of range", id);
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  FX_TRY(prof_drain(ctx));
  if (launches) *launches = ctx->prof_launches[id];
  if (total_ms) *total_ms = ctx->prof_ms[id];
  if (work) *work = ctx->prof_work[id];
  return FX_OK;
}

fx_status fx_memory(const fx_ctx* ctx, size_t* in_use, size_t* peak) {
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  if (in_use) *in_use = ctx->in_use;
  if (peak) *peak = ctx->peak;
  return FX_OK;
}

}  // extern "C"
