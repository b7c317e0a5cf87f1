// fx_serve: continuous batching of V_X and K_ACE requests over orbitals kept
// resident on the device (the host scheduling is in serve_sched.hpp).
//
// One host loop replays the arrivals.  Waiting requests of one operation are
// merged into one launch (their target orbitals gathered into one block) up
// to max_batch_pairs pairs: ACE requests of one trajectory; V_X requests of
// up to eight trajectories that share the grid, kernel, orbital count and
// precision (on the specialised grids), each target paired with its own
// trajectory's orbitals.  A merged batch runs on a free slot, each slot
// owning a stream and a workspace, so batches that are in flight overlap on
// the device.  A slot's completion event stamps the latency of every request
// in it.  Admission keeps resident orbitals, ACE factors and slot workspaces
// inside the HBM budget: a batch whose workspace does not fit waits for a
// slot to drain, and is refused (FX_ERR_OOM) only if it cannot fit with every
// slot idle; an arrival that finds max_queue requests waiting is refused
// (FX_ERR_BUSY); fx_serve_cancel drops a request that has not started.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <set>
#include <cmath>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "ace.hpp"
#include "serve_sched.hpp"
#include "vx.hpp"

using namespace fx;

namespace {

struct Traj {
  fx_cell cell;
  fx_kernel kern;
  int n = 0;
  int64_t nr = 0;
  fx_dtype dtype = FX_C64;
  fx_prec vx_prec = FX_PREC_FP32_ACC64, ace_prec = FX_PREC_ACE_FP32R;
  void* psi = nullptr;  // owned, ld nr
  size_t psi_bytes = 0;
  fx_ace* ace = nullptr;
  int vx_class = 0;  // V_X requests of trajectories with the same class may share a launch
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  Workspace ws;
};

// gather columns [first, first+count) of each request's trajectory into a
// contiguous block, or scatter a contiguous block back to request outputs
__global__ void k_copy_cols(const char* __restrict__ src, int64_t ld_src_bytes, char* __restrict__ dst,
                            int64_t ld_dst_bytes, int64_t col_bytes, int ncols) {
  const int c = blockIdx.y;
  if (c >= ncols) return;
  const uint4* s = reinterpret_cast<const uint4*>(src + c * ld_src_bytes);
  uint4* d = reinterpret_cast<uint4*>(dst + c * ld_dst_bytes);
  const int64_t nv = col_bytes / 16;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

fx_status copy_cols(const void* src, int64_t ld_src_bytes, void* dst, int64_t ld_dst_bytes, int64_t col_bytes,
                    int ncols, hipStream_t st) {
  if (col_bytes % 16 || ld_src_bytes % 16 || ld_dst_bytes % 16 || ((uintptr_t)src % 16) || ((uintptr_t)dst % 16)) {
    for (int c = 0; c < ncols; ++c)
      FX_HIP(hipMemcpyAsync((char*)dst + c * ld_dst_bytes, (const char*)src + c * ld_src_bytes, col_bytes,
                            hipMemcpyDeviceToDevice, st));
    return FX_OK;
  }
  const int64_t nv = col_bytes / 16;
  dim3 grid((unsigned)std::min<int64_t>((nv + 255) / 256, 1024), (unsigned)ncols);
  hipLaunchKernelGGL(k_copy_cols, grid, dim3(256), 0, st, (const char*)src, ld_src_bytes, (char*)dst, ld_dst_bytes,
                     col_bytes, ncols);
  FX_LAUNCH_CHECK();
  return FX_OK;
}

}  // namespace

struct fx_server {
  fx_ctx* ctx = nullptr;
  fx_serve_cfg cfg;
  size_t saved_budget = 0;  // the context budget before the server capped it
  std::map<int, Traj> trajs;
  std::vector<Slot> slots;
  // requests of the running (or next) fx_serve call cancelled by
  // fx_serve_cancel, which takes only this lock (fx_serve holds the context's)
  std::mutex cancel_mu;
  std::set<int> cancelled;
  std::atomic<int> n_cancelled{0};
};

static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Device resources of a server: resident orbitals and ACE factors of its
// trajectories, slot workspaces, events and streams; the context budget it
// capped is restored.  The device has been synchronised by the caller.
static void serve_release(fx_server* srv) {
  fx_ctx* ctx = srv->ctx;
  for (auto& kv : srv->trajs) {
    Traj& t = kv.second;
    if (t.ace) {
      for (auto& b : t.ace->owned) ctx_free(ctx, b.first, b.second);
      ws_release(ctx, &t.ace->ws);
      delete t.ace;
      t.ace = nullptr;
    }
    ctx_free(ctx, t.psi, t.psi_bytes);
  }
  srv->trajs.clear();
  std::vector<hipStream_t> streams;
  for (auto& sl : srv->slots) {
    ws_release(ctx, &sl.ws);
    if (sl.done) (void)hipEventDestroy(sl.done);
    sl.done = nullptr;
    if (std::find(streams.begin(), streams.end(), sl.st) == streams.end()) streams.push_back(sl.st);
  }
  srv->slots.clear();
  for (auto st : streams) (void)hipStreamDestroy(st);
  ctx->budget = srv->saved_budget;
}

namespace fx {
void serve_detach_all(fx_ctx* ctx) {
  for (fx_server* srv : ctx->servers) {
    serve_release(srv);
    srv->ctx = nullptr;
  }
  ctx->servers.clear();
}
}  // namespace fx

// The device side of the serving loop: slot streams, events and workspaces.
namespace {
struct HipExec final : ServeExecutor {
  fx_server* srv;
  fx_ctx* ctx;
  const fx_request* reqs;
  std::vector<int> stream_id;
  HipExec(fx_server* s, const fx_request* r) : srv(s), ctx(s->ctx), reqs(r) {
    const int ns = (int)srv->slots.size();
    stream_id.resize(ns);
    for (int i = 0; i < ns; ++i) {
      stream_id[i] = i;
      for (int j = 0; j < i; ++j)
        if (srv->slots[j].st == srv->slots[i].st) {
          stream_id[i] = stream_id[j];
          break;
        }
    }
  }
  int n_slots() const override { return (int)srv->slots.size(); }
  int stream_of(int slot) const override { return stream_id[slot]; }
  int orbitals(int traj) const override { return srv->trajs.at(traj).n; }
  int merge_class(int traj, int op) const override { return op == 0 ? srv->trajs.at(traj).vx_class : traj; }
  bool cancelled(int req) const override {
    if (srv->n_cancelled.load(std::memory_order_acquire) == 0) return false;
    std::lock_guard<std::mutex> lk(srv->cancel_mu);
    return srv->cancelled.count(req) != 0;
  }
  fx_status launch(int slot, const std::vector<int>& batch_in) override {
    Slot& sl = srv->slots[slot];
    // the batch's requests grouped by trajectory (first appearance first), each
    // trajectory's requests in batch order: the targets of one trajectory are
    // contiguous in the gathered block
    std::vector<int> trajs_in, batch;
    for (int i : batch_in)
      if (std::find(trajs_in.begin(), trajs_in.end(), reqs[i].traj) == trajs_in.end()) trajs_in.push_back(reqs[i].traj);
    for (int tj : trajs_in)
      for (int i : batch_in)
        if (reqs[i].traj == tj) batch.push_back(i);
    const fx_request& r0 = reqs[batch[0]];
    Traj& t = srv->trajs[r0.traj];
    const size_t esz = dtype_size(t.dtype);
    const int64_t cb = (int64_t)esz * t.nr;
    int total = 0;
    for (int i : batch) total += reqs[i].count;
    const void* phi = nullptr;
    void* out = nullptr;
    const bool single = batch.size() == 1;
    TrajSegs segs;
    if (trajs_in.size() > 1) {
      if ((int)trajs_in.size() > kMaxTrajSegs) FX_FAIL(FX_ERR_INVALID, "batch over %d trajectories", kMaxTrajSegs);
      int off = 0;
      for (int i : batch) {
        if (segs.n == 0 || srv->trajs[reqs[i].traj].psi != segs.psi[segs.n - 1]) {
          segs.start[segs.n] = off;
          segs.psi[segs.n] = srv->trajs[reqs[i].traj].psi;
          ++segs.n;
        }
        off += reqs[i].count;
      }
      segs.start[segs.n] = off;
    }
    if (single) {
      phi = (const char*)t.psi + (int64_t)r0.first * cb;
      out = r0.out;
    } else {
      void *g = nullptr, *o = nullptr;
      FX_TRY(ws_get(ctx, &sl.ws, "srv_gather", (size_t)cb * total, &g));
      FX_TRY(ws_get(ctx, &sl.ws, "srv_out", (size_t)cb * total, &o));
      int off = 0;
      for (int i : batch) {
        const Traj& ti = srv->trajs[reqs[i].traj];
        FX_TRY(copy_cols((const char*)ti.psi + (int64_t)reqs[i].first * cb, cb, (char*)g + (int64_t)off * cb, cb, cb,
                         reqs[i].count, sl.st));
        off += reqs[i].count;
      }
      phi = g;
      out = o;
    }
    const int64_t ld_out = single ? r0.ld_out : t.nr;
    if (r0.op == 0) {
      VxArgs va;
      va.segs = segs;
      va.cell = &t.cell;
      va.kern = &t.kern;
      va.psi = t.psi;
      va.n_psi = t.n;
      va.ld_psi = t.nr;
      va.phi = phi;
      va.n_phi = total;
      va.ld_phi = t.nr;
      va.out = out;
      va.ld_out = ld_out;
      va.in_dtype = t.dtype;
      va.out_dtype = t.dtype;
      va.prec = t.vx_prec;
      va.work_cap = (size_t)(srv->cfg.vx_work_mb > 0 ? srv->cfg.vx_work_mb : 1024) << 20;
      FX_TRY(vx_apply(ctx, &sl.ws, va, sl.st, nullptr));
    } else {
      FX_TRY(ace_apply_impl(ctx, &sl.ws, t.ace, phi, total, t.nr, out, ld_out, t.dtype, t.dtype, t.ace_prec, sl.st));
    }
    if (!single) {
      int off = 0;
      for (int i : batch) {
        FX_TRY(copy_cols((char*)out + (int64_t)off * cb, cb, reqs[i].out, reqs[i].ld_out * (int64_t)esz, cb,
                         reqs[i].count, sl.st));
        off += reqs[i].count;
      }
    }
    FX_HIP(hipEventRecord(sl.done, sl.st));
    return FX_OK;
  }
  bool release_idle(const std::vector<char>& idle) override {
    for (size_t i = 0; i < srv->slots.size(); ++i) {
      if (!idle[i]) continue;
      // a failed launch may have queued copies on this slot's stream
      if (hipStreamSynchronize(srv->slots[i].st) != hipSuccess) return false;
      ws_release(ctx, &srv->slots[i].ws);
    }
    clear_error();
    return true;
  }
  int poll(int slot) override {
    const hipError_t q = hipEventQuery(srv->slots[slot].done);
    if (q == hipSuccess) return 1;
    if (q == hipErrorNotReady) return 0;
    set_error("device error while serving: %s", hipGetErrorString(q));
    return -1;
  }
  double now() override { return now_s(); }
  void idle_wait(double seconds) override { std::this_thread::sleep_for(std::chrono::duration<double>(seconds)); }
  size_t mem_in_use() const override { return ctx->in_use; }
};
}  // namespace

extern "C" {

fx_status fx_serve_create(fx_ctx* ctx, const fx_serve_cfg* cfg, fx_server** srv) {
  clear_error();
  if (!ctx || !cfg || !srv) FX_FAIL(FX_ERR_INVALID, "NULL argument");
  if (cfg->max_slots <= 0 || cfg->max_slots > 64) FX_FAIL(FX_ERR_INVALID, "max_slots = %d not in [1, 64]", cfg->max_slots);
  if (cfg->n_streams <= 0 || cfg->n_streams > cfg->max_slots)
    FX_FAIL(FX_ERR_INVALID, "n_streams = %d not in [1, max_slots]", cfg->n_streams);
  if (cfg->max_batch_pairs <= 0) FX_FAIL(FX_ERR_INVALID, "max_batch_pairs must be positive");
  if (cfg->max_queue < 0) FX_FAIL(FX_ERR_INVALID, "max_queue = %d must be >= 0", cfg->max_queue);
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  FX_HIP(hipSetDevice(ctx->device));
  fx_server* s = new fx_server();
  s->ctx = ctx;
  s->cfg = *cfg;
  s->saved_budget = ctx->budget;
  if (cfg->hbm_budget_bytes && cfg->hbm_budget_bytes < ctx->budget) ctx->budget = cfg->hbm_budget_bytes;
  s->slots.resize(cfg->max_slots);
  std::vector<hipStream_t> streams;
  auto undo = [&]() {
    for (auto& sl : s->slots)
      if (sl.done) (void)hipEventDestroy(sl.done);
    for (auto st : streams) (void)hipStreamDestroy(st);
    ctx->budget = s->saved_budget;
    delete s;
  };
  for (int i = 0; i < cfg->n_streams; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      undo();
      FX_FAIL(FX_ERR_DEVICE, "stream creation failed");
    }
    streams.push_back(st);
  }
  for (int i = 0; i < cfg->max_slots; ++i) {
    s->slots[i].st = streams[i % cfg->n_streams];
    if (hipEventCreateWithFlags(&s->slots[i].done, hipEventDisableTiming) != hipSuccess) {
      undo();
      FX_FAIL(FX_ERR_DEVICE, "event creation failed");
    }
  }
  ctx->servers.insert(s);
  *srv = s;
  return FX_OK;
}

fx_status fx_serve_register(fx_server* srv, int32_t traj, const fx_cell* cell, const fx_kernel* kernel,
                            const void* psi, int32_t n, int64_t ld, fx_dtype dtype, fx_prec vx_prec,
                            fx_prec ace_prec) {
  clear_error();
  if (!srv) FX_FAIL(FX_ERR_INVALID, "srv is NULL");
  if (!srv->ctx) FX_FAIL(FX_ERR_INVALID, "the context of this server was finalized");
  fx_ctx* ctx = srv->ctx;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->capturing = false;  // the serving loop runs on its own, uncaptured streams
  FX_HIP(hipSetDevice(ctx->device));
  FX_TRY(check_cell(cell));
  FX_TRY(check_kernel(kernel));
  if (srv->trajs.count(traj)) FX_FAIL(FX_ERR_INVALID, "trajectory %d already registered", traj);
  if (!psi || n <= 0) FX_FAIL(FX_ERR_INVALID, "psi NULL or n <= 0");
  const int64_t nr = (int64_t)cell->n[0] * cell->n[1] * cell->n[2];
  if (ld < nr) FX_FAIL(FX_ERR_INVALID, "ld < N_r");
  if (dtype != FX_C128 && dtype != FX_C64) FX_FAIL(FX_ERR_UNSUPPORTED, "unknown dtype");
  Traj t;
  t.cell = *cell;
  t.kern = *kernel;
  t.n = n;
  t.nr = nr;
  t.dtype = dtype;
  t.vx_prec = vx_prec;
  t.ace_prec = ace_prec;
  t.psi_bytes = dtype_size(dtype) * (size_t)nr * n;
  FX_TRY(ctx_alloc(ctx, t.psi_bytes, &t.psi));
  const int64_t cb = (int64_t)dtype_size(dtype) * nr;
  fx_status s = copy_cols(psi, ld * (int64_t)dtype_size(dtype), t.psi, cb, cb, n, nullptr);
  if (s == FX_OK && srv->cfg.autotune) {
    // configurations for this grid's requests (blocks of targets against all
    // n orbitals) and for the ACE build (phi == psi), unless already held
    const int nt = std::min(n, srv->cfg.autotune_targets > 0 ? srv->cfg.autotune_targets : 8);
    if (!ctx->vx_tuning.count(vx_tune_key(cell, vx_prec, false)))
      s = vx_autotune_impl(ctx, cell, kernel, n, nt, false, vx_prec, nullptr, nullptr, nullptr);
    if (s == FX_OK && !ctx->vx_tuning.count(vx_tune_key(cell, vx_prec, true)))
      s = vx_autotune_impl(ctx, cell, kernel, n, n, true, vx_prec, nullptr, nullptr, nullptr);
  }
  if (s == FX_OK) {
    s = ace_build_impl(ctx, &ctx->ws, cell, kernel, t.psi, n, nr, dtype, vx_prec, ace_prec, nullptr, &t.ace,
                       nullptr);
  }
  if (s != FX_OK) {
    ctx_free(ctx, t.psi, t.psi_bytes);
    return s;
  }
  // the build's scratch is not needed while serving
  FX_HIP(hipDeviceSynchronize());
  ws_release(ctx, &ctx->ws);
  // V_X requests may share launches with those of trajectories that pair the
  // same way: same grid (specialised kernels), cell, kernel, orbital count,
  // dtype and precision, with no conversion of the orbitals
  t.vx_class = traj;
  const bool conv = (dtype == FX_C128) != (vx_prec == FX_PREC_FP64);
  if (ct_supported(cell) && !conv) {
    for (const auto& kv : srv->trajs) {
      const Traj& u = kv.second;
      bool same = u.n == t.n && u.dtype == t.dtype && u.vx_prec == t.vx_prec && u.kern.kind == t.kern.kind &&
                  u.kern.scale == t.kern.scale && (t.kern.kind != FX_HSE || u.kern.omega == t.kern.omega);
      for (int a = 0; a < 3; ++a) same = same && u.cell.n[a] == t.cell.n[a] && u.cell.len[a] == t.cell.len[a];
      if (same && ct_supported(&u.cell)) {
        t.vx_class = u.vx_class;
        break;
      }
    }
  }
  srv->trajs[traj] = t;
  return FX_OK;
}

fx_status fx_serve(fx_server* srv, const fx_request* reqs, int32_t n_reqs, fx_status* per_status,
                   double* per_lat_ms, fx_serve_report* report) {
  clear_error();
  if (!srv) FX_FAIL(FX_ERR_INVALID, "srv is NULL");
  if (n_reqs < 0 || (n_reqs > 0 && !reqs)) FX_FAIL(FX_ERR_INVALID, "bad request array");
  if (!srv->ctx) FX_FAIL(FX_ERR_INVALID, "the context of this server was finalized");
  fx_ctx* ctx = srv->ctx;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->capturing = false;  // the serving loop runs on its own, uncaptured streams
  FX_HIP(hipSetDevice(ctx->device));
  const int nq = n_reqs;
  std::vector<char> valid(nq, 1);
  for (int i = 0; i < nq; ++i) {
    const fx_request& r = reqs[i];
    auto it = srv->trajs.find(r.traj);
    if (it == srv->trajs.end() || (r.op != 0 && r.op != 1) || r.count <= 0 || r.first < 0 ||
        r.first + r.count > it->second.n || !r.out || r.ld_out < it->second.nr)
      valid[i] = 0;
  }
  HipExec ex(srv, reqs);
  ServeOutcome o;
  serve_schedule(ex, reqs, nq, valid, srv->cfg.max_batch_pairs, &o, srv->cfg.max_queue);
  {
    // cancellations refer to this call's requests only
    std::lock_guard<std::mutex> lk(srv->cancel_mu);
    srv->cancelled.clear();
    srv->n_cancelled.store(0, std::memory_order_release);
  }
  if (o.fatal != FX_OK) {
    (void)hipDeviceSynchronize();
    return o.fatal;
  }
  std::vector<double> ok;
  for (int i = 0; i < nq; ++i) {
    if (per_status) per_status[i] = o.status[i];
    if (per_lat_ms) per_lat_ms[i] = o.lat_ms[i];
    if (o.status[i] == FX_OK) ok.push_back(o.lat_ms[i]);
  }
  if (report) {
    fx_serve_report& R = *report;
    R.p50_ms = serve_percentile(ok, 0.50);
    R.p99_ms = serve_percentile(ok, 0.99);
    double sum = 0, mx = 0;
    for (double v : ok) {
      sum += v;
      mx = std::max(mx, v);
    }
    R.mean_ms = ok.empty() ? 0.0 : sum / ok.size();
    R.max_ms = mx;
    R.wall_s = o.wall;
    R.req_per_s = o.wall > 0 ? ok.size() / o.wall : 0.0;
    R.pairs_per_s = o.wall > 0 ? o.pairs_done / o.wall : 0.0;
    R.busy_frac = o.wall > 0 ? o.busy_time / o.wall : 0.0;
    R.n_done = (int64_t)ok.size();
    R.n_rejected = o.rejected;
    R.n_batches = o.batches;
    R.hbm_peak_bytes = o.hbm_peak;
    R.n_cancelled = o.cancelled;
  }
  return FX_OK;
}

fx_status fx_serve_cancel(fx_server* srv, int32_t request) {
  clear_error();
  if (!srv) FX_FAIL(FX_ERR_INVALID, "srv is NULL");
  if (request < 0) FX_FAIL(FX_ERR_INVALID, "request index %d is negative", request);
  std::lock_guard<std::mutex> lk(srv->cancel_mu);
  srv->cancelled.insert(request);
  srv->n_cancelled.fetch_add(1, std::memory_order_release);
  return FX_OK;
}

fx_status fx_serve_destroy(fx_server* srv) {
  clear_error();
  if (!srv) FX_FAIL(FX_ERR_INVALID, "srv is NULL");
  // a server whose context was finalized holds no device resources any more
  if (fx_ctx* ctx = srv->ctx) {
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    FX_HIP(hipSetDevice(ctx->device));
    FX_HIP(hipDeviceSynchronize());
    serve_release(srv);
    ctx->servers.erase(srv);
  }
  delete srv;
  return FX_OK;
}

}  // extern "C"
