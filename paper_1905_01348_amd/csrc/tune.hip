// Launch-configuration autotuner of the V_X pair path and the per-context
// configuration store (fx_vx_autotune, fx_vx_set_config, fx_vx_get_config).
//
// Candidates are timed on synthetic orbitals the tuner writes itself (the
// values do not matter for speed), on a probe of up to two full batches of
// pairs, with HIP events on the caller's stream.  The search is coordinate
// descent from the automatic configuration: the kernel family, then the
// family's own knobs (specialised: plane-forward prefetch form, z-pass tile;
// generic: the radix schedule of each axis, z-pass tile and threads), then
// the batch volume.  A candidate replaces the incumbent only when it is at
// least 2% faster, so timing noise does not flip settled choices.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "common.hpp"
#include "vx.hpp"

namespace fx {

// Deterministic filler: a splitmix-style hash of the element index, mapped to
// [-1, 1) and scaled so a column has norm ~1 (sizes like real orbitals).
template <typename T>
__global__ void k_fill_probe(cpx<T>* p, int64_t n, uint64_t seed, T scale) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + seed;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const T re = (T)((double)(z >> 40) * (1.0 / 8388608.0) - 1.0);
    const T im = (T)((double)((z >> 16) & 0xFFFFFF) * (1.0 / 8388608.0) - 1.0);
    p[i] = cpx<T>{re * scale, im * scale};
  }
}

static fx_status check_config(const fx_cell* cell, const fx_vx_config& c) {
  if (c.kernels < 0 || c.kernels > 2) FX_FAIL(FX_ERR_INVALID, "kernels = %d not in {0, 1, 2}", c.kernels);
  if (c.work_mb < 0 || c.work_mb > (1 << 20)) FX_FAIL(FX_ERR_INVALID, "work_mb = %d out of range", c.work_mb);
  if (c.a_prefetch < -1 || c.a_prefetch > 1) FX_FAIL(FX_ERR_INVALID, "a_prefetch = %d not in {-1, 0, 1}", c.a_prefetch);
  if (c.b_variant < 0 || c.b_variant > 4) FX_FAIL(FX_ERR_INVALID, "b_variant = %d not in {0, ..., 4}", c.b_variant);
  if (c.c_variant < 0 || c.c_variant > 5) FX_FAIL(FX_ERR_INVALID, "c_variant = %d not in {0, ..., 5}", c.c_variant);
  if (c.a_variant < 0 || c.a_variant > 3) FX_FAIL(FX_ERR_INVALID, "a_variant = %d not in {0, ..., 3}", c.a_variant);
  if (c.nt_hint < -1 || c.nt_hint > 1) FX_FAIL(FX_ERR_INVALID, "nt_hint = %d not in {-1, 0, 1}", c.nt_hint);
  if (c.c_split != 0 && c.c_split != 1 && c.c_split != 2 && c.c_split != 4 && c.c_split != 8)
    FX_FAIL(FX_ERR_INVALID, "c_split = %d not in {0, 1, 2, 4, 8}", c.c_split);
  if (c.b_xtile < 0 || c.b_xtile > cell->n[0]) FX_FAIL(FX_ERR_INVALID, "b_xtile = %d not in [0, n_x]", c.b_xtile);
  if (c.b_threads != 0 && (c.b_threads < 64 || c.b_threads > 256 || c.b_threads % 64))
    FX_FAIL(FX_ERR_INVALID, "b_threads = %d must be 0 or a multiple of 64 in [64, 256]", c.b_threads);
  PlanSet ps;
  bool any = false;
  if (!plans_from_radix(cell, c.radix, &ps, &any))
    FX_FAIL(FX_ERR_INVALID, "a radix row is not a schedule of its edge (radices from {2,3,4,6,8,9,12}, product n)");
  if (c.kernels == 1) {
    if (!ct_supported(cell)) FX_FAIL(FX_ERR_INVALID, "no specialised kernels for this grid");
    PlanSet d;
    default_plans(cell, &d);
    if (any && !same_plans(ps, d)) FX_FAIL(FX_ERR_INVALID, "specialised kernels run the default radix schedule only");
  }
  return FX_OK;
}

static bool is_vx_prec(fx_prec p) { return p == FX_PREC_FP64 || p == FX_PREC_FP32 || p == FX_PREC_FP32_ACC64; }

// ---- configuration file -------------------------------------------------------
// One configuration per line:
//   fxcfg <device> <nx> <ny> <nz> <prec> <phi_is_psi> <kernels> <work_mb> <a_prefetch>
//         <b_variant> <c_variant> <a_variant> <nt_hint> <b_xtile> <b_threads> <12 radix entries>
//         [<c_split>]
// (lines without c_split, written before it existed, read it as 0)
// where <device> is the architecture and CU count ("gfx950/256"): a tuned
// launch shape holds for that kind of device only.  Lines starting with '#'
// are comments; lines for other devices are kept when the file is rewritten.
static std::string device_tag(int device) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
  std::string arch(p.gcnArchName);
  const size_t c = arch.find(':');
  if (c != std::string::npos) arch.resize(c);
  return arch + "/" + std::to_string(p.multiProcessorCount);
}

static std::string config_line(const std::string& tag, const std::array<int, 5>& k, const fx_vx_config& c) {
  std::string s = "fxcfg " + tag;
  for (int v : k) s += " " + std::to_string(v);
  const int f[9] = {c.kernels, c.work_mb, c.a_prefetch, c.b_variant, c.c_variant, c.a_variant, c.nt_hint, c.b_xtile,
                    c.b_threads};
  for (int v : f) s += " " + std::to_string(v);
  for (int a = 0; a < 3; ++a)
    for (int r = 0; r < 4; ++r) s += " " + std::to_string(c.radix[a][r]);
  s += " " + std::to_string(c.c_split);
  return s;
}

// Parse one line; false if it is not a configuration line.
static bool parse_config_line(const char* line, std::string* tag, std::array<int, 5>* k, fx_vx_config* c) {
  char tg[128];
  int v[5 + 9 + 12 + 1];
  int used = 0;
  if (std::sscanf(line, "fxcfg %127s%n", tg, &used) != 1) return false;
  const char* p = line + used;
  for (int i = 0; i < 26; ++i) {
    int adv = 0;
    if (std::sscanf(p, "%d%n", &v[i], &adv) != 1) return false;
    p += adv;
  }
  int adv = 0;
  if (std::sscanf(p, "%d%n", &v[26], &adv) != 1) v[26] = 0;
  *tag = tg;
  for (int i = 0; i < 5; ++i) (*k)[i] = v[i];
  int* f[9] = {&c->kernels, &c->work_mb, &c->a_prefetch, &c->b_variant, &c->c_variant, &c->a_variant, &c->nt_hint,
               &c->b_xtile, &c->b_threads};
  for (int i = 0; i < 9; ++i) *f[i] = v[5 + i];
  for (int a = 0; a < 3; ++a)
    for (int r = 0; r < 4; ++r) c->radix[a][r] = v[14 + 4 * a + r];
  c->c_split = v[26];
  return true;
}

fx_status load_configs_impl(fx_ctx* ctx, const char* path, int* n_loaded) {
  if (n_loaded) *n_loaded = 0;
  FILE* f = std::fopen(path, "r");
  if (!f) FX_FAIL(FX_ERR_INVALID, "cannot open configuration file %s", path);
  const std::string tag = device_tag(ctx->device);
  char line[1024];
  int n = 0, lineno = 0;
  fx_status st = FX_OK;
  while (std::fgets(line, sizeof line, f)) {
    ++lineno;
    if (line[0] == '#' || line[0] == '\n') continue;
    std::string tg;
    std::array<int, 5> k;
    fx_vx_config c{};
    if (!parse_config_line(line, &tg, &k, &c)) {
      set_error("%s:%d: not a configuration line", path, lineno);
      st = FX_ERR_INVALID;
      break;
    }
    if (tg != tag) continue;
    fx_cell cell{{k[0], k[1], k[2]}, {1.0, 1.0, 1.0}};
    if (check_cell(&cell) != FX_OK || !is_vx_prec((fx_prec)k[3]) || (k[4] != 0 && k[4] != 1) ||
        check_config(&cell, c) != FX_OK) {
      set_error("%s:%d: invalid configuration", path, lineno);
      st = FX_ERR_INVALID;
      break;
    }
    ctx->vx_tuning[k] = c;
    ++n;
  }
  std::fclose(f);
  if (n_loaded) *n_loaded = n;
  return st;
}

fx_status save_configs_impl(fx_ctx* ctx, const char* path) {
  const std::string tag = device_tag(ctx->device);
  // keep the lines of other devices and of shapes this context does not hold
  std::vector<std::string> keep;
  if (FILE* f = std::fopen(path, "r")) {
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
      std::string tg;
      std::array<int, 5> k;
      fx_vx_config c{};
      std::string ln(line);
      while (!ln.empty() && (ln.back() == '\n' || ln.back() == '\r')) ln.pop_back();
      if (ln.empty() || ln.rfind("# libfock", 0) == 0) continue;
      // this device's shapes that the context holds are rewritten; any other
      // line (other devices, other shapes, foreign text) is kept as it was
      if (parse_config_line(line, &tg, &k, &c) && tg == tag && ctx->vx_tuning.count(k)) continue;
      keep.push_back(ln);
    }
    std::fclose(f);
  }
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) FX_FAIL(FX_ERR_INVALID, "cannot write configuration file %s", tmp.c_str());
  std::fprintf(f, "# libfock V_X launch configurations (fx_vx_save_configs); one per device kind, grid, precision "
                  "and form\n");
  for (const auto& ln : keep) std::fprintf(f, "%s\n", ln.c_str());
  for (const auto& kv : ctx->vx_tuning) std::fprintf(f, "%s\n", config_line(tag, kv.first, kv.second).c_str());
  const bool ok = std::fclose(f) == 0;
  if (!ok || std::rename(tmp.c_str(), path) != 0) FX_FAIL(FX_ERR_INVALID, "cannot replace configuration file %s", path);
  return FX_OK;
}

// One timed candidate: a warm-up apply (allocations, tables), then the best
// of two.  Returns +inf when the candidate cannot run (budget, launch shape).
static fx_status time_candidate(fx_ctx* ctx, const VxArgs& base, const fx_vx_config& c, hipStream_t st,
                                hipEvent_t e0, hipEvent_t e1, double* ms) {
  *ms = std::numeric_limits<double>::infinity();
  VxArgs a = base;
  a.kernels = c.kernels;
  a.work_cap = c.work_mb > 0 ? (size_t)c.work_mb << 20 : 0;
  a.a_pipe = c.a_prefetch;
  a.b_var = c.b_variant;
  a.c_var = c.c_variant;
  a.a_var = c.a_variant;
  a.nt_hint = c.nt_hint;
  a.c_split = c.c_split;
  a.xtile = c.b_xtile;
  a.nthr_b = c.b_threads;
  bool any = false;
  if (!plans_from_radix(a.cell, c.radix, &a.plans, &any)) return FX_OK;
  a.plans_set = any;
  fx_status s = vx_apply(ctx, &ctx->ws, a, st, nullptr);
  if (s == FX_ERR_OOM || s == FX_ERR_UNSUPPORTED) {
    clear_error();
    FX_HIP(hipStreamSynchronize(st));
    return FX_OK;
  }
  FX_TRY(s);
  FX_HIP(hipStreamSynchronize(st));
  for (int r = 0; r < 2; ++r) {
    FX_HIP(hipEventRecord(e0, st));
    FX_TRY(vx_apply(ctx, &ctx->ws, a, st, nullptr));
    FX_HIP(hipEventRecord(e1, st));
    FX_HIP(hipEventSynchronize(e1));
    float t = 0.f;
    FX_HIP(hipEventElapsedTime(&t, e0, e1));
    *ms = std::min(*ms, (double)t);
  }
  return FX_OK;
}

static fx_status autotune(fx_ctx* ctx, const fx_cell* cell, const fx_kernel* kernel, int n_psi, int n_phi, bool square,
                          fx_prec prec, hipStream_t st, fx_vx_config* out, double* ms_per_kpair) {
  const int64_t nr = (int64_t)cell->n[0] * cell->n[1] * cell->n[2];
  const bool t64 = prec == FX_PREC_FP64;
  const fx_dtype in_dt = t64 ? FX_C128 : FX_C64;
  const fx_dtype out_dt = prec == FX_PREC_FP32 ? FX_C64 : FX_C128;
  const size_t esz = dtype_size(in_dt), osz = dtype_size(out_dt);
  // probe: about two batches of the largest volume tried
  const size_t max_cap = std::min<size_t>((size_t)16 << 30, ctx->budget / 4);
  const int64_t pair_bytes = nr * (int64_t)esz;
  const int64_t probe = std::min<int64_t>((int64_t)n_psi * n_phi,
                                          std::max<int64_t>(64, 2 * (int64_t)(max_cap / pair_bytes)));
  int np_psi, np_phi;
  if (square) {
    np_psi = np_phi = (int)std::min<int64_t>(n_psi, (int64_t)std::ceil(std::sqrt(2.0 * (double)probe)));
  } else {
    np_phi = (int)std::min<int64_t>(n_phi, std::max<int64_t>(1, probe / std::min(n_psi, 16)));
    np_psi = (int)std::min<int64_t>(n_psi, std::max<int64_t>(1, probe / np_phi));
  }
  Workspace tws;
  void *psi = nullptr, *phi = nullptr, *out_p = nullptr;
  fx_status s = ws_get(ctx, &tws, "tune_psi", (size_t)np_psi * nr * esz, &psi);
  if (s == FX_OK && !square) s = ws_get(ctx, &tws, "tune_phi", (size_t)np_phi * nr * esz, &phi);
  if (s == FX_OK) s = ws_get(ctx, &tws, "tune_out", (size_t)np_phi * nr * osz, &out_p);
  if (s != FX_OK) {
    ws_release(ctx, &tws);
    return s;
  }
  if (square) phi = psi;
  const double scale = 1.0 / std::sqrt((double)nr);
  if (t64) {
    hipLaunchKernelGGL(k_fill_probe<double>, dim3(1024), dim3(256), 0, st, (cpx<double>*)psi, (int64_t)np_psi * nr,
                       (uint64_t)12345, scale);
    if (!square)
      hipLaunchKernelGGL(k_fill_probe<double>, dim3(1024), dim3(256), 0, st, (cpx<double>*)phi,
                         (int64_t)np_phi * nr, (uint64_t)67890, scale);
  } else {
    hipLaunchKernelGGL(k_fill_probe<float>, dim3(1024), dim3(256), 0, st, (cpx<float>*)psi, (int64_t)np_psi * nr,
                       (uint64_t)12345, (float)scale);
    if (!square)
      hipLaunchKernelGGL(k_fill_probe<float>, dim3(1024), dim3(256), 0, st, (cpx<float>*)phi, (int64_t)np_phi * nr,
                         (uint64_t)67890, (float)scale);
  }
  if (hipGetLastError() != hipSuccess) {
    ws_release(ctx, &tws);
    FX_FAIL(FX_ERR_DEVICE, "launch of the probe filler failed");
  }

  VxArgs base;
  base.cell = cell;
  base.kern = kernel;
  base.psi = psi;
  base.n_psi = np_psi;
  base.ld_psi = nr;
  base.phi = phi;
  base.n_phi = np_phi;
  base.ld_phi = nr;
  base.out = out_p;
  base.ld_out = nr;
  base.in_dtype = in_dt;
  base.out_dtype = out_dt;
  base.prec = prec;

  hipEvent_t e0 = nullptr, e1 = nullptr;
  fx_status rs = FX_OK;
  fx_vx_config cur{};
  double best = std::numeric_limits<double>::infinity();
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    ws_release(ctx, &tws);
    // the context workspace grew to the largest batch tried; later calls
    // allocate what they need
    ws_release(ctx, &ctx->ws);
  };
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    FX_FAIL(FX_ERR_DEVICE, "hipEventCreate failed");
  }
  auto trial = [&](const fx_vx_config& c) -> fx_status {
    double ms = 0;
    FX_TRY(time_candidate(ctx, base, c, st, e0, e1, &ms));
    if (ms < 0.98 * best) {
      best = ms;
      cur = c;
    }
    return FX_OK;
  };
  const bool spec = ct_supported(cell);
  cur.kernels = spec ? 1 : 2;
  cur.a_prefetch = 0;
  cur.b_variant = spec ? (cell->n[0] == 96 ? 4 : (cell->n[0] == 72 ? 3 : 1)) : 0;
  cur.c_variant = spec ? (cell->n[0] == 96 || cell->n[0] == 72 ? 5 : 1) : 0;
  cur.a_variant = spec ? (t64 && (cell->n[0] == 96 || cell->n[0] == 72) ? 3 : 1) : 0;
  cur.nt_hint = spec ? 1 : 0;
  rs = trial(cur);
  if (rs == FX_OK && best == std::numeric_limits<double>::infinity()) {
    cleanup();
    FX_FAIL(FX_ERR_OOM, "the automatic configuration does not run on this budget");
  }
  if (rs == FX_OK && spec) {
    fx_vx_config c = cur;
    c.kernels = 2;
    c.b_variant = 0;
    c.c_variant = 0;
    c.a_variant = 0;
    rs = trial(c);
  }
  if (rs == FX_OK && cur.kernels == 1) {
    if (!t64) {
      fx_vx_config c = cur;
      c.a_prefetch = 1;
      rs = trial(c);
    }
    const fx_vx_config bstart = cur;
    for (int bv = 1; bv <= 4 && rs == FX_OK; ++bv) {
      if (bv == bstart.b_variant) continue;
      fx_vx_config c = bstart;
      c.b_variant = bv;
      rs = trial(c);
    }
    const fx_vx_config cstart = cur;
    for (int cv = 1; cv <= 5 && rs == FX_OK; ++cv) {
      if (cv == cstart.c_variant) continue;
      fx_vx_config c = cstart;
      c.c_variant = cv;
      rs = trial(c);
    }
    const int astart = cur.a_variant;
    for (int av = 1; av <= 3 && rs == FX_OK; ++av) {
      if (av == astart) continue;
      fx_vx_config c = cur;
      c.a_variant = av;
      rs = trial(c);
    }
    if (rs == FX_OK) {
      fx_vx_config c = cur;
      c.nt_hint = 1 - cur.nt_hint;
      rs = trial(c);
    }
    // sum groups of the plane-inverse pass (pays where targets are few)
    const fx_vx_config sstart = cur;
    for (int sp = 2; sp <= 8 && rs == FX_OK; sp *= 2) {
      fx_vx_config c = sstart;
      c.c_split = sp;
      rs = trial(c);
    }
  }
  if (rs == FX_OK && cur.kernels == 2) {
    for (int ax = 0; ax < 3 && rs == FX_OK; ++ax) {
      AxisPlan plans[8];
      const int np = enumerate_axis_plans(cell->n[ax], plans, 6);
      const fx_vx_config start = cur;
      for (int i = 1; i < np && rs == FX_OK; ++i) {  // plan 0 is the default
        fx_vx_config c = start;
        for (int r = 0; r < 4; ++r) c.radix[ax][r] = r < plans[i].nst ? plans[i].R[r] : 0;
        rs = trial(c);
      }
    }
    const int xts[] = {4, 8, 16, 24, 32, 48, 64, 96};
    const fx_vx_config start = cur;
    for (int xt : xts) {
      if (rs != FX_OK || xt > cell->n[0]) break;
      fx_vx_config c = start;
      c.b_xtile = xt;
      rs = trial(c);
    }
    const fx_vx_config start2 = cur;
    for (int nt : {64, 128, 256}) {
      if (rs != FX_OK) break;
      fx_vx_config c = start2;
      c.b_threads = nt;
      rs = trial(c);
    }
  }
  if (rs == FX_OK) {
    const fx_vx_config start = cur;
    for (int mb : {2048, 4096, 16384}) {
      if (rs != FX_OK || ((size_t)mb << 20) > ctx->budget / 4) continue;
      fx_vx_config c = start;
      c.work_mb = mb;
      rs = trial(c);
    }
  }
  cleanup();
  FX_TRY(rs);
  ctx->vx_tuning[vx_tune_key(cell, prec, square)] = cur;
  if (out) *out = cur;
  if (ms_per_kpair) *ms_per_kpair = best / ((double)np_psi * np_phi) * 1000.0;
  return FX_OK;
}

fx_status vx_autotune_impl(fx_ctx* ctx, const fx_cell* cell, const fx_kernel* kernel, int n_psi, int n_phi,
                           bool square, fx_prec prec, hipStream_t st, fx_vx_config* best, double* ms_per_kpair) {
  // a stored configuration for this key must not fill in the candidates'
  // automatic fields; it comes back if tuning fails
  const auto key = vx_tune_key(cell, prec, square);
  auto it = ctx->vx_tuning.find(key);
  const bool had = it != ctx->vx_tuning.end();
  fx_vx_config old{};
  if (had) {
    old = it->second;
    ctx->vx_tuning.erase(it);
  }
  // probe launches are not the caller's work: keep them out of the timing
  const bool prof = ctx->prof;
  ctx->prof = false;
  fx_status s = autotune(ctx, cell, kernel, n_psi, n_phi, square, prec, st, best, ms_per_kpair);
  ctx->prof = prof;
  if (s != FX_OK && had) ctx->vx_tuning[key] = old;
  return s;
}

}  // namespace fx

using namespace fx;

extern "C" {

fx_status fx_vx_autotune(fx_ctx* ctx, const fx_cell* cell, const fx_kernel* kernel, int32_t n_psi, int32_t n_phi,
                         int32_t phi_is_psi, fx_prec prec, void* stream, fx_vx_config* best,
                         double* best_ms_per_kpair) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  FX_TRY(check_cell(cell));
  FX_TRY(check_kernel(kernel));
  if (!is_vx_prec(prec)) FX_FAIL(FX_ERR_UNSUPPORTED, "precision %d is not a V_X precision", prec);
  if (n_psi <= 0 || n_phi <= 0) FX_FAIL(FX_ERR_INVALID, "n_psi = %d and n_phi = %d must be positive", n_psi, n_phi);
  if (phi_is_psi && n_phi != n_psi) FX_FAIL(FX_ERR_INVALID, "phi_is_psi needs n_phi == n_psi");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  FX_HIP(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  FX_TRY(note_capture(ctx, st));
  if (ctx->capturing) FX_FAIL(FX_ERR_INVALID, "fx_vx_autotune waits on its stream and cannot be captured");
  FX_TRY(vx_autotune_impl(ctx, cell, kernel, n_psi, n_phi, phi_is_psi != 0, prec, st, best, best_ms_per_kpair));
  ctx->cfg_gen++;
  // FX_TUNE_CACHE: keep the file of tuned configurations up to date
  if (const char* e = getenv("FX_TUNE_CACHE"))
    if (*e) FX_TRY(save_configs_impl(ctx, e));
  return FX_OK;
}

fx_status fx_vx_load_configs(fx_ctx* ctx, const char* path, int32_t* n_loaded) {
  clear_error();
  if (!ctx || !path) FX_FAIL(FX_ERR_INVALID, "NULL argument");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  int n = 0;
  const fx_status s = load_configs_impl(ctx, path, &n);
  if (n_loaded) *n_loaded = n;
  ctx->cfg_gen++;
  return s;
}

fx_status fx_vx_save_configs(fx_ctx* ctx, const char* path) {
  clear_error();
  if (!ctx || !path) FX_FAIL(FX_ERR_INVALID, "NULL argument");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  return save_configs_impl(ctx, path);
}

fx_status fx_vx_set_config(fx_ctx* ctx, const fx_cell* cell, fx_prec prec, int32_t phi_is_psi,
                           const fx_vx_config* cfg) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  FX_TRY(check_cell(cell));
  if (!is_vx_prec(prec)) FX_FAIL(FX_ERR_UNSUPPORTED, "precision %d is not a V_X precision", prec);
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  const auto key = vx_tune_key(cell, prec, phi_is_psi != 0);
  ctx->cfg_gen++;
  if (!cfg) {
    ctx->vx_tuning.erase(key);
    return FX_OK;
  }
  FX_TRY(check_config(cell, *cfg));
  ctx->vx_tuning[key] = *cfg;
  return FX_OK;
}

fx_status fx_vx_get_config(fx_ctx* ctx, const fx_cell* cell, fx_prec prec, int32_t phi_is_psi, fx_vx_config* cfg,
                           int32_t* is_set) {
  clear_error();
  if (!ctx || !cfg || !is_set) FX_FAIL(FX_ERR_INVALID, "NULL argument");
  FX_TRY(check_cell(cell));
  if (!is_vx_prec(prec)) FX_FAIL(FX_ERR_UNSUPPORTED, "precision %d is not a V_X precision", prec);
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  auto it = ctx->vx_tuning.find(vx_tune_key(cell, prec, phi_is_psi != 0));
  *is_set = it != ctx->vx_tuning.end();
  if (*is_set) {
    *cfg = it->second;
  } else {
    *cfg = fx_vx_config{};
    cfg->a_prefetch = -1;
    cfg->nt_hint = -1;
  }
  return FX_OK;
}

}  // extern "C"
