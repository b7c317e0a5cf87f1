// Host checks of the serving scheduler (paper_1905_01348_amd/csrc/serve_sched.hpp)
// against a simulated executor: a virtual clock, batch service times that grow
// with the pairs, slot workspaces held against a byte budget, and injected
// allocation and device failures.  Built with g++ (address and undefined-
// behaviour sanitizers) and run by tests/test_serve_sched.py.  Prints one line
// per failed check and "ok <checks>" at the end; exits 1 on any failure.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "serve_sched.hpp"

using namespace fx;

static int g_checks = 0, g_fail = 0;
#define CHECK(cond, ...)                              \
  do {                                                \
    ++g_checks;                                       \
    if (!(cond)) {                                    \
      ++g_fail;                                       \
      std::printf("FAIL %s:%d ", __FILE__, __LINE__); \
      std::printf(__VA_ARGS__);                       \
      std::printf("\n");                              \
    }                                                 \
  } while (0)

struct Launch {
  double t_start, t_end;
  int slot, stream;
  std::vector<int> batch;
};

struct FakeExec final : ServeExecutor {
  int ns, nstreams;
  std::map<int, int> norb;         // trajectory -> orbitals
  std::map<int, int> cls;          // trajectory -> merge class of its V_X requests (none: the trajectory)
  std::set<int> cancel;            // requests the caller has cancelled
  double c0 = 1e-4, c1 = 2e-8;     // service time = c0 + c1 * pairs (seconds)
  size_t bytes_per_pair = 1000, budget = (size_t)1 << 40, in_use = 0;
  std::vector<size_t> ws;          // workspace held by each slot
  std::vector<double> t_end;       // completion time of each slot's batch
  std::vector<char> running;
  double clock = 100.0;
  int fail_launch_at = -1, launches_tried = 0;  // injected OOM on this launch attempt
  int poll_error_at = -1, polls = 0;            // injected device error on this poll
  int releases = 0;
  const fx_request* reqs = nullptr;
  std::vector<Launch> log;

  FakeExec(int slots, int streams) : ns(slots), nstreams(streams), ws(slots, 0), t_end(slots, 0), running(slots, 0) {}
  int n_slots() const override { return ns; }
  int stream_of(int s) const override { return s % nstreams; }
  int orbitals(int traj) const override { return norb.at(traj); }
  int merge_class(int traj, int op) const override {
    auto it = cls.find(traj);
    return op == 0 && it != cls.end() ? it->second : traj;
  }
  bool cancelled(int req) const override { return cancel.count(req) != 0; }
  int64_t pairs_of(const std::vector<int>& b) const {
    int64_t p = 0;
    for (int i : b) p += (int64_t)norb.at(reqs[i].traj) * reqs[i].count;
    return p;
  }
  fx_status launch(int s, const std::vector<int>& batch) override {
    const int attempt = launches_tried++;
    if (attempt == fail_launch_at) return FX_ERR_OOM;
    const size_t need = bytes_per_pair * (size_t)pairs_of(batch);
    if (need > ws[s]) {
      if (in_use - ws[s] + need > budget) return FX_ERR_OOM;
      in_use = in_use - ws[s] + need;
      ws[s] = need;
    }
    running[s] = 1;
    t_end[s] = clock + c0 + c1 * (double)pairs_of(batch);
    log.push_back({clock, t_end[s], s, stream_of(s), batch});
    return FX_OK;
  }
  bool release_idle(const std::vector<char>& idle) override {
    ++releases;
    for (int s = 0; s < ns; ++s)
      if (idle[s]) {
        in_use -= ws[s];
        ws[s] = 0;
      }
    return true;
  }
  int poll(int s) override {
    if (polls++ == poll_error_at) return -1;
    if (running[s] && clock >= t_end[s]) {
      running[s] = 0;
      return 1;
    }
    return running[s] ? 0 : 1;
  }
  double now() override { return clock; }
  void idle_wait(double dt) override { clock += dt; }
  size_t mem_in_use() const override { return in_use; }
};

// seeded request stream: Poisson arrivals over three trajectories, blocks of targets
static std::vector<fx_request> make_requests(unsigned seed, int n, double rate) {
  std::vector<fx_request> r(n);
  uint64_t x = seed * 0x9E3779B97F4A7C15ull + 1;
  auto u01 = [&]() {
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
    return ((x >> 11) + 0.5) / 9007199254740992.0;
  };
  double t = 0;
  for (int i = 0; i < n; ++i) {
    t += -std::log(u01()) / rate;
    const double c = u01();
    r[i].traj = c < 0.5 ? 0 : (c < 0.85 ? 1 : 2);
    r[i].op = u01() < 0.5 ? 0 : 1;
    r[i].first = 0;
    r[i].count = 1 + (int)(u01() * 8);
    r[i].t_arrival_s = t;
    r[i].out = nullptr;
    r[i].ld_out = 0;
  }
  return r;
}

static void check_log(const FakeExec& ex, const std::vector<fx_request>& reqs, const std::vector<char>& valid,
                      const ServeOutcome& o, int64_t max_pairs, const char* what) {
  std::vector<int> seen(reqs.size(), 0);
  for (const Launch& l : ex.log) {
    const fx_request& h = reqs[l.batch[0]];
    int64_t pairs = 0;
    std::set<int> trajs;
    for (size_t k = 0; k < l.batch.size(); ++k) {
      const fx_request& r = reqs[l.batch[k]];
      ++seen[l.batch[k]];
      trajs.insert(r.traj);
      CHECK(r.op == h.op && ex.merge_class(r.traj, r.op) == ex.merge_class(h.traj, h.op),
            "%s: batch mixes operations or merge classes", what);
      CHECK(r.t_arrival_s <= l.t_start - 100.0 + 1e-12, "%s: request %d launched before it arrived", what,
            l.batch[k]);
      if (k) CHECK(reqs[l.batch[k - 1]].t_arrival_s <= r.t_arrival_s, "%s: batch not in arrival order", what);
      pairs += (int64_t)ex.norb.at(r.traj) * r.count;
    }
    CHECK(l.batch.size() == 1 || pairs <= max_pairs, "%s: merged batch of %lld pairs over the cap", what,
          (long long)pairs);
    CHECK((int)trajs.size() <= kServeMaxTrajs, "%s: batch draws on %zu trajectories", what, trajs.size());
  }
  // one stream runs one batch at a time
  for (size_t a = 0; a < ex.log.size(); ++a)
    for (size_t b = a + 1; b < ex.log.size(); ++b)
      if (ex.log[a].stream == ex.log[b].stream)
        CHECK(ex.log[a].t_end <= ex.log[b].t_start + 1e-12 || ex.log[b].t_end <= ex.log[a].t_start + 1e-12,
              "%s: batches %zu and %zu overlap on stream %d", what, a, b, ex.log[a].stream);
  // batch heads are dispatched oldest first
  for (size_t a = 1; a < ex.log.size(); ++a)
    CHECK(reqs[ex.log[a - 1].batch[0]].t_arrival_s <= reqs[ex.log[a].batch[0]].t_arrival_s,
          "%s: a younger head went first", what);
  for (size_t i = 0; i < reqs.size(); ++i) {
    if (!valid[i]) {
      CHECK(seen[i] == 0 && o.status[i] == FX_ERR_INVALID, "%s: invalid request %zu ran or lost its status", what, i);
      continue;
    }
    if (o.status[i] == FX_OK) {
      CHECK(seen[i] == 1, "%s: request %zu served %d times", what, i, seen[i]);
      CHECK(o.lat_ms[i] >= 1e3 * ex.c0 - 1e-9, "%s: latency %g below the service time", what, o.lat_ms[i]);
    } else {
      CHECK((o.status[i] == FX_ERR_OOM || o.status[i] == FX_ERR_BUSY || o.status[i] == FX_ERR_CANCELLED) &&
                seen[i] == 0,
            "%s: request %zu status %d", what, i, (int)o.status[i]);
    }
  }
}

int main() {
  // nearest-rank percentiles
  {
    std::vector<double> v;
    for (int i = 100; i >= 1; --i) v.push_back(i);
    CHECK(serve_percentile(v, 0.5) == 50 && serve_percentile(v, 0.99) == 99 && serve_percentile(v, 1.0) == 100,
          "percentiles of 1..100");
    CHECK(serve_percentile({7.0}, 0.5) == 7.0 && serve_percentile({}, 0.99) == 0.0, "percentiles of 1 and 0 values");
  }
  // merge: oldest first, then the same trajectory and operation in arrival order, within the cap
  {
    FakeExec ex(1, 1);
    ex.norb = {{0, 10}, {1, 10}};
    std::vector<fx_request> r(5);
    int tr[5] = {0, 1, 0, 0, 0}, op[5] = {0, 0, 1, 0, 0}, cnt[5] = {2, 2, 2, 3, 2};
    for (int i = 0; i < 5; ++i) {
      r[i] = fx_request{};
      r[i].traj = tr[i];
      r[i].op = op[i];
      r[i].count = cnt[i];
      r[i].t_arrival_s = i;
    }
    ex.reqs = r.data();
    std::deque<int> w{0, 1, 2, 3, 4};
    std::vector<int> b = serve_merge(w, r.data(), ex, 50);
    CHECK(b == std::vector<int>({0, 3}), "merge skips other trajectories and operations, stops at the cap");
    b = serve_merge(w, r.data(), ex, 1000);
    CHECK(b == std::vector<int>({0, 3, 4}), "merge takes every match under a large cap");
    b = serve_merge(w, r.data(), ex, 5);
    CHECK(b == std::vector<int>({0}), "a request over the cap alone still forms a batch");
  }
  const int64_t cap = 4096;
  // a replay with merging and overlap; then the same replay again (determinism)
  std::vector<fx_request> reqs = make_requests(7, 600, 2000.0);
  std::vector<char> valid(reqs.size(), 1);
  for (size_t i = 0; i < reqs.size(); i += 37) valid[i] = 0;
  std::vector<Launch> first_log;
  for (int rep = 0; rep < 2; ++rep) {
    FakeExec ex(4, 2);
    ex.norb = {{0, 16}, {1, 128}, {2, 432}};
    ex.reqs = reqs.data();
    ServeOutcome o;
    serve_schedule(ex, reqs.data(), (int)reqs.size(), valid, cap, &o);
    CHECK(o.fatal == FX_OK, "replay: fatal %d", (int)o.fatal);
    int64_t nv = 0;
    for (char v : valid) nv += v;
    CHECK(o.done == nv && o.rejected == 0, "replay: %lld done of %lld", (long long)o.done, (long long)nv);
    CHECK(o.batches < o.done, "replay: no request was merged");
    check_log(ex, reqs, valid, o, cap, "replay");
    if (rep == 0) {
      first_log = ex.log;
    } else {
      bool same = first_log.size() == ex.log.size();
      for (size_t i = 0; same && i < ex.log.size(); ++i)
        same = first_log[i].slot == ex.log[i].slot && first_log[i].batch == ex.log[i].batch &&
               first_log[i].t_start == ex.log[i].t_start;
      CHECK(same, "replay: a second run scheduled differently");
    }
  }
  // a small budget: batches wait while others run and are refused only when nothing runs
  {
    FakeExec ex(3, 3);
    ex.norb = {{0, 16}, {1, 128}, {2, 432}};
    ex.reqs = reqs.data();
    ex.budget = 1000 * 432 * 6;  // fits one 432-orbital request of up to 6 targets
    std::vector<char> all(reqs.size(), 1);
    ServeOutcome o;
    serve_schedule(ex, reqs.data(), (int)reqs.size(), all, cap, &o);
    CHECK(o.fatal == FX_OK, "budget: fatal %d", (int)o.fatal);
    int64_t refused = 0;
    for (size_t i = 0; i < reqs.size(); ++i) {
      const int64_t p = (int64_t)ex.norb.at(reqs[i].traj) * reqs[i].count;
      if (o.status[i] == FX_ERR_OOM) {
        ++refused;
        CHECK(p * 1000 > (int64_t)ex.budget, "budget: request %zu of %lld pairs refused though it fits alone", i,
              (long long)p);
      }
    }
    CHECK(refused > 0 && o.done + o.rejected == (int64_t)reqs.size(), "budget: %lld refused, %lld done",
          (long long)refused, (long long)o.done);
    CHECK(ex.in_use <= ex.budget, "budget exceeded");
    check_log(ex, reqs, all, o, cap, "budget");
  }
  // an allocation failure on one launch: idle workspaces are handed back and the launch retried
  {
    FakeExec ex(2, 2);
    ex.norb = {{0, 16}, {1, 128}, {2, 432}};
    ex.reqs = reqs.data();
    ex.fail_launch_at = 5;
    std::vector<fx_request> few(reqs.begin(), reqs.begin() + 40);
    std::vector<char> all(few.size(), 1);
    ex.reqs = few.data();
    ServeOutcome o;
    serve_schedule(ex, few.data(), (int)few.size(), all, cap, &o);
    CHECK(o.fatal == FX_OK && o.done == (int64_t)few.size() && ex.releases == 1, "retry: done %lld, releases %d",
          (long long)o.done, ex.releases);
  }
  // a device error while polling ends the loop with FX_ERR_DEVICE
  {
    FakeExec ex(2, 2);
    ex.norb = {{0, 16}, {1, 128}, {2, 432}};
    std::vector<fx_request> few(reqs.begin(), reqs.begin() + 40);
    std::vector<char> all(few.size(), 1);
    ex.reqs = few.data();
    ex.poll_error_at = 3;
    ServeOutcome o;
    serve_schedule(ex, few.data(), (int)few.size(), all, cap, &o);
    CHECK(o.fatal == FX_ERR_DEVICE, "device error: fatal %d", (int)o.fatal);
  }
  // no slots: the loop refuses instead of waiting forever
  {
    FakeExec ex(0, 1);
    ex.norb = {{0, 16}, {1, 128}, {2, 432}};
    std::vector<fx_request> few(reqs.begin(), reqs.begin() + 3);
    std::vector<char> all(few.size(), 1);
    ex.reqs = few.data();
    ServeOutcome o;
    serve_schedule(ex, few.data(), (int)few.size(), all, cap, &o);
    CHECK(o.fatal == FX_ERR_INVALID && o.done == 0, "no slots: fatal %d", (int)o.fatal);
  }
  // merge classes: V_X requests of trajectories of one class share launches
  // (at most kServeMaxTrajs trajectories each), never across classes or with ACE
  {
    std::vector<fx_request> r = make_requests(11, 800, 4000.0);
    for (size_t i = 0; i < r.size(); ++i) r[i].traj = (int)(i * 7 % 13);  // 13 trajectories
    FakeExec ex(4, 2);
    for (int t = 0; t < 13; ++t) {
      ex.norb[t] = t < 10 ? 32 : 64;
      if (t < 10) ex.cls[t] = 100;      // ten of one class: more than one launch may hold
      else if (t < 12) ex.cls[t] = 200;  // two of another
    }
    ex.reqs = r.data();
    std::vector<char> all(r.size(), 1);
    ServeOutcome o;
    serve_schedule(ex, r.data(), (int)r.size(), all, cap, &o);
    CHECK(o.fatal == FX_OK && o.done == (int64_t)r.size(), "classes: done %lld", (long long)o.done);
    check_log(ex, r, all, o, cap, "classes");
    int mixed = 0;
    for (const Launch& l : ex.log) {
      std::set<int> t;
      for (int i : l.batch) t.insert(r[i].traj);
      if (t.size() > 1) {
        ++mixed;
        CHECK(r[l.batch[0]].op == 0, "classes: an ACE batch mixes trajectories");
      }
    }
    CHECK(mixed > 0, "classes: no launch merged trajectories of one class");
  }
  // admission: an arrival that finds max_queue requests waiting is refused with FX_ERR_BUSY
  {
    std::vector<fx_request> r = make_requests(13, 300, 1e6);  // a burst
    FakeExec ex(1, 1);
    ex.norb = {{0, 16}, {1, 128}, {2, 432}};
    ex.reqs = r.data();
    std::vector<char> all(r.size(), 1);
    ServeOutcome o;
    serve_schedule(ex, r.data(), (int)r.size(), all, 1, &o, 4);
    int64_t busy = 0;
    for (auto st : o.status) busy += st == FX_ERR_BUSY;
    CHECK(o.fatal == FX_OK && busy > 0 && o.done + busy == (int64_t)r.size() && o.rejected == busy,
          "queue cap: done %lld busy %lld", (long long)o.done, (long long)busy);
    check_log(ex, r, all, o, 1, "queue cap");
    ServeOutcome o2;
    FakeExec ex2(1, 1);
    ex2.norb = ex.norb;
    ex2.reqs = r.data();
    serve_schedule(ex2, r.data(), (int)r.size(), all, 1, &o2, 0);
    CHECK(o2.done == (int64_t)r.size(), "no queue cap: every request served");
  }
  // cancellation: cancelled requests never run and report FX_ERR_CANCELLED
  {
    std::vector<fx_request> r = make_requests(17, 200, 3000.0);
    FakeExec ex(2, 2);
    ex.norb = {{0, 16}, {1, 128}, {2, 432}};
    ex.reqs = r.data();
    for (int i = 0; i < 200; i += 9) ex.cancel.insert(i);
    std::vector<char> all(r.size(), 1);
    ServeOutcome o;
    serve_schedule(ex, r.data(), (int)r.size(), all, cap, &o);
    bool ok = o.fatal == FX_OK && o.cancelled == (int64_t)ex.cancel.size() &&
              o.done + o.cancelled == (int64_t)r.size();
    for (int i : ex.cancel) ok = ok && o.status[i] == FX_ERR_CANCELLED;
    CHECK(ok, "cancel: done %lld cancelled %lld", (long long)o.done, (long long)o.cancelled);
    check_log(ex, r, all, o, cap, "cancel");
  }
  // no requests at all
  {
    FakeExec ex(2, 1);
    ServeOutcome o;
    serve_schedule(ex, nullptr, 0, {}, cap, &o);
    CHECK(o.fatal == FX_OK && o.done == 0 && o.batches == 0, "empty replay");
  }
  std::printf("%s %d checks, %d failed\n", g_fail ? "FAILED" : "ok", g_checks, g_fail);
  return g_fail ? 1 : 0;
}
