// Host scheduling of the serving loop, separate from the device work so that
// it can be built and tested on a CPU with a simulated executor.
//
// The loop replays arrivals in time order.  An arrival that finds max_queue
// requests already waiting is refused (FX_ERR_BUSY); a request the caller has
// cancelled before it was dispatched is dropped (FX_ERR_CANCELLED).  Waiting
// requests are dispatched oldest first; a dispatch merges the oldest waiting
// request with later ones of the same operation and merge class (requests
// that can share one launch: for V_X, trajectories on the same grid with the
// same kernel, orbital count and precision; otherwise one trajectory), in
// arrival order, from at most kServeMaxTrajs trajectories, while the batch
// stays within max_batch_pairs pairs (pairs = orbitals x targets).  A batch
// goes to an idle slot whose stream has nothing running.  If its workspace
// does not fit, the idle slots hand back their workspaces and the launch is
// tried once more; if it still does not fit it waits for a running batch to
// finish, or is refused (FX_ERR_OOM) when nothing is running.  A request's
// latency runs from its arrival to the completion of its batch.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <vector>

#include "../../include/fock.h"

namespace fx {

// Trajectories one merged launch may draw on (the pass kernels take a table of
// this many orbital blocks).
constexpr int kServeMaxTrajs = 8;

// What the scheduler needs from the device side.
struct ServeExecutor {
  virtual ~ServeExecutor() = default;
  virtual int n_slots() const = 0;
  // slots with the same stream id never run batches at the same time
  virtual int stream_of(int slot) const = 0;
  // orbitals of a trajectory (a request of `count` targets is orbitals x count pairs)
  virtual int orbitals(int traj) const = 0;
  // requests of one operation whose trajectories have the same class may share
  // a launch (the trajectory itself: never merged with other trajectories)
  virtual int merge_class(int traj, int op) const {
    (void)op;
    return traj;
  }
  // the caller has cancelled request `req` (checked before it is dispatched)
  virtual bool cancelled(int req) const {
    (void)req;
    return false;
  }
  // enqueue `batch` (request indices, merged in this order) on `slot`:
  // FX_OK, FX_ERR_OOM if its workspace does not fit now, or another error
  virtual fx_status launch(int slot, const std::vector<int>& batch) = 0;
  // hand back the workspaces of the idle slots (idle[s] != 0) once their
  // streams have drained; false on a device error
  virtual bool release_idle(const std::vector<char>& idle) = 0;
  // 1 the slot's batch has finished, 0 still running, -1 device error
  virtual int poll(int slot) = 0;
  // clock in seconds, and a pause of the loop when it has nothing to do
  virtual double now() = 0;
  virtual void idle_wait(double seconds) = 0;
  // device bytes in use (for the peak in the report)
  virtual size_t mem_in_use() const = 0;
};

struct ServeOutcome {
  // per request: FX_OK, FX_ERR_INVALID, FX_ERR_OOM, FX_ERR_BUSY, or
  // FX_ERR_CANCELLED (cancelled by the caller, or never reached because the
  // loop ended on an error)
  std::vector<fx_status> status;
  std::vector<double> lat_ms;     // per request, -1 when not served
  int64_t done = 0, rejected = 0, cancelled = 0, batches = 0;
  double pairs_done = 0.0, busy_time = 0.0, wall = 0.0;
  size_t hbm_peak = 0;
  fx_status fatal = FX_OK;  // a device error or a launch failure other than FX_ERR_OOM
};

// Nearest-rank percentile (q in [0, 1]) of a sample; 0 for an empty one.
inline double serve_percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  size_t k = (size_t)std::ceil(q * (double)v.size());
  if (k < 1) k = 1;
  if (k > v.size()) k = v.size();
  return v[k - 1];
}

// The merge of one dispatch: the oldest waiting request, then later waiting
// requests of the same operation and merge class in arrival order, from at
// most kServeMaxTrajs trajectories, while the pairs stay within max_pairs (the
// first request that would exceed it ends the merge).
inline std::vector<int> serve_merge(const std::deque<int>& waiting, const fx_request* reqs, const ServeExecutor& ex,
                                    int64_t max_pairs) {
  std::vector<int> batch;
  if (waiting.empty()) return batch;
  const int head = waiting.front();
  const fx_request& rh = reqs[head];
  const int cls = ex.merge_class(rh.traj, rh.op);
  std::vector<int> trajs{rh.traj};
  batch.push_back(head);
  int64_t pairs = (int64_t)ex.orbitals(rh.traj) * rh.count;
  for (size_t w = 1; w < waiting.size(); ++w) {
    const fx_request& rw = reqs[waiting[w]];
    if (rw.op != rh.op || ex.merge_class(rw.traj, rw.op) != cls) continue;
    const bool new_traj = std::find(trajs.begin(), trajs.end(), rw.traj) == trajs.end();
    if (new_traj && (int)trajs.size() >= kServeMaxTrajs) continue;
    const int64_t p = (int64_t)ex.orbitals(rw.traj) * rw.count;
    if (pairs + p > max_pairs) break;
    batch.push_back(waiting[w]);
    if (new_traj) trajs.push_back(rw.traj);
    pairs += p;
  }
  return batch;
}

// Run the loop over nq requests; valid[i] == 0 marks a request the caller has
// rejected (its status stays FX_ERR_INVALID).
inline void serve_schedule(ServeExecutor& ex, const fx_request* reqs, int nq, const std::vector<char>& valid,
                           int64_t max_batch_pairs, ServeOutcome* out, int64_t max_queue = 0) {
  ServeOutcome& o = *out;
  o = ServeOutcome();
  o.status.assign(nq, FX_ERR_CANCELLED);
  o.lat_ms.assign(nq, -1.0);
  int64_t n_valid = 0;
  for (int i = 0; i < nq; ++i) {
    if (valid[i])
      ++n_valid;
    else
      o.status[i] = FX_ERR_INVALID;
  }
  std::vector<int> order(nq);
  for (int i = 0; i < nq; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return reqs[a].t_arrival_s < reqs[b].t_arrival_s; });
  const int ns = ex.n_slots();
  if (ns <= 0 && n_valid > 0) {  // nowhere to run: refuse rather than wait forever
    o.fatal = FX_ERR_INVALID;
    return;
  }
  std::vector<char> busy(ns, 0);
  std::vector<std::vector<int>> in_slot(ns);
  std::deque<int> waiting;
  size_t next = 0;
  int nbusy = 0;
  double busy_since = -1.0;
  const double t0 = ex.now();
  o.hbm_peak = ex.mem_in_use();

  auto finish = [&](int s, double t) {
    for (int i : in_slot[s]) {
      o.lat_ms[i] = 1e3 * (t - (t0 + reqs[i].t_arrival_s));
      o.status[i] = FX_OK;
      ++o.done;
    }
    in_slot[s].clear();
    busy[s] = 0;
    if (--nbusy == 0 && busy_since >= 0) {
      o.busy_time += t - busy_since;
      busy_since = -1.0;
    }
  };

  while (o.done + o.rejected + o.cancelled < n_valid || !waiting.empty() || nbusy) {
    const double t = ex.now() - t0;
    while (next < (size_t)nq && reqs[order[next]].t_arrival_s <= t) {
      const int i = order[next++];
      if (!valid[i]) continue;
      if (ex.cancelled(i)) {
        o.status[i] = FX_ERR_CANCELLED;
        ++o.cancelled;
      } else if (max_queue > 0 && (int64_t)waiting.size() >= max_queue) {
        o.status[i] = FX_ERR_BUSY;  // admission control: the queue is full
        ++o.rejected;
      } else {
        waiting.push_back(i);
      }
    }
    // waiting requests cancelled since they arrived leave the queue
    if (!waiting.empty()) {
      std::deque<int> keep;
      for (int w : waiting) {
        if (ex.cancelled(w)) {
          o.status[w] = FX_ERR_CANCELLED;
          ++o.cancelled;
        } else {
          keep.push_back(w);
        }
      }
      waiting.swap(keep);
    }
    for (int s = 0; s < ns; ++s) {
      if (!busy[s]) continue;
      const int q = ex.poll(s);
      if (q == 1) {
        finish(s, ex.now());
      } else if (q < 0) {
        o.fatal = FX_ERR_DEVICE;
        break;
      }
    }
    if (o.fatal != FX_OK) break;
    bool progressed = false;
    for (int s = 0; s < ns; ++s) {
      if (busy[s] || waiting.empty()) continue;
      bool stream_busy = false;
      for (int u = 0; u < ns; ++u)
        if (busy[u] && ex.stream_of(u) == ex.stream_of(s)) stream_busy = true;
      if (stream_busy) continue;
      const std::vector<int> batch = serve_merge(waiting, reqs, ex, max_batch_pairs);
      fx_status st = ex.launch(s, batch);
      if (st == FX_ERR_OOM) {
        std::vector<char> idle(ns);
        for (int u = 0; u < ns; ++u) idle[u] = busy[u] ? 0 : 1;
        if (!ex.release_idle(idle)) {
          o.fatal = FX_ERR_DEVICE;
          break;
        }
        st = ex.launch(s, batch);
      }
      if (st == FX_ERR_OOM) {
        if (nbusy > 0) break;  // wait for memory to drain
        for (int i : batch) {
          o.status[i] = FX_ERR_OOM;
          ++o.rejected;
        }
      } else if (st != FX_OK) {
        o.fatal = st;
        break;
      } else {
        busy[s] = 1;
        in_slot[s] = batch;
        if (nbusy++ == 0) busy_since = ex.now();
        ++o.batches;
        for (int i : batch) o.pairs_done += (double)ex.orbitals(reqs[i].traj) * reqs[i].count;
        progressed = true;
      }
      std::deque<int> rest;
      for (int w : waiting)
        if (std::find(batch.begin(), batch.end(), w) == batch.end()) rest.push_back(w);
      waiting.swap(rest);
      o.hbm_peak = std::max(o.hbm_peak, ex.mem_in_use());
    }
    if (o.fatal != FX_OK) break;
    if (!progressed) {
      // nothing launched: pause until the next arrival, at most a short poll
      // interval and at least 1 us (a pause that rounds to nothing on the
      // clock would leave the arrival unreached)
      double wait = 2e-4;
      if (next < (size_t)nq && waiting.empty() && nbusy == 0) wait = reqs[order[next]].t_arrival_s - t;
      ex.idle_wait(std::min(std::max(wait, 1e-6), 5e-5));
    }
    if (next >= (size_t)nq && waiting.empty() && nbusy == 0) break;
  }
  o.wall = ex.now() - t0;
}

}  // namespace fx
