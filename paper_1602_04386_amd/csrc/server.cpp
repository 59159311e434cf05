// Serving: continuous batching of Fiedler requests on one GPU.
//
// Worker threads, each with its own HIP stream, take requests from the queue
// as in-flight slots free up, build (or reuse from the cache) their
// hierarchies, and run small ones (finest level up to kServeBatchMaxN
// vertices) together as one persistent batched launch, one workgroup per
// graph, and a large one alone through the multi-workgroup single-graph path
// with the worker's own workspace.  With two or more workers the first one
// takes only small requests, so they never queue behind a multi-million-vertex
// solve.  A request that arrives while others run on the device is admitted by
// the next worker that is free, launches from different workers overlap on
// the device, and each result is published as soon as its own work ends.  Device memory for hierarchies and launch workspaces comes out
// of the context's HBM budget; cached hierarchies not in use are evicted
// least-recently-used first when a reservation does not fit.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>

#include "fv_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  fv_request req;
  fv_csr graph;
  bool has_graph = false;
  int state = 0;  // 0 queued, 1 running, 2 done
  fv_result res{};
  Clock::time_point t_submit, t_start;
};

struct CacheEntry {
  fv_hierarchy* h = nullptr;
  int refs = 0;
  uint64_t last_use = 0;
  bool building = false;
};

}  // namespace

struct fv_server {
  fv_context* ctx = nullptr;
  fv_server_opts opts{};
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Request> reqs;
  std::unordered_map<uint64_t, CacheEntry> cache;
  std::vector<std::thread> workers;
  bool stop = false;
  uint64_t next_ticket = 1;
  uint64_t use_clock = 0;
  int inflight = 0;
  // Deadlock-free waiting for memory: `holders` workers have an admitted batch
  // (and may hold hierarchies and workspaces until it ends); `waiters` of them
  // are blocked, waiting for memory or for another worker's build of the same
  // graph.  `released` counts events that can free memory (a batch ended, a
  // build ended, a hierarchy was evicted).
  int holders = 0;
  int waiters = 0;
  uint64_t released = 0;
};

namespace {

// Frees one unreferenced cached hierarchy (least recently used); returns false
// when none can be freed.  Caller holds s->mu.
bool evict_one(fv_server* s) {
  auto victim = s->cache.end();
  for (auto it = s->cache.begin(); it != s->cache.end(); ++it)
    if (it->second.refs == 0 && !it->second.building && it->second.h &&
        (victim == s->cache.end() || it->second.last_use < victim->second.last_use))
      victim = it;
  if (victim == s->cache.end()) return false;
  // refs == 0: every batch that used it has ended, and a batch ends only after
  // its stream has finished, so no device work reads it any more.
  fv::free_hierarchy(victim->second.h, /*sync_device=*/false);
  s->cache.erase(victim);
  ++s->released;
  return true;
}

// True while another worker holds an admitted batch and is not blocked itself:
// that worker will end its batch (or give up) and release memory, so waiting
// for it cannot deadlock.  Caller holds s->mu and is a holder.
bool others_progress(const fv_server* s) { return s->holders - s->waiters - 1 > 0; }

// Blocks (caller holds lk on s->mu) until the next release event, counted as
// a waiter meanwhile.
void wait_release(fv_server* s, std::unique_lock<std::mutex>& lk) {
  const uint64_t seen = s->released;
  ++s->waiters;
  s->cv.wait(lk, [&] { return s->released != seen; });
  --s->waiters;
}

// Runs f(); on FV_E_BUDGET evicts cached hierarchies not in use, or waits for
// another worker's batch to release memory, then retries.  Gives up (rethrows)
// when nothing can be evicted and no other worker is making progress: the
// memory is then held by this worker's own batch, by blocked workers, or
// outside the server, and waiting could last forever.
template <class F>
auto with_budget(fv_server* s, F f) -> decltype(f()) {
  for (;;) {
    try {
      return f();
    } catch (const fv::Error& e) {
      if (e.st != FV_E_BUDGET) throw;
      std::unique_lock<std::mutex> lk(s->mu);
      if (evict_one(s)) continue;
      if (!others_progress(s)) throw;
      wait_release(s, lk);
    }
  }
}

// Finest-level size above which a request leaves the batched launch: one
// workgroup per graph stops paying off once a level no longer fits its LDS.
constexpr int kServeBatchMaxN = 16384;

// Finest-level size of a queued request: its graph's, or its cached
// hierarchy's; 0 when unknown (treated as small).  Caller holds s->mu.
size_t request_n(const fv_server* s, const Request& r) {
  if (r.has_graph) return (size_t)r.graph.n;
  auto it = s->cache.find(r.req.graph_id);
  if (it != s->cache.end() && it->second.h) return fv::hierarchy_nmax(it->second.h);
  return 0;
}

bool is_large(const fv_server* s, uint64_t t) {
  return request_n(s, s->reqs.at(t)) > (size_t)kServeBatchMaxN;
}

// Admission.  A worker of the small lane takes only small requests; the
// others take the oldest request, alone when it is large, else together with
// the next small ones (up to `room`, skipping large ones, which stay queued
// in order).  So a small request never waits behind a large one in the same
// worker, and the oldest request is always the next one a general worker
// admits.  Returns false when this worker has nothing it may take.  Caller
// holds s->mu.
bool admit(fv_server* s, bool small_lane, int room, std::vector<uint64_t>& batch) {
  auto& q = s->queue;
  if (q.empty() || room < 1) return false;
  if (!small_lane && is_large(s, q.front())) {
    batch.push_back(q.front());
    q.pop_front();
    return true;
  }
  for (auto it = q.begin(); it != q.end() && (int)batch.size() < room;) {
    if (is_large(s, *it)) {
      ++it;
      continue;
    }
    batch.push_back(*it);
    it = q.erase(it);
  }
  return !batch.empty();
}

bool has_eligible(const fv_server* s, bool small_lane) {
  if (!small_lane) return !s->queue.empty();
  for (uint64_t t : s->queue)
    if (!is_large(s, t)) return true;
  return false;
}

void worker_main(fv_server* s, int share, bool small_lane) {
  (void)hipSetDevice(s->ctx->device);
  hipStream_t stream = nullptr;
  if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) return;
  fv::SolveScratch scratch;
  std::vector<uint64_t> batch;
  for (;;) {
    batch.clear();
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] {
        return (s->inflight < s->opts.max_inflight && has_eligible(s, small_lane)) ||
               (s->stop && !has_eligible(s, small_lane));
      });
      const int room = std::min(share, s->opts.max_inflight - s->inflight);
      if (!admit(s, small_lane, room, batch)) break;  // stopping, nothing left for this lane
      const auto now = Clock::now();
      for (uint64_t t : batch) {
        Request& r = s->reqs[t];
        r.state = 1;
        r.t_start = now;
      }
      s->inflight += (int)batch.size();
      ++s->holders;
    }
    // Hierarchies: cache hit, or build on this worker's stream.
    std::vector<fv_hierarchy*> hs(batch.size(), nullptr);
    std::vector<fv_status> st(batch.size(), FV_OK);
    std::vector<int> owned(batch.size(), 0);
    for (size_t k = 0; k < batch.size(); ++k) {
      Request* r;
      uint64_t gid;
      {
        std::unique_lock<std::mutex> lk(s->mu);
        r = &s->reqs[batch[k]];
        gid = r->req.graph_id;
        if (s->opts.cache_hierarchies) {
          for (;;) {
            auto it = s->cache.find(gid);
            if (it == s->cache.end()) {
              CacheEntry ce;
              ce.building = true;
              s->cache[gid] = ce;
              break;
            }
            if (!it->second.building) {
              it->second.refs++;
              it->second.last_use = ++s->use_clock;
              hs[k] = it->second.h;
              r->res.cache_hit = 1;
              break;
            }
            // Another worker builds this graph; its build ends with a
            // release event (success or failure).
            wait_release(s, lk);
          }
        }
      }
      if (hs[k]) continue;
      if (!r->has_graph) {
        st[k] = FV_E_INVALID;
      } else {
        try {
          hs[k] = with_budget(s, [&] {
            return fv::build_hierarchy(s->ctx, &r->graph, &s->opts.hier, stream);
          });
        } catch (const fv::Error& e) {
          st[k] = e.st;
        } catch (...) {
          st[k] = FV_E_DEVICE;
        }
      }
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->opts.cache_hierarchies) {
        CacheEntry& ce = s->cache[gid];
        ce.building = false;
        if (hs[k]) {
          ce.h = hs[k];
          ce.refs = 1;
          ce.last_use = ++s->use_clock;
        } else {
          s->cache.erase(gid);
        }
        ++s->released;
        s->cv.notify_all();
      } else {
        owned[k] = hs[k] ? 1 : 0;
      }
    }
    // Completes item k of the batch as soon as its own device work has ended
    // (its stream has finished it): the result becomes visible to fv_poll,
    // its slot and its hierarchy reference are given back.
    auto complete = [&](size_t k, double lam, double res, long long bytes) {
      const auto t_done = Clock::now();
      std::lock_guard<std::mutex> g(s->mu);
      Request& r = s->reqs[batch[k]];
      r.res.status = st[k];
      r.res.lambda = lam;
      r.res.residual = res;
      r.res.alg_bytes = bytes;
      r.res.queue_ms = std::chrono::duration<double, std::milli>(r.t_start - r.t_submit).count();
      r.res.latency_ms = std::chrono::duration<double, std::milli>(t_done - r.t_submit).count();
      r.state = 2;
      if (s->opts.cache_hierarchies) {
        auto it = s->cache.find(r.req.graph_id);
        if (it != s->cache.end() && hs[k] == it->second.h) it->second.refs--;
      } else if (owned[k]) {
        fv::free_hierarchy(hs[k], /*sync_device=*/false);
      }
      --s->inflight;
      ++s->released;
      s->cv.notify_all();
    };
    // Requests without a hierarchy (build failed) complete at once.
    for (size_t k = 0; k < batch.size(); ++k)
      if (!hs[k] || st[k] != FV_OK) complete(k, 0.0, 0.0, 0);
    // One batched launch for the small admitted requests; the large ones run
    // one by one below (a general worker admits a large request alone).
    std::vector<const fv_hierarchy*> run_h;
    std::vector<double*> run_x;
    std::vector<size_t> run_k, solo_k;
    for (size_t k = 0; k < batch.size(); ++k)
      if (hs[k] && st[k] == FV_OK) {
        if (fv::hierarchy_nmax(hs[k]) > (size_t)kServeBatchMaxN) {
          solo_k.push_back(k);
          continue;
        }
        run_h.push_back(hs[k]);
        std::lock_guard<std::mutex> g(s->mu);
        run_x.push_back(s->reqs[batch[k]].req.x_out);
        run_k.push_back(k);
      }
    if (!run_h.empty()) {
      std::vector<double> lam(run_h.size(), 0.0);
      std::vector<fv_solve_stats> stats(run_h.size());
      std::vector<fv_status> ist(run_h.size(), FV_OK);
      try {
        // the autotuner's cached configuration for this size class, if any
        // (a request never waits for a tuning run)
        fv_batch_opts bo;
        fv_batch_opts_default(&bo);
        bo.autotune = 2;
        with_budget(s, [&] {
          return fv::solve_batch(s->ctx, (int)run_h.size(), run_h.data(), &s->opts.solve, &bo,
                                 run_x.data(), 0, lam.data(), stats.data(), ist.data(), stream);
        });
      } catch (const fv::Error& e) {
        for (auto& v : ist) v = e.st;
      } catch (...) {
        for (auto& v : ist) v = FV_E_DEVICE;
      }
      for (size_t j = 0; j < run_k.size(); ++j) {
        st[run_k[j]] = ist[j];
        complete(run_k[j], lam[j], stats[j].residual, stats[j].alg_bytes);
      }
    }
    for (size_t k : solo_k) {
      double* xo;
      {
        std::lock_guard<std::mutex> g(s->mu);
        xo = s->reqs[batch[k]].req.x_out;
      }
      fv_solve_stats S{};
      double lam = 0.0;
      try {
        st[k] = with_budget(s, [&] {
          return fv::solve_one_with(s->ctx, scratch, hs[k], &s->opts.solve, xo, 0, &lam, &S,
                                    stream);
        });
      } catch (const fv::Error& e) {
        st[k] = e.st;
      } catch (...) {
        st[k] = FV_E_DEVICE;
      }
      // FV_E_NOT_CONVERGED still fills x and lambda
      complete(k, lam, S.residual, S.alg_bytes);
    }
    std::lock_guard<std::mutex> g(s->mu);
    --s->holders;
    ++s->released;
    s->cv.notify_all();
  }
  (void)hipStreamSynchronize(stream);
  fv::release_scratch(s->ctx, scratch);
  (void)hipStreamDestroy(stream);
}

}  // namespace

extern "C" {

fv_status fv_server_create(fv_context* ctx, const fv_server_opts* opts, fv_server** out) {
  if (!ctx || !opts || !out) return FV_E_INVALID;
  *out = nullptr;
  if (opts->max_inflight < 1 || opts->queue_capacity < 1 || opts->workers < 0)
    return FV_E_INVALID;
  if (opts->solve.replay || opts->solve.stream) return FV_E_INVALID;
  try {
    fv_server* s = new fv_server();
    s->ctx = ctx;
    s->opts = *opts;
    if (opts->hbm_budget_bytes) ctx->budget = opts->hbm_budget_bytes;
    // 8 by default: a solve is a chain of short dependent launches, so more
    // streams keep more of the GPU busy (on the serving pool 4, 8 and 16
    // workers gave 38, 52 and 56 solves/s in a closed loop)
    const int nworkers = std::max(1, std::min(opts->workers ? opts->workers : 8,
                                              opts->max_inflight));
    const int share = std::max(1, opts->max_inflight / nworkers);
    // with two or more workers the first one is the small-request lane
    for (int w = 0; w < nworkers; ++w)
      s->workers.emplace_back(worker_main, s, share, nworkers > 1 && w == 0);
    *out = s;
    return FV_OK;
  } catch (...) {
    return FV_E_DEVICE;
  }
}

fv_status fv_submit(fv_server* s, const fv_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket || !req->x_out) return FV_E_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  if ((int)s->queue.size() >= s->opts.queue_capacity) return FV_E_BUSY;
  if (!req->graph && !(s->opts.cache_hierarchies && s->cache.count(req->graph_id)))
    return FV_E_INVALID;
  if (req->graph && s->ctx->budget) {
    // A graph whose input alone exceeds the budget can never be admitted.
    const size_t in_bytes = (size_t)req->graph->nnz * 12 + (size_t)(req->graph->n + 1) * 4;
    if (in_bytes > s->ctx->budget) return FV_E_BUDGET;
  }
  Request r;
  r.req = *req;
  if (req->graph) {
    r.graph = *req->graph;
    r.has_graph = true;
  }
  r.t_submit = Clock::now();
  const uint64_t t = s->next_ticket++;
  s->reqs.emplace(t, r);
  s->queue.push_back(t);
  *ticket = t;
  s->cv.notify_all();
  return FV_OK;
}

fv_status fv_poll(fv_server* s, uint64_t ticket, fv_result* out) {
  if (!s || !out) return FV_E_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return FV_E_UNKNOWN_TICKET;
  if (it->second.state != 2) return FV_PENDING;
  *out = it->second.res;
  s->reqs.erase(it);
  return FV_OK;
}

void fv_server_destroy(fv_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto& t : s->workers) t.join();
  (void)hipSetDevice(s->ctx->device);
  for (auto& kv : s->cache)
    if (kv.second.h) fv::free_hierarchy(kv.second.h);
  delete s;
}

}  // extern "C"
