// C entry points of include/fiedler.h: argument checks, exception-to-status
// mapping, contexts and device-memory accounting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <new>
#include <thread>

#include "fv_internal.h"

namespace fv {

void budget_reserve(fv_context* ctx, size_t bytes) {
  std::lock_guard<std::mutex> g(ctx->mu);
  if (ctx->budget && ctx->in_use + bytes > ctx->budget)
    throw Error(FV_E_BUDGET, "HBM budget exceeded");
  ctx->in_use += bytes;
}

void budget_release(fv_context* ctx, size_t bytes) {
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->in_use -= std::min(ctx->in_use, bytes);
}

// Cached blocks are reused for requests up to 1/8 smaller than the block; new
// blocks are rounded up to 256 B (4 KiB above 64 KiB).  At most kCacheCap
// bytes stay cached; beyond that a released block goes back to HIP.
constexpr size_t kCacheCap = size_t(8) << 30;

static size_t block_round(size_t bytes) {
  const size_t g = bytes >= (size_t(64) << 10) ? 4096 : 256;
  return (std::max<size_t>(bytes, 1) + g - 1) / g * g;
}

void* block_get(fv_context* ctx, size_t bytes) {
  const size_t want = block_round(bytes);
  {
    std::lock_guard<std::mutex> g(ctx->cache_mu);
    auto it = ctx->cache.lower_bound(want);
    if (it != ctx->cache.end() && it->first <= want + want / 8) {
      void* p = it->second;
      ctx->live[p] = it->first;
      ctx->cached -= it->first;
      ctx->cache.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    block_trim(ctx);
    if (hipMalloc(&p, want) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(FV_E_NOMEM, "device allocation failed");
    }
  }
  std::lock_guard<std::mutex> g(ctx->cache_mu);
  ctx->live[p] = want;
  return p;
}

void block_put(fv_context* ctx, void* p) {
  if (!p) return;
  std::unique_lock<std::mutex> g(ctx->cache_mu);
  auto it = ctx->live.find(p);
  if (it == ctx->live.end()) return;
  const size_t sz = it->second;
  ctx->live.erase(it);
  if (ctx->cached + sz > kCacheCap) {
    g.unlock();
    (void)hipFree(p);
    return;
  }
  ctx->cache.emplace(sz, p);
  ctx->cached += sz;
}

void block_trim(fv_context* ctx) {
  std::multimap<size_t, void*> drop;
  {
    std::lock_guard<std::mutex> g(ctx->cache_mu);
    drop.swap(ctx->cache);
    ctx->cached = 0;
  }
  for (auto& kv : drop) (void)hipFree(kv.second);
}

void* pin_get(fv_context* ctx) {
  {
    std::lock_guard<std::mutex> g(ctx->pin_mu);
    if (!ctx->pins.empty()) {
      void* p = ctx->pins.back();
      ctx->pins.pop_back();
      return p;
    }
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, kPinBytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    throw Error(FV_E_NOMEM, "pinned host allocation failed");
  }
  return p;
}

void pin_put(fv_context* ctx, void* p, hipStream_t s) {
  if (!p) return;
  (void)hipStreamSynchronize(s);
  std::lock_guard<std::mutex> g(ctx->pin_mu);
  ctx->pins.push_back(p);
}

void pin_trim(fv_context* ctx) {
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> g(ctx->pin_mu);
    drop.swap(ctx->pins);
  }
  for (void* p : drop) (void)hipHostFree(p);
}

void* dev_alloc(fv_context* ctx, size_t bytes, size_t* counter) {
  budget_reserve(ctx, bytes);
  void* p = nullptr;
  try {
    p = block_get(ctx, bytes);
  } catch (...) {
    budget_release(ctx, bytes);
    throw;
  }
  if (counter) *counter += bytes;
  return p;
}

void dev_free(fv_context* ctx, void* p, size_t bytes, size_t* counter) {
  if (!p) return;
  block_put(ctx, p);
  budget_release(ctx, bytes);
  if (counter) *counter -= std::min(*counter, bytes);
}

}  // namespace fv

using fv::Error;

#define FV_GUARD(body)                                  \
  try {                                                 \
    body                                                \
  } catch (const Error& e) {                            \
    return e.st;                                        \
  } catch (const std::bad_alloc&) {                     \
    return FV_E_NOMEM;                                  \
  } catch (...) {                                       \
    return FV_E_DEVICE;                                 \
  }

extern "C" {

void fv_hier_opts_default(fv_hier_opts* o) {
  if (!o) return;
  o->n_coarse = 25;
  o->max_levels = FV_MAX_LEVELS;
  o->colour_seed = 0;
  o->ell = 0;
}

void fv_solve_opts_default(fv_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->prec = FV_PREC_FP64;
  o->seed = 1;
  o->tol_cos = 1e-6;
  o->tol_res = 0.0;
  o->omega = 1.0;
  o->max_gs = 100;
  o->max_pi = 100;
  o->max_outer = 50;
  o->max_coarsest = 100000;
  o->replay = nullptr;
  o->replay_len = 0;
  o->stream = nullptr;
  o->tol_coarse = 1e-13;
  o->time_finest = 0;
  o->early_exit = 0;
}

const char* fv_status_str(fv_status st) {
  switch (st) {
    case FV_OK: return "ok";
    case FV_PENDING: return "pending";
    case FV_E_INVALID: return "invalid argument or CSR structure";
    case FV_E_NOT_SYMMETRIC: return "matrix not symmetric";
    case FV_E_NOT_LAPLACIAN: return "not a graph Laplacian / adjacency";
    case FV_E_ISOLATED: return "isolated vertex";
    case FV_E_NOMEM: return "out of device memory";
    case FV_E_BUDGET: return "HBM budget exceeded";
    case FV_E_NOT_CONVERGED: return "not converged";
    case FV_E_DEVICE: return "device error";
    case FV_E_UNKNOWN_TICKET: return "unknown ticket";
    case FV_E_BUSY: return "server queue full";
    case FV_E_SCRATCH: return "graph exceeds the fixed scratch of the allocation-free solve";
  }
  return "unknown status";
}

fv_status fv_context_create(int device, size_t hbm_budget_bytes, fv_context** out) {
  if (!out) return FV_E_INVALID;
  *out = nullptr;
  FV_GUARD({
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
      return FV_E_INVALID;
    FV_HIP(hipSetDevice(device));
    fv_context* c = new fv_context();
    c->device = device;
    c->budget = hbm_budget_bytes;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return FV_E_DEVICE;
    }
    try {
      // Host buffers and events of the context's solves, and the device
      // address of the allocation-free solve's scratch on this device.
      fv::scratch_host_init(c->scratch);
      (void)fv::noalloc_scratch_init(device);
    } catch (...) {
      fv::release_scratch(c, c->scratch);
      (void)hipStreamDestroy(c->stream);
      delete c;
      throw;
    }
    *out = c;
    return FV_OK;
  })
}

void fv_context_destroy(fv_context* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  fv::release_batch_graph(c);
  fv::release_scratch(c, c->scratch);
  fv::block_trim(c);
  fv::pin_trim(c);
  (void)hipStreamDestroy(c->stream);
  delete c;
}

fv_status fv_build_hierarchy(fv_context* ctx, const fv_csr* L, const fv_hier_opts* opts,
                             fv_hierarchy** out) {
  if (!ctx || !L || !out) return FV_E_INVALID;
  *out = nullptr;
  FV_GUARD({
    FV_HIP(hipSetDevice(ctx->device));
    fv_hier_opts o;
    fv_hier_opts_default(&o);
    if (opts) o = *opts;
    *out = fv::build_hierarchy(ctx, L, &o, ctx->stream);
    return FV_OK;
  })
}

fv_status fv_build_hierarchies(fv_context* ctx, int32_t count, const fv_csr* const* graphs,
                               const fv_hier_opts* opts, int32_t threads, fv_hierarchy** out,
                               fv_status* item_status) {
  if (!ctx || count < 0 || (count > 0 && (!graphs || !out))) return FV_E_INVALID;
  fv_hier_opts o;
  fv_hier_opts_default(&o);
  if (opts) o = *opts;
  std::vector<fv_status> st(count, FV_OK);
  for (int i = 0; i < count; ++i) out[i] = nullptr;
  int nt = threads > 0 ? threads : 8;
  nt = std::max(1, std::min(nt, count));
  std::atomic<int> next{0};
  auto work = [&] {
    fv_status ts = FV_OK;
    hipStream_t s = nullptr;
    if (hipSetDevice(ctx->device) != hipSuccess ||
        hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      ts = FV_E_DEVICE;
    }
    for (int i = next++; i < count; i = next++) {
      if (ts != FV_OK) {
        st[i] = ts;
        continue;
      }
      try {
        out[i] = fv::build_hierarchy(ctx, graphs[i], &o, s);
        FV_HIP(hipStreamSynchronize(s));
      } catch (const fv::Error& e) {
        st[i] = e.st;
      } catch (const std::bad_alloc&) {
        st[i] = FV_E_NOMEM;
      } catch (...) {
        st[i] = FV_E_DEVICE;
      }
      if (st[i] != FV_OK && out[i]) {
        fv::free_hierarchy(out[i]);
        out[i] = nullptr;
      }
    }
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  };
  std::vector<std::thread> pool;
  try {
    for (int t = 1; t < nt; ++t) pool.emplace_back(work);
  } catch (...) {
    // fewer threads: the calling thread and those already started do the work
  }
  work();
  for (auto& t : pool) t.join();
  fv_status first = FV_OK;
  for (int i = 0; i < count; ++i) {
    if (item_status) item_status[i] = st[i];
    if (first == FV_OK && st[i] != FV_OK) first = st[i];
  }
  return first;
}

fv_status fv_hierarchy_info(const fv_hierarchy* h, int32_t* levels, int32_t* n, int64_t* nnz,
                            int32_t* colours, double* sigma) {
  if (!h) return FV_E_INVALID;
  if (levels) *levels = h->levels;
  for (int l = 0; l < h->levels; ++l) {
    if (n) n[l] = h->lv[l].n;
    if (nnz) nnz[l] = h->lv[l].m;
    if (colours) colours[l] = l == h->levels - 1 ? 0 : h->lv[l].ncol;
    if (sigma) sigma[l] = h->lv[l].sigma;
  }
  return FV_OK;
}

fv_status fv_hierarchy_bytes(const fv_hierarchy* h, int64_t* bytes) {
  if (!h || !bytes) return FV_E_INVALID;
  *bytes = (int64_t)h->bytes;
  return FV_OK;
}

fv_status fv_hierarchy_ell_width(const fv_hierarchy* h, int32_t level, int32_t colour,
                                 int32_t* width) {
  if (!h || !width || level < 0 || level >= h->levels) return FV_E_INVALID;
  *width = h->lv[level].ell_width(colour);
  return FV_OK;
}

fv_status fv_hierarchy_export_level(const fv_hierarchy* h, int32_t level, int32_t* row_ptr,
                                    int32_t* col, double* w, int32_t* q, int32_t* colour) {
  if (!h || level < 0 || level >= h->levels) return FV_E_INVALID;
  FV_GUARD({
    const fv::Level& L = h->lv[level];
    hipStream_t s = h->ctx->stream;
    FV_HIP(hipSetDevice(h->ctx->device));
    if (row_ptr)
      FV_HIP(hipMemcpyAsync(row_ptr, L.rp_c, sizeof(int) * (L.n + 1), hipMemcpyDeviceToHost, s));
    if (col && L.m)
      FV_HIP(hipMemcpyAsync(col, L.col_c, sizeof(int) * L.m, hipMemcpyDeviceToHost, s));
    if (w && L.m)
      FV_HIP(hipMemcpyAsync(w, L.w_c, sizeof(double) * L.m, hipMemcpyDeviceToHost, s));
    if (q && L.q_c)
      FV_HIP(hipMemcpyAsync(q, L.q_c, sizeof(int) * L.n, hipMemcpyDeviceToHost, s));
    if (colour && L.colour_c)
      FV_HIP(hipMemcpyAsync(colour, L.colour_c, sizeof(int) * L.n, hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    return FV_OK;
  })
}

void fv_free_hierarchy(fv_hierarchy* h) {
  if (!h) return;
  (void)hipSetDevice(h->ctx->device);
  (void)hipStreamSynchronize(h->ctx->stream);
  fv::free_hierarchy(h);
}

static fv_status check_solve_opts(const fv_solve_opts* o) {
  if (o->prec != FV_PREC_FP64 && o->prec != FV_PREC_FP32_MIXED) return FV_E_INVALID;
  if (!(o->tol_cos >= 0.0) || !(o->tol_res >= 0.0) || !(o->tol_coarse >= 0.0))
    return FV_E_INVALID;
  if (!(o->omega > 0.0 && o->omega < 2.0)) return FV_E_INVALID;
  if (o->max_gs < 0 || o->max_pi < 0 || o->max_outer < 0 || o->max_coarsest < 0)
    return FV_E_INVALID;
  if (o->replay && (o->replay_len < 0 || o->replay_len > FV_SCHEDULE_CAP)) return FV_E_INVALID;
  for (int k = 0; o->replay && k < o->replay_len; ++k)
    if (o->replay[k] < 0) return FV_E_INVALID;
  return FV_OK;
}

fv_status fv_fiedler_solve(fv_context* ctx, const fv_hierarchy* h, const fv_solve_opts* opts,
                           double* x_out, int32_t x_on_device, double* lambda_out,
                           fv_solve_stats* stats) {
  if (!ctx || !h || !x_out || h->ctx != ctx) return FV_E_INVALID;
  fv_solve_opts o;
  fv_solve_opts_default(&o);
  if (opts) o = *opts;
  fv_status st = check_solve_opts(&o);
  if (st != FV_OK) return st;
  FV_GUARD({
    FV_HIP(hipSetDevice(ctx->device));
    return fv::solve_one(ctx, h, &o, x_out, x_on_device, lambda_out, stats);
  })
}

fv_status fv_fiedler_solve_noalloc(fv_context* ctx, const fv_hierarchy* h,
                                   const fv_solve_opts* opts, double* x_out,
                                   int32_t x_on_device, double* lambda_out,
                                   fv_solve_stats* stats) {
  if (!ctx || !h || !x_out || h->ctx != ctx) return FV_E_INVALID;
  fv_solve_opts o;
  fv_solve_opts_default(&o);
  if (opts) o = *opts;
  fv_status st = check_solve_opts(&o);
  if (st != FV_OK) return st;
  FV_GUARD({
    FV_HIP(hipSetDevice(ctx->device));
    return fv::solve_noalloc(ctx, h, &o, x_out, x_on_device, lambda_out, stats);
  })
}

void fv_batch_opts_default(fv_batch_opts* o) {
  if (o) std::memset(o, 0, sizeof(*o));
}

fv_status fv_fiedler_solve_batch(fv_context* ctx, int32_t count, const fv_hierarchy* const* h,
                                 const fv_solve_opts* opts, double* const* x_out,
                                 int32_t x_on_device, double* lambda_out, fv_solve_stats* stats,
                                 fv_status* item_status) {
  return fv_fiedler_solve_batch_ex(ctx, count, h, opts, nullptr, x_out, x_on_device, lambda_out,
                                   stats, item_status);
}

fv_status fv_fiedler_solve_batch_ex(fv_context* ctx, int32_t count,
                                    const fv_hierarchy* const* h, const fv_solve_opts* opts,
                                    fv_batch_opts* batch, double* const* x_out,
                                    int32_t x_on_device, double* lambda_out,
                                    fv_solve_stats* stats, fv_status* item_status) {
  if (!ctx || count < 0 || (count > 0 && (!h || !x_out))) return FV_E_INVALID;
  for (int k = 0; k < count; ++k)
    if (!h[k] || !x_out[k] || h[k]->ctx != ctx) return FV_E_INVALID;
  fv_solve_opts o;
  fv_solve_opts_default(&o);
  if (opts) o = *opts;
  fv_status st = check_solve_opts(&o);
  if (st != FV_OK) return st;
  if (o.replay) return FV_E_INVALID;
  FV_GUARD({
    FV_HIP(hipSetDevice(ctx->device));
    hipStream_t s = o.stream ? static_cast<hipStream_t>(o.stream) : ctx->stream;
    if (batch && (batch->autotune < 0 || batch->autotune > 2 || batch->lds_bytes < 0))
      return FV_E_INVALID;
    return fv::solve_batch(ctx, count, h, &o, batch, x_out, x_on_device, lambda_out, stats,
                           item_status, s);
  })
}

fv_status fv_spectral_partition(fv_context* ctx, const fv_csr* graph,
                                const fv_hier_opts* hopts, const fv_solve_opts* sopts,
                                const fv_partition_opts* popts, int32_t* part_out,
                                int32_t part_on_device, fv_partition_stats* stats) {
  if (!ctx || !graph || !popts || !part_out) return FV_E_INVALID;
  if (popts->parts < 2 || (popts->parts & (popts->parts - 1)) || popts->cut < 0 ||
      popts->cut > 1 || graph->n < 2)
    return FV_E_INVALID;
  fv_hier_opts ho;
  fv_hier_opts_default(&ho);
  if (hopts) ho = *hopts;
  fv_solve_opts o;
  fv_solve_opts_default(&o);
  if (sopts) o = *sopts;
  fv_status st = check_solve_opts(&o);
  if (st != FV_OK) return st;
  if (o.replay) return FV_E_INVALID;
  FV_GUARD({
    FV_HIP(hipSetDevice(ctx->device));
    return fv::spectral_partition(ctx, graph, &ho, &o, popts, part_out, part_on_device, stats);
  })
}

}  // extern "C"
