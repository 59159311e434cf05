// Internal declarations shared by the library's translation units (host and
// device).  Not part of the public ABI (include/fiedler.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "fiedler.h"

namespace fv {

// ---------------------------------------------------------------------------
// Errors: HIP failures and status-carrying errors are C++ exceptions inside
// the library and become fv_status at the C boundary.
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
  fv_status st;
  Error(fv_status s, const std::string& what) : std::runtime_error(what), st(s) {}
};

#define FV_HIP(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      throw ::fv::Error(e_ == hipErrorOutOfMemory ? FV_E_NOMEM : FV_E_DEVICE,        \
                        std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

// ---------------------------------------------------------------------------
// Launch geometry.
// ---------------------------------------------------------------------------
constexpr int kBlock = 256;    // threads per block of the multi-workgroup row passes
constexpr int kWGSolo = 512;  // engine threads for the small levels of one graph
constexpr int kWGBatch = 512;  // engine threads per graph of a batch
constexpr size_t kSoloLds = 144 * 1024;  // engine LDS for one graph's level vector
constexpr size_t kBatchLds = 64 * 1024;  // per graph of a batch
constexpr int kNP = 5;         // FP64 partial sums carried by a refinement pass
constexpr int kXCD = 8;        // accelerator complex dies on MI355X


// ---------------------------------------------------------------------------
// Device-resident solve state of one graph (scalars of the current phase).
// ---------------------------------------------------------------------------
struct DevState {
  double mu;      // pending normalisation of the stored vector: xhat = (x - mu) * inv_s
  double inv_s;
  double rho;     // shift of the next smoothing sweep
  double cos;     // cosine of the last step
  double tol;     // 1 - tol_cos threshold is (1 - tol)
  double lambda;  // finest Rayleigh quotient
  double res;     // finest residual
  double sumsq;   // sum of xhat^2 in the Rayleigh pass
  double xmax;    // max |xhat|
  double sign;    // output sign
  int done;       // current phase finished
  int iters;      // steps executed in the current phase
  int cap;        // step limit of the current phase
  int forced;     // 1: run exactly cap steps
  int cur;        // which ping-pong buffer holds the iterate
  unsigned counter;  // last-block-done counter
  int sign_idx;   // first (canonical) index with |x_i| >= 1e-3 max|x|
  int err;
  int halt;       // finest residual reached the tolerance: later phases do nothing
};

// Per-level descriptor as the kernels see it (solve order: rows of one colour
// contiguous, ascending original index inside a colour).
// The finest rounds' early exit (fv_solve_opts.early_exit): true when the
// residual res, multiplied round after round by its last reduction factor
// res / res_prev, falls to tol within `left` more rounds (the products taken
// one at a time in double); false when it did not fall.
__host__ __device__ inline bool can_reach(double res, double res_prev, double tol, int left) {
  if (!(res < res_prev)) return false;
  const double q = res / res_prev;
  double v = res;
  for (int k = 0; k < left; ++k) {
    v *= q;
    if (v <= tol) return true;
  }
  return false;
}

struct LevelDesc {
  int n;
  int ncol;
  long long m;
  const int* rp;
  const int* col;
  const double* w64;
  const float* w32;
  const int* cptr;   // colour row ranges, ncol + 1 entries
  const int* qs;     // aggregate (solve order of the next level) of each row; null on coarsest
  const int* perm;   // original index -> solve position
  const int* iperm;  // solve position -> original index
  double sigma;
  // Slot-major (ELL) blocks of some colours of the solve-order matrix (null:
  // none): colour c's block starts at the host's Level::ecoff[c]; entry k of
  // its row r0 + i at k * rows + i (CSR order; padding slots hold column -1
  // and weight 0).
  const int* ecol;
  const double* ew64;
  const float* ew32;
};

// One graph's work for the one-workgroup engine.
struct GraphTask {
  const LevelDesc* lv;  // device array, levels 0..J
  int J;                // coarsest level
  int stop;             // finest level refined by the engine
  int prec;             // fv_precision
  int finalize;         // 1: stop == 0 and the engine also does the Rayleigh quotient,
                        //    finest repeats and the output
  void* xa;             // two vector buffers of nmax entries (8-byte capacity each)
  void* xb;
  double* lx;           // FP64 scratch of nmax entries
  double* x_out;        // canonical FP64 output (finalize), device pointer
  DevState* st;         // where the engine leaves its scalars
  const int* replay;    // device array or null
  int replay_len;
  int* sched;           // device schedule output, FV_SCHEDULE_CAP entries
  int* sched_len;
  int out_buf;          // 0: iterate ends in xa, 1: in xb (written by the engine)
  unsigned long long seed;
  double tol_cos, tol_res, omega, tol_coarse;
  int max_gs, max_pi, max_outer, max_coarsest;
  int early_exit;       // fv_solve_opts.early_exit
  long long work;       // ordering key (bigger first)
};

// ---------------------------------------------------------------------------
// Host-side level storage.
// ---------------------------------------------------------------------------
struct Level {
  int n = 0;
  long long m = 0;
  int ncol = 0;
  double sigma = 0.0;
  // canonical numbering
  int* rp_c = nullptr;
  int* col_c = nullptr;
  double* w_c = nullptr;
  int* q_c = nullptr;
  int* colour_c = nullptr;
  // solve order
  int* rp = nullptr;
  int* col = nullptr;
  double* w64 = nullptr;
  float* w32 = nullptr;
  int* cptr = nullptr;
  std::vector<int> cptr_h;
  std::vector<long long> cnnz_h;  // solve-order row pointer at each colour start (and m)
  int* perm = nullptr;
  int* iperm = nullptr;
  int* qs = nullptr;
  // Slot-major (ELL) blocks for the smoothing sweeps: ew slots per row (0:
  // none); ecoff[c] the slot offset of colour c's block, or -1 when colour c
  // is swept from CSR; eslots the slots of all blocks.
  int ew = 0;
  std::vector<long long> ecoff;
  long long eslots = 0;
  int* ecol = nullptr;
  double* ew64 = nullptr;
  float* ew32 = nullptr;
  int ell_width(int c) const { return c >= 0 && c < (int)ecoff.size() && ecoff[c] >= 0 ? ew : 0; }
};

// The device descriptor of a level.
inline LevelDesc desc_of(const Level& F) {
  LevelDesc d;
  std::memset(&d, 0, sizeof(d));
  d.n = F.n;
  d.ncol = F.ncol;
  d.m = F.m;
  d.rp = F.rp;
  d.col = F.col;
  d.w64 = F.w64;
  d.w32 = F.w32;
  d.cptr = F.cptr;
  d.qs = F.qs;
  d.perm = F.perm;
  d.iperm = F.iperm;
  d.sigma = F.sigma;
  d.ecol = F.ecol;
  d.ew64 = F.ew64;
  d.ew32 = F.ew32;
  return d;
}

}  // namespace fv

// Opaque handles of the public ABI.
namespace fv {
// Workspace of the single-graph solve: device scratch (grown on demand,
// counted against the budget), a small pinned host buffer for read-backs, and
// a mapped, coherent host buffer that the finishing kernels write the phase's
// stop flag and the finest residual into (hflags_dev is its device address).
// The context owns one; each serving worker owns its own so that solves on
// different streams never share it.
struct SolveScratch {
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int* pinned = nullptr;
  int* hflags = nullptr;
  int* hflags_dev = nullptr;
  // Events of a solve: start and end of the timed region, the two chunk
  // events of the early stop, and the event after a residual pass.
  hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr, ev_chunk[2] = {nullptr, nullptr},
             ev_res = nullptr;
  // Event pairs of the opt-in per-launch timing (created on first use).
  std::vector<hipEvent_t> tev;
};
}  // namespace fv

struct fv_context {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;   // 0 = unbounded
  size_t in_use = 0;   // bytes held by live hierarchies and workspaces
  std::mutex mu;       // guards in_use (the server's threads share the context)
  fv::SolveScratch scratch;  // workspace of fv_fiedler_solve
  void* bgraph = nullptr;    // the last captured batch launch (fv_fiedler_solve_batch_ex)
  // Device blocks released by finished work, kept for reuse so that building
  // and freeing hierarchies does not pay hipMalloc / hipFree every time.
  std::multimap<size_t, void*> cache;      // block size -> block
  std::unordered_map<void*, size_t> live;  // block handed out -> block size
  size_t cached = 0;
  std::mutex cache_mu;
  // Small pinned host buffers for read-backs (kPinBytes each), reused so that
  // builds on concurrent streams do not pay hipHostMalloc / hipHostFree (which
  // synchronises) every time; freed with the context.
  std::vector<void*> pins;
  std::mutex pin_mu;
};

struct fv_hierarchy {
  fv_context* ctx = nullptr;
  uint64_t serial = 0;  // unique per built hierarchy in the process (never reused)
  int levels = 0;
  fv::Level lv[FV_MAX_LEVELS];
  fv::LevelDesc* d_desc = nullptr;  // device copy of the level descriptors
  size_t bytes = 0;
};

namespace fv {

// Device blocks from the context's cache (not counted against the budget).
// block_put requires that no queued or running device work still uses the
// block: the caller has synchronised the streams that used it.
void* block_get(fv_context* ctx, size_t bytes);
void block_put(fv_context* ctx, void* p);
void block_trim(fv_context* ctx);  // hipFree every cached block

// A pinned host buffer of kPinBytes from the context's pool.  pin_put
// requires that no copy into or out of it is still queued: it synchronises
// stream s (the stream that used it) before returning the buffer.
constexpr size_t kPinBytes = 4096;
void* pin_get(fv_context* ctx);
void pin_put(fv_context* ctx, void* p, hipStream_t s);
void pin_trim(fv_context* ctx);

// Device allocation accounted against the context budget (blocks from the
// cache; dev_free has block_put's precondition).
void* dev_alloc(fv_context* ctx, size_t bytes, size_t* counter);
void dev_free(fv_context* ctx, void* p, size_t bytes, size_t* counter);
void budget_reserve(fv_context* ctx, size_t bytes);
void budget_release(fv_context* ctx, size_t bytes);

// Setup (setup.hip).
fv_hierarchy* build_hierarchy(fv_context* ctx, const fv_csr* L, const fv_hier_opts* o,
                              hipStream_t s);
// sync_device: wait for every stream first (solves on any stream may still
// read the levels); false when the caller knows no queued work uses h.
void free_hierarchy(fv_hierarchy* h, bool sync_device = true);
size_t hierarchy_nmax(const fv_hierarchy* h);

// Solve (solve.hip).
fv_status solve_one(fv_context* ctx, const fv_hierarchy* h, const fv_solve_opts* o,
                    double* x_out, int x_on_device, double* lambda_out, fv_solve_stats* stats);
// The same on a given stream and workspace (the server's workers).
fv_status solve_one_with(fv_context* ctx, SolveScratch& sc, const fv_hierarchy* h,
                         const fv_solve_opts* o, double* x_out, int x_on_device,
                         double* lambda_out, fv_solve_stats* stats, hipStream_t s);
void release_scratch(fv_context* ctx, SolveScratch& sc);
// Pinned and mapped host buffers and events of a workspace (created once).
void scratch_host_init(SolveScratch& sc);
// Device address of the fixed scratch of the allocation-free solve on the
// current device (looked up once per device; fv_context_create calls it).
void* noalloc_scratch_init(int device);
// fv_fiedler_solve without any allocation: the workspace is the fixed scratch.
fv_status solve_noalloc(fv_context* ctx, const fv_hierarchy* h, const fv_solve_opts* o,
                        double* x_out, int x_on_device, double* lambda_out,
                        fv_solve_stats* stats);
fv_status solve_batch(fv_context* ctx, int count, const fv_hierarchy* const* h,
                      const fv_solve_opts* o, fv_batch_opts* bo, double* const* x_out,
                      int x_on_device, double* lambda_out, fv_solve_stats* stats,
                      fv_status* item_status, hipStream_t s);
void release_batch_graph(fv_context* ctx);
// Recursive spectral bisection (partition.hip).
fv_status spectral_partition(fv_context* ctx, const fv_csr* g, const fv_hier_opts* ho,
                             const fv_solve_opts* so, const fv_partition_opts* po,
                             int32_t* part_out, int part_on_device, fv_partition_stats* st);
size_t solve_workspace_bytes(size_t nmax, int maxcol);

// Algorithmic bytes of one refinement pass over a level.
inline long long pass_bytes(int n, long long m, int prec) {
  return prec == FV_PREC_FP32_MIXED ? 8LL * m + 4LL * (n + 1) + 8LL * n
                                    : 12LL * m + 4LL * (n + 1) + 16LL * n;
}

}  // namespace fv
