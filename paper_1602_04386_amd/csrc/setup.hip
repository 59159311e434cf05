// Setup phase on the device (Algorithm 3, Step 1; Algorithm 1): input
// validation, heavy-edge matching, aggregation, Galerkin coarse graphs,
// first-fit colouring for the multicolour smoother and the colour-ordered copy
// of every level that the refinement kernels read.
#include <hip/hip_runtime.h>

#include <atomic>

#include <algorithm>
#include <climits>
#include <cmath>
#include <initializer_list>
#include <type_traits>

#include "fv_device.h"
#include "fv_internal.h"

namespace fv {

// ---------------------------------------------------------------------------
// Temporary device buffers of one build (not counted against the budget).
// ---------------------------------------------------------------------------
struct Tmp {
  fv_context* ctx;
  hipStream_t s;
  std::vector<void*> ptrs;
  template <class T>
  T* get(size_t count) {
    ptrs.push_back(block_get(ctx, std::max<size_t>(count, 1) * sizeof(T)));
    return static_cast<T*>(ptrs.back());
  }
  ~Tmp() {
    (void)hipStreamSynchronize(s);  // the build's work is the only user
    for (void* p : ptrs) block_put(ctx, p);
  }
};

static inline int nblk(long long n, int b = kBlock) { return (int)std::max<long long>(1, (n + b - 1) / b); }

// Sets *flag to 1: one plain store per wave, by the lowest of the lanes that
// reach this call.  Every writer stores the same value, so no read-modify-write
// is needed; same-address atomics from thousands of waves serialise and made a
// round over a million vertices take ~180 us.
__device__ inline void wave_flag(int* flag) {
  const unsigned long long m = __ballot(1);
  if ((threadIdx.x & 63) == __ffsll((long long)m) - 1) *flag = 1;
}

// Round kernels walk the vertices with a grid-stride loop over at most
// kRoundGrid blocks: one vertex per thread up to a million vertices, since a
// working round is a chain of dependent loads per vertex (4096 instead of 1024
// blocks cut the rounds' kernel time per build by ~0.16 ms), while a round
// that exits at once still costs only its launch.
constexpr int kRoundGrid = 4096;
static inline int round_grid(int n) { return std::min(nblk(n), kRoundGrid); }



// ---------------------------------------------------------------------------
// Exclusive scan of f(0..n-1) (int64 accumulation).
// ---------------------------------------------------------------------------
constexpr int kScanPer = 8;
constexpr int kScanTile = kBlock * kScanPer;

__device__ inline long long block_inclusive_scan_ll(long long v, long long* lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    long long t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  if (lane == 63) lds[wid] = v;
  __syncthreads();
  long long pre = 0;
  for (int w = 0; w < wid; ++w) pre += lds[w];
  __syncthreads();
  return v + pre;
}

template <class F>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(F f, int n, long long* bsum) {
  __shared__ long long lds[kBlock / 64];
  long long s = 0;
  const int base = blockIdx.x * kScanTile;
  for (int k = threadIdx.x; k < kScanTile; k += kBlock) {
    int i = base + k;
    if (i < n) s += f(i);
  }
  s = block_sum_ll(s, lds);
  if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_scan_blocks(long long* bsum, int nb) {
  __shared__ long long lds[kBlock / 64];
  __shared__ long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += kBlock) {
    int i = base + threadIdx.x;
    long long v = i < nb ? bsum[i] : 0;
    long long inc = block_inclusive_scan_ll(v, lds);
    long long c = carry;
    if (i < nb) bsum[i] = c + inc - v;
    __syncthreads();
    if (threadIdx.x == kBlock - 1) carry = c + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

template <class F, class OUT>
__global__ __launch_bounds__(kBlock) void k_scan_apply(F f, int n, const long long* boff, OUT* out) {
  __shared__ long long lds[kBlock / 64];
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanPer;
  long long vals[kScanPer];
  long long s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    int i = base + k;
    vals[k] = i < n ? (long long)f(i) : 0;
    s += vals[k];
  }
  long long inc = block_inclusive_scan_ll(s, lds);
  long long run = boff[blockIdx.x] + inc - s;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    int i = base + k;
    if (i < n) out[i] = (OUT)run;
    run += vals[k];
  }
}

__global__ void k_write_total(const long long* src, int* dst) { *dst = (int)*src; }

// The whole scan in one block when n fits one tile: exclusive scan into out
// (if non-null), the total into *total and, when write_total, into out[n].
template <class F>
__global__ __launch_bounds__(kBlock) void k_scan_small(F f, int n, int* out, bool write_total,
                                                     long long* total) {
  __shared__ long long lds[kBlock / 64];
  const int base = threadIdx.x * kScanPer;
  long long vals[kScanPer];
  long long s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int i = base + k;
    vals[k] = i < n ? (long long)f(i) : 0;
    s += vals[k];
  }
  const long long inc = block_inclusive_scan_ll(s, lds);
  long long run = inc - s;
  if (out) {
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      const int i = base + k;
      if (i < n) out[i] = (int)run;
      run += vals[k];
    }
  }
  if (threadIdx.x == blockDim.x - 1) {
    *total = inc;
    if (out && write_total) out[n] = (int)inc;
  }
}

struct Scanner {
  Tmp* tmp = nullptr;
  long long* bsum = nullptr;
  int cap = 0;
  hipStream_t s = nullptr;
  long long* host = nullptr;  // pinned
  const long long* last = nullptr;
  // Queues the exclusive scan of f over [0, n) into out (if non-null) and,
  // when write_total, the total into out[n].  Nothing is read back.
  template <class F>
  void enqueue(F f, int n, int* out, bool write_total) {
    const int nb = std::max(1, (n + kScanTile - 1) / kScanTile);
    if (nb + 1 > cap) {
      cap = nb + 4;
      bsum = tmp->get<long long>(cap);
    }
    if (nb == 1) {
      k_scan_small<<<1, kBlock, 0, s>>>(f, n, out, write_total, bsum + 1);
      FV_HIP(hipGetLastError());
      last = bsum + 1;
      return;
    }
    k_scan_reduce<<<nb, kBlock, 0, s>>>(f, n, bsum);
    k_scan_blocks<<<1, kBlock, 0, s>>>(bsum, nb);
    if (out) {
      k_scan_apply<<<nb, kBlock, 0, s>>>(f, n, bsum, out);
      if (write_total) k_write_total<<<1, 1, 0, s>>>(bsum + nb, out + n);
    }
    FV_HIP(hipGetLastError());
    last = bsum + nb;
  }
  // enqueue, then waits for the stream and returns the total.
  template <class F>
  long long run(F f, int n, int* out, bool write_total) {
    enqueue(f, n, out, write_total);
    FV_HIP(hipMemcpyAsync(host, last, sizeof(long long), hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    return *host;
  }
};

struct FromArray {
  const int* a;
  __device__ int operator()(int i) const { return a[i]; }
};
struct LeaderFlag {
  const int* root;
  const int* minmem;
  __device__ int operator()(int v) const { return minmem[root[v]] == v ? 1 : 0; }
};
struct PermDeg {
  const int* rp;
  const int* iperm;
  __device__ int operator()(int i) const {
    int v = iperm[i];
    return rp[v + 1] - rp[v];
  }
};
struct BigRow {
  const int* tstart;
  __device__ int operator()(int i) const { return (tstart[i + 1] - tstart[i]) > 64 ? 1 : 0; }
};

// ---------------------------------------------------------------------------
// Small utility kernels.
// ---------------------------------------------------------------------------
__global__ void k_fill_int(int* a, long long n, int v) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// Several int arrays filled by one launch (each fill of a level's scratch
// arrays was a launch of its own).
constexpr int kFillMax = 12;
struct FillSet {
  int* p[kFillMax];
  long long n[kFillMax];
  int v[kFillMax];
  int k;
};
__global__ void k_fill_multi(FillSet f) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (int a = 0; a < f.k; ++a)
    if (i < f.n[a]) f.p[a][i] = f.v[a];
}

struct FillItem {
  int* p;
  long long n;
  int v;
};
// Fills every listed array (p[0, n) = v) in one launch.
static void fill_multi(hipStream_t s, std::initializer_list<FillItem> items) {
  FillSet f{};
  long long nmax = 0;
  for (const FillItem& it : items) {
    if (f.k == kFillMax) throw Error(FV_E_DEVICE, "too many arrays for one fill");
    f.p[f.k] = it.p;
    f.n[f.k] = it.n;
    f.v[f.k] = it.v;
    ++f.k;
    nmax = std::max(nmax, it.n);
  }
  if (nmax > 0) k_fill_multi<<<nblk(nmax), kBlock, 0, s>>>(f);
}
__global__ void k_iota(int* a, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = i;
}
__global__ void k_f64_to_f32(const double* a, float* b, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// ---------------------------------------------------------------------------
// Input validation (Definition 2.1) and extraction of the weights W.
// flags: 1 structure, 2 values / Laplacian form, 4 symmetry, 8 isolated vertex.
// ---------------------------------------------------------------------------
__global__ void k_val_structure(int n, int nnz, const int* rp, const int* col, int* flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int a = rp[i], b = rp[i + 1];
  if (i == 0 && a != 0) atomicOr(flags, 1);
  if (i == n - 1 && b != nnz) atomicOr(flags, 1);
  if (a < 0 || b < a || b > nnz) {
    atomicOr(flags, 1);
    return;
  }
  for (int p = a; p < b; ++p) {
    int c = col[p];
    if (c < 0 || c >= n || (p > a && c <= col[p - 1])) {
      atomicOr(flags, 1);
      return;
    }
  }
}

__device__ inline int find_col(const int* rp, const int* col, int i, int j) {
  int lo = rp[i], hi = rp[i + 1] - 1;
  while (lo <= hi) {
    int mid = lo + ((hi - lo) >> 1);
    int c = col[mid];
    if (c == j) return mid;
    if (c < j) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

// G lanes per row (a group of consecutive lanes): lane j checks entries j,
// j + G, ... of row i (finite, off-diagonal weights positive, the mirror
// entry present with the same bits), so a row's mirror searches run side by
// side; the group's first lane then adds the row's degree in CSR order and
// checks the diagonal against it.
template <int G>
__global__ void k_val_values(int n, const int* rp, const int* col, const double* val, int adj,
                             int* offdeg, int* flags) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(g / G), j = (int)(g % G);
  if (i >= n) return;
  const int a = rp[i], b = rp[i + 1];
  int f = 0;
  for (int p = a + j; p < b; p += G) {
    const double v = val[p];
    const int c = col[p];
    if (!isfinite(v)) f |= 2;
    if (c == i) {
      if (adj) f |= 2;
    } else {
      const double wij = adj ? v : -v;
      if (!(wij > 0.0)) f |= 2;
      const int t = find_col(rp, col, c, i);
      if (t < 0 || __double_as_longlong(val[t]) != __double_as_longlong(v)) f |= 4;
    }
  }
  if (j == 0) {
    bool has_diag = false;
    double diag = 0.0, deg = 0.0;
    int nd = 0;
    for (int p = a; p < b; ++p) {
      const double v = val[p];
      if (col[p] == i) {
        has_diag = true;
        diag = v;
      } else {
        deg += adj ? v : -v;
        ++nd;
      }
    }
    if (!adj && b > a) {
      if (!has_diag) {
        f |= 2;
      } else {
        double tol = 1e-12 * (fabs(diag) > 1.0 ? fabs(diag) : 1.0);
        if (fabs(diag - deg) > tol) f |= 2;
      }
    }
    if (nd == 0) f |= 8;
    offdeg[i] = nd;
  }
  if (f) atomicOr(flags, f);
}

__global__ void k_extract(int n, const int* __restrict__ rp, const int* __restrict__ col,
                          const double* __restrict__ val, int adj, const int* __restrict__ rpw,
                          int* __restrict__ colw, double* __restrict__ ww) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int k = rpw[i];
  for (int p = rp[i]; p < rp[i + 1]; ++p) {
    int j = col[p];
    if (j == i) continue;
    colw[k] = j;
    ww[k] = adj ? val[p] : -val[p];
    ++k;
  }
}

// ---------------------------------------------------------------------------
// Shift sigma = 2 max_i d_i, d_i summed in row order.
// ---------------------------------------------------------------------------
// Rows are strided over at most kDegreeGrid blocks: one atomicMax per block,
// and atomics on one address serialise (one block per 256 rows of a
// 1M-vertex level took ~50 us, nearly all of it in the atomics).  The same
// pass finds the longest row (*lmax), which decides the level's ELL copy.
constexpr int kDegreeGrid = 512;

__global__ __launch_bounds__(kBlock) void k_degree_max(int n, const int* rp, const double* w,
                                                     unsigned long long* dmax,
                                                     unsigned long long* lmax) {
  __shared__ double lds[kBlock / 64];
  double m = 0.0, len = 0.0;
  // The next row's pointers are requested before this row is summed, and a
  // row's weights eight at a time before any is added (in row order).
  const int stride = gridDim.x * blockDim.x;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int a = 0, e = 0;
  if (i < n) {
    a = rp[i];
    e = rp[i + 1];
  }
  for (; i < n; i += stride) {
    int an = 0, en = 0;
    if (i + stride < n) {
      an = rp[i + stride];
      en = rp[i + stride + 1];
    }
    double d = 0.0;
    for (int p = a; p < e; p += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = w[min(p + u, e - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (p + u < e) d += v[u];
    }
    m = fmax(m, d);
    len = fmax(len, (double)(e - a));
    a = an;
    e = en;
  }
  m = block_max(m, lds);
  len = block_max(len, lds);
  if (threadIdx.x == 0) {
    atomicMax(dmax, (unsigned long long)__double_as_longlong(m));
    atomicMax(lmax, (unsigned long long)len);
  }
}

// ELL blocks (the sweeps' storage for the rows of regular enough colours).  On
// a level that the multi-workgroup sweeps visit (more than kEllMinRows rows)
// whose longest row has at most kEllMaxWidth entries, every row gets that
// length rounded up to a multiple of 4 slots, and each of the first
// kEllMaxCol colours gets a block when its padding is cheap: at most an eighth
// more slots than entries, or at most kEllPadBytes of padding read per launch
// (FP32 index and weight).  A CSR tile launch pays a dependent load phase
// (the row pointers), and on dense rows more (one per staging chunk), that the
// ELL launch does not, worth about that many bytes at the bandwidth such
// launches reach.  So large near-regular colours (grid levels) and the small
// dense colours of irregular levels (the last colours of a random geometric
// graph) take ELL; the large colours of irregular levels keep CSR.
constexpr int kEllMinRows = 8192;
constexpr int kEllMaxWidth = 32;
constexpr int kEllMaxCol = 32;
constexpr long long kEllPadBytes = 8LL << 20;

// The ELL blocks of one level: slot width and, per colour, row range and slot
// offset (count colours with a block, in colour order).
struct EllBlocks {
  int count;
  int ew;
  int r0[kEllMaxCol];
  int rows[kEllMaxCol];
  long long off[kEllMaxCol];
};

// Decides a level's ELL blocks from its longest row and its colours' row and
// entry counts; fills F.ew, F.ecoff, F.eslots and B.  Blocks start at
// multiples of 64 slots.
static void ell_plan(Level& F, long long longest, EllBlocks& B) {
  B.count = 0;
  F.ew = 0;
  F.ecoff.assign(F.ncol, -1);
  F.eslots = 0;
  if (F.n <= kEllMinRows || longest < 1 || longest > kEllMaxWidth) return;
  const int ew = (int)((longest + 3) / 4) * 4;
  B.ew = ew;
  long long off = 0;
  for (int c = 0; c < std::min(F.ncol, kEllMaxCol); ++c) {
    const long long rows = F.cptr_h[c + 1] - F.cptr_h[c];
    const long long ent = F.cnnz_h[c + 1] - F.cnnz_h[c];
    const long long slots = (long long)ew * rows;
    if (rows <= 0 || off + slots >= INT_MAX) continue;
    if (!(slots <= ent + ent / 8 || (slots - ent) * 8 <= kEllPadBytes)) continue;
    F.ecoff[c] = off;
    B.r0[B.count] = F.cptr_h[c];
    B.rows[B.count] = (int)rows;
    B.off[B.count] = off;
    ++B.count;
    off += (slots + 63) / 64 * 64;
  }
  if (B.count == 0) return;
  F.ew = ew;
  F.eslots = off;
}

// Copies the rows of the ELL colours into their slot-major blocks: block y of
// the grid is ELL colour y; entry k of its row r0 + i goes to off + k * rows +
// i, the slots past the row's end hold column -1 and weight 0.
__global__ void k_ell_fill(EllBlocks B, const int* __restrict__ rp, const int* __restrict__ col,
                           const double* __restrict__ w64, const float* __restrict__ w32,
                           int* __restrict__ ecol, double* __restrict__ ew64,
                           float* __restrict__ ew32) {
  const int c = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int rows = B.rows[c];
  if (i >= rows) return;
  const int a = rp[B.r0[c] + i], e = rp[B.r0[c] + i + 1];
  for (int k = 0; k < B.ew; ++k) {
    const long long o = B.off[c] + (long long)k * rows + i;
    const bool in = a + k < e;
    ecol[o] = in ? col[a + k] : -1;
    ew64[o] = in ? w64[a + k] : 0.0;
    ew32[o] = in ? w32[a + k] : 0.0f;
  }
}

// Neighbours loaded per batch by the matching and colouring kernels: every
// column index and weight of a batch, then the state of those neighbours,
// before any is used (a row of up to eight neighbours costs two dependent
// loads instead of two per neighbour).
constexpr int kNbU = 8;

// v's best free neighbour in the strict edge order (-1: none).  Positions
// past the row end repeat its last entry: an edge is never strictly before
// itself, so a repeat changes nothing.
__device__ inline int pick_best(int v, int a, int b, const int* col, const double* w,
                                const int* mate) {
  int best = -1;
  double bw = 0.0;
  for (int pb = a; pb < b; pb += kNbU) {
    int u[kNbU], mu[kNbU];
    double wu[kNbU];
#pragma unroll
    for (int k = 0; k < kNbU; ++k) u[k] = col[min(pb + k, b - 1)];
#pragma unroll
    for (int k = 0; k < kNbU; ++k) wu[k] = w[min(pb + k, b - 1)];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < kNbU; ++k) mu[k] = mate[u[k]];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < kNbU; ++k)
      if (mu[k] == -1 && (best < 0 || edge_before(wu[k], v, u[k], bw, v, best))) {
        best = u[k];
        bw = wu[k];
      }
  }
  return best;
}

// pick_best by one wavefront for a long row: each lane keeps the best of
// every 64th entry, then the lanes' choices are reduced by the same strict
// order (a total order, so the result does not depend on how the entries
// were split).  Every lane of the wave calls it with the same v and returns
// the same vertex.
__device__ inline int pick_best_wave(int v, int a, int b, const int* col, const double* w,
                                     const int* mate) {
  int best = -1;
  double bw = 0.0;
  for (int p = a + (int)(threadIdx.x & 63); p < b; p += 64) {
    const int u = col[p];
    const double wu = w[p];
    if (mate[u] == -1 && (best < 0 || edge_before(wu, v, u, bw, v, best))) {
      best = u;
      bw = wu;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const int ob = __shfl_xor(best, off, 64);
    const double ow = __shfl_xor(bw, off, 64);
    if (ob >= 0 && (best < 0 || edge_before(ow, v, ob, bw, v, best))) {
      best = ob;
      bw = ow;
    }
  }
  return best;
}

// A level is dense for the one-workgroup kernels when its rows average at
// least this many entries: each row is then scanned by a whole wavefront
// instead of one thread (coarse levels of random graphs grow dense: on an
// 11k-vertex Erdos-Renyi graph a 517-vertex level has 81 neighbours per
// vertex and 27 colours, and one thread per row took milliseconds).
constexpr int kDenseRow = 24;
__host__ __device__ inline bool dense_level(int n, long long m) {
  return m >= (long long)kDenseRow * n;
}

// ---------------------------------------------------------------------------
// Heavy-edge matching by locally dominant rounds: every free vertex points at
// its best free neighbour in the strict edge order; mutual pointers match.
// Under a strict total order this yields the greedy matching that takes the
// edges from heaviest down.  mate: -1 free, -2 free without free neighbours.
// ---------------------------------------------------------------------------
// Rounds are launched in batches; round r > 0 returns at once when round r - 1
// left no vertex pending (prev points at that round's flag).  Rounds after the
// last productive one change nothing either way.
__global__ void k_match_pick(int n, const int* rp, const int* col, const double* w,
                             const int* mate, int* ptr, const int* prev) {
  if (prev && *prev == 0) return;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    if (mate[v] != -1) continue;
    ptr[v] = pick_best(v, rp[v], rp[v + 1], col, w, mate);
  }
}

__global__ void k_match_commit(int n, int* mate, const int* ptr, int* active, const int* prev) {
  if (prev && *prev == 0) return;
  bool pending = false;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    if (mate[v] != -1) continue;
    int u = ptr[v];
    if (u < 0) {
      mate[v] = -2;
    } else if (ptr[u] == v) {
      mate[v] = u;
    } else {
      pending = true;
    }
  }
  if (__ballot(pending) != 0ULL && (threadIdx.x & 63) == 0) *active = 1;
}

// The whole matching of a small level in one workgroup: the same pick and
// commit rounds, separated by barriers instead of kernel boundaries.
constexpr int kLocalBlock = 1024;
constexpr int kLocalMaxN = 4096;

__global__ __launch_bounds__(kLocalBlock) void k_match_local(int n, const int* rp, const int* col,
                                                           const double* w, int* mate, int* ptr,
                                                           int* err) {
  __shared__ int pending;
  const bool dense = dense_level(n, rp[n]);
  const int wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  for (int v = threadIdx.x; v < n; v += blockDim.x) mate[v] = -1;
  __syncthreads();
  for (int round = 0;; ++round) {
    if (dense) {
      for (int v = wave; v < n; v += nwave) {
        if (mate[v] != -1) continue;  // uniform over the wave
        const int b = pick_best_wave(v, rp[v], rp[v + 1], col, w, mate);
        if ((threadIdx.x & 63) == 0) ptr[v] = b;
      }
    } else {
      for (int v = threadIdx.x; v < n; v += blockDim.x) {
        if (mate[v] != -1) continue;
        ptr[v] = pick_best(v, rp[v], rp[v + 1], col, w, mate);
      }
    }
    if (threadIdx.x == 0) pending = 0;
    __syncthreads();
    for (int v = threadIdx.x; v < n; v += blockDim.x) {
      if (mate[v] != -1) continue;
      const int u = ptr[v];
      if (u < 0) mate[v] = -2;
      else if (ptr[u] == v) mate[v] = u;
      else pending = 1;
    }
    __syncthreads();
    if (!pending) break;
    if (round > n) {  // cannot happen under a strict order; never spin
      if (threadIdx.x == 0) *err = 1;
      break;
    }
    __syncthreads();
  }
}

// Smallest colour >= 0 that no neighbour in col[a, b) has in c (-1: none).
template <class IP, class CP>
__device__ inline int first_fit(int a, int b, IP col, CP c) {
  for (int base = 0;; base += 64) {
    unsigned long long mask = 0;
    for (int p = a; p < b; ++p) {
      const int k = c[col[p]];
      if (k >= base && k < base + 64) mask |= 1ULL << (k - base);
    }
    if (mask != ~0ULL) return base + __builtin_ctzll(~mask);
  }
}

// A batch of kNbU neighbours for the colouring kernels: all column indices,
// then all their colours.  Positions past the row end repeat its last
// neighbour, which changes neither a wait test nor a set of used colours.
template <class IP, class CP>
__device__ inline void load_nb(int pb, int b, IP col, CP c, int (&u)[kNbU], int (&cu)[kNbU]) {
#pragma unroll
  for (int k = 0; k < kNbU; ++k) u[k] = col[min(pb + k, b - 1)];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < kNbU; ++k) cu[k] = c[u[k]];
  __builtin_amdgcn_sched_barrier(0);
}

// first_fit with batched loads: the colours below 64 that the neighbours
// use, as a bit mask; the rare full mask falls back to first_fit.
template <class IP, class CP>
__device__ inline int first_fit_batched(int a, int b, IP col, CP c) {
  unsigned long long mask = 0;
  for (int pb = a; pb < b; pb += kNbU) {
    int u[kNbU], cu[kNbU];
    load_nb(pb, b, col, c, u, cu);
#pragma unroll
    for (int k = 0; k < kNbU; ++k)
      if (cu[k] >= 0 && cu[k] < 64) mask |= 1ULL << cu[k];
  }
  return mask != ~0ULL ? __builtin_ctzll(~mask) : first_fit(a, b, col, c);
}

// One Jones-Plassmann test of uncoloured vertex v with row [a, b): returns
// true when an uncoloured neighbour of higher priority (ties: smaller index)
// makes v wait; otherwise *fit is v's first-fit colour.  The colours read for
// the test are final for every coloured neighbour (each has higher priority,
// and no lower-priority neighbour can be coloured before v), so the first fit
// is taken from the same loads.
template <class IP, class CP>
__device__ inline bool jp_try(int v, int a, int b, IP col, CP colour, uint32_t seed, int* fit) {
  const uint32_t pv = colour_priority(v, seed);
  bool wait = false;
  unsigned long long mask = 0;
  for (int pb = a; pb < b; pb += kNbU) {
    int u[kNbU], cu[kNbU];
    load_nb(pb, b, col, colour, u, cu);
#pragma unroll
    for (int k = 0; k < kNbU; ++k) {
      if (cu[k] < 0) {
        const uint32_t pu = colour_priority(u[k], seed);
        wait = wait || pu > pv || (pu == pv && u[k] < v);
      } else if (cu[k] < 64) {
        mask |= 1ULL << cu[k];
      }
    }
  }
  if (wait) return true;
  *fit = mask != ~0ULL ? __builtin_ctzll(~mask) : first_fit(a, b, col, colour);
  return false;
}

__device__ inline unsigned long long wave_or(unsigned long long m) {
  for (int off = 32; off > 0; off >>= 1) m |= __shfl_xor(m, off, 64);
  return m;
}

// first_fit by one wavefront (every lane of the wave calls it with the same
// row and gets the same colour): the lanes take every 64th entry, windows of
// 64 colours from `base` on.
template <class IP, class CP>
__device__ inline int first_fit_wave(int a, int b, IP col, CP c, int base) {
  for (;; base += 64) {
    unsigned long long mask = 0;
    for (int p = a + (int)(threadIdx.x & 63); p < b; p += 64) {
      const int k = c[col[p]];
      if (k >= base && k < base + 64) mask |= 1ULL << (k - base);
    }
    mask = wave_or(mask);
    if (mask != ~0ULL) return base + __builtin_ctzll(~mask);
  }
}

// jp_try by one wavefront (same v in every lane; same answer in every lane).
template <class IP, class CP>
__device__ inline bool jp_try_wave(int v, int a, int b, IP col, CP colour, uint32_t seed,
                                   int* fit) {
  const uint32_t pv = colour_priority(v, seed);
  bool wait = false;
  unsigned long long mask = 0;
  for (int p = a + (int)(threadIdx.x & 63); p < b; p += 64) {
    const int u = col[p];
    const int cu = colour[u];
    if (cu < 0) {
      const uint32_t pu = colour_priority(u, seed);
      wait = wait || pu > pv || (pu == pv && u < v);
    } else if (cu < 64) {
      mask |= 1ULL << cu;
    }
  }
  if (__ballot(wait) != 0ULL) return true;
  mask = wave_or(mask);
  *fit = mask != ~0ULL ? __builtin_ctzll(~mask) : first_fit_wave(a, b, col, colour, 64);
  return false;
}

// ---------------------------------------------------------------------------
// Two-colouring of a bipartite level (the optimal colouring when there is one;
// on a 5-point grid the red-black order).  A union-find forest with parities:
// word W[v] = 2 * parent(v) + (colour of v xor colour of its parent), a root
// holding 2 v.  Each edge {u, v} is united with "different colours": when the
// roots differ, the larger root is hooked under the smaller one by a
// compare-and-swap that succeeds only while it is still a root, with the link
// parity that makes u and v differ.  Parents only ever point to smaller
// indices, so the forest has no cycles, and a root's word changes once (when
// it is hooked), so a failed swap means another edge made progress.  Every
// parity relation, once stored, stays true (path compression stores a
// vertex's relation to an ancestor), so the end result does not depend on the
// order in which edges were united: a component's root is its smallest vertex
// (colour 0) and every vertex's colour is its parity to the root -- the unique
// two-colouring of a connected bipartite graph with that vertex at colour 0.
// An edge whose ends end up with equal colours (an odd cycle) marks the level
// as not bipartite.  Scope: the memory scope of the atomics (agent for a level
// spread over the grid, workgroup for one workgroup's LDS).
// ---------------------------------------------------------------------------
template <int Scope, class WP>
__device__ inline unsigned uf_find(WP W, unsigned x, unsigned* parity) {
  unsigned par = 0, cur = x;
  for (;;) {
    const unsigned w = __hip_atomic_load(&W[cur], __ATOMIC_RELAXED, Scope);
    if ((w >> 1) == cur) break;
    par ^= w & 1u;
    cur = w >> 1;
  }
  // x is not a root: store its relation to the root found (still an ancestor)
  if (cur != x) __hip_atomic_store(&W[x], (cur << 1) | par, __ATOMIC_RELAXED, Scope);
  *parity = par;
  return cur;
}

// Unites u and v as differently coloured; returns false when they are already
// in one tree with equal colours (an odd cycle).
template <int Scope, class WP>
__device__ inline bool uf_unite_diff(WP W, unsigned u, unsigned v) {
  for (;;) {
    unsigned pu, pv;
    unsigned ru = uf_find<Scope>(W, u, &pu);
    unsigned rv = uf_find<Scope>(W, v, &pv);
    if (ru == rv) return pu != pv;
    if (ru < rv) {
      const unsigned t = ru, tp = pu;
      ru = rv;
      pu = pv;
      rv = t;
      pv = tp;
    }
    unsigned expected = ru << 1;
    const unsigned desired = (rv << 1) | (pu ^ pv ^ 1u);
    if (__hip_atomic_compare_exchange_strong(&W[ru], &expected, desired, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, Scope))
      return true;
  }
}

// Multi-workgroup form: the same forest built in bulk-synchronous rounds
// (hooking and compression, after Shiloach and Vishkin) instead of
// concurrent unions.  Round: every tree root fu adjacent (through an edge
// {u, v} with f(u) = fu) to a tree with a smaller parent fv hooks under the
// smallest such fv, with the link parity p(u) ^ p(v) ^ 1 that makes u and v
// differ; then every vertex's path is compressed to its root.  Hooks only go
// to smaller indices (no cycles), roots change only in the hook kernel, and
// the rounds end when a hook kernel hooks nothing: one tree per component,
// rooted at its smallest vertex, whose colour is 0.  On a grid the first round
// already joins everything under vertex 0, but into paths as long as a row
// plus a column; compression therefore runs in launches of at most kBipHops
// jumps per vertex (each launch shortens every path by that factor, since it
// also follows the jumps other vertices stored).  A level with a triangle is
// not bipartite; it is recognised first and skips the rest.  An edge whose
// ends get equal colours (a longer odd cycle) sets bad as well.
constexpr int kBipHops = 32;

// bad = 1 when one of the first kTriRows rows shows a triangle: row v, its
// first neighbour u above v, and a common neighbour among the first kTriU
// entries of both rows.  A certificate, not a decision: a level whose
// triangles this misses goes through the hooking rounds and the edge check,
// which decide exactly.  One row per thread and no dependent loads inside the
// comparison (the old row-by-row sorted merge, one dependent load per step,
// took 211 us on the 4M-point random geometric graph).
constexpr int kTriU = 8;
constexpr int kTriRows = 1 << 16;

__global__ void k_bip_triangle(int n, const int* __restrict__ rp, const int* __restrict__ col,
                               int* bad) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  bool tri = false;
  if (v < n) {
    const int a0 = rp[v], a1 = rp[v + 1];
    int nv[kTriU];
#pragma unroll
    for (int k = 0; k < kTriU; ++k) {
      const int c = col[min(a0 + k, max(a1 - 1, 0))];  // unconditional: all loads in flight
      nv[k] = a0 + k < a1 ? c : -1;
    }
    int u = -1;
#pragma unroll
    for (int k = kTriU - 1; k >= 0; --k)
      if (nv[k] > v) u = nv[k];  // the smallest listed neighbour above v
    if (u >= 0) {
      const int b0 = rp[u], b1 = rp[u + 1];
      int nu[kTriU];
#pragma unroll
      for (int k = 0; k < kTriU; ++k) {
        const int c = col[min(b0 + k, max(b1 - 1, 0))];
        nu[k] = b0 + k < b1 ? c : -2;
      }
#pragma unroll
      for (int i = 0; i < kTriU; ++i)
#pragma unroll
        for (int j = 0; j < kTriU; ++j) tri = tri || nv[i] == nu[j];
    }
  }
  if (__ballot(tri) != 0ULL && (threadIdx.x & 63) == 0) *bad = 1;
}

__global__ void k_bip_init(int n, unsigned* W) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    W[v] = (unsigned)v << 1;
}

// One hooking step.  *work is set when this round has work for its
// compression launches: a root was hooked, or the previous round's
// compression left paths unfinished (prev_more).  The round has nothing to do
// when the previous one had no work (prev_work == 0), and the rounds are over
// once a round ends with *work == 0.
__global__ void k_bip_hook(int n, const int* __restrict__ rp, const int* __restrict__ col,
                           unsigned* W, const int* bad, int* work, const int* prev_work,
                           const int* prev_more) {
  if (*bad || (prev_work && *prev_work == 0)) return;  // uniform over the grid
  const bool pending = prev_more && *prev_more;
  bool any = false;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const unsigned wv = W[v];
    const unsigned fu = wv >> 1;
    if ((W[fu] >> 1) != fu) continue;  // v's parent is not a root (yet)
    unsigned best = fu, bpar = 0;
    for (int p = rp[v], e = rp[v + 1]; p < e; ++p) {
      const unsigned wu = W[col[p]];
      const unsigned fv = wu >> 1;
      if (fv < best) {
        best = fv;
        bpar = (wv ^ wu ^ 1u) & 1u;
      }
    }
    if (best < fu) {
      W[fu] = (best << 1) | bpar;  // one 32-bit word: parent and parity together
      any = true;
    }
  }
  if ((__ballot(any) != 0ULL || (pending && blockIdx.x == 0)) && (threadIdx.x & 63) == 0)
    *work = 1;
}

// Up to kBipHops jumps towards the root per vertex (roots do not change inside
// this kernel).  *more is set when some vertex has not reached its root;
// go: the flag that says this launch has work (the round hooked something,
// or the previous compression launch left paths unfinished).
__global__ void k_bip_compress(int n, unsigned* W, const int* bad, const int* go, int* more) {
  if (*bad || *go == 0) return;
  bool left = false;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    unsigned w = W[v];
    int h = 0;
    for (;; ++h) {
      const unsigned f = w >> 1;
      const unsigned wf = W[f];
      if ((wf >> 1) == f) break;
      if (h == kBipHops) {
        left = true;
        break;
      }
      w = (wf & ~1u) | ((w ^ wf) & 1u);
    }
    if (h > 0) W[v] = w;
  }
  if (__ballot(left) != 0ULL && (threadIdx.x & 63) == 0) *more = 1;
}

// Every vertex points at its root now: its colour is its parity bit.
__global__ void k_bip_check(int n, const int* __restrict__ rp, const int* __restrict__ col,
                            const unsigned* __restrict__ W, int* bad) {
  if (*bad) return;
  bool clash = false;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const unsigned w = W[v];
    for (int p = rp[v], e = rp[v + 1]; p < e; ++p) clash = clash || ((W[col[p]] ^ w) & 1u) == 0;
  }
  if (__ballot(clash) != 0ULL && (threadIdx.x & 63) == 0) *bad = 1;
}

__global__ void k_bip_commit(int n, const unsigned* __restrict__ W, int* colour, const int* bad) {
  if (*bad) return;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    colour[v] = (int)(W[v] & 1u);
}

// One-workgroup form over n vertices (W and colour in LDS or global memory):
// returns true and leaves the two-colouring in colour when the level is
// bipartite.  Every thread of the block must call; bad is a shared flag.
template <class IP, class CP, class WP>
__device__ bool two_colour_local(int n, IP rp, IP col, CP colour, WP W, int& bad) {
  if (threadIdx.x == 0) bad = 0;
  for (int v = threadIdx.x; v < n; v += blockDim.x) W[v] = (unsigned)v << 1;
  __syncthreads();
  for (int v = threadIdx.x; v < n; v += blockDim.x) {
    if (__hip_atomic_load(&bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
    for (int p = rp[v], e = rp[v + 1]; p < e; ++p) {
      const int u = col[p];
      if (u > v && !uf_unite_diff<__HIP_MEMORY_SCOPE_WORKGROUP>(W, (unsigned)v, (unsigned)u)) {
        __hip_atomic_store(&bad, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        break;
      }
    }
  }
  __syncthreads();
  if (bad) return false;  // uniform: read after the barrier
  for (int v = threadIdx.x; v < n; v += blockDim.x) {
    unsigned p;
    (void)uf_find<__HIP_MEMORY_SCOPE_WORKGROUP>(W, (unsigned)v, &p);
    colour[v] = (int)p;
  }
  __syncthreads();
  bool clash = false;
  for (int v = threadIdx.x; v < n; v += blockDim.x)
    for (int p = rp[v], e = rp[v + 1]; p < e; ++p) clash = clash || colour[col[p]] == colour[v];
  if (clash) bad = 1;
  __syncthreads();
  return !bad;
}

// The whole Jones-Plassmann colouring of a small level in one workgroup,
// then the iterated-greedy pass (cnew: scratch of n); *maxc receives the
// largest colour.  IP / CP are the pointer types of the CSR and of the two
// colour arrays (LDS when the level fits, global otherwise).
template <class IP, class CP, class WP>
__device__ void colour_local_body(int n, IP rp, IP col, uint32_t seed, int two, CP colour,
                                  CP cnew, WP W, int* maxc, int* err, int& waiting, int* lmax) {
  // With `two` (the finest level) a bipartite level takes its two-colouring
  // (W: n words of scratch, the same memory as cnew); first fit and the
  // iterated-greedy pass colour every other level.
  if (two && two_colour_local(n, rp, col, colour, W, waiting)) {
    int m = -1;
    for (int v = threadIdx.x; v < n; v += blockDim.x) m = max(m, colour[v]);
    m = block_max_int(m, lmax);
    if (threadIdx.x == 0) *maxc = m;
    return;
  }
  __syncthreads();
  for (int v = threadIdx.x; v < n; v += blockDim.x) colour[v] = -1;
  __syncthreads();
  // dense levels: one wavefront per row (lane 0 stores the wave's result)
  const bool dense = dense_level(n, rp[n]);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  for (int round = 0;; ++round) {
    if (threadIdx.x == 0) waiting = 0;
    __syncthreads();
    if (dense) {
      for (int v = wave; v < n; v += nwave) {
        if (colour[v] >= 0) continue;  // only this wave writes colour[v]
        int fit;
        if (jp_try_wave(v, rp[v], rp[v + 1], col, colour, seed, &fit)) {
          if (lane == 0) waiting = 1;
          continue;
        }
        if (lane == 0) colour[v] = fit;
      }
    } else {
      for (int v = threadIdx.x; v < n; v += blockDim.x) {
        if (colour[v] >= 0) continue;
        int fit;
        if (jp_try(v, rp[v], rp[v + 1], col, colour, seed, &fit)) {
          waiting = 1;
          continue;
        }
        colour[v] = fit;
      }
    }
    __syncthreads();
    if (!waiting) break;
    if (round > n) {
      if (threadIdx.x == 0) *err = 1;
      break;
    }
    __syncthreads();  // every thread has read `waiting` before it is reset
  }
  int m = -1;
  for (int v = threadIdx.x; v < n; v += blockDim.x) m = max(m, colour[v]);
  m = block_max_int(m, lmax);
  // One iterated-greedy pass (k_recolour_class, class by class in this block).
  for (int v = threadIdx.x; v < n; v += blockDim.x) cnew[v] = -1;
  __syncthreads();
  for (int c = m; c >= 0; --c) {
    if (dense) {
      for (int v = wave; v < n; v += nwave)
        if (colour[v] == c) {
          const int f = first_fit_wave(rp[v], rp[v + 1], col, cnew, 0);
          if (lane == 0) cnew[v] = f;
        }
    } else {
      for (int v = threadIdx.x; v < n; v += blockDim.x)
        if (colour[v] == c) cnew[v] = first_fit_batched(rp[v], rp[v + 1], col, cnew);
    }
    __syncthreads();
  }
  int m2 = -1;
  for (int v = threadIdx.x; v < n; v += blockDim.x) {
    colour[v] = cnew[v];
    m2 = max(m2, cnew[v]);
  }
  m2 = block_max_int(m2, lmax);
  if (threadIdx.x == 0) *maxc = m2;
}

// Bytes of dynamic LDS that k_colour_local stages a level into: row
// pointers, column indices and both colour arrays.  Levels whose CSR does
// not fit run on global memory.
__host__ __device__ inline size_t colour_local_lds(int n, long long m) {
  return 4 * ((size_t)n + 1) + 4 * (size_t)m + 8 * (size_t)n;
}
constexpr size_t kColourLocalLds = 144 * 1024;

// lds_bytes: the dynamic LDS the launch provides (0: none).  With the level
// in LDS every neighbour test is an LDS access instead of a dependent global
// load (the largest local level coloured in ~140 us on global memory).
__global__ __launch_bounds__(kLocalBlock) void k_colour_local(int n, long long m, const int* rp,
                                                            const int* col, uint32_t seed,
                                                            int two, int* colour, int* cnew,
                                                            int* maxc, int* err, int lds_bytes) {
  extern __shared__ __align__(16) unsigned char cl_dyn[];
  __shared__ int waiting;
  __shared__ int lmax[kLocalBlock / 64];
  using lint = __attribute__((address_space(3))) int*;
  using luint = __attribute__((address_space(3))) unsigned*;
  if (lds_bytes > 0 && colour_local_lds(n, m) <= (size_t)lds_bytes) {
    lint lrp = (lint)(reinterpret_cast<int*>(cl_dyn));
    lint lcol = lrp + (n + 1);
    lint lc = lcol + m;
    lint lnew = lc + n;
    for (int k = threadIdx.x; k <= n; k += blockDim.x) lrp[k] = rp[k];
    for (long long k = threadIdx.x; k < m; k += blockDim.x) lcol[k] = col[k];
    __syncthreads();
    colour_local_body(n, lrp, lcol, seed, two, lc, lnew, (luint)lnew, maxc, err, waiting, lmax);
    __syncthreads();
    for (int v = threadIdx.x; v < n; v += blockDim.x) colour[v] = lc[v];
  } else {
    colour_local_body(n, rp, col, seed, two, colour, cnew, reinterpret_cast<unsigned*>(cnew),
                      maxc, err, waiting, lmax);
  }
}

// Aggregates (Algorithm 1): pairs; an unmatched vertex joins the aggregate of
// its best neighbour; aggregates numbered by smallest member.
__global__ void k_agg_root(int n, const int* rp, const int* col, const double* w,
                           const int* mate, int* root, int* err) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int m = mate[v];
  if (m >= 0) {
    root[v] = v < m ? v : m;
    return;
  }
  int a = rp[v], b = rp[v + 1];
  if (a == b) {
    root[v] = v;
    return;
  }
  int best = col[a];
  double bw = w[a];
  for (int p = a + 1; p < b; ++p)
    if (edge_before(w[p], v, col[p], bw, v, best)) {
      best = col[p];
      bw = w[p];
    }
  int mb = mate[best];
  if (mb < 0) {
    wave_flag(err);
    root[v] = v;
    return;
  }
  root[v] = best < mb ? best : mb;
}

__global__ void k_agg_minmem(int n, const int* root, int* minmem) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) atomicMin(&minmem[root[v]], v);
}

__global__ void k_agg_q(int n, const int* root, const int* minmem, const int* id, int* q) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) q[v] = id[minmem[root[v]]];
}

// ---------------------------------------------------------------------------
// Iterated greedy (one pass): the classes of a first-fit colouring, from the
// highest colour down, are recoloured first-fit against the vertices already
// recoloured.  A class is an independent set, so one launch per class gives
// the sequential pass exactly, and the result never has more colours; the
// small last classes that first-fit leaves are mostly absorbed, each of which
// would cost a launch per sweep.
// ---------------------------------------------------------------------------
__global__ void k_recolour_class(int n, const int* __restrict__ rp, const int* __restrict__ col,
                                 const int* __restrict__ old, int* cnew, int c) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    if (old[v] == c) cnew[v] = first_fit_batched(rp[v], rp[v + 1], col, cnew);
}

// ---------------------------------------------------------------------------
// Jones-Plassmann rounds: a vertex takes the smallest colour absent among its
// neighbours once every neighbour of higher priority is coloured.  This equals
// sequential first-fit in priority order.
// ---------------------------------------------------------------------------
__global__ void k_colour_round(int n, const int* rp, const int* col, uint32_t seed, int* colour,
                               int* active, const int* prev) {
  if (prev && *prev == 0) return;  // uniform over the grid
  bool wait_any = false;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    if (colour[v] >= 0) continue;
    int fit;
    if (jp_try(v, rp[v], rp[v + 1], col, colour, seed, &fit)) {
      wait_any = true;
      continue;
    }
    colour[v] = fit;
  }
  if (__ballot(wait_any) != 0ULL && (threadIdx.x & 63) == 0) *active = 1;
}

// Largest colour: per-block maxima, then one block over those.
__global__ __launch_bounds__(kBlock) void k_max_blocks(int n, const int* a, int* bmax) {
  __shared__ int lds[kBlock / 64];
  int m = -1;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    m = max(m, a[v]);
  m = block_max_int(m, lds);
  if (threadIdx.x == 0) bmax[blockIdx.x] = m;
}

__global__ __launch_bounds__(kBlock) void k_max_final(int nb, const int* bmax, int* out) {
  __shared__ int lds[kBlock / 64];
  int m = -1;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) m = max(m, bmax[b]);
  m = block_max_int(m, lds);
  if (threadIdx.x == 0) *out = m;
}

// Solve order: rows sorted by colour, ascending original index inside a
// colour (a stable counting sort).  Block b counts its kBlock vertices per
// colour into cnt[c * nb + b]; an exclusive scan of cnt in that (colour-major)
// order gives every (colour, block) run its start; each vertex then adds the
// number of earlier vertices of its block with its colour.
__global__ __launch_bounds__(kBlock) void k_colour_block_count(int n, const int* colour, int ncol,
                                                             int nb, int* cnt) {
  extern __shared__ int hist[];
  for (int c = threadIdx.x; c < ncol; c += kBlock) hist[c] = 0;
  __syncthreads();
  const int v = blockIdx.x * kBlock + threadIdx.x;
  if (v < n) atomicAdd(&hist[colour[v]], 1);
  __syncthreads();
  for (int c = threadIdx.x; c < ncol; c += kBlock) cnt[(size_t)c * nb + blockIdx.x] = hist[c];
}

__global__ __launch_bounds__(kBlock) void k_colour_scatter(int n, const int* colour, int nb,
                                                         const int* off, int* perm, int* iperm) {
  __shared__ int sc[kBlock];
  const int v = blockIdx.x * kBlock + threadIdx.x;
  const int c = v < n ? colour[v] : -1;
  sc[threadIdx.x] = c;
  __syncthreads();
  if (v >= n) return;
  int r = 0;
  for (int t = 0; t < (int)threadIdx.x; ++t) r += sc[t] == c;
  const int p = off[(size_t)c * nb + blockIdx.x] + r;
  perm[v] = p;
  iperm[p] = v;
}

// cptr[c] = first solve-order row of colour c; cptr[ncol] = n.
__global__ void k_colour_ptr(int n, int ncol, int nb, const int* off, int* cptr) {
  for (int c = threadIdx.x; c <= ncol; c += blockDim.x) cptr[c] = c < ncol ? off[(size_t)c * nb] : n;
}

// Colour-ordered copy: row i of the solve order is original row iperm[i];
// columns are relabelled but keep their original order (so row sums add in
// the same order as in the original numbering).
// G lanes per row (a group of consecutive lanes): lane j of row i's group
// copies entries j, j + G, ... of the canonical row iperm[i] to solve-order
// row i, so the reads of a row and the writes of its copy are consecutive
// words across the group instead of one word per lane.
template <int G>
__global__ void k_solve_fill(int n, const int* __restrict__ rp_c, const int* __restrict__ col_c,
                             const double* __restrict__ w_c, const int* __restrict__ iperm,
                             const int* __restrict__ perm, const int* __restrict__ rp,
                             int* __restrict__ col, double* __restrict__ w64,
                             float* __restrict__ w32) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(g / G), j = (int)(g % G);
  if (i >= n) return;
  const int v = iperm[i];
  const int a = rp_c[v], b = rp_c[v + 1];
  const int k = rp[i] - a;
  for (int p = a + j; p < b; p += G) {
    col[k + p] = perm[col_c[p]];
    const double wv = w_c[p];
    w64[k + p] = wv;
    w32[k + p] = (float)wv;
  }
}

// Lanes per row of the row-group kernels: about one entry per lane of an
// average row, between 4 and 16.
static int row_group(long long rows, long long entries) {
  const long long mean = entries / std::max<long long>(rows, 1);
  return mean <= 4 ? 4 : mean <= 8 ? 8 : 16;
}

static void launch_solve_fill(int n, long long m, hipStream_t s, const int* rp_c,
                              const int* col_c, const double* w_c, const int* iperm,
                              const int* perm, const int* rp, int* col, double* w64, float* w32) {
  switch (row_group(n, m)) {
    case 4:
      k_solve_fill<4><<<nblk(4LL * n), kBlock, 0, s>>>(n, rp_c, col_c, w_c, iperm, perm, rp, col,
                                                        w64, w32);
      break;
    case 8:
      k_solve_fill<8><<<nblk(8LL * n), kBlock, 0, s>>>(n, rp_c, col_c, w_c, iperm, perm, rp, col,
                                                        w64, w32);
      break;
    default:
      k_solve_fill<16><<<nblk(16LL * n), kBlock, 0, s>>>(n, rp_c, col_c, w_c, iperm, perm, rp,
                                                          col, w64, w32);
  }
}

// ---- solve-order copies of the small levels, one workgroup per level -------
// The colour-ordered copy (stable counting sort by colour in 256-row
// segments, colour ranges, solve-order row pointers, relabelled CSR) of every
// level of at most kSmallCopyRows rows in one launch: the same arrays the
// multi-block kernels above produce (k_colour_block_count, the cell scan,
// k_colour_scatter, k_colour_ptr, the PermDeg scan, k_solve_fill), with the
// colours, counters, permutations and row pointers in LDS.  A level without
// colours (the coarsest) keeps its order.  The aggregate maps (k_qs) follow in
// a launch of their own, since they read the next level's permutation.
constexpr int kSmallCopyRows = 4096;
constexpr int kSmallCopyCells = 4096;  // colours x 256-row segments
constexpr int kSmallCopyThreads = 1024;
constexpr int kSmallCopyMax = 16;      // levels per launch

struct SmallCopy {
  int n, ncol;
  const int* colour;  // canonical colours, or null: one colour
  const int* rp_c;
  const int* col_c;
  const double* w_c;
  const int* q_c;        // aggregate of each row (k_qs_small), null on the coarsest level
  const int* perm_next;  // the next level's permutation (k_qs_small)
  int* perm;
  int* iperm;
  int* cptr;
  int* rp;
  int* col;
  double* w64;
  float* w32;
  int* qs;
};
struct SmallCopies {
  int count;
  SmallCopy lv[kSmallCopyMax];
};

// Dynamic LDS ints of a level: colours, counters (+1), iperm, perm, row pointers (+1).
__host__ __device__ inline int small_copy_ints(int n, int ncol) {
  const int nb = (n + kBlock - 1) / kBlock;
  return 4 * n + ncol * nb + 2;
}

// Exclusive scan over a[0, len) in place (len <= 4 * blockDim.x); returns the total.
__device__ inline int block_excl_scan4(int* a, int len, long long* lds) {
  const int base = 4 * (int)threadIdx.x;
  int v[4];
  long long sum = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = base + k < len ? a[base + k] : 0;
    sum += v[k];
  }
  __syncthreads();  // every value read before any is overwritten
  const long long inc = block_inclusive_scan_ll(sum, lds);
  long long run = inc - sum;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < len) a[base + k] = (int)run;
    run += v[k];
  }
  __shared__ int total;
  if (threadIdx.x == blockDim.x - 1) total = (int)inc;
  __syncthreads();
  return total;
}

__global__ __launch_bounds__(kSmallCopyThreads) void k_small_copy(SmallCopies S) {
  extern __shared__ int sm[];
  __shared__ long long lds[kSmallCopyThreads / 64];
  const SmallCopy& C = S.lv[blockIdx.x];
  const int n = C.n, ncol = C.ncol, nb = (n + kBlock - 1) / kBlock, cells = ncol * nb;
  const int T = blockDim.x, t = threadIdx.x;
  int* cl = sm;
  int* cnt = cl + n;
  int* ip = cnt + cells + 1;
  int* pm = ip + n;
  int* rpl = pm + n;
  for (int v = t; v < n; v += T) cl[v] = C.colour ? C.colour[v] : 0;
  for (int k = t; k < cells; k += T) cnt[k] = 0;
  __syncthreads();
  for (int v = t; v < n; v += T) atomicAdd(&cnt[cl[v] * nb + v / kBlock], 1);
  __syncthreads();
  block_excl_scan4(cnt, cells, lds);  // ends with a barrier
  for (int v = t; v < n; v += T) {
    const int c = cl[v], seg = v / kBlock;
    int r = 0;
    for (int u = seg * kBlock; u < v; ++u) r += cl[u] == c;
    const int p = cnt[c * nb + seg] + r;
    pm[v] = p;
    ip[p] = v;
    C.perm[v] = p;
    C.iperm[p] = v;
  }
  for (int c = t; c <= ncol; c += T) C.cptr[c] = c < ncol ? cnt[c * nb] : n;
  __syncthreads();
  for (int i = t; i < n; i += T) rpl[i] = C.rp_c[ip[i] + 1] - C.rp_c[ip[i]];
  __syncthreads();
  const int m = block_excl_scan4(rpl, n, lds);
  for (int i = t; i < n; i += T) C.rp[i] = rpl[i];
  if (t == 0) C.rp[n] = m;
  for (int i = t; i < n; i += T) {
    const int v = ip[i];
    int k = rpl[i];
    for (int p = C.rp_c[v]; p < C.rp_c[v + 1]; ++p, ++k) {
      C.col[k] = pm[C.col_c[p]];
      const double wv = C.w_c[p];
      C.w64[k] = wv;
      C.w32[k] = (float)wv;
    }
  }
}

// k_qs for the levels of a SmallCopies batch that have a next level.
__global__ void k_qs_small(SmallCopies S) {
  const SmallCopy& C = S.lv[blockIdx.y];
  if (!C.q_c) return;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < C.n; v += gridDim.x * blockDim.x)
    C.qs[C.perm[v]] = C.perm_next[C.q_c[v]];
}

__global__ void k_qs(int n, const int* perm, const int* q, const int* perm_next, int* qs) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int c = q[v];
  qs[perm[v]] = perm_next ? perm_next[c] : c;
}

// ---------------------------------------------------------------------------
// Galerkin coarse graph I L I^T.  For coarse row I the terms are the fine
// edges (v, j) with q(v) = I != q(j) = J; they are ordered by (J, min(v,j),
// max(v,j)) and each run of equal J is summed sequentially in that order, so
// W_c(I,J) and W_c(J,I) add the same fine weights in the same order.
// ---------------------------------------------------------------------------
// A batch of a row's neighbours for the Galerkin kernels: column indices and
// weights, then the neighbours' aggregates (positions past the row end repeat
// its last entry; callers skip them).
__device__ inline void gal_batch(int pb, int b, const int* __restrict__ col,
                                 const double* __restrict__ w, const int* __restrict__ q,
                                 int (&jj)[kNbU], int (&JJ)[kNbU], double (&ww)[kNbU]) {
#pragma unroll
  for (int k = 0; k < kNbU; ++k) jj[k] = col[min(pb + k, b - 1)];
  if (w)
#pragma unroll
    for (int k = 0; k < kNbU; ++k) ww[k] = w[min(pb + k, b - 1)];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < kNbU; ++k) JJ[k] = q[jj[k]];
  __builtin_amdgcn_sched_barrier(0);
}

// G lanes per fine row (a group of consecutive lanes of one wave): lane j
// takes entries j, j + G, ... of row v.  ext_mask gives the group's lanes
// whose entry in this pass is a term of v's coarse row (its neighbour in
// another aggregate), as bits of the wave.
template <int G>
__device__ inline unsigned long long gal_group_mask() {
  const int lane = threadIdx.x & 63;
  return (G == 64 ? ~0ULL : ((1ULL << G) - 1ULL)) << (lane & ~(G - 1));
}

template <int G>
__global__ void k_gal_count(int n, const int* __restrict__ rp, const int* __restrict__ col,
                            const int* __restrict__ q, int* __restrict__ tcount) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = (int)(g / G), j = (int)(g % G);
  if (v >= n) return;  // the whole group leaves together
  const int I = q[v], a = rp[v], b = rp[v + 1];
  const unsigned long long gm = gal_group_mask<G>();
  int c = 0;
  for (int pb = a; pb < b; pb += G) {
    const int p = pb + j;
    const bool ext = p < b && q[col[p]] != I;
    c += __popcll(__ballot(ext) & gm);
  }
  if (j == 0 && c) atomicAdd(&tcount[I], c);
}

// The terms of fine row v at v's place in its coarse row's list (lane order
// within each pass of the group; the rows are sorted afterwards, so the order
// in the list does not matter).  The group's first pass stays in registers
// between the count and the fill (most rows fit one pass).
template <int G>
__global__ void k_gal_fill(int n, const int* __restrict__ rp, const int* __restrict__ col,
                           const double* __restrict__ w, const int* __restrict__ q,
                           const int* __restrict__ tstart, int* __restrict__ tfill,
                           int* __restrict__ tJ, int* __restrict__ ta, int* __restrict__ tb,
                           double* __restrict__ tw) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = (int)(g / G), j = (int)(g % G);
  if (v >= n) return;  // the whole group leaves together
  const int I = q[v], a = rp[v], b = rp[v + 1];
  const int lane = threadIdx.x & 63;
  const unsigned long long gm = gal_group_mask<G>();
  const unsigned long long below = gm & ((1ULL << lane) - 1ULL);
  int j0 = 0, J0 = I;
  double w0 = 0.0;
  if (a + j < b) {
    j0 = col[a + j];
    w0 = w[a + j];
    J0 = q[j0];
  }
  const bool ext0 = a + j < b && J0 != I;
  const unsigned long long m0 = __ballot(ext0) & gm;
  int c = __popcll(m0);
  for (int pb = a + G; pb < b; pb += G) {
    const int p = pb + j;
    const bool ext = p < b && q[col[p]] != I;
    c += __popcll(__ballot(ext) & gm);
  }
  if (!c) return;
  int base = 0;
  if (j == 0) base = atomicAdd(&tfill[I], c);
  int k = tstart[I] + __shfl(base, lane & ~(G - 1));
  auto emit = [&](int jv, int J, double wv, int pos) {
    tJ[pos] = J;
    ta[pos] = v < jv ? v : jv;
    tb[pos] = v < jv ? jv : v;
    tw[pos] = wv;
  };
  if (ext0) emit(j0, J0, w0, k + __popcll(m0 & below));
  k += __popcll(m0);
  for (int pb = a + G; pb < b; pb += G) {
    const int p = pb + j;
    int jv = 0, J = I;
    double wv = 0.0;
    if (p < b) {
      jv = col[p];
      wv = w[p];
      J = q[jv];
    }
    const bool ext = p < b && J != I;
    const unsigned long long m = __ballot(ext) & gm;
    if (ext) emit(jv, J, wv, k + __popcll(m & below));
    k += __popcll(m);
  }
}

__device__ inline bool term_less(int J1, int a1, int b1, int J2, int a2, int b2) {
  if (J1 != J2) return J1 < J2;
  if (a1 != a2) return a1 < a2;
  return b1 < b2;
}

// Makes a wave's LDS stores visible to the wave's other lanes (the sorting
// helpers below use a region of their own per wave, so no block barrier).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Coarse row I with at most 64 terms sorted by one wavefront: each lane ranks
// its term against the row's others (broadcast with readlane), the terms go
// to the wave's LDS region (64 slots) in rank order, and each run of equal J
// is summed in that order.  Every lane of the wave calls; rows with more
// terms, and I >= nc, leave the wave idle.
__device__ inline void gal_row64(int I, int nc, const int* tstart, const int* tJ, const int* ta,
                                 const int* tb, const double* tw, int* sJ, double* sw, int* cJ,
                                 double* cw, int* uniq) {
  const int lane = threadIdx.x & 63;
  int s = 0, T = 0;
  if (I < nc) {
    s = tstart[I];
    T = tstart[I + 1] - s;
  }
  const bool active = I < nc && T <= 64;
  int myJ = INT_MAX, mya = 0, myb = 0;
  double myw = 0.0;
  if (active && lane < T) {
    myJ = tJ[s + lane];
    mya = ta[s + lane];
    myb = tb[s + lane];
    myw = tw[s + lane];
  }
  // T is the same in every lane of the wave, so the terms are broadcast with
  // readlane (scalar) instead of a cross-lane shuffle.
  int rank = 0;
  const int Tl = active ? T : 0;
  for (int l = 0; l < Tl; ++l) {
    const int J2 = __builtin_amdgcn_readlane(myJ, l), a2 = __builtin_amdgcn_readlane(mya, l),
              b2 = __builtin_amdgcn_readlane(myb, l);
    if (term_less(J2, a2, b2, myJ, mya, myb)) ++rank;
  }
  if (active && lane < T) {
    sJ[rank] = myJ;
    sw[rank] = myw;
  }
  wave_lds_sync();
  bool head = false;
  if (active && lane < T) head = lane == 0 || sJ[lane] != sJ[lane - 1];
  unsigned long long mask = __ballot(head);
  if (head) {
    int pos = __popcll(mask & ((1ULL << lane) - 1ULL));
    int J = sJ[lane];
    double sum = 0.0;
    for (int p = lane; p < T && sJ[p] == J; ++p) sum += sw[p];
    cJ[s + pos] = J;
    cw[s + pos] = sum;
  }
  if (active && lane == 0) uniq[I] = __popcll(mask);
  wave_lds_sync();  // the next call reuses sJ / sw
}


// Two coarse rows of at most 32 terms each, one per half of the wave (row I
// in lanes h * 32 + l, h = 0, 1): the same ranks and sums as gal_row64, the
// terms broadcast within each half by a cross-lane read.
__device__ inline void gal_row32(int I, int nc, const int* tstart, const int* tJ, const int* ta,
                                 const int* tb, const double* tw, int* sJ, double* sw, int* cJ,
                                 double* cw, int* uniq) {
  const int lane = threadIdx.x & 63, h = lane >> 5, l = lane & 31;
  int s = 0, T = 0;
  if (I < nc) {
    s = tstart[I];
    T = tstart[I + 1] - s;
  }
  const bool mine = I < nc && l < T;
  int myJ = INT_MAX, mya = 0, myb = 0;
  double myw = 0.0;
  if (mine) {
    myJ = tJ[s + l];
    mya = ta[s + l];
    myb = tb[s + l];
    myw = tw[s + l];
  }
  // Padding lanes hold (INT_MAX, 0, 0), after every real term of the row.
  const int Tm = max(__builtin_amdgcn_readlane(T, 0), __builtin_amdgcn_readlane(T, 32));
  int rank = 0;
  for (int k = 0; k < Tm; ++k) {
    const int src = (h << 5) + k;
    const int J2 = __shfl(myJ, src), a2 = __shfl(mya, src), b2 = __shfl(myb, src);
    if (term_less(J2, a2, b2, myJ, mya, myb)) ++rank;
  }
  int* rJ = sJ + (h << 5);
  double* rw = sw + (h << 5);
  if (mine) {
    rJ[rank] = myJ;
    rw[rank] = myw;
  }
  wave_lds_sync();
  bool head = false;
  if (mine) head = l == 0 || rJ[l] != rJ[l - 1];
  const unsigned long long rowmask = (__ballot(head) >> (h << 5)) & 0xFFFFFFFFULL;
  if (head) {
    const int pos = __popcll(rowmask & ((1ULL << l) - 1ULL));
    const int J = rJ[l];
    double sum = 0.0;
    for (int p = l; p < T && rJ[p] == J; ++p) sum += rw[p];
    cJ[s + pos] = J;
    cw[s + pos] = sum;
  }
  if (I < nc && l == 0) uniq[I] = __popcll(rowmask);
  wave_lds_sync();  // the next call reuses sJ / sw
}

// Lane value of the lane k places further round its row of 16 (DPP row_ror).
template <int K>
__device__ inline int row_ror(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x120 + K, 0xf, 0xf, false);
}

// Rows with at most 64 terms.  With packed set, a block of four waves takes
// Four consecutive rows per wave: when each of the four has at most 16 terms
// (the common case on large levels: a pair of fine rows of a 5-point grid
// gives six), the wave sorts them at once in rows of 16 lanes, ranking each
// term against the 15 others of its row by DPP rotations; when each has at
// most 32 (a pair of rows of a random geometric graph gives 14 on average, up
// to ~50), two at a time in halves of the wave; otherwise one after another
// across all 64 lanes.  Without packed (levels with few rows, where latency
// decides), one row per wave.  Same ranks, same sums either way.
constexpr int kGalPackedRows = 32768;  // coarse rows from which packed pays

__global__ __launch_bounds__(kBlock) void k_gal_rows_small(int nc, int packed, const int* tstart,
                                                         const int* tJ, const int* ta,
                                                         const int* tb, const double* tw,
                                                         int* cJ, double* cw, int* uniq) {
  __shared__ int sJ[kBlock / 64][64];
  __shared__ double sw[kBlock / 64][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (!packed) {
    gal_row64(blockIdx.x * (kBlock / 64) + wave, nc, tstart, tJ, ta, tb, tw, sJ[wave], sw[wave],
              cJ, cw, uniq);
    return;
  }
  const int I0 = (blockIdx.x * (kBlock / 64) + wave) * 4;  // the wave's first row
  const int g = lane >> 4, l16 = lane & 15;
  const int I = I0 + g;
  int s = 0, T = 0;
  if (I < nc) {
    s = tstart[I];
    T = tstart[I + 1] - s;
  }
  // the longest of the wave's four rows (lanes 0, 16, 32, 48 hold them)
  const int Tw = max(max(__builtin_amdgcn_readlane(T, 0), __builtin_amdgcn_readlane(T, 16)),
                     max(__builtin_amdgcn_readlane(T, 32), __builtin_amdgcn_readlane(T, 48)));
  if (Tw > 32) {
    for (int r = 0; r < 4; ++r)
      gal_row64(I0 + r, nc, tstart, tJ, ta, tb, tw, sJ[wave], sw[wave], cJ, cw, uniq);
    return;
  }
  if (Tw > 16) {
    for (int r = 0; r < 4; r += 2)
      gal_row32(I0 + r + (lane >> 5), nc, tstart, tJ, ta, tb, tw, sJ[wave], sw[wave], cJ, cw,
                uniq);
    return;
  }
  const bool mine = I < nc && l16 < T;
  int myJ = INT_MAX, mya = 0, myb = 0;
  double myw = 0.0;
  if (mine) {
    myJ = tJ[s + l16];
    mya = ta[s + l16];
    myb = tb[s + l16];
    myw = tw[s + l16];
  }
  int rank = 0;
  // Padding lanes hold (INT_MAX, 0, 0), after every real term of the row.
#define FV_RANK_STEP(K) \
  rank += term_less(row_ror<K>(myJ), row_ror<K>(mya), row_ror<K>(myb), myJ, mya, myb) ? 1 : 0;
  FV_RANK_STEP(1) FV_RANK_STEP(2) FV_RANK_STEP(3) FV_RANK_STEP(4) FV_RANK_STEP(5)
  FV_RANK_STEP(6) FV_RANK_STEP(7) FV_RANK_STEP(8) FV_RANK_STEP(9) FV_RANK_STEP(10)
  FV_RANK_STEP(11) FV_RANK_STEP(12) FV_RANK_STEP(13) FV_RANK_STEP(14) FV_RANK_STEP(15)
#undef FV_RANK_STEP
  int* rJ = sJ[wave] + g * 16;
  double* rw = sw[wave] + g * 16;
  if (mine) {
    rJ[rank] = myJ;
    rw[rank] = myw;
  }
  wave_lds_sync();
  bool head = false;
  if (mine) head = l16 == 0 || rJ[l16] != rJ[l16 - 1];
  const unsigned long long rowmask = (__ballot(head) >> (g * 16)) & 0xFFFFULL;
  if (head) {
    const int pos = __popcll(rowmask & ((1ULL << l16) - 1ULL));
    const int J = rJ[l16];
    double sum = 0.0;
    for (int p = l16; p < T && rJ[p] == J; ++p) sum += rw[p];
    cJ[s + pos] = J;
    cw[s + pos] = sum;
  }
  if (I < nc && l16 == 0) uniq[I] = __popcll(rowmask);
}

// Rows with more than 64 terms: one workgroup per listed row, rank sort into
// global scratch, then a sequential collapse.
__device__ inline void gal_big_row(int I, const int* tstart, const int* tJ, const int* ta,
                                   const int* tb, const double* tw, int* sJ, double* sw, int* cJ,
                                   double* cw, int* uniq) {
  const int s = tstart[I], T = tstart[I + 1] - s;
  for (int k = threadIdx.x; k < T; k += blockDim.x) {
    int J = tJ[s + k], a = ta[s + k], b = tb[s + k];
    int rank = 0;
    for (int l = 0; l < T; ++l)
      if (term_less(tJ[s + l], ta[s + l], tb[s + l], J, a, b)) ++rank;
    sJ[s + rank] = J;
    sw[s + rank] = tw[s + k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int u = 0;
    int p = 0;
    while (p < T) {
      int J = sJ[s + p];
      double sum = 0.0;
      while (p < T && sJ[s + p] == J) sum += sw[s + p++];
      cJ[s + u] = J;
      cw[s + u] = sum;
      ++u;
    }
    uniq[I] = u;
  }
}

__global__ __launch_bounds__(kBlock) void k_gal_rows_big(const int* list, const int* nlist,
                                                       const int* tstart, const int* tJ,
                                                       const int* ta, const int* tb,
                                                       const double* tw, int* sJ, double* sw,
                                                       int* cJ, double* cw, int* uniq) {
  const int nbig = *nlist;
  for (int row = blockIdx.x; row < nbig; row += gridDim.x) {
    gal_big_row(list[row], tstart, tJ, ta, tb, tw, sJ, sw, cJ, cw, uniq);
    __syncthreads();
  }
}

__global__ void k_list_fill(int n, const int* tstart, const int* pos, int* list) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (tstart[i + 1] - tstart[i]) > 64) list[pos[i]] = i;
}

// G lanes per coarse row: lane j moves entries j, j + G, ... of the row.
template <int G>
__global__ void k_gal_compact(int nc, const int* tstart, const int* uniq, const int* crp,
                              const int* cJ, const double* cw, int* col, double* w) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int I = (int)(g / G), j = (int)(g % G);
  if (I >= nc) return;
  const int s = tstart[I], d = crp[I], u = uniq[I];
  for (int k = j; k < u; k += G) {
    col[d + k] = cJ[s + k];
    w[d + k] = cw[s + k];
  }
}

// ---------------------------------------------------------------------------
// Host orchestration.
// ---------------------------------------------------------------------------
template <class T>
static T* halloc(fv_hierarchy* h, size_t count) {
  return static_cast<T*>(dev_alloc(h->ctx, std::max<size_t>(count, 1) * sizeof(T), &h->bytes));
}

static int read_int(const int* d, hipStream_t s, int* pinned) {
  FV_HIP(hipMemcpyAsync(pinned, d, sizeof(int), hipMemcpyDeviceToHost, s));
  FV_HIP(hipStreamSynchronize(s));
  return *pinned;
}

// The per-level maxima of the degree (as 64-bit words) and every level's
// colour ranges, packed into out in one launch, so that the end of a build
// reads them back with a single copy.
struct LevelRanges {
  const int* cptr[FV_MAX_LEVELS];
  const int* rp[FV_MAX_LEVELS];  // solve-order row pointers
  int len[FV_MAX_LEVELS];
  int off[FV_MAX_LEVELS];
};
// out[off + k]: colour k's first row; out[total + off + k]: the row pointer
// there (the colour's first entry).
__global__ void k_gather_ranges(LevelRanges R, int nlev, const unsigned long long* dmax,
                                int ndm, unsigned long long* out_dm, int* out, int total) {
  for (int k = threadIdx.x; k < ndm; k += blockDim.x) out_dm[k] = dmax[k];
  for (int l = 0; l < nlev; ++l)
    for (int k = threadIdx.x; k < R.len[l]; k += blockDim.x) {
      const int r = R.cptr[l][k];
      out[R.off[l] + k] = r;
      out[total + R.off[l] + k] = R.rp[l][r];
    }
}

// Copies up to 8 device ints into out[0..7] (one launch, so that one
// read-back returns them all).
struct IntSrc {
  const int* p[8];
};
__global__ void k_gather_ints(IntSrc src, int count, int* out) {
  const int t = threadIdx.x;
  if (t < count) out[t] = src.p[t] ? *src.p[t] : 0;
}

static void free_level(fv_hierarchy* h, Level& L) {
  auto f = [&](void* p, size_t bytes) {
    if (p) dev_free(h->ctx, p, bytes, &h->bytes);
  };
  size_t n = std::max(L.n, 1), m = std::max<long long>(L.m, 1), c = std::max(L.ncol + 1, 1);
  f(L.rp_c, (L.n + 1) * sizeof(int));
  f(L.col_c, m * sizeof(int));
  f(L.w_c, m * sizeof(double));
  f(L.q_c, n * sizeof(int));
  f(L.colour_c, n * sizeof(int));
  f(L.rp, (L.n + 1) * sizeof(int));
  f(L.col, m * sizeof(int));
  f(L.w64, m * sizeof(double));
  f(L.w32, m * sizeof(float));
  f(L.cptr, c * sizeof(int));
  f(L.perm, n * sizeof(int));
  f(L.iperm, n * sizeof(int));
  f(L.qs, n * sizeof(int));
  const size_t slots = (size_t)std::max<long long>(L.eslots, 1);
  f(L.ecol, slots * sizeof(int));
  f(L.ew64, slots * sizeof(double));
  f(L.ew32, slots * sizeof(float));
  L = Level();
}

void free_hierarchy(fv_hierarchy* h, bool sync_device) {
  if (!h) return;
  // Solves on any stream may still read the levels; wait for them before the
  // blocks go back to the cache (hipFree would synchronise the same way).
  if (sync_device) (void)hipDeviceSynchronize();
  for (int l = 0; l < FV_MAX_LEVELS; ++l) free_level(h, h->lv[l]);
  if (h->d_desc) dev_free(h->ctx, h->d_desc, sizeof(LevelDesc) * FV_MAX_LEVELS, &h->bytes);
  delete h;
}

size_t hierarchy_nmax(const fv_hierarchy* h) { return h->levels ? (size_t)h->lv[0].n : 0; }

// Allows k_colour_local more than the 64 KiB of dynamic LDS a launch gets by
// default; done once per process.
static void enable_small_copy_lds() {
  static std::once_flag once;
  std::call_once(once, [] {
    FV_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_small_copy),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(sizeof(int) * small_copy_ints(kSmallCopyRows, kSmallCopyCells / nblk(kSmallCopyRows)))));
  });
}

static void enable_colour_local_lds() {
  static std::once_flag once;
  std::call_once(once, [] {
    FV_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_colour_local),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kColourLocalLds));
  });
}

fv_hierarchy* build_hierarchy(fv_context* ctx, const fv_csr* Lin, const fv_hier_opts* o,
                              hipStream_t s) {
  if (!Lin) throw Error(FV_E_INVALID, "null graph");
  const int n = Lin->n;
  const int nnz = Lin->nnz;
  if (n < 2 || nnz < 0 || !Lin->row_ptr || (nnz > 0 && (!Lin->col || !Lin->val)))
    throw Error(FV_E_INVALID, "bad CSR header");
  int n_coarse = o ? o->n_coarse : 25;
  int max_levels = o ? o->max_levels : FV_MAX_LEVELS;
  unsigned long long cseed = o ? o->colour_seed : 0ULL;
  const int ell = o ? o->ell : 0;
  if (n_coarse < 1) throw Error(FV_E_INVALID, "n_coarse < 1");
  if (max_levels < 1 || max_levels > FV_MAX_LEVELS) max_levels = FV_MAX_LEVELS;

  Tmp tmp{ctx, s, {}};
  int* pin_i = static_cast<int*>(pin_get(ctx));
  long long* pin_ll = nullptr;
  struct PinGuard {
    fv_context* c;
    void* p;
    hipStream_t s;
    ~PinGuard() { pin_put(c, p, s); }
  } pg{ctx, pin_i, s};
  pin_ll = reinterpret_cast<long long*>(pin_i + 8);

  // Stage the input on the device.
  const int* rp_in = Lin->row_ptr;
  const int* col_in = Lin->col;
  const double* val_in = Lin->val;
  if (!Lin->on_device) {
    int* r = tmp.get<int>(n + 1);
    int* c = tmp.get<int>(nnz);
    double* v = tmp.get<double>(nnz);
    FV_HIP(hipMemcpyAsync(r, Lin->row_ptr, sizeof(int) * (n + 1), hipMemcpyHostToDevice, s));
    if (nnz) {
      FV_HIP(hipMemcpyAsync(c, Lin->col, sizeof(int) * nnz, hipMemcpyHostToDevice, s));
      FV_HIP(hipMemcpyAsync(v, Lin->val, sizeof(double) * nnz, hipMemcpyHostToDevice, s));
    }
    rp_in = r;
    col_in = c;
    val_in = v;
  }

  Scanner sc;
  sc.tmp = &tmp;
  sc.s = s;
  sc.host = pin_ll;

  // Validation (Definition 2.1): the structure first (the value check reads
  // through it), then values, symmetry and degrees.
  int* flags = tmp.get<int>(8);
  int* gath = tmp.get<int>(8);
  FV_HIP(hipMemsetAsync(flags, 0, 8 * sizeof(int), s));
  k_val_structure<<<nblk(n), kBlock, 0, s>>>(n, nnz, rp_in, col_in, flags);
  FV_HIP(hipGetLastError());
  if (read_int(flags, s, pin_i) & 1) throw Error(FV_E_INVALID, "CSR structure invalid");
  int* offdeg = tmp.get<int>(n);
  int* rp0 = tmp.get<int>(n + 1);
  const int adj = Lin->is_adjacency ? 1 : 0;
  switch (row_group(n, nnz)) {
    case 4:
      k_val_values<4><<<nblk(4LL * n), kBlock, 0, s>>>(n, rp_in, col_in, val_in, adj, offdeg, flags);
      break;
    case 8:
      k_val_values<8><<<nblk(8LL * n), kBlock, 0, s>>>(n, rp_in, col_in, val_in, adj, offdeg, flags);
      break;
    default:
      k_val_values<16><<<nblk(16LL * n), kBlock, 0, s>>>(n, rp_in, col_in, val_in, adj, offdeg,
                                                          flags);
  }
  FV_HIP(hipGetLastError());
  sc.enqueue(FromArray{offdeg}, n, rp0, true);
  k_gather_ints<<<1, 64, 0, s>>>(IntSrc{{flags, rp0 + n}}, 2, gath);
  FV_HIP(hipMemcpyAsync(pin_i, gath, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  FV_HIP(hipStreamSynchronize(s));
  const int f = pin_i[0];
  const long long m0 = pin_i[1];
  if (f & 2) throw Error(FV_E_NOT_LAPLACIAN, "not a graph Laplacian / adjacency");
  if (f & 4) throw Error(FV_E_NOT_SYMMETRIC, "not symmetric");
  if (f & 8) throw Error(FV_E_ISOLATED, "isolated vertex");

  static std::atomic<uint64_t> serials{0};
  fv_hierarchy* h = new fv_hierarchy();
  h->serial = ++serials;
  h->ctx = ctx;
  try {
    Level& L0 = h->lv[0];
    L0.n = n;
    L0.rp_c = halloc<int>(h, n + 1);
    FV_HIP(hipMemcpyAsync(L0.rp_c, rp0, sizeof(int) * (n + 1), hipMemcpyDeviceToDevice, s));
    L0.m = m0;
    L0.col_c = halloc<int>(h, m0);
    L0.w_c = halloc<double>(h, m0);
    if (Lin->is_adjacency) {
      // W itself: validation rejected self-loops, so W is the input verbatim
      // (and rp0 equals the input's row pointers); two copies at full bandwidth
      // instead of a row-per-thread walk.
      if (m0 > 0) {
        FV_HIP(hipMemcpyAsync(L0.col_c, col_in, sizeof(int) * m0, hipMemcpyDeviceToDevice, s));
        FV_HIP(hipMemcpyAsync(L0.w_c, val_in, sizeof(double) * m0, hipMemcpyDeviceToDevice, s));
      }
    } else {
      k_extract<<<nblk(n), kBlock, 0, s>>>(n, rp_in, col_in, val_in, 0, L0.rp_c, L0.col_c,
                                           L0.w_c);
      FV_HIP(hipGetLastError());
    }

    // Scratch sized by level 0 and reused on every level.
    const long long mcap = std::max<long long>(m0, 1);
    int* mate = tmp.get<int>(n);
    int* ptr = tmp.get<int>(n);
    int* root = tmp.get<int>(n);
    int* minmem = tmp.get<int>(n);
    int* id = tmp.get<int>(n + 1);
    int* cnew = tmp.get<int>(n);  // the recolouring pass's output
    unsigned* bipw = tmp.get<unsigned>(n);  // union-find words of the two-colouring
    int* bipbad = tmp.get<int>(1);           // the level is not bipartite
    int* tcount = tmp.get<int>(n + 1);
    int* tstart = tmp.get<int>(n + 1);
    int* tfill = tmp.get<int>(n);
    int* uniq = tmp.get<int>(n + 1);
    int* list = tmp.get<int>(n);
    int* lpos = tmp.get<int>(n + 1);
    int* tJ = tmp.get<int>(mcap);
    int* ta = tmp.get<int>(mcap);
    int* tb = tmp.get<int>(mcap);
    double* tw = tmp.get<double>(mcap);
    int* cJ = tmp.get<int>(mcap);
    double* cw = tmp.get<double>(mcap);
    int* sJ = tmp.get<int>(mcap);
    double* sw = tmp.get<double>(mcap);
    // [l]: level l's largest degree (bits of the double); [FV_MAX_LEVELS + l]: its
    // longest row
    unsigned long long* dmax = tmp.get<unsigned long long>(2 * FV_MAX_LEVELS);
    FV_HIP(hipMemsetAsync(dmax, 0, sizeof(unsigned long long) * 2 * FV_MAX_LEVELS, s));
    // Per-round progress flags of the matching and colouring rounds.
    constexpr int kRoundCap = 4096;
    int* mflag = tmp.get<int>(kRoundCap);
    int* cflag = tmp.get<int>(kRoundCap);
    int* bflag = tmp.get<int>(kRoundCap);  // per hooking round: something was hooked
    // [0] aggregation error, [1] largest colour, [2] a one-workgroup loop
    // overran, [3] always 0
    int* lflag = flags + 4;
    int* bmax = tmp.get<int>(kRoundGrid);

    int l = 0;
    for (;;) {
      Level& F = h->lv[l];
      k_degree_max<<<std::min(nblk(F.n), kDegreeGrid), kBlock, 0, s>>>(F.n, F.rp_c, F.w_c, dmax + l,
                                                                         dmax + FV_MAX_LEVELS + l);
      FV_HIP(hipGetLastError());
      if (F.n <= n_coarse || l + 1 >= max_levels) break;
      const int fn = F.n;
      // Matching and colouring rounds run in batches; the host reads the
      // progress flag of the last round of each batch, together with the
      // aggregate count, in one read-back when the first batches suffice.
      const bool local = fn <= kLocalMaxN;
      int mr = 0, cr = 0;
      F.colour_c = halloc<int>(h, fn);
      // The level's scratch in one launch: round flags, matching and colour
      // state, and the Galerkin term counters (nc < fn terms rows).
      if (!local)
        fill_multi(s, {{mflag, kRoundCap, 0}, {cflag, kRoundCap, 0}, {mate, fn, -1},
                       {F.colour_c, fn, -1}, {cnew, fn, -1}, {tcount, fn, 0}, {tfill, fn, 0},
                       {bipbad, 1, 0}, {bflag, kRoundCap, 0}});
      else
        fill_multi(s, {{tcount, fn, 0}, {tfill, fn, 0}, {bipbad, 1, 0}});
      auto match_rounds = [&](int b) {
        if (mr + b > kRoundCap) throw Error(FV_E_DEVICE, "matching did not terminate");
        for (int r = mr; r < mr + b; ++r) {
          const int* prev = r ? mflag + r - 1 : nullptr;
          k_match_pick<<<round_grid(fn), kBlock, 0, s>>>(fn, F.rp_c, F.col_c, F.w_c, mate, ptr,
                                                         prev);
          k_match_commit<<<round_grid(fn), kBlock, 0, s>>>(fn, mate, ptr, mflag + r, prev);
        }
        mr += b;
        FV_HIP(hipGetLastError());
      };
      auto aggregate = [&]() {
        fill_multi(s, {{lflag, 1, 0}, {minmem, fn, INT_MAX}});
        k_agg_root<<<nblk(fn), kBlock, 0, s>>>(fn, F.rp_c, F.col_c, F.w_c, mate, root, lflag);
        k_agg_minmem<<<nblk(fn), kBlock, 0, s>>>(fn, root, minmem);
        FV_HIP(hipGetLastError());
        sc.enqueue(LeaderFlag{root, minmem}, fn, id, true);
      };
      const uint32_t lseed = level_seed(cseed, l);
      // A bipartite finest level is two-coloured before the first-fit rounds,
      // which then find every vertex coloured and stop after one round.
      int br = 0;
      // Hooking rounds: per round r, flag bflag[S r] (the round has work) and
      // bflag[S r + c + 1] (its compression launch c left paths unfinished),
      // S = kBipStride; kBipCompress compression launches per round finish
      // paths of up to kBipHops^3 links, and a longer one carries over to the
      // next round as work.
      constexpr int kBipCompress = 3;
      constexpr int kBipStride = 1 + kBipCompress;
      auto two_colour_rounds = [&](int b) {
        if ((br + b) * kBipStride > kRoundCap)
          throw Error(FV_E_DEVICE, "two-colouring did not terminate");
        if (br == 0) {
          k_bip_triangle<<<nblk(std::min(fn, kTriRows)), kBlock, 0, s>>>(
              std::min(fn, kTriRows), F.rp_c, F.col_c, bipbad);
          k_bip_init<<<round_grid(fn), kBlock, 0, s>>>(fn, bipw);
        }
        for (int r = br; r < br + b; ++r) {
          int* f = bflag + r * kBipStride;
          k_bip_hook<<<round_grid(fn), kBlock, 0, s>>>(
              fn, F.rp_c, F.col_c, bipw, bipbad, f, r ? f - kBipStride : nullptr,
              r ? f - 1 : nullptr);
          for (int c = 0; c < kBipCompress; ++c)
            k_bip_compress<<<round_grid(fn), kBlock, 0, s>>>(fn, bipw, bipbad, f + c, f + c + 1);
        }
        br += b;
        FV_HIP(hipGetLastError());
      };
      // After the rounds: the edge check and (bipartite) the colouring
      // itself, which the first-fit rounds then leave alone.
      auto two_colour_finish = [&]() {
        k_bip_check<<<round_grid(fn), kBlock, 0, s>>>(fn, F.rp_c, F.col_c, bipw, bipbad);
        k_bip_commit<<<round_grid(fn), kBlock, 0, s>>>(fn, bipw, F.colour_c, bipbad);
        FV_HIP(hipGetLastError());
      };
      auto colour_rounds = [&](int b) {
        if (cr + b > kRoundCap) throw Error(FV_E_DEVICE, "colouring did not terminate");
        for (int r = cr; r < cr + b; ++r)
          k_colour_round<<<round_grid(fn), kBlock, 0, s>>>(fn, F.rp_c, F.col_c, lseed,
                                                           F.colour_c, cflag + r,
                                                           r ? cflag + r - 1 : nullptr);
        cr += b;
        k_max_blocks<<<round_grid(fn), kBlock, 0, s>>>(fn, F.colour_c, bmax);
        k_max_final<<<1, kBlock, 0, s>>>(round_grid(fn), bmax, lflag + 1);
        FV_HIP(hipGetLastError());
      };
      auto read_back = [&]() {
        // lflag[3] is never written: it stands for "no round pending" on the
        // one-workgroup path, whose loops run to the end
        const int* mdone = local ? lflag + 3 : mflag + mr - 1;
        const int* cdone = local ? lflag + 3 : cflag + cr - 1;
        // the two-colouring rounds are unfinished while the last one had work
        const int* bdone = (local || br == 0) ? lflag + 3 : bflag + (br - 1) * kBipStride;
        k_gather_ints<<<1, 64, 0, s>>>(
            IntSrc{{mdone, cdone, lflag, lflag + 1, id + fn, lflag + 2, bipbad, bdone}}, 8, gath);
        FV_HIP(hipMemcpyAsync(pin_i, gath, 8 * sizeof(int), hipMemcpyDeviceToHost, s));
        FV_HIP(hipStreamSynchronize(s));
      };
      if (local) {
        // one workgroup runs every round of both loops
        k_match_local<<<1, kLocalBlock, 0, s>>>(fn, F.rp_c, F.col_c, F.w_c, mate, ptr, lflag + 2);
        aggregate();
        const size_t cl_bytes = colour_local_lds(fn, F.m);
        const int cl_lds = cl_bytes <= kColourLocalLds ? (int)cl_bytes : 0;
        if (cl_lds > 64 * 1024) enable_colour_local_lds();
        k_colour_local<<<1, kLocalBlock, cl_lds, s>>>(fn, F.m, F.rp_c, F.col_c, lseed,
                                                      l == 0 ? 1 : 0, F.colour_c, cnew,
                                                      lflag + 1, lflag + 2, cl_lds);
        FV_HIP(hipGetLastError());
      } else {
        match_rounds(8);
        aggregate();
        if (l == 0) {
          two_colour_rounds(2);
          two_colour_finish();
        }
        colour_rounds(16);
      }
      read_back();
      if (pin_i[5]) throw Error(FV_E_DEVICE, "matching or colouring did not terminate");
      if (pin_i[7]) {
        // The hooking rounds enqueued did not reach the end (rare: very
        // long trees): finish them, then redo the colouring from scratch.
        while (pin_i[7]) {
          two_colour_rounds(8);
          read_back();
        }
        fill_multi(s, {{cflag, kRoundCap, 0}, {F.colour_c, fn, -1}, {bipbad, 1, 0}});
        cr = 0;
        two_colour_finish();
        colour_rounds(16);
        read_back();
      }
      while (pin_i[0]) {
        match_rounds(8);
        aggregate();
        read_back();
      }
      while (pin_i[1]) {
        colour_rounds(8);
        read_back();
      }
      if (pin_i[2]) throw Error(FV_E_DEVICE, "matching not maximal");
      // ncol: exact on the one-workgroup path (its kernel recolours too); an
      // upper bound after the recolouring pass below, trimmed once the colour
      // ranges are read back at the end of the build.
      F.ncol = pin_i[3] + 1;
      // (the one-workgroup kernel decides and recolours itself)
      const bool two_coloured = l == 0 && pin_i[6] == 0;
      if (!local && !two_coloured) {
        for (int c = F.ncol - 1; c >= 0; --c)
          k_recolour_class<<<round_grid(fn), kBlock, 0, s>>>(fn, F.rp_c, F.col_c, F.colour_c, cnew,
                                                             c);
        FV_HIP(hipGetLastError());
        FV_HIP(hipMemcpyAsync(F.colour_c, cnew, sizeof(int) * fn, hipMemcpyDeviceToDevice, s));
      }
      const int nc = pin_i[4];
      if (nc < 2 || nc >= fn) {
        dev_free(ctx, F.colour_c, sizeof(int) * fn, &h->bytes);
        F.colour_c = nullptr;
        F.ncol = 0;
        break;
      }
      F.q_c = halloc<int>(h, fn);
      k_agg_q<<<nblk(fn), kBlock, 0, s>>>(fn, root, minmem, id, F.q_c);
      // Galerkin coarse graph
      Level& Cl = h->lv[l + 1];
      Cl.n = nc;
      auto gal_terms = [&](auto G) {
        constexpr int kG = decltype(G)::value;
        k_gal_count<kG><<<nblk((long long)kG * fn), kBlock, 0, s>>>(fn, F.rp_c, F.col_c, F.q_c,
                                                                    tcount);
        FV_HIP(hipGetLastError());
        sc.enqueue(FromArray{tcount}, nc, tstart, true);
        k_gal_fill<kG><<<nblk((long long)kG * fn), kBlock, 0, s>>>(
            fn, F.rp_c, F.col_c, F.w_c, F.q_c, tstart, tfill, tJ, ta, tb, tw);
      };
      switch (row_group(fn, F.m)) {
        case 4: gal_terms(std::integral_constant<int, 4>{}); break;
        case 8: gal_terms(std::integral_constant<int, 8>{}); break;
        default: gal_terms(std::integral_constant<int, 16>{});
      }
      {
        const int packed = nc >= kGalPackedRows ? 1 : 0;
        k_gal_rows_small<<<nblk(nc, (packed ? 4 : 1) * (kBlock / 64)), kBlock, 0, s>>>(
            nc, packed, tstart, tJ, ta, tb, tw, cJ, cw, uniq);
      }
      FV_HIP(hipGetLastError());
      sc.enqueue(BigRow{tstart}, nc, lpos, true);
      k_list_fill<<<nblk(nc), kBlock, 0, s>>>(nc, tstart, lpos, list);
      k_gal_rows_big<<<std::min(nc, 512), kBlock, 0, s>>>(list, lpos + nc, tstart, tJ, ta, tb, tw,
                                                          sJ, sw, cJ, cw, uniq);
      FV_HIP(hipGetLastError());
      Cl.rp_c = halloc<int>(h, nc + 1);
      const long long mc = sc.run(FromArray{uniq}, nc, Cl.rp_c, true);
      Cl.m = mc;
      Cl.col_c = halloc<int>(h, mc);
      Cl.w_c = halloc<double>(h, mc);
      switch (row_group(nc, mc)) {
        case 4:
          k_gal_compact<4><<<nblk(4LL * nc), kBlock, 0, s>>>(nc, tstart, uniq, Cl.rp_c, cJ, cw,
                                                              Cl.col_c, Cl.w_c);
          break;
        case 8:
          k_gal_compact<8><<<nblk(8LL * nc), kBlock, 0, s>>>(nc, tstart, uniq, Cl.rp_c, cJ, cw,
                                                              Cl.col_c, Cl.w_c);
          break;
        default:
          k_gal_compact<16><<<nblk(16LL * nc), kBlock, 0, s>>>(nc, tstart, uniq, Cl.rp_c, cJ, cw,
                                                                Cl.col_c, Cl.w_c);
      }
      FV_HIP(hipGetLastError());
      ++l;
    }
    const int J = l;
    h->levels = J + 1;

    // Solve-order copies, coarsest first so that q can use the next perm.  The
    // small levels (the coarsest run of levels that fit one workgroup each)
    // in one launch, then their aggregate maps in another.
    int kbig = J;  // levels above kbig go through the per-level kernels
    {
      SmallCopies S;
      std::memset(&S, 0, sizeof(S));
      int lds_ints = 0;
      for (int k = J; k >= 0 && S.count < kSmallCopyMax; --k) {
        Level& F = h->lv[k];
        const int fn = F.n;
        const int ncol = k == J ? 1 : F.ncol;
        if (fn > kSmallCopyRows || (long long)ncol * nblk(fn) > kSmallCopyCells) break;
        if (k == J) {
          F.ncol = 1;
          F.cptr_h = {0, fn};
        }
        F.perm = halloc<int>(h, fn);
        F.iperm = halloc<int>(h, fn);
        F.cptr = halloc<int>(h, ncol + 1);
        F.rp = halloc<int>(h, fn + 1);
        F.col = halloc<int>(h, F.m);
        F.w64 = halloc<double>(h, F.m);
        F.w32 = halloc<float>(h, F.m);
        if (k < J) F.qs = halloc<int>(h, fn);
        SmallCopy& C = S.lv[S.count++];
        C.n = fn;
        C.ncol = ncol;
        C.colour = k == J ? nullptr : F.colour_c;
        C.rp_c = F.rp_c;
        C.col_c = F.col_c;
        C.w_c = F.w_c;
        C.q_c = k < J ? F.q_c : nullptr;
        C.perm_next = k < J ? h->lv[k + 1].perm : nullptr;
        C.perm = F.perm;
        C.iperm = F.iperm;
        C.cptr = F.cptr;
        C.rp = F.rp;
        C.col = F.col;
        C.w64 = F.w64;
        C.w32 = F.w32;
        C.qs = F.qs;
        lds_ints = std::max(lds_ints, small_copy_ints(fn, ncol));
        kbig = k - 1;
      }
      if (S.count > 0) {
        const size_t lds = sizeof(int) * (size_t)lds_ints;
        if (lds > 64 * 1024) enable_small_copy_lds();
        k_small_copy<<<S.count, kSmallCopyThreads, lds, s>>>(S);
        k_qs_small<<<dim3(nblk(kSmallCopyRows), S.count), kBlock, 0, s>>>(S);
        FV_HIP(hipGetLastError());
      }
    }
    for (int k = kbig; k >= 0; --k) {
      Level& F = h->lv[k];
      const int fn = F.n;
      F.perm = halloc<int>(h, fn);
      F.iperm = halloc<int>(h, fn);
      if (k == J) {
        F.ncol = 1;
        F.cptr_h = {0, fn};
        k_iota<<<nblk(fn), kBlock, 0, s>>>(F.perm, fn);
        k_iota<<<nblk(fn), kBlock, 0, s>>>(F.iperm, fn);
        F.cptr = halloc<int>(h, 2);
        FV_HIP(hipMemcpyAsync(F.cptr, F.cptr_h.data(), sizeof(int) * 2, hipMemcpyHostToDevice, s));
      } else {
        const int nb = nblk(fn);
        const long long cells = (long long)F.ncol * nb;
        if (cells >= INT_MAX) throw Error(FV_E_INVALID, "too many colours");
        int* cnt = tmp.get<int>(cells);
        int* off = tmp.get<int>(cells + 1);
        k_colour_block_count<<<nb, kBlock, sizeof(int) * F.ncol, s>>>(fn, F.colour_c, F.ncol, nb,
                                                                      cnt);
        FV_HIP(hipGetLastError());
        sc.enqueue(FromArray{cnt}, (int)cells, off, false);
        k_colour_scatter<<<nb, kBlock, 0, s>>>(fn, F.colour_c, nb, off, F.perm, F.iperm);
        F.cptr = halloc<int>(h, F.ncol + 1);
        k_colour_ptr<<<1, kBlock, 0, s>>>(fn, F.ncol, nb, off, F.cptr);
        FV_HIP(hipGetLastError());
      }
      F.rp = halloc<int>(h, fn + 1);
      sc.enqueue(PermDeg{F.rp_c, F.iperm}, fn, F.rp, true);
      F.col = halloc<int>(h, F.m);
      F.w64 = halloc<double>(h, F.m);
      F.w32 = halloc<float>(h, F.m);
      launch_solve_fill(fn, F.m, s, F.rp_c, F.col_c, F.w_c, F.iperm, F.perm, F.rp, F.col, F.w64,
                        F.w32);
      FV_HIP(hipGetLastError());
      if (k < J) {
        F.qs = halloc<int>(h, fn);
        k_qs<<<nblk(fn), kBlock, 0, s>>>(fn, F.perm, F.q_c, h->lv[k + 1].perm, F.qs);
        FV_HIP(hipGetLastError());
      }
    }
    // Read back the shifts and colour ranges of every level at once: one
    // gather into a staging block, one copy.
    LevelRanges R;
    std::memset(&R, 0, sizeof(R));
    int total = 0;
    for (int k = 0; k < J; ++k) {
      R.cptr[k] = h->lv[k].cptr;
      R.rp[k] = h->lv[k].rp;
      R.len[k] = h->lv[k].ncol + 1;
      R.off[k] = total;
      total += R.len[k];
    }
    const size_t dm_bytes = sizeof(unsigned long long) * 2 * FV_MAX_LEVELS;
    unsigned char* stage = tmp.get<unsigned char>(dm_bytes + sizeof(int) * 2 * total);
    k_gather_ranges<<<1, kBlock, 0, s>>>(R, J, dmax, 2 * FV_MAX_LEVELS,
                                         reinterpret_cast<unsigned long long*>(stage),
                                         reinterpret_cast<int*>(stage + dm_bytes), total);
    FV_HIP(hipGetLastError());
    std::vector<unsigned char> host(dm_bytes + sizeof(int) * 2 * total);
    FV_HIP(hipMemcpyAsync(host.data(), stage, host.size(), hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    std::vector<unsigned long long> dm(2 * FV_MAX_LEVELS);
    std::memcpy(dm.data(), host.data(), dm_bytes);
    for (int k = 0; k < J; ++k) {
      Level& F = h->lv[k];
      F.cptr_h.assign(F.ncol + 1, 0);
      std::memcpy(F.cptr_h.data(), host.data() + dm_bytes + sizeof(int) * R.off[k],
                  sizeof(int) * R.len[k]);
      std::vector<int> e(R.len[k]);
      std::memcpy(e.data(), host.data() + dm_bytes + sizeof(int) * (total + R.off[k]),
                  sizeof(int) * R.len[k]);
      F.cnnz_h.assign(e.begin(), e.end());
    }
    for (int k = 0; k < J; ++k) {  // drop the empty last classes the recolouring left
      Level& F = h->lv[k];
      while (F.ncol > 1 && F.cptr_h[F.ncol - 1] == F.n) --F.ncol;
      F.cptr_h.resize(F.ncol + 1);
      F.cnnz_h.resize(F.ncol + 1);
    }
    for (int k = 0; k <= J; ++k) {
      double d;
      std::memcpy(&d, &dm[k], sizeof(double));
      h->lv[k].sigma = 2.0 * d;
    }
    // ELL blocks of the colours the multi-workgroup sweeps visit.
    for (int k = 0; k < J && ell >= 0; ++k) {
      Level& F = h->lv[k];
      EllBlocks B;
      ell_plan(F, (long long)dm[FV_MAX_LEVELS + k], B);
      if (!F.ew) continue;
      F.ecol = halloc<int>(h, F.eslots);
      F.ew64 = halloc<double>(h, F.eslots);
      F.ew32 = halloc<float>(h, F.eslots);
      int maxrows = 1;
      for (int b = 0; b < B.count; ++b) maxrows = std::max(maxrows, B.rows[b]);
      k_ell_fill<<<dim3(nblk(maxrows), B.count), kBlock, 0, s>>>(B, F.rp, F.col, F.w64, F.w32,
                                                                 F.ecol, F.ew64, F.ew32);
      FV_HIP(hipGetLastError());
    }
    // Device descriptors.
    std::vector<LevelDesc> d(FV_MAX_LEVELS);
    std::memset(d.data(), 0, sizeof(LevelDesc) * FV_MAX_LEVELS);
    for (int k = 0; k <= J; ++k) d[k] = desc_of(h->lv[k]);
    h->d_desc = static_cast<LevelDesc*>(
        dev_alloc(ctx, sizeof(LevelDesc) * FV_MAX_LEVELS, &h->bytes));
    FV_HIP(hipMemcpyAsync(h->d_desc, d.data(), sizeof(LevelDesc) * FV_MAX_LEVELS,
                          hipMemcpyHostToDevice, s));
    FV_HIP(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    free_hierarchy(h, /*sync_device=*/false);  // only this build's stream used it
    throw;
  }
  return h;
}

}  // namespace fv
