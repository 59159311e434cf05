// Spectral partitioning by recursive bisection of the Fiedler vector: the use
// of phi_2 that the paper names (graph partitioning, spectral clustering; see
// its introduction and conclusion).  Each part of the current level is cut in
// two by its own Fiedler vector: the induced subgraph is extracted on the
// device, the library builds its hierarchy and solves it, and the vertices
// are split at the median of phi_2 (the smaller half by value, ties to the
// smaller index) or by its sign.  Vertices left without an edge inside their
// part (they cannot take part in a solve) go to the smaller half.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>

#include "fv_device.h"
#include "fv_internal.h"

namespace fv {
namespace {

constexpr int kPB = 256;   // threads per block
constexpr int kPer = 8;    // scan elements per thread
constexpr int kTile = kPB * kPer;

// ---- exclusive scan of an int array (three launches) ------------------------

__device__ inline long long block_incl_scan(long long v, long long* lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const long long t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  if (lane == 63) lds[wid] = v;
  __syncthreads();
  long long pre = 0;
  for (int w = 0; w < wid; ++w) pre += lds[w];
  __syncthreads();
  return v + pre;
}

__global__ __launch_bounds__(kPB) void k_ps_reduce(const int* a, int n, long long* bsum) {
  __shared__ long long lds[kPB / 64];
  long long s = 0;
  for (int k = threadIdx.x; k < kTile; k += kPB) {
    const int i = blockIdx.x * kTile + k;
    if (i < n) s += a[i];
  }
  s = block_sum_ll(s, lds);
  if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

__global__ __launch_bounds__(kPB) void k_ps_blocks(long long* bsum, int nb) {
  __shared__ long long lds[kPB / 64];
  __shared__ long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += kPB) {
    const int i = base + threadIdx.x;
    const long long v = i < nb ? bsum[i] : 0;
    const long long inc = block_incl_scan(v, lds);
    const long long c = carry;
    if (i < nb) bsum[i] = c + inc - v;
    __syncthreads();
    if (threadIdx.x == kPB - 1) carry = c + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(kPB) void k_ps_apply(const int* a, int n, const long long* boff,
                                                 int* out) {
  __shared__ long long lds[kPB / 64];
  const int base = blockIdx.x * kTile + threadIdx.x * kPer;
  long long v[kPer], s = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    v[k] = base + k < n ? a[base + k] : 0;
    s += v[k];
  }
  long long run = boff[blockIdx.x] + block_incl_scan(s, lds) - s;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (base + k < n) out[base + k] = (int)run;
    run += v[k];
  }
}

// ---- induced subgraph ---------------------------------------------------------

// For every vertex of part p: its degree inside the part; in[v] = 1 when it
// has one (it enters the subgraph), iso[v] = 1 when it has none.
__global__ void k_part_degree(int n, const int* __restrict__ rp, const int* __restrict__ col,
                              const int* __restrict__ part, int p, int* deg, int* in, int* iso) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int d = 0;
  const bool mine = part[v] == p;
  if (mine)
    for (int k = rp[v]; k < rp[v + 1]; ++k) d += part[col[k]] == p;
  deg[v] = d;
  in[v] = mine && d > 0;
  iso[v] = mine && d == 0;
}

// Subgraph CSR in the part's vertex order (which keeps each row's columns
// ascending): row newid[v] of the subgraph is v's row restricted to the part.
__global__ void k_part_fill(int n, const int* __restrict__ rp, const int* __restrict__ col,
                            const double* __restrict__ w, const int* __restrict__ part, int p,
                            const int* __restrict__ in, const int* __restrict__ newid,
                            const int* __restrict__ off, int* srp, int* scol, double* sw,
                            int* orig) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || !in[v]) return;
  const int j = newid[v];
  int o = off[v];
  srp[j] = o;
  orig[j] = v;
  for (int k = rp[v]; k < rp[v + 1]; ++k) {
    const int u = col[k];
    if (part[u] == p) {
      scol[o] = newid[u];
      sw[o] = w[k];
      ++o;
    }
  }
}

__global__ void k_set_int(int* a, int v) { *a = v; }

// ---- median selection (most significant digit first radix select) -------------

// A total order on doubles as unsigned integers (no NaNs here); -0 and +0 are
// made equal first.
__device__ inline unsigned long long order_key(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x + 0.0);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ULL);
}

// 256-bin histogram of digit `shift` of the keys whose higher digits equal
// prefix (under mask).
__global__ __launch_bounds__(kPB) void k_digit_hist(int n, const double* __restrict__ x,
                                                   unsigned long long prefix,
                                                   unsigned long long mask, int shift,
                                                   unsigned* hist) {
  __shared__ unsigned h[256];
  for (int b = threadIdx.x; b < 256; b += kPB) h[b] = 0;
  __syncthreads();
  for (int i = blockIdx.x * kPB + threadIdx.x; i < n; i += gridDim.x * kPB) {
    const unsigned long long k = order_key(x[i]);
    if ((k & mask) == prefix) atomicAdd(&h[(k >> shift) & 255], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < 256; b += kPB)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// Median cut: child 0 for keys below K, and for keys equal to K the first
// `need` in index order (tie_rank: their exclusive rank among the ties).
__global__ void k_tie_flags(int n, const double* __restrict__ x, unsigned long long K, int* tie) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) tie[i] = order_key(x[i]) == K;
}

__global__ void k_split_median(int n, const double* __restrict__ x, unsigned long long K,
                               const int* __restrict__ tie_rank, int need,
                               const int* __restrict__ orig, int base, int* next) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned long long k = order_key(x[i]);
  const int c = k < K ? 0 : (k > K ? 1 : (tie_rank[i] < need ? 0 : 1));
  next[orig[i]] = base + c;
}

__global__ void k_split_sign(int n, const double* __restrict__ x, const int* __restrict__ orig,
                             int base, int* next, int* count0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool neg = false;
  if (i < n) {
    neg = x[i] + 0.0 < 0.0;  // -0 counts as 0: child 1
    next[orig[i]] = base + (neg ? 0 : 1);
  }
  const unsigned long long b = __ballot(neg);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(count0, (int)__popcll(b));
}

__global__ void k_assign_iso(int n, const int* __restrict__ iso, int label, int* next) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && iso[v]) next[v] = label;
}

// Cut weight (each undirected edge once), total weight, part sizes.
__global__ __launch_bounds__(kPB) void k_part_stats(int n, const int* __restrict__ rp,
                                                   const int* __restrict__ col,
                                                   const double* __restrict__ w,
                                                   const int* __restrict__ part, double* sums,
                                                   int* sizes) {
  __shared__ double lds[block_sum_lds(kPB)];
  double s[2] = {0.0, 0.0};
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) {
    const int pv = part[v];
    for (int k = rp[v]; k < rp[v + 1]; ++k)
      if (col[k] > v) {
        s[1] += w[k];
        if (part[col[k]] != pv) s[0] += w[k];
      }
    atomicAdd(&sizes[pv], 1);
  }
  block_sum<2>(s, lds);
  if (threadIdx.x == 0) {
    atomicAdd(&sums[0], s[0]);
    atomicAdd(&sums[1], s[1]);
  }
}

inline int nb_of(long long n, int b = kPB) { return (int)std::max<long long>(1, (n + b - 1) / b); }

struct DevBuf {
  fv_context* ctx;
  void* p = nullptr;
  DevBuf(fv_context* c, size_t bytes) : ctx(c) { p = block_get(c, bytes); }
  ~DevBuf() { block_put(ctx, p); }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

}  // namespace

__global__ void k_iota_int(int n, int* a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = i;
}

fv_status spectral_partition(fv_context* ctx, const fv_csr* g, const fv_hier_opts* ho,
                             const fv_solve_opts* so, const fv_partition_opts* po,
                             int32_t* part_out, int part_on_device, fv_partition_stats* st) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!g->is_adjacency) return FV_E_INVALID;  // the weights W, no diagonal
  hipStream_t s = so->stream ? static_cast<hipStream_t>(so->stream) : ctx->stream;
  const int n = g->n;
  const long long m = g->nnz;
  // The first cut solves the whole graph: its hierarchy build also validates
  // the input (errors as fv_build_hierarchy) before any kernel here reads it.
  fv_hierarchy* h0 = build_hierarchy(ctx, g, ho, s);
  struct HGuard {
    fv_hierarchy* h;
    ~HGuard() {
      if (h) free_hierarchy(h, true);
    }
  } hg{h0};
  DevBuf rp(ctx, sizeof(int) * (n + 1)), col(ctx, sizeof(int) * std::max<long long>(m, 1)),
      w(ctx, sizeof(double) * std::max<long long>(m, 1));
  const hipMemcpyKind kind = g->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  FV_HIP(hipMemcpyAsync(rp.p, g->row_ptr, sizeof(int) * (n + 1), kind, s));
  if (m) {
    FV_HIP(hipMemcpyAsync(col.p, g->col, sizeof(int) * m, kind, s));
    FV_HIP(hipMemcpyAsync(w.p, g->val, sizeof(double) * m, kind, s));
  }
  DevBuf part(ctx, sizeof(int) * n), next(ctx, sizeof(int) * n), deg(ctx, sizeof(int) * n),
      in(ctx, sizeof(int) * n), iso(ctx, sizeof(int) * n), newid(ctx, sizeof(int) * (n + 1)),
      off(ctx, sizeof(int) * (n + 1)), orig(ctx, sizeof(int) * n), tie(ctx, sizeof(int) * (n + 1)),
      srp(ctx, sizeof(int) * (n + 1)), scol(ctx, sizeof(int) * std::max<long long>(m, 1)),
      sw(ctx, sizeof(double) * std::max<long long>(m, 1)), x(ctx, sizeof(double) * n),
      bsum(ctx, sizeof(long long) * (nb_of(n + 1, kTile) + 2)),
      misc(ctx, sizeof(unsigned) * (512 + 16 + (size_t)po->parts));
  int* pin = static_cast<int*>(pin_get(ctx));  // kPinBytes
  struct PinGuard {
    fv_context* c;
    void* p;
    hipStream_t s;
    ~PinGuard() { pin_put(c, p, s); }
  } pg{ctx, pin, s};
  FV_HIP(hipMemsetAsync(part.p, 0, sizeof(int) * n, s));

  // Exclusive scan of a[0, cnt) into out (out[cnt] = total); returns the total.
  auto scan = [&](const int* a, int cnt, int* out) -> long long {
    const int nb = nb_of(cnt, kTile);
    long long* bs = bsum.as<long long>();
    k_ps_reduce<<<nb, kPB, 0, s>>>(a, cnt, bs);
    k_ps_blocks<<<1, kPB, 0, s>>>(bs, nb);
    k_ps_apply<<<nb, kPB, 0, s>>>(a, cnt, bs, out);
    FV_HIP(hipMemcpyAsync(pin, bs + nb, sizeof(long long), hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    const long long total = *reinterpret_cast<long long*>(pin);
    k_set_int<<<1, 1, 0, s>>>(out + cnt, (int)total);
    return total;
  };

  int solves = 0, not_conv = 0;
  // Solves h (nsub vertices, orig[j] the input vertex of its vertex j) and
  // labels its vertices base or base + 1 in next; returns the two sizes.
  auto solve_split = [&](fv_hierarchy* h, int nsub, int base, int* c0, int* c1) -> fv_status {
    const fv_status rs = solve_one_with(ctx, ctx->scratch, h, so, x.as<double>(), 1, nullptr,
                                        nullptr, s);
    ++solves;
    if (rs == FV_E_NOT_CONVERGED) ++not_conv;
    else if (rs != FV_OK) return rs;
    if (po->cut == 1) {
      int* cnt0 = reinterpret_cast<int*>(misc.p);
      k_set_int<<<1, 1, 0, s>>>(cnt0, 0);
      k_split_sign<<<nb_of(nsub), kPB, 0, s>>>(nsub, x.as<double>(), orig.as<int>(), base,
                                               next.as<int>(), cnt0);
      FV_HIP(hipMemcpyAsync(pin, cnt0, sizeof(int), hipMemcpyDeviceToHost, s));
      FV_HIP(hipStreamSynchronize(s));
      *c0 = pin[0];
      *c1 = nsub - *c0;
      return FV_OK;
    }
    // Median: the hs = nsub / 2 smallest (value, index) pairs form child 0.
    // Radix-select the hs-th smallest key K, 8 bits at a time from the top,
    // then give child 0 the first `need` vertices (in index order) whose key
    // equals K.
    const int hs = nsub / 2;
    unsigned* hist = reinterpret_cast<unsigned*>(misc.p);
    unsigned long long prefix = 0, mask = 0;
    long long below = 0;  // keys below the selected bucket so far
    long long rank = hs;  // rank of K (1-based) among the keys matching prefix
    for (int shift = 56; shift >= 0; shift -= 8) {
      FV_HIP(hipMemsetAsync(hist, 0, sizeof(unsigned) * 256, s));
      k_digit_hist<<<std::min(nb_of(nsub), 1024), kPB, 0, s>>>(nsub, x.as<double>(), prefix,
                                                                mask, shift, hist);
      FV_HIP(hipMemcpyAsync(pin, hist, sizeof(unsigned) * 256, hipMemcpyDeviceToHost, s));
      FV_HIP(hipStreamSynchronize(s));
      const unsigned* hh = reinterpret_cast<const unsigned*>(pin);
      int b = 0;
      long long acc = 0;
      while (b < 255 && acc + (long long)hh[b] < rank) acc += hh[b++];
      rank -= acc;
      below += acc;
      prefix |= (unsigned long long)b << shift;
      mask |= 255ULL << shift;
    }
    const int need = hs - (int)below;
    k_tie_flags<<<nb_of(nsub), kPB, 0, s>>>(nsub, x.as<double>(), prefix, tie.as<int>());
    scan(tie.as<int>(), nsub, off.as<int>());
    k_split_median<<<nb_of(nsub), kPB, 0, s>>>(nsub, x.as<double>(), prefix, off.as<int>(), need,
                                               orig.as<int>(), base, next.as<int>());
    FV_HIP(hipGetLastError());
    *c0 = hs;
    *c1 = nsub - hs;
    return FV_OK;
  };

  int levels = 0;
  while ((1 << levels) < po->parts) ++levels;
  for (int d = 0; d < levels; ++d) {
    FV_HIP(hipMemcpyAsync(next.p, part.p, sizeof(int) * n, hipMemcpyDeviceToDevice, s));
    for (int p = 0; p < (1 << d); ++p) {
      const int base = 2 * p;
      int c0 = 0, c1 = 0;
      if (d == 0) {
        // the whole (validated, isolated-free) graph
        k_iota_int<<<nb_of(n), kPB, 0, s>>>(n, orig.as<int>());
        const fv_status rs = solve_split(h0, n, base, &c0, &c1);
        free_hierarchy(h0, true);
        hg.h = nullptr;
        if (rs != FV_OK) return rs;
        continue;
      }
      k_part_degree<<<nb_of(n), kPB, 0, s>>>(n, rp.as<int>(), col.as<int>(), part.as<int>(), p,
                                            deg.as<int>(), in.as<int>(), iso.as<int>());
      const int nsub = (int)scan(in.as<int>(), n, newid.as<int>());
      const long long niso = scan(iso.as<int>(), n, off.as<int>());
      // row starts of the subgraph: the in-part degrees (zero outside it)
      const long long msub = scan(deg.as<int>(), n, off.as<int>());
      // A vertex with an edge inside the part has a neighbour there with one
      // too, so nsub is 0 or at least 2.
      if (nsub >= 2) {
        k_part_fill<<<nb_of(n), kPB, 0, s>>>(n, rp.as<int>(), col.as<int>(), w.as<double>(),
                                            part.as<int>(), p, in.as<int>(), newid.as<int>(),
                                            off.as<int>(), srp.as<int>(), scol.as<int>(),
                                            sw.as<double>(), orig.as<int>());
        k_set_int<<<1, 1, 0, s>>>(srp.as<int>() + nsub, (int)msub);
        FV_HIP(hipGetLastError());
        fv_csr sub{nsub, (int32_t)msub, srp.as<int>(), scol.as<int>(), sw.as<double>(), 1, 1};
        fv_hierarchy* h = build_hierarchy(ctx, &sub, ho, s);
        fv_status rs;
        try {
          rs = solve_split(h, nsub, base, &c0, &c1);
        } catch (...) {
          (void)hipStreamSynchronize(s);
          free_hierarchy(h, false);
          throw;
        }
        FV_HIP(hipStreamSynchronize(s));
        free_hierarchy(h, false);
        if (rs != FV_OK) return rs;
      }
      // vertices without an edge inside the part join the smaller half
      if (niso > 0)
        k_assign_iso<<<nb_of(n), kPB, 0, s>>>(n, iso.as<int>(), base + (c1 < c0 ? 1 : 0),
                                              next.as<int>());
      FV_HIP(hipGetLastError());
    }
    FV_HIP(hipMemcpyAsync(part.p, next.p, sizeof(int) * n, hipMemcpyDeviceToDevice, s));
  }
  // statistics and output
  const int parts = 1 << levels;
  double* sums = reinterpret_cast<double*>(misc.p);
  int* sizes = reinterpret_cast<int*>(misc.as<char>() + 64);
  FV_HIP(hipMemsetAsync(misc.p, 0, 64 + sizeof(int) * parts, s));
  k_part_stats<<<nb_of(n), kPB, 0, s>>>(n, rp.as<int>(), col.as<int>(), w.as<double>(),
                                        part.as<int>(), sums, sizes);
  FV_HIP(hipGetLastError());
  std::vector<int> hsz(parts);
  double hs[2];
  FV_HIP(hipMemcpyAsync(hs, sums, sizeof(hs), hipMemcpyDeviceToHost, s));
  FV_HIP(hipMemcpyAsync(hsz.data(), sizes, sizeof(int) * parts, hipMemcpyDeviceToHost, s));
  FV_HIP(hipMemcpyAsync(part_out, part.p, sizeof(int) * n,
                        part_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  FV_HIP(hipStreamSynchronize(s));
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->parts = parts;
    st->cut_weight = hs[0];
    st->total_weight = hs[1];
    st->part_size_min = *std::min_element(hsz.begin(), hsz.end());
    st->part_size_max = *std::max_element(hsz.begin(), hsz.end());
    st->solves = solves;
    st->not_converged = not_conv;
    st->t_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return FV_OK;
}

}  // namespace fv
