// One-workgroup engine driver (included by solve.hip): one workgroup runs the
// coarsest solve and then every level from the coarsest up to T.stop, all
// phases and sweeps, without leaving the kernel.
//
// A level is worked on through a view whose pointer types are template
// parameters, so the compiler emits LDS instructions (ds_read/ds_write) when
// the data sits in LDS rather than generic flat accesses:
//   * vector and CSR in LDS (small levels: everything stays on chip),
//   * vector, column indices and row pointers in LDS, weights from global
//     memory (L2-resident),
//   * vector in LDS, CSR read from global memory (L2-resident),
//   * everything in global memory.
// Between levels the vector passes through one of two global buffers, which
// also serve as the scratch output of the power steps.
#pragma once

template <class T>
using lds_ptr = __attribute__((address_space(3))) T*;

// Workgroup-wide copy between any two pointers (global, LDS or generic).
template <class DP, class SP>
__device__ inline void wg_copy(DP dst, SP src, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
}

template <class XP, class IP, class WP>
struct LView {
  int n, ncol;
  IP rp, col;   // CSR (solve order)
  WP w;         // working-precision weights
  const int* cptr;
  const int* qs;
  const int* perm;
  const int* iperm;
  const double* w64;  // FP64 weights (global), for the Rayleigh quotient
  double sigma;
};

// ---- per-row arithmetic on a view (same operation order as row_gs & co.) --

// Neighbours of a row are fetched in batches of kRowU entries: the batch's
// column indices and weights are loaded first (indices past the row end
// repeat its last entry, so no load is conditional), then the neighbour
// values, and only then is any of them used.  The scheduling barriers keep
// the compiler from interleaving loads and uses (it otherwise waits for each
// weight before issuing the next load: one memory round trip per entry).
// The first batch's values stay in registers for the edge-energy pass; later
// batches are fetched again for it.  The sums take the same terms in the same
// order as a plain loop over the row (padding entries add exact zeros at the
// end).  Eight entries cover most coarse rows in one batch (four left the
// engine's sweeps 8 % slower: a second dependent round trip).
constexpr int kRowU = 8;

template <class VT, class V, class XP>
__device__ __forceinline__ void vrow_batch(const V& L, XP x, int pb, int p1, int (&jj)[kRowU],
                                           double (&ww)[kRowU], double (&xx)[kRowU]) {
  VT wr[kRowU], xr[kRowU];
#pragma unroll
  for (int u = 0; u < kRowU; ++u) jj[u] = L.col[min(pb + u, p1 - 1)];
#pragma unroll
  for (int u = 0; u < kRowU; ++u) wr[u] = L.w[min(pb + u, p1 - 1)];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < kRowU; ++u) xr[u] = x[jj[u]];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < kRowU; ++u) {
    ww[u] = pb + u < p1 ? (double)wr[u] : 0.0;
    xx[u] = (double)xr[u];
  }
}

// A row's bounds, own value and first batch of neighbours (indices, weights,
// values), loaded before any is used.
struct RowHead {
  int p0, p1;
  double xr;
  int jj[kRowU];
  double ww[kRowU], xx[kRowU];
};

// The update of row i from its loaded head: later batches are fetched here,
// the new value stored, and the row's sums added to acc.
template <class VT, class V, class XP>
__device__ __forceinline__ void vrow_finish(int i, const RowHead& H, const V& L, XP x,
                                            int lower_end, double mu, double inv_s, double rho,
                                            double omega, double (&acc)[kNP]) {
  const int p0 = H.p0, p1 = H.p1;
  const double xo = (H.xr - mu) * inv_s;
  double num = 0.0, den = 0.0;
  if (p1 > p0)
#pragma unroll
    for (int u = 0; u < kRowU; ++u) {
      num += H.ww[u] * (H.jj[u] < lower_end ? H.xx[u] : (H.xx[u] - mu) * inv_s);
      den += H.ww[u];
    }
  for (int pb = p0 + kRowU; pb < p1; pb += kRowU) {
    int jj[kRowU];
    double ww[kRowU], xx[kRowU];
    vrow_batch<VT>(L, x, pb, p1, jj, ww, xx);
#pragma unroll
    for (int u = 0; u < kRowU; ++u) {
      num += ww[u] * (jj[u] < lower_end ? xx[u] : (xx[u] - mu) * inv_s);
      den += ww[u];
    }
  }
  double u = xo;
  if (den > 0.0) {
    const double g = (num + rho * xo) / den;
    u = omega == 1.0 ? g : (1.0 - omega) * xo + omega * g;
  }
  const VT us = (VT)u;
  x[i] = us;
  const double ud = (double)us;
  double e = 0.0;
  if (p1 > p0)
#pragma unroll
    for (int k = 0; k < kRowU; ++k) {
      const double d = ud - H.xx[k];
      e += (H.jj[k] < lower_end ? H.ww[k] : 0.0) * d * d;
    }
  for (int pb = p0 + kRowU; pb < p1; pb += kRowU) {
    int jj[kRowU];
    double ww[kRowU], xx[kRowU];
    vrow_batch<VT>(L, x, pb, p1, jj, ww, xx);
#pragma unroll
    for (int k = 0; k < kRowU; ++k) {
      const double d = ud - xx[k];
      e += (jj[k] < lower_end ? ww[k] : 0.0) * d * d;
    }
  }
  acc[0] += ud;
  acc[1] += ud * ud;
  acc[2] += ud * xo;
  acc[3] += xo;
  acc[4] += e;
}

template <class VT, class V, class XP>
__device__ __forceinline__ void vrow_gs(int i, const V& L, XP x, int lower_end, double mu, double inv_s,
                               double rho, double omega, double (&acc)[kNP]) {
  RowHead H;
  H.p0 = L.rp[i];
  H.p1 = L.rp[i + 1];
  H.xr = (double)x[i];
  if (H.p1 > H.p0) vrow_batch<VT>(L, x, H.p0, H.p1, H.jj, H.ww, H.xx);
  vrow_finish<VT>(i, H, L, x, lower_end, mu, inv_s, rho, omega, acc);
}

// Rows iA and iB (iA first) of one colour with their first batches loaded
// together: both rows' pointers and own values, then both batches' indices and
// weights, then both batches' gathers, so the two rows cost the dependent load
// phases of one.  Rows of one colour have no edges among them, so neither
// reads the other's new value; the sums are added in the order of two
// vrow_gs calls.  A row without entries takes the plain path.
template <class VT, class V, class XP>
__device__ __forceinline__ void vrow_gs2(int iA, int iB, const V& L, XP x, int lower_end,
                                         double mu, double inv_s, double rho, double omega,
                                         double (&acc)[kNP]) {
  RowHead A, B;
  A.p0 = L.rp[iA];
  A.p1 = L.rp[iA + 1];
  B.p0 = L.rp[iB];
  B.p1 = L.rp[iB + 1];
  const VT xa = x[iA], xb = x[iB];
  if (A.p1 <= A.p0 || B.p1 <= B.p0) {
    vrow_gs<VT>(iA, L, x, lower_end, mu, inv_s, rho, omega, acc);
    vrow_gs<VT>(iB, L, x, lower_end, mu, inv_s, rho, omega, acc);
    return;
  }
  A.xr = (double)xa;
  B.xr = (double)xb;
  VT wa[kRowU], wb[kRowU], ga[kRowU], gb[kRowU];
#pragma unroll
  for (int u = 0; u < kRowU; ++u) A.jj[u] = L.col[min(A.p0 + u, A.p1 - 1)];
#pragma unroll
  for (int u = 0; u < kRowU; ++u) B.jj[u] = L.col[min(B.p0 + u, B.p1 - 1)];
#pragma unroll
  for (int u = 0; u < kRowU; ++u) wa[u] = L.w[min(A.p0 + u, A.p1 - 1)];
#pragma unroll
  for (int u = 0; u < kRowU; ++u) wb[u] = L.w[min(B.p0 + u, B.p1 - 1)];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < kRowU; ++u) ga[u] = x[A.jj[u]];
#pragma unroll
  for (int u = 0; u < kRowU; ++u) gb[u] = x[B.jj[u]];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < kRowU; ++u) {
    A.ww[u] = A.p0 + u < A.p1 ? (double)wa[u] : 0.0;
    A.xx[u] = (double)ga[u];
    B.ww[u] = B.p0 + u < B.p1 ? (double)wb[u] : 0.0;
    B.xx[u] = (double)gb[u];
  }
  vrow_finish<VT>(iA, A, L, x, lower_end, mu, inv_s, rho, omega, acc);
  vrow_finish<VT>(iB, B, L, x, lower_end, mu, inv_s, rho, omega, acc);
}

template <class VT, class V, class XP>
__device__ __forceinline__ Scal vsweep(const V& L, XP x, Scal s, double omega, EngineCtx& E) {
  double acc[kNP] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int c = 0; c < L.ncol; ++c) {
    const int r0 = L.cptr[c], r1 = L.cptr[c + 1];
    const int bd = blockDim.x;
    int i = r0 + threadIdx.x;
    if constexpr (sizeof(VT) == 4)  // FP64 pairs would spill registers
      for (; i + bd < r1; i += 2 * bd)
        vrow_gs2<VT>(i, i + bd, L, x, r0, s.mu, s.inv_s, s.rho, omega, acc);
    for (; i < r1; i += bd) vrow_gs<VT>(i, L, x, r0, s.mu, s.inv_s, s.rho, omega, acc);
    if (c + 1 < L.ncol) __syncthreads();  // the last colour: block_allsum's barrier
  }
  block_allsum<kNP>(acc, E.red, E.flip);
  return after_gs(acc, L.n);
}

// Power step: y (global scratch) = sigma xhat - L xhat, then y is copied back
// into x, so the vector keeps its place.
template <class VT, class V, class XP>
__device__ __forceinline__ Scal vpi_step(const V& L, XP x, VT* y, Scal s, EngineCtx& E) {
  double acc[kNP] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < L.n; i += blockDim.x) {
    const double xi = (double)x[i];
    double lx = 0.0;
    for (int p = L.rp[i]; p < L.rp[i + 1]; ++p)
      lx += (double)L.w[p] * (xi - (double)x[L.col[p]]);
    const double xo = (xi - s.mu) * s.inv_s;
    const VT ys = (VT)(L.sigma * xo - lx * s.inv_s);
    y[i] = ys;
    const double yd = (double)ys;
    acc[0] += yd;
    acc[1] += yd * yd;
    acc[2] += yd * xo;
    acc[3] += xo;
  }
  block_allsum<kNP>(acc, E.red, E.flip);  // its barrier also orders the y writes
  for (int i = threadIdx.x; i < L.n; i += blockDim.x) x[i] = y[i];
  __syncthreads();
  Scal r = after_gs(acc, L.n);
  r.rho = s.rho;
  return r;
}

// Prolongation from a global coarse vector into x, plus v^T L v for the shift.
template <class VT, class SRC, class V, class XP>
__device__ __forceinline__ Scal vprolong(const V& L, const SRC* xc, XP xf, Scal s, EngineCtx& E) {
  double acc[kNP] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < L.n; i += blockDim.x) {
    const VT vs = (VT)(((double)xc[L.qs[i]] - s.mu) * s.inv_s);
    xf[i] = vs;
    const double v = (double)vs;
    double e = 0.0;
    for (int p = L.rp[i]; p < L.rp[i + 1]; ++p) {
      const double vj = (double)(VT)(((double)xc[L.qs[L.col[p]]] - s.mu) * s.inv_s);
      const double d = v - vj;
      e += (double)L.w[p] * d * d;
    }
    acc[0] += v;
    acc[1] += v * v;
    acc[4] += 0.5 * e;
  }
  block_allsum<kNP>(acc, E.red, E.flip);  // its barrier also orders the xf writes
  return after_prolong(acc, L.n);
}

// Rayleigh quotient (FP64 weights), residual and sign on the finest level.
template <class VT, class V, class XP>
__device__ __forceinline__ void vrq_residual(const V& L, XP x, const Scal& s, double* lx, double& lam,
                             double& res, double& sign, EngineCtx& E) {
  double a3[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < L.n; i += blockDim.x) {
    const double xi = ((double)x[i] - s.mu) * s.inv_s;
    double l = 0.0, e = 0.0;
    for (int p = L.rp[i]; p < L.rp[i + 1]; ++p) {
      const double d = xi - ((double)x[L.col[p]] - s.mu) * s.inv_s;
      l += L.w64[p] * d;
      e += L.w64[p] * d * d;
    }
    lx[i] = l;
    a3[0] += xi * xi;
    a3[1] += 0.5 * e;
    a3[2] = fmax(a3[2], fabs(xi));
  }
  __syncthreads();
  const double mx = block_max(a3[2], E.lds);
  double t[2] = {a3[0], a3[1]};
  block_sum<2>(t, E.lds);
  lam = t[1] / t[0];
  const double thr = 1e-3 * mx;
  double r[1] = {0.0};
  int cand = INT_MAX;
  for (int i = threadIdx.x; i < L.n; i += blockDim.x) {
    const double xh = ((double)x[i] - s.mu) * s.inv_s;
    const double d = lx[i] - lam * xh;
    r[0] += d * d;
    if (fabs(xh) >= thr) cand = min(cand, L.iperm[i]);
  }
  block_sum<1>(r, E.lds);
  cand = block_min_int(cand, E.ilds);
  res = sqrt(r[0] / t[0]);
  const double xv = cand < INT_MAX ? ((double)x[L.perm[cand]] - s.mu) * s.inv_s : 1.0;
  sign = xv < 0.0 ? -1.0 : 1.0;
}

template <class VT, class V, class XP>
__device__ __forceinline__ int vgs_phase(const V& L, XP x, Scal& s, double omega, PhaseCfg P, EngineCtx& E) {
  const int lim = P.forced >= 0 ? P.forced : P.cap;
  int k = 0;
  while (k < lim) {
    s = vsweep<VT>(L, x, s, omega, E);
    ++k;
    if (P.forced < 0 && P.tol > 0.0 && s.cos > 1.0 - P.tol) break;
  }
  return k;
}

template <class VT, class V, class XP>
__device__ __forceinline__ int vpi_phase(const V& L, XP x, VT* y, Scal& s, PhaseCfg P, EngineCtx& E) {
  const int lim = P.forced >= 0 ? P.forced : P.cap;
  int k = 0;
  while (k < lim) {
    s = vpi_step<VT>(L, x, y, s, E);
    ++k;
    if (P.forced < 0 && P.tol > 0.0 && s.cos > 1.0 - P.tol) break;
  }
  return k;
}

// ---- views ------------------------------------------------------------------

template <class VT>
using GView = LView<VT*, const int*, const VT*>;
template <class VT>
using XView = LView<lds_ptr<VT>, const int*, const VT*>;
template <class VT>
using SView = LView<lds_ptr<VT>, lds_ptr<const int>, lds_ptr<const VT>>;
template <class VT>
using IView = LView<lds_ptr<VT>, lds_ptr<const int>, const VT*>;

// The colour ranges of the level in LDS (when there are at most kEngineMaxCol
// colours): every colour step reads its bounds, and a global load there would
// put a memory round trip on the critical path of each colour.
__device__ __forceinline__ const int* stage_cptr(const LevelDesc& D, EngineCtx& E) {
  if (D.ncol > kEngineMaxCol) return D.cptr;
  __syncthreads();  // the previous level's steps are done with E.cptr
  for (int k = threadIdx.x; k <= D.ncol; k += blockDim.x) E.cptr[k] = D.cptr[k];
  __syncthreads();
  return E.cptr;
}

template <class V, class IP, class WP>
__device__ __forceinline__ V make_view(const LevelDesc& D, const int* cptr, IP rp, IP col, WP w) {
  V v;
  v.n = D.n;
  v.ncol = D.ncol;
  v.rp = rp;
  v.col = col;
  v.w = w;
  v.cptr = cptr;
  v.qs = D.qs;
  v.perm = D.perm;
  v.iperm = D.iperm;
  v.w64 = D.w64;
  v.sigma = D.sigma;
  return v;
}

// LDS layout of a level: the vector at offset 0, then (when it fits) the
// weights, column indices and row pointers.  Returns true when the CSR was
// staged.
template <class VT>
__device__ __forceinline__ bool stage_csr(const LevelDesc& D, EngineCtx& E, size_t& w_off, size_t& c_off,
                                 size_t& r_off) {
  w_off = ((size_t)D.n * sizeof(VT) + 15) & ~(size_t)15;
  c_off = w_off + (((size_t)D.m * sizeof(VT) + 15) & ~(size_t)15);
  r_off = c_off + (((size_t)D.m * 4 + 15) & ~(size_t)15);
  if (r_off + (size_t)(D.n + 1) * 4 > (size_t)E.bytes) return false;
  unsigned char* base = static_cast<unsigned char*>(E.xl);
  wg_copy(reinterpret_cast<VT*>(base + w_off), WSel<VT>::w(D), (int)D.m);
  wg_copy(reinterpret_cast<int*>(base + c_off), D.col, (int)D.m);
  wg_copy(reinterpret_cast<int*>(base + r_off), D.rp, D.n + 1);
  return true;
}

// When the whole CSR does not fit: the vector, the column indices and the row
// pointers (in that order) without the weights.  A row's weight loads then
// come from L2 alongside its index loads from LDS instead of after a row
// pointer load from L2.  Returns true when staged.
template <class VT>
__device__ __forceinline__ bool stage_index(const LevelDesc& D, EngineCtx& E, size_t& c_off,
                                            size_t& r_off) {
  c_off = ((size_t)D.n * sizeof(VT) + 15) & ~(size_t)15;
  r_off = c_off + (((size_t)D.m * 4 + 15) & ~(size_t)15);
  if (r_off + (size_t)(D.n + 1) * 4 > (size_t)E.bytes) return false;
  unsigned char* base = static_cast<unsigned char*>(E.xl);
  wg_copy(reinterpret_cast<int*>(base + c_off), D.col, (int)D.m);
  wg_copy(reinterpret_cast<int*>(base + r_off), D.rp, D.n + 1);
  return true;
}

// Processes one level in a given view: prolongation from the global coarse
// vector, smoothing phase, power phase.  Returns (g, p) through refs.
template <class VT, class SRC, class V, class XP>
__device__ __forceinline__ void run_level(const V& L, XP x, const SRC* xc, VT* ytmp, Scal& s, const GraphTask& T,
                          int fg, int fp, int& g, int& p, EngineCtx& E) {
  s = vprolong<VT>(L, xc, x, s, E);
  PhaseCfg pg{fg, T.max_gs, T.tol_cos};
  g = vgs_phase<VT>(L, x, s, T.omega, pg, E);
  PhaseCfg pp{fp, T.max_pi, T.tol_cos};
  p = vpi_phase<VT>(L, x, ytmp, s, pp, E);
}

// Finest-level repeats, Rayleigh quotient, residual and output.
template <class VT, class V, class XP>
__device__ __forceinline__ void finish_level0(const V& L, XP x, VT* ytmp, Scal& s, const GraphTask& T, int J,
                              int& si, int& slen, double& lam, double& res, EngineCtx& E) {
  double sign = 1.0;
  vrq_residual<VT>(L, x, s, T.lx, lam, res, sign, E);
  double res_prev = res;
  int outer = 0;
  if (J > 0) {
    for (;;) {
      int fg, fp;
      if (T.replay) {
        if (si >= T.replay_len) break;
        fg = T.replay[si++];
        fp = si < T.replay_len ? T.replay[si++] : -1;
      } else {
        if (!(T.tol_res > 0.0) || res <= T.tol_res || outer >= T.max_outer) break;
        if (T.early_exit && outer > 0 &&
            !can_reach(res, res_prev, T.tol_res, T.max_outer - outer))
          break;
        fg = fp = -1;
      }
      s.rho = lam;
      PhaseCfg pg{fg, T.max_gs, T.tol_cos};
      const int g = vgs_phase<VT>(L, x, s, T.omega, pg, E);
      PhaseCfg pp{fp, T.max_pi, T.tol_cos};
      const int p = vpi_phase<VT>(L, x, ytmp, s, pp, E);
      if (threadIdx.x == 0 && slen + 1 < FV_SCHEDULE_CAP) {
        T.sched[slen] = g;
        T.sched[slen + 1] = p;
      }
      slen += 2;
      ++outer;
      __syncthreads();
      res_prev = res;
      vrq_residual<VT>(L, x, s, T.lx, lam, res, sign, E);
    }
  }
  for (int v = threadIdx.x; v < L.n; v += blockDim.x)
    T.x_out[v] = sign * (((double)x[L.perm[v]] - s.mu) * s.inv_s);
}

template <class VT>
__device__ void engine_run(const GraphTask& T, EngineCtx& E) {
  const LevelDesc* lv = T.lv;
  const int J = T.J;
  int si = 0;  // replay cursor
  auto next_forced = [&]() -> int { return (T.replay && si < T.replay_len) ? T.replay[si++] : -1; };
  int slen = 0;
  auto push = [&](int v) {
    if (threadIdx.x == 0 && slen < FV_SCHEDULE_CAP) T.sched[slen] = v;
    ++slen;
  };
  VT* const Ga = static_cast<VT*>(T.xa);
  VT* const Gb = static_cast<VT*>(T.xb);
  auto G = [&](int k) -> VT* { return k ? Gb : Ga; };
  double* xa64 = static_cast<double*>(T.xa);
  unsigned char* lbase = static_cast<unsigned char*>(E.xl);
  lds_ptr<VT> xl = (lds_ptr<VT>)(reinterpret_cast<VT*>(lbase));
  int conv = 0;
  const int cit =
      engine_coarsest(lv[J], T.seed, T.max_coarsest, next_forced(), T.tol_coarse, xa64, T.lx,
                      &conv, E);
  push(cit);
  __syncthreads();
  Scal s{0.0, 1.0, 1.0, 0.0};
  int gsrc = 0;         // global buffer holding the current vector between levels
  bool src64 = true;    // it is the FP64 coarsest iterate
  int final_mode = -1;  // how level 0 was kept: 0 global, 1 LDS vector, 2 LDS vector + CSR
  for (int l = J - 1; l >= T.stop; --l) {
    const LevelDesc D = lv[l];
    const int gfree = 1 - gsrc;
    const bool keep = (l == 0 && T.finalize);  // level 0 stays where it is for the finish
    int g = 0, p = 0;
    const int fg = next_forced(), fp = next_forced();
    if (D.n <= E.cap) {
      size_t wo, co, ro;
      const bool staged = stage_csr<VT>(D, E, wo, co, ro);
      if (staged) {
        SView<VT> L = make_view<SView<VT>>(D, stage_cptr(D, E), (lds_ptr<const int>)(reinterpret_cast<const int*>(lbase + ro)),
            (lds_ptr<const int>)(reinterpret_cast<const int*>(lbase + co)),
            (lds_ptr<const VT>)(reinterpret_cast<const VT*>(lbase + wo)));
        if (src64) run_level<VT>(L, xl, xa64, G(gfree), s, T, fg, fp, g, p, E);
        else run_level<VT>(L, xl, G(gsrc), G(gfree), s, T, fg, fp, g, p, E);
        if (keep) final_mode = 2;
      } else if (!keep && !src64 && stage_index<VT>(D, E, co, ro)) {
        IView<VT> L = make_view<IView<VT>>(D, stage_cptr(D, E), (lds_ptr<const int>)(reinterpret_cast<const int*>(lbase + ro)),
            (lds_ptr<const int>)(reinterpret_cast<const int*>(lbase + co)), WSel<VT>::w(D));
        run_level<VT>(L, xl, G(gsrc), G(gfree), s, T, fg, fp, g, p, E);
      } else {
        XView<VT> L = make_view<XView<VT>>(D, stage_cptr(D, E), (const int*)D.rp, (const int*)D.col,
                                           WSel<VT>::w(D));
        if (src64) run_level<VT>(L, xl, xa64, G(gfree), s, T, fg, fp, g, p, E);
        else run_level<VT>(L, xl, G(gsrc), G(gfree), s, T, fg, fp, g, p, E);
        if (keep) final_mode = 1;
      }
      if (!keep) {
        wg_copy(G(gfree), xl, D.n);
        gsrc = gfree;
      }
    } else {
      GView<VT> L = make_view<GView<VT>>(D, stage_cptr(D, E), (const int*)D.rp, (const int*)D.col, WSel<VT>::w(D));
      if (src64) run_level<VT>(L, G(gfree), xa64, G(gsrc), s, T, fg, fp, g, p, E);
      else run_level<VT>(L, G(gfree), G(gsrc), G(gsrc), s, T, fg, fp, g, p, E);
      gsrc = gfree;
      if (keep) final_mode = 0;
    }
    src64 = false;
    push(g);
    push(p);
    __syncthreads();
  }
  if (src64 && J == 0) {
    // One-level hierarchy: the coarsest iterate is the answer; store it in the
    // working precision of the finest level.
    double acc[kNP] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < lv[0].n; i += blockDim.x) {
      const VT v = (VT)xa64[i];
      G(1)[i] = v;
      acc[0] += (double)v;
      acc[1] += (double)v * (double)v;
    }
    __syncthreads();
    block_sum<kNP>(acc, E.lds);
    gsrc = 1;
    final_mode = 0;
    s = after_prolong(acc, lv[0].n);
  }
  if (!T.finalize) {
    if (threadIdx.x == 0) {
      T.st->mu = s.mu;
      T.st->inv_s = s.inv_s;
      T.st->rho = s.rho;
      T.st->cos = s.cos;
      T.st->cur = gsrc;
      T.st->err = conv ? 0 : 1;
      *T.sched_len = slen;
    }
    return;
  }
  const LevelDesc D0 = lv[0];
  double lam = 0.0, res = 0.0;
  if (final_mode == 2) {
    // the CSR of level 0 is still staged from its level pass
    size_t wo = ((size_t)D0.n * sizeof(VT) + 15) & ~(size_t)15;
    size_t co = wo + (((size_t)D0.m * sizeof(VT) + 15) & ~(size_t)15);
    size_t ro = co + (((size_t)D0.m * 4 + 15) & ~(size_t)15);
    SView<VT> L = make_view<SView<VT>>(D0, stage_cptr(D0, E), (lds_ptr<const int>)(reinterpret_cast<const int*>(lbase + ro)),
        (lds_ptr<const int>)(reinterpret_cast<const int*>(lbase + co)),
        (lds_ptr<const VT>)(reinterpret_cast<const VT*>(lbase + wo)));
    finish_level0<VT>(L, xl, G(0), s, T, J, si, slen, lam, res, E);
  } else if (final_mode == 1) {
    XView<VT> L = make_view<XView<VT>>(D0, stage_cptr(D0, E), (const int*)D0.rp, (const int*)D0.col,
                                       WSel<VT>::w(D0));
    finish_level0<VT>(L, xl, G(0), s, T, J, si, slen, lam, res, E);
  } else {
    GView<VT> L = make_view<GView<VT>>(D0, stage_cptr(D0, E), (const int*)D0.rp, (const int*)D0.col,
                                       WSel<VT>::w(D0));
    finish_level0<VT>(L, G(gsrc), G(1 - gsrc), s, T, J, si, slen, lam, res, E);
  }
  if (threadIdx.x == 0) {
    T.st->lambda = lam;
    T.st->res = res;
    T.st->cos = s.cos;
    T.st->mu = s.mu;
    T.st->inv_s = s.inv_s;
    T.st->cur = gsrc;
    const bool nc = !conv || (!T.replay && T.tol_res > 0.0 && res > T.tol_res);
    T.st->err = nc ? 1 : 0;
    *T.sched_len = slen;
  }
}

// Persistent engine: each workgroup takes graphs from the queue until it is
// empty.  Dynamic LDS holds lds_cap vector entries (and staged CSRs).
template <class VT, int NT>
__global__ __launch_bounds__(NT) void k_engine(const GraphTask* tasks, int ntasks,
                                             unsigned* queue, int lds_cap) {
  extern __shared__ __align__(16) unsigned char fv_dyn_lds[];
  __shared__ double lds[block_sum_lds(NT)];
  __shared__ int ilds[NT / 64];
  __shared__ int s_cptr[kEngineMaxCol + 1];
  __shared__ int s_task;
  __shared__ double red[2 * block_sum_lds(NT)];
  EngineCtx E{lds, ilds, fv_dyn_lds, lds_cap, lds_cap * (int)sizeof(VT), s_cptr,
              (__attribute__((address_space(3))) double*)red, 0};
  for (;;) {
    if (threadIdx.x == 0) s_task = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int t = s_task;
    __syncthreads();
    if (t >= ntasks) break;
    engine_run<VT>(tasks[t], E);
    __syncthreads();
  }
}
