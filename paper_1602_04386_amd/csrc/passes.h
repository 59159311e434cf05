// Multi-workgroup passes over one large level (included by solve.hip after the
// per-row arithmetic).
//
// Each pass kernel handles tiles of kBlock consecutive rows (solve order).  A
// tile first stages its row pointers, the column indices and weights of its
// CSR slice, and the neighbour values those columns gather, in LDS: the CSR
// slice is read with unit-stride loads and all gathers of the tile are in
// flight together.  Each thread then reduces its own row from LDS in CSR
// order, the same arithmetic as the direct row functions.  A tile whose slice
// exceeds kTileNnz entries falls back to direct loads.
//
// A pass writes one partial-sum slot per block; a one-block finishing kernel
// reduces the slots in a fixed order and updates the device state.  The
// kernel boundary makes the partials visible, so no block needs a
// device-scope fence.
#pragma once

constexpr int kTileNnz = 2048;

template <class WT, class XT>
struct TileLds {
  int rp[kBlock + 1];
  int col[kTileNnz];
  WT w[kTileNnz];
  XT x[kTileNnz];
};

// Stages rows [rs, re) (re - rs <= kBlock).  Returns the CSR offset of the
// tile, or -1 when the slice is too long to stage.
template <class WT, class XT, class G>
__device__ inline int stage_tile(const LevelDesc& L, const WT* __restrict__ w, int rs, int re,
                                 TileLds<WT, XT>& T, G gather) {
  const int nr = re - rs;
  for (int k = threadIdx.x; k <= nr; k += blockDim.x) T.rp[k] = L.rp[rs + k];
  __syncthreads();
  const int p0 = T.rp[0], cnt = T.rp[nr] - p0;
  if (cnt > kTileNnz) return -1;
  const int* __restrict__ col = L.col;
  for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
    const int c = col[p0 + k];
    T.col[k] = c;
    T.w[k] = w[p0 + k];
    T.x[k] = gather(c);
  }
  __syncthreads();
  return p0;
}

__global__ void k_phase_begin(DevState* st, int cap, int forced, double tol) {
  st->done = cap <= 0 ? 1 : 0;
  st->iters = 0;
  st->cap = cap;
  st->forced = forced;
  st->tol = tol;
}

__device__ inline void write_slot(double* part, int stride, int slot, const double (&S)[kNP]) {
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < kNP; ++k) part[k * stride + slot] = S[k];
}

// ---- smoothing sweep, one colour -------------------------------------------

template <class VT>
__global__ __launch_bounds__(kBlock) void k_gs_tile(LevelDesc L, int r0, int r1, VT* xa, VT* xb,
                                                  const DevState* st, double* part, int stride,
                                                  int slot_base, double omega) {
  __shared__ TileLds<VT, VT> T;
  __shared__ double lds[block_sum_lds(kBlock)];
  if (st->done) return;
  VT* x = st->cur ? xb : xa;
  const double mu = st->mu, inv_s = st->inv_s, rho = st->rho;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int rs = r0 + b * kBlock, re = min(rs + kBlock, r1);
  const auto* w = WSel<VT>::w(L);
  double acc[kNP] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int p0 = stage_tile<VT, VT>(L, w, rs, re, T, [&](int c) { return x[c]; });
  const int t = threadIdx.x, i = rs + t;
  if (i < re) {
    if (p0 < 0) {
      row_gs<VT>(i, L, x, r0, mu, inv_s, rho, omega, acc);
    } else {
      const int a = T.rp[t] - p0, e = T.rp[t + 1] - p0;
      const double xo = ((double)x[i] - mu) * inv_s;
      double num = 0.0, den = 0.0;
      for (int k = a; k < e; ++k) {
        const double wj = (double)T.w[k];
        const double xj = (double)T.x[k];
        num += wj * (T.col[k] < r0 ? xj : (xj - mu) * inv_s);
        den += wj;
      }
      double u = xo;
      if (den > 0.0) {
        const double g = (num + rho * xo) / den;
        u = omega == 1.0 ? g : (1.0 - omega) * xo + omega * g;
      }
      const VT us = (VT)u;
      x[i] = us;
      const double ud = (double)us;
      double en = 0.0;
      for (int k = a; k < e; ++k)
        if (T.col[k] < r0) {
          const double d = ud - (double)T.x[k];
          en += (double)T.w[k] * d * d;
        }
      acc[0] += ud;
      acc[1] += ud * ud;
      acc[2] += ud * xo;
      acc[3] += xo;
      acc[4] += en;
    }
  }
  block_sum<kNP>(acc, lds);
  write_slot(part, stride, slot_base + blockIdx.x, acc);
}

// ---- power step ------------------------------------------------------------

template <class VT>
__global__ __launch_bounds__(kBlock) void k_pi_tile(LevelDesc L, VT* xa, VT* xb,
                                                  const DevState* st, double* part, int stride) {
  __shared__ TileLds<VT, VT> T;
  __shared__ double lds[block_sum_lds(kBlock)];
  if (st->done) return;
  const int cur = st->cur;
  const VT* x = cur ? xb : xa;
  VT* y = cur ? xa : xb;
  const double mu = st->mu, inv_s = st->inv_s, sigma = L.sigma;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int rs = b * kBlock, re = min(rs + kBlock, L.n);
  const auto* w = WSel<VT>::w(L);
  double acc[kNP] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int p0 = stage_tile<VT, VT>(L, w, rs, re, T, [&](int c) { return x[c]; });
  const int t = threadIdx.x, i = rs + t;
  if (i < re) {
    if (p0 < 0) {
      row_pi<VT>(i, L, x, y, mu, inv_s, sigma, acc);
    } else {
      const int a = T.rp[t] - p0, e = T.rp[t + 1] - p0;
      const double xi = (double)x[i];
      double lx = 0.0;
      for (int k = a; k < e; ++k) lx += (double)T.w[k] * (xi - (double)T.x[k]);
      const double xo = (xi - mu) * inv_s;
      const VT ys = (VT)(sigma * xo - lx * inv_s);
      y[i] = ys;
      const double yd = (double)ys;
      acc[0] += yd;
      acc[1] += yd * yd;
      acc[2] += yd * xo;
      acc[3] += xo;
    }
  }
  block_sum<kNP>(acc, lds);
  write_slot(part, stride, blockIdx.x, acc);
}

// ---- prolongation ----------------------------------------------------------

template <class SRC, class VT>
__global__ __launch_bounds__(kBlock) void k_prolong_tile(LevelDesc L, const SRC* xc_a,
                                                       const SRC* xc_b, VT* xf_a, VT* xf_b,
                                                       const DevState* st, double* part,
                                                       int stride) {
  __shared__ TileLds<VT, VT> T;
  __shared__ double lds[block_sum_lds(kBlock)];
  const int cur = st->cur;
  const SRC* xc = cur ? xc_b : xc_a;
  VT* xf = cur ? xf_a : xf_b;
  const double mu = st->mu, inv_s = st->inv_s;
  const int* __restrict__ qs = L.qs;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int rs = b * kBlock, re = min(rs + kBlock, L.n);
  const auto* w = WSel<VT>::w(L);
  double acc[kNP] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int p0 = stage_tile<VT, VT>(L, w, rs, re, T, [&](int c) {
    return (VT)(((double)xc[qs[c]] - mu) * inv_s);
  });
  const int t = threadIdx.x, i = rs + t;
  if (i < re) {
    if (p0 < 0) {
      row_prolong<SRC, VT>(i, L, xc, xf, mu, inv_s, acc);
    } else {
      const VT vs = (VT)(((double)xc[qs[i]] - mu) * inv_s);
      xf[i] = vs;
      const double v = (double)vs;
      const int a = T.rp[t] - p0, e = T.rp[t + 1] - p0;
      double en = 0.0;
      for (int k = a; k < e; ++k) {
        const double d = v - (double)T.x[k];
        en += (double)T.w[k] * d * d;
      }
      acc[0] += v;
      acc[1] += v * v;
      acc[4] += 0.5 * en;
    }
  }
  block_sum<kNP>(acc, lds);
  write_slot(part, stride, blockIdx.x, acc);
}

// ---- Rayleigh quotient and residual (FP64 weights) -------------------------

template <class VT>
__global__ __launch_bounds__(kBlock) void k_rq_tile(LevelDesc L, const VT* xa, const VT* xb,
                                                  const DevState* st, double* lxo, double* part,
                                                  int stride) {
  __shared__ TileLds<double, VT> T;
  __shared__ double lds[block_sum_lds(kBlock)];
  const VT* x = st->cur ? xb : xa;
  const double mu = st->mu, inv_s = st->inv_s;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int rs = b * kBlock, re = min(rs + kBlock, L.n);
  double a3[3] = {0.0, 0.0, 0.0};
  const int p0 = stage_tile<double, VT>(L, L.w64, rs, re, T, [&](int c) { return x[c]; });
  const int t = threadIdx.x, i = rs + t;
  if (i < re) {
    if (p0 < 0) {
      row_rq<VT>(i, L, x, mu, inv_s, lxo, a3);
    } else {
      const double xi = ((double)x[i] - mu) * inv_s;
      double lx = 0.0, e = 0.0;
      for (int k = T.rp[t] - p0; k < T.rp[t + 1] - p0; ++k) {
        const double d = xi - ((double)T.x[k] - mu) * inv_s;
        lx += T.w[k] * d;
        e += T.w[k] * d * d;
      }
      lxo[i] = lx;
      a3[0] += xi * xi;
      a3[1] += 0.5 * e;
      a3[2] = fmax(a3[2], fabs(xi));
    }
  }
  const double mx = block_max(a3[2], lds);
  double t2[2] = {a3[0], a3[1]};
  block_sum<2>(t2, lds);
  double S[kNP] = {t2[0], t2[1], mx, 0.0, 0.0};
  write_slot(part, stride, blockIdx.x, S);
}

template <class VT>
__global__ __launch_bounds__(kBlock) void k_res_tile(LevelDesc L, const VT* xa, const VT* xb,
                                                   const DevState* st, const double* lx,
                                                   double* part, int* ipart) {
  __shared__ double lds[block_sum_lds(kBlock)];
  __shared__ int ilds[kBlock / 64];
  const VT* x = st->cur ? xb : xa;
  const double mu = st->mu, inv_s = st->inv_s, lam = st->lambda, thr = 1e-3 * st->xmax;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int i = b * kBlock + threadIdx.x;
  double r2[1] = {0.0};
  int cand = INT_MAX;
  if (i < L.n) {
    const double xh = ((double)x[i] - mu) * inv_s;
    const double r = lx[i] - lam * xh;
    r2[0] = r * r;
    if (fabs(xh) >= thr) cand = L.iperm[i];
  }
  block_sum<1>(r2, lds);
  cand = block_min_int(cand, ilds);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = r2[0];
    ipart[blockIdx.x] = cand;
  }
}

// ---- finishing kernels (one block) -----------------------------------------

enum FinishMode { kFinGS = 0, kFinPI = 1, kFinProlong = 2, kFinRQ = 3 };

__global__ __launch_bounds__(kBlock) void k_finish(DevState* st, const double* part, int stride,
                                                 int nslots, int n, int mode) {
  __shared__ double lds[block_sum_lds(kBlock)];
  if ((mode == kFinGS || mode == kFinPI) && st->done) return;
  double S[kNP] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double mx = 0.0;
  for (int s = threadIdx.x; s < nslots; s += blockDim.x) {
    if (mode == kFinRQ) {
      S[0] += part[s];
      S[1] += part[stride + s];
      mx = fmax(mx, part[2 * stride + s]);
    } else {
#pragma unroll
      for (int k = 0; k < kNP; ++k) S[k] += part[k * stride + s];
    }
  }
  block_sum<kNP>(S, lds);
  if (mode == kFinRQ) mx = block_max(mx, lds);
  if (threadIdx.x != 0) return;
  if (mode == kFinRQ) {
    st->sumsq = S[0];
    st->lambda = S[1] / S[0];
    st->xmax = mx;
    st->rho = st->lambda;
    return;
  }
  const Scal r = mode == kFinProlong ? after_prolong(S, n) : after_gs(S, n);
  st->mu = r.mu;
  st->inv_s = r.inv_s;
  if (mode == kFinProlong) {
    st->rho = r.rho;
    st->cur = 1 - st->cur;
    return;
  }
  st->cos = r.cos;
  if (mode == kFinGS) st->rho = r.rho;
  if (mode == kFinPI) st->cur = 1 - st->cur;
  const int it = st->iters + 1;
  st->iters = it;
  st->done = (it >= st->cap || (!st->forced && r.cos > 1.0 - st->tol)) ? 1 : 0;
}

template <class VT>
__global__ __launch_bounds__(kBlock) void k_finish_res(LevelDesc L, const VT* xa, const VT* xb,
                                                     DevState* st, const double* part,
                                                     const int* ipart, int nslots) {
  __shared__ double lds[block_sum_lds(kBlock)];
  __shared__ int ilds[kBlock / 64];
  double s[1] = {0.0};
  int c = INT_MAX;
  for (int k = threadIdx.x; k < nslots; k += blockDim.x) {
    s[0] += part[k];
    c = min(c, ipart[k]);
  }
  block_sum<1>(s, lds);
  c = block_min_int(c, ilds);
  if (threadIdx.x != 0) return;
  const VT* x = st->cur ? xb : xa;
  st->res = sqrt(s[0] / st->sumsq);
  st->sign_idx = c;
  const double xv = c < INT_MAX ? ((double)x[L.perm[c]] - st->mu) * st->inv_s : 1.0;
  st->sign = xv < 0.0 ? -1.0 : 1.0;
}

template <class VT>
__global__ void k_output(LevelDesc L, const VT* xa, const VT* xb, const DevState* st,
                         double* out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= L.n) return;
  const VT* x = st->cur ? xb : xa;
  out[v] = st->sign * (((double)x[L.perm[v]] - st->mu) * st->inv_s);
}
