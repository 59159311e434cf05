// Refinement on the device (Algorithm 3, Steps 2-3, and the finest Rayleigh
// quotient): coarsest power iteration, prolongation, multicolour Gauss-Seidel
// smoothing on (L - rho I) x = 0, power iteration on sigma I - L, the
// cosine stopping test, and the finest-level Rayleigh quotient and residual.
//
// Two engines share the per-row arithmetic below:
//  * multi-workgroup passes (one launch per colour / step) for large levels,
//    reductions closed by the last block to finish, decisions kept on device;
//  * a one-workgroup-per-graph engine that runs whole levels (all phases, all
//    sweeps) inside one launch, used for the small levels of a big graph and
//    for every graph of a batch (a persistent grid with a work queue).
//
// The stored iterate x carries a pending normalisation (mu, inv_s): the unit,
// mean-free iterate is xhat = (x - mu) * inv_s.  Every pass applies it on the
// fly and returns the sums that define the next one, so projection and
// normalisation never need a pass of their own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <tuple>
#include <climits>
#include <cmath>
#include <cstdlib>

#include "fv_device.h"
#include "fv_internal.h"

namespace fv {

template <class VT>
struct WSel;
template <>
struct WSel<float> {
  __device__ static const float* w(const LevelDesc& L) { return L.w32; }
};
template <>
struct WSel<double> {
  __device__ static const double* w(const LevelDesc& L) { return L.w64; }
};

// ---------------------------------------------------------------------------
// Per-row arithmetic.
// ---------------------------------------------------------------------------

// Row arithmetic of the multi-workgroup sweeps (the tile and ELL kernels, the
// direct path of long rows and the finishing block's rows): one fixed
// sequence of roundings (contraction off, the fused multiply-adds written
// out), so that the kernels give bitwise-equal sweeps whatever the compiler
// makes of the surrounding code.  Entry (wj, xj) of a row: xj is already this sweep's
// value when `updated` (an earlier colour), else it still needs the pending
// shift and scale.
__device__ inline void gs_entry(double& num, double& den, double wj, double xj, bool updated,
                                double mu, double inv_s) {
#pragma clang fp contract(off)
  num = fma(wj, updated ? xj : (xj - mu) * inv_s, num);
  den = den + wj;
}

// The relaxed update of a row from its sums (the row's value xo when it has
// no entries).
__device__ inline double gs_relax(double num, double den, double xo, double rho,
                                  double omega) {
#pragma clang fp contract(off)
  double u = xo;
  if (den > 0.0) {
    const double g = fma(rho, xo, num) / den;
    u = omega == 1.0 ? g : fma(omega, g, (1.0 - omega) * xo);
  }
  return u;
}

// Adds w (u - xj)^2 of an edge to an earlier colour to the sweep's energy term.
__device__ inline void gs_energy(double& en, double wj, double ud, double xj) {
#pragma clang fp contract(off)
  const double d = ud - xj;
  en = fma(wj * d, d, en);
}

// Adds a row's terms to the sweep's sums.
__device__ inline void gs_sums(double (&acc)[kNP], double ud, double xo, double en) {
#pragma clang fp contract(off)
  acc[0] = acc[0] + ud;
  acc[1] = fma(ud, ud, acc[1]);
  acc[2] = fma(ud, xo, acc[2]);
  acc[3] = acc[3] + xo;
  acc[4] = acc[4] + en;
}

// Shifted Gauss-Seidel update of row i (Algorithm 2 on (L - rho I) x = 0 with
// the splitting (D - W_l) x' = (W_u + rho I) x):
// x_i <- (sum_j w_ij x_j + rho xhat_i) / d_i, relaxed by omega (an eigenvector
// with rho its eigenvalue is a fixed point).  Rows below lower_end were
// already updated in this sweep and are read as stored; the others are read
// through the pending normalisation.  Accumulates
// {sum u, sum u^2, sum u xhat_i, sum xhat_i, sum over already-updated
// neighbours of w (u - x_j)^2} where u is the stored new value; the last term
// adds up to u^T L u over the sweep (each edge counted by its later colour).
template <class VT>
__device__ inline void row_gs(int i, const LevelDesc& L, VT* __restrict__ x, int lower_end,
                              double mu, double inv_s, double rho, double omega,
                              double (&acc)[kNP]) {
  const auto* __restrict__ w = WSel<VT>::w(L);
  const int* __restrict__ col = L.col;
  const int p0 = L.rp[i], p1 = L.rp[i + 1];
  const double xo = ((double)x[i] - mu) * inv_s;
  double num = 0.0, den = 0.0;
  for (int p = p0; p < p1; ++p) {
    const int j = col[p];
    gs_entry(num, den, (double)w[p], (double)x[j], j < lower_end, mu, inv_s);
  }
  const VT us = (VT)gs_relax(num, den, xo, rho, omega);
  x[i] = us;
  const double ud = (double)us;
  double e = 0.0;
  for (int p = p0; p < p1; ++p) {
    const int j = col[p];
    if (j < lower_end) gs_energy(e, (double)w[p], ud, (double)x[j]);
  }
  gs_sums(acc, ud, xo, e);
}

// row_gs with the row's pointers given and its neighbours fetched kRowB at a
// time (every index and weight load of a batch, then every gather): the same
// terms added in the same order, for the rows a single block sweeps.  The
// first batch stays in registers for the edge-energy pass (most rows have at
// most kRowB entries, so that pass issues no loads).
constexpr int kRowB = 8;

template <class VT>
__device__ inline void row_gs_batched(int i, int p0, int p1, const LevelDesc& L,
                                      VT* __restrict__ x, int lower_end, double mu,
                                      double inv_s, double rho, double omega,
                                      double (&acc)[kNP]) {
  const auto* __restrict__ w = WSel<VT>::w(L);
  const int* __restrict__ col = L.col;
  const double xo = ((double)x[i] - mu) * inv_s;
  double num = 0.0, den = 0.0;
  int j0[kRowB];
  double w0[kRowB], x0[kRowB];
  auto batch = [&](int pb, int (&jj)[kRowB], double (&ww)[kRowB], double (&xx)[kRowB]) {
#pragma unroll
    for (int u = 0; u < kRowB; ++u) {
      const int q = min(pb + u, p1 - 1);
      jj[u] = col[q];
      ww[u] = (double)w[q];
    }
#pragma unroll
    for (int u = 0; u < kRowB; ++u) xx[u] = (double)x[jj[u]];
  };
  for (int pb = p0; pb < p1; pb += kRowB) {
    int jj[kRowB];
    double ww[kRowB], xx[kRowB];
    batch(pb, jj, ww, xx);
#pragma unroll
    for (int u = 0; u < kRowB; ++u)
      if (pb + u < p1) gs_entry(num, den, ww[u], xx[u], jj[u] < lower_end, mu, inv_s);
    if (pb == p0)
#pragma unroll
      for (int u = 0; u < kRowB; ++u) {
        j0[u] = jj[u];
        w0[u] = ww[u];
        x0[u] = xx[u];
      }
  }
  const VT us = (VT)gs_relax(num, den, xo, rho, omega);
  x[i] = us;
  const double ud = (double)us;
  double e = 0.0;
  if (p1 > p0)
#pragma unroll
    for (int u = 0; u < kRowB; ++u)
      if (p0 + u < p1 && j0[u] < lower_end) gs_energy(e, w0[u], ud, x0[u]);
  for (int pb = p0 + kRowB; pb < p1; pb += kRowB) {
    int jj[kRowB];
    double ww[kRowB], xx[kRowB];
    batch(pb, jj, ww, xx);
#pragma unroll
    for (int u = 0; u < kRowB; ++u)
      if (pb + u < p1 && jj[u] < lower_end) gs_energy(e, ww[u], ud, xx[u]);
  }
  gs_sums(acc, ud, xo, e);
}

// Power-iteration step of row i: y_i = sigma xhat_i - (L xhat)_i with
// (L x)_i = sum_j w_ij (x_i - x_j).  Accumulates {sum y, sum y^2,
// sum y xhat_i, sum xhat_i}.
template <class VT>
__device__ inline void row_pi(int i, const LevelDesc& L, const VT* __restrict__ x,
                              VT* __restrict__ y, double mu, double inv_s, double sigma,
                              double (&acc)[kNP]) {
  const auto* __restrict__ w = WSel<VT>::w(L);
  const int* __restrict__ col = L.col;
  const double xi = (double)x[i];
  double lx = 0.0;
  for (int p = L.rp[i]; p < L.rp[i + 1]; ++p) lx += (double)w[p] * (xi - (double)x[col[p]]);
  const double xo = (xi - mu) * inv_s;
  const VT ys = (VT)(sigma * xo - lx * inv_s);
  y[i] = ys;
  const double yd = (double)ys;
  acc[0] += yd;
  acc[1] += yd * yd;
  acc[2] += yd * xo;
  acc[3] += xo;
}

// Prolongation of row i (Algorithm 3, Step 3): v_i = xhat_c[q(i)], plus the
// row's share of v^T L v (half of sum_j w_ij (v_i - v_j)^2) for the first
// shift.  Accumulates {sum v, sum v^2, -, -, energy}.
template <class SRC, class VT>
__device__ inline void row_prolong(int i, const LevelDesc& L, const SRC* __restrict__ xc,
                                   VT* __restrict__ xf, double muc, double inv_sc,
                                   double (&acc)[kNP]) {
  const auto* __restrict__ w = WSel<VT>::w(L);
  const int* __restrict__ col = L.col;
  const int* __restrict__ qs = L.qs;
  const VT vs = (VT)(((double)xc[qs[i]] - muc) * inv_sc);
  xf[i] = vs;
  const double v = (double)vs;
  double e = 0.0;
  for (int p = L.rp[i]; p < L.rp[i + 1]; ++p) {
    const double vj = (double)(VT)(((double)xc[qs[col[p]]] - muc) * inv_sc);
    const double d = v - vj;
    e += (double)w[p] * d * d;
  }
  acc[0] += v;
  acc[1] += v * v;
  acc[4] += 0.5 * e;
}

// Rayleigh-quotient row (FP64 weights): lx_i = (L xhat)_i, half edge energy,
// xhat_i^2 and |xhat_i|.
template <class VT>
__device__ inline void row_rq(int i, const LevelDesc& L, const VT* __restrict__ x, double mu,
                              double inv_s, double* __restrict__ lxo, double (&acc)[3]) {
  const double* __restrict__ w = L.w64;
  const int* __restrict__ col = L.col;
  const double xi = ((double)x[i] - mu) * inv_s;
  double lx = 0.0, e = 0.0;
  for (int p = L.rp[i]; p < L.rp[i + 1]; ++p) {
    const double d = xi - ((double)x[col[p]] - mu) * inv_s;
    lx += w[p] * d;
    e += w[p] * d * d;
  }
  lxo[i] = lx;
  acc[0] += xi * xi;
  acc[1] += 0.5 * e;
  acc[2] = fmax(acc[2], fabs(xi));
}

// ---------------------------------------------------------------------------
// Scalar updates after a pass (sums -> next pending normalisation).
// ---------------------------------------------------------------------------
struct Scal {
  double mu, inv_s, cos, rho;
};

__device__ inline Scal after_gs(const double (&S)[kNP], int n) {
  Scal r;
  r.mu = S[0] / n;
  double var = S[1] - S[0] * r.mu;
  r.inv_s = var > 0.0 ? 1.0 / sqrt(var) : 1.0;
  r.cos = (S[2] - r.mu * S[3]) * r.inv_s;
  r.rho = var > 0.0 ? S[4] / var : 0.0;
  return r;
}

__device__ inline Scal after_prolong(const double (&S)[kNP], int n) {
  Scal r;
  r.mu = S[0] / n;
  double var = S[1] - S[0] * r.mu;
  r.inv_s = var > 0.0 ? 1.0 / sqrt(var) : 1.0;
  r.cos = 1.0;
  r.rho = var > 0.0 ? S[4] / var : 0.0;
  return r;
}

#include "passes.h"

// ---------------------------------------------------------------------------
// One-workgroup engine.
// ---------------------------------------------------------------------------
constexpr int kEngineMaxCol = 255;

struct EngineCtx {
  double* lds;  // (threads / 64) * kNP doubles
  int* ilds;
  void* xl;     // dynamic LDS: one level vector, then optionally its CSR
  int cap;      // capacity in vector entries
  int bytes;    // size in bytes
  int* cptr;    // LDS, kEngineMaxCol + 1 entries: the current level's colour ranges
  __attribute__((address_space(3))) double* red;  // 2 * block_sum_lds(threads) doubles
  int flip;     // block_allsum's region toggle
};

// Sum over lanes 0..31 of a wave whose lanes 32..63 hold zeros: the same
// value as wave_sum (whose upper half adds two exact zeros) with half the
// read-outs.
__device__ inline double wave_sum_low32(double v) {
  v = row_sum16(v);
  auto lane_val = [&](int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
  };
  return lane_val(0) + lane_val(16);
}

// The power-iteration steps of the one-wavefront coarsest solve, lane i
// holding x_i (lanes >= n hold 0); rowl(x) returns lane i's (L x)_i.  Sums run
// over half a wave when n <= 32 (half).  Runs until the stop test passes
// (cv = 1), max_it steps, or exactly forced steps; returns the steps taken
// and leaves the iterate in x.
template <class RowL>
__device__ int coarsest_iterate(RowL rowl, bool half, int n, bool has, double sigma, double tol,
                                int max_it, int forced, double& x, int& cv) {
  auto sum = [half](double v) { return half ? wave_sum_low32(v) : wave_sum(v); };
  int it = 0;
  cv = 0;
  for (;;) {
    double l = rowl(x);
    l = has ? l : 0.0;
    // The shifted step does not depend on the stop test, so its mean is
    // reduced together with the Rayleigh quotient.
    double y = has ? sigma * x - l : 0.0;
    const double rho = sum(x * l);
    const double my = sum(y) / n;
    y = has ? y - my : 0.0;
    if (forced >= 0) {
      if (it >= forced) {
        cv = 1;
        break;
      }
    } else {
      const double r = l - rho * x;
      const double rr = sum(r * r);
      const double yy = sum(y * y);
      if (sqrt(rr) <= tol * sigma) {
        cv = 1;
        break;
      }
      if (it >= max_it) break;
      x = y * (1.0 / sqrt(yy));
      ++it;
      continue;
    }
    x = y * (1.0 / sqrt(sum(y * y)));
    ++it;
  }
  return it;
}

__device__ inline double lane_bcast(double v, int j) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), j),
                          __builtin_amdgcn_readlane(__double2loint(v), j));
}

// Dense form: lane i's row of W in R registers (columns j >= n are zero),
// n <= R <= 32, or read from LDS (R = 0, any n <= 64); x_j is broadcast with
// readlane, j ascending.
template <int R>
__device__ int coarsest_steps(__attribute__((address_space(3))) const double* Wd, int n, int base,
                              bool has, double sigma, double tol, int max_it, int forced,
                              double& x, int& cv) {
  double wr[R > 0 ? R : 1];
#pragma unroll
  for (int j = 0; j < R; ++j) wr[j] = j < n ? Wd[j * n + base] : 0.0;
  auto rowl = [&](double xv) {
    double l = 0.0;
    if (R > 0) {
#pragma unroll
      for (int j = 0; j < R; ++j) l += wr[j] * (xv - lane_bcast(xv, j));
    } else {
      for (int j = 0; j < n; ++j) l += Wd[j * n + base] * (xv - lane_bcast(xv, j));
    }
    return l;
  };
  return coarsest_iterate(rowl, R > 0, n, has, sigma, tol, max_it, forced, x, cv);
}

// Sparse form for levels whose rows hold at most K entries: lane i keeps its
// row's columns and weights (column order; padded with its own index and
// weight 0, which add exact zeros) and fetches x_j with a lane shuffle.  The
// terms are the dense form's nonzero ones in the same order, and the zero
// terms the dense form adds leave its sums unchanged, so both give the same
// iterates; the shuffles replace R broadcasts by K.
template <int K>
__device__ int coarsest_steps_sparse(const int* __restrict__ rp, const int* __restrict__ col,
                                     const double* __restrict__ w, int n, int lane, bool has,
                                     double sigma, double tol, int max_it, int forced, double& x,
                                     int& cv) {
  int ck[K];
  double wk[K];
  const int p0 = has ? rp[lane] : 0, p1 = has ? rp[lane + 1] : 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const bool in = p0 + k < p1;
    ck[k] = in ? col[p0 + k] : lane;
    wk[k] = in ? w[p0 + k] : 0.0;
  }
  auto rowl = [&](double xv) {
    double xj[K];
#pragma unroll
    for (int k = 0; k < K; ++k) xj[k] = __shfl(xv, ck[k], 64);
    double l = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) l += wk[k] * (xv - xj[k]);
    return l;
  };
  return coarsest_iterate(rowl, n <= 32, n, has, sigma, tol, max_it, forced, x, cv);
}

// Coarsest solve in FP64 (Algorithm 3, Step 2): power iteration on
// sigma I - L with projection, from the seeded start, stopping when
// ||L x - rho x|| <= tol sigma or at the cap (forced >= 0: exactly forced
// steps).  Writes the unit iterate to out; returns steps, sets *conv.
__device__ int engine_coarsest(const LevelDesc& L, unsigned long long seed, int max_it,
                               int forced, double tol, double* out, double* lx, int* conv,
                               EngineCtx& E) {
  const int n = __builtin_amdgcn_readfirstlane(L.n);  // uniform: keeps loop branches scalar
  const double sigma = L.sigma;
  const double* __restrict__ w = L.w64;
  const int* __restrict__ col = L.col;
  int it = 0;
  if (n <= 64 && n * n * (int)sizeof(double) <= E.bytes) {
    // One wavefront: lane i owns row i.  W is staged densely in LDS, column
    // j contiguous, so that (L x)_i = sum_j W_ij (x_i - x_j) runs over j in
    // ascending order (the CSR order of this level, whose rows are in
    // original order) with x_j broadcast by readlane; absent edges add
    // 0 * (x_i - x_j) = 0 exactly.
    __attribute__((address_space(3))) double* Wd =
        (__attribute__((address_space(3))) double*)(static_cast<double*>(E.xl));
    for (int k = threadIdx.x; k < n * n; k += blockDim.x) Wd[k] = 0.0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x)
      for (int p = L.rp[i]; p < L.rp[i + 1]; ++p) Wd[col[p] * n + i] = w[p];
    __syncthreads();
    __shared__ int s_it, s_conv;
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      const bool has = lane < n;
      const int base = has ? lane : 0;
      double x = has ? 2.0 * splitmix_uniform(seed, (unsigned long long)lane + 1ULL) - 1.0 : 0.0;
      double m = wave_sum(x) / n;
      x = has ? x - m : 0.0;
      x *= 1.0 / sqrt(wave_sum(x * x));
      int cv = 0;
      // Rows of at most 16 entries (the usual coarsest level: ~4 a row) take
      // the sparse form.  Otherwise, up to 32 vertices the row is also held in
      // registers, so an iteration touches no memory at all; the row length is
      // rounded up to 8, 16, 24 or 32 (the padding columns add exact zeros).
      const int len = has ? L.rp[lane + 1] - L.rp[lane] : 0;
      int maxlen = len;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) maxlen = max(maxlen, __shfl_xor(maxlen, off, 64));
      maxlen = __builtin_amdgcn_readfirstlane(maxlen);
      if (maxlen <= 4)
        it = coarsest_steps_sparse<4>(L.rp, col, w, n, lane, has, sigma, tol, max_it, forced, x, cv);
      else if (maxlen <= 8)
        it = coarsest_steps_sparse<8>(L.rp, col, w, n, lane, has, sigma, tol, max_it, forced, x, cv);
      else if (maxlen <= 16)
        it = coarsest_steps_sparse<16>(L.rp, col, w, n, lane, has, sigma, tol, max_it, forced, x, cv);
      else if (n <= 8) it = coarsest_steps<8>(Wd, n, base, has, sigma, tol, max_it, forced, x, cv);
      else if (n <= 16) it = coarsest_steps<16>(Wd, n, base, has, sigma, tol, max_it, forced, x, cv);
      else if (n <= 24) it = coarsest_steps<24>(Wd, n, base, has, sigma, tol, max_it, forced, x, cv);
      else if (n <= 32) it = coarsest_steps<32>(Wd, n, base, has, sigma, tol, max_it, forced, x, cv);
      else it = coarsest_steps<0>(Wd, n, base, has, sigma, tol, max_it, forced, x, cv);
      if (has) out[lane] = x;
      if (lane == 0) {
        s_it = it;
        s_conv = cv;
      }
    }
    __syncthreads();
    it = s_it;
    *conv = s_conv;
    __syncthreads();
    return it;
  }
  // General size: rows strided over the workgroup.
  double* x = out;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    x[i] = 2.0 * splitmix_uniform(seed, (unsigned long long)i + 1ULL) - 1.0;
  __syncthreads();
  auto project_normalise = [&](double* v) {
    double t[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) t[0] += v[i];
    block_sum<1>(t, E.lds);
    const double m = t[0] / n;
    double q[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      v[i] -= m;
      q[0] += v[i] * v[i];
    }
    block_sum<1>(q, E.lds);
    const double inv = 1.0 / sqrt(q[0]);
    for (int i = threadIdx.x; i < n; i += blockDim.x) v[i] *= inv;
    __syncthreads();
  };
  project_normalise(x);
  int cv = 0;
  for (;;) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      double l = 0.0;
      for (int p = L.rp[i]; p < L.rp[i + 1]; ++p) l += w[p] * (x[i] - x[col[p]]);
      lx[i] = l;
    }
    __syncthreads();
    if (forced >= 0) {
      if (it >= forced) {
        cv = 1;
        break;
      }
    } else {
      double t[1] = {0.0};
      for (int i = threadIdx.x; i < n; i += blockDim.x) t[0] += x[i] * lx[i];
      block_sum<1>(t, E.lds);
      double r[1] = {0.0};
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double d = lx[i] - t[0] * x[i];
        r[0] += d * d;
      }
      block_sum<1>(r, E.lds);
      if (sqrt(r[0]) <= tol * sigma) {
        cv = 1;
        break;
      }
      if (it >= max_it) break;
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = sigma * x[i] - lx[i];
    __syncthreads();
    project_normalise(x);
    ++it;
  }
  *conv = cv;
  return it;
}

// Phase counts: forced (replay) or free with the cosine test.
struct PhaseCfg {
  int forced;  // -1 = free
  int cap;
  double tol;
};

#include "engine.h"

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
static inline int nblk(long long n, int b = kBlock) {
  return (int)std::max<long long>(1, (n + b - 1) / b);
}

// Rows per thread of a tile pass over `rows` rows holding `entries` entries:
// two when tiles of kBlock rows would need more than one round of resident
// blocks (the CU count times the blocks per CU that the tile's LDS allows) and
// a tile of two rows per thread still fits one staging chunk on average (at
// most four entries a row), one otherwise: more, smaller blocks spread a small
// level over more CUs, and on denser levels a two-row tile takes two or three
// chunks, each two more dependent load phases (the 4M-point random geometric
// graph's level-0 sweep: 281 us with two rows per thread, 256 us with one).
// The ELL sweep takes the same count, so both give the same block sums.
// FV_TILE_RPT=1 or 2 forces it.
template <class VT>
static int tile_rpt(long long rows, long long entries) {
  static const long long one_round = [] {
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    return (long long)ncu * tile_waves<VT>() * kBlock;
  }();
  static const int forced = [] {
    const char* e = std::getenv("FV_TILE_RPT");
    return e ? std::atoi(e) : 0;
  }();
  if (forced == 1 || forced == 2) return forced;
  return rows > one_round && entries <= 4 * rows ? 2 : 1;
}

// Blocks of a tile kernel that one round of residency holds: the CU count
// times the blocks per CU the tile's LDS allows.
template <class VT>
static int resident_tiles(int rpt) {
  static const int ncu = [] {
    int dev = 0, n = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    return n;
  }();
  return ncu * (rpt == 2 ? tile_waves<VT, 2>() : tile_waves<VT, 1>());
}

// Allows an engine instantiation the dynamic LDS it is launched with (more
// than the 64 KiB default); done once per instantiation and process.
template <class VT, int NT>
static void enable_engine_lds(size_t bytes) {
  static std::once_flag once;
  std::call_once(once, [&] {
    FV_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_engine<VT, NT>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  });
}

struct Workspace {
  void* xa;
  void* xb;
  double* lx;
  double* part;
  int* ipart;
  DevState* st;
  GraphTask* task;
  int* sched;
  int* sched_len;
  int* replay;
  int* rec;  // step count of each multi-workgroup phase, one slot spare
  unsigned* queue;
  int stride;
};

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Partial-sum slots: a sweep launches ceil(rows_c / kBlock) blocks per colour,
// at most n / kBlock + ncolours in total.
static size_t slot_count(size_t nmax, int maxcol) {
  return nmax / kBlock + (size_t)maxcol + 2 * FV_MAX_LEVELS + 1024;
}

size_t solve_workspace_bytes(size_t nmax, int maxcol) {
  const size_t slots = slot_count(nmax, maxcol);
  return 3 * align_up(8 * std::max<size_t>(nmax, 1)) + align_up(8 * kNP * slots) +
         align_up(4 * slots) + align_up(sizeof(DevState)) + align_up(sizeof(GraphTask)) +
         2 * align_up(4 * FV_SCHEDULE_CAP) + align_up(4 * (FV_SCHEDULE_CAP + 1)) + align_up(64);
}

static Workspace carve(void* base, size_t nmax, int maxcol) {
  Workspace w;
  char* p = static_cast<char*>(base);
  const size_t slots = slot_count(nmax, maxcol);
  auto take = [&](size_t b) {
    char* r = p;
    p += align_up(b);
    return r;
  };
  w.xa = take(8 * std::max<size_t>(nmax, 1));
  w.xb = take(8 * std::max<size_t>(nmax, 1));
  w.lx = reinterpret_cast<double*>(take(8 * std::max<size_t>(nmax, 1)));
  w.part = reinterpret_cast<double*>(take(8 * kNP * slots));
  w.ipart = reinterpret_cast<int*>(take(4 * slots));
  w.st = reinterpret_cast<DevState*>(take(sizeof(DevState)));
  w.task = reinterpret_cast<GraphTask*>(take(sizeof(GraphTask)));
  w.sched = reinterpret_cast<int*>(take(4 * FV_SCHEDULE_CAP));
  w.replay = reinterpret_cast<int*>(take(4 * FV_SCHEDULE_CAP));
  w.rec = reinterpret_cast<int*>(take(4 * (FV_SCHEDULE_CAP + 1)));
  w.queue = reinterpret_cast<unsigned*>(take(64));
  w.sched_len = reinterpret_cast<int*>(w.queue + 4);
  w.stride = (int)slots;
  return w;
}

// Host side of the early stop.  The host enqueues a phase in chunks of
// kChunk steps and reads the phase's done flag after each, but it enqueues
// chunk k+1 before it waits for chunk k: the device always has queued work
// while the host waits, and a phase that has ended leaves at most one chunk of
// launches that return at once.  The finishing kernels write the flag (and
// the finest residual) into mapped host memory, so no copy enters the stream;
// once the event after chunk k has completed, the flag holds the state after
// chunk k or later, and a later state of the same phase is as good (the flag
// only goes from 0 to 1 within a phase).
struct HostSync {
  volatile int* hdone;     // host view of the flag
  volatile double* hres;   // host view of the residual
  int* hdone_dev;          // device addresses of the same
  double* hres_dev;
  hipEvent_t ev[2];        // recorded after chunk k (alternating)
  hipEvent_t ev_res;       // recorded after the residual pass
};

constexpr int kChunk = 2;

// Opt-in timing of the finest level's smoothing launches: a pair of HIP
// events around each launch, read after the solve has finished.  Events come
// from the scratch's pool, created on first use, at most kTimedLaunches pairs
// per solve (later launches run untimed).
constexpr int kTimedLaunches = 2048;
struct LaunchTimer {
  std::vector<hipEvent_t>* pool = nullptr;
  int used = 0;
  std::vector<long long> bytes;
  bool on() const { return pool != nullptr; }
  // the event before launch `used`, or nullptr when the pool is exhausted
  hipEvent_t* pair() {
    if (!pool || used >= kTimedLaunches) return nullptr;
    while ((int)pool->size() < 2 * (used + 1)) {
      hipEvent_t e = nullptr;
      FV_HIP(hipEventCreate(&e));
      pool->push_back(e);
    }
    return pool->data() + 2 * used;
  }
};

// Launches colour c's sweep from its ELL block when it has one (returns false
// otherwise): EW the level's slot count, RPT the tile sweep's rows per thread
// (two only with at most 8 slots).
template <class VT, int EW>
static void gs_ell_launch(const Level& Lh, int c, int rpt, int nb, hipStream_t s, int r0, int r1,
                          VT* xa, VT* xb, const Workspace& W, int base, double omega) {
  const int* ec = Lh.ecol + Lh.ecoff[c];
  const VT* ev = sizeof(VT) == 4 ? reinterpret_cast<const VT*>(Lh.ew32 + Lh.ecoff[c])
                                 : reinterpret_cast<const VT*>(Lh.ew64 + Lh.ecoff[c]);
  if constexpr (EW <= 8) {
    if (rpt == 2) {
      k_gs_ell<VT, EW, 2><<<nb, kBlock, 0, s>>>(r0, r1, ec, ev, xa, xb, W.st, W.part, W.stride,
                                                base, omega);
      return;
    }
  }
  k_gs_ell<VT, EW, 1><<<nb, kBlock, 0, s>>>(r0, r1, ec, ev, xa, xb, W.st, W.part, W.stride, base,
                                            omega);
}

template <class VT>
static bool launch_gs_ell(const Level& Lh, int c, int rpt, int nb, hipStream_t s, int r0, int r1,
                          VT* xa, VT* xb, const Workspace& W, int base, double omega) {
  const int ew = Lh.ell_width(c);
  if (!ew || (rpt == 2 && ew > 8)) return false;
  switch (ew) {
    case 4: gs_ell_launch<VT, 4>(Lh, c, rpt, nb, s, r0, r1, xa, xb, W, base, omega); break;
    case 8: gs_ell_launch<VT, 8>(Lh, c, rpt, nb, s, r0, r1, xa, xb, W, base, omega); break;
    case 12: gs_ell_launch<VT, 12>(Lh, c, rpt, nb, s, r0, r1, xa, xb, W, base, omega); break;
    case 16: gs_ell_launch<VT, 16>(Lh, c, rpt, nb, s, r0, r1, xa, xb, W, base, omega); break;
    case 20: gs_ell_launch<VT, 20>(Lh, c, rpt, nb, s, r0, r1, xa, xb, W, base, omega); break;
    case 24: gs_ell_launch<VT, 24>(Lh, c, rpt, nb, s, r0, r1, xa, xb, W, base, omega); break;
    case 28: gs_ell_launch<VT, 28>(Lh, c, rpt, nb, s, r0, r1, xa, xb, W, base, omega); break;
    case 32: gs_ell_launch<VT, 32>(Lh, c, rpt, nb, s, r0, r1, xa, xb, W, base, omega); break;
    default: return false;
  }
  return true;
}

// Launches the finishing block of a sweep whose colours from ct on are swept
// by it, with the ELL blocks of those colours where they have them.
template <class VT, int EW>
static void gs_tail_launch(const Level& Lh, const LevelDesc& L, int ct, hipStream_t s, VT* xa,
                           VT* xb, const Workspace& W, int nslots, double omega, int* rec,
                           int* hdone, const TailEll& te) {
  k_finish_gs_tail<VT, EW><<<1, kTailBlock, 0, s>>>(L, xa, xb, W.st, W.part, W.stride, nslots,
                                                    ct, Lh.cptr_h[ct], Lh.cptr_h[ct + 1], omega,
                                                    te, rec, hdone);
}

template <class VT>
static void launch_gs_tail(const Level& Lh, const LevelDesc& L, int ct, hipStream_t s, VT* xa,
                           VT* xb, const Workspace& W, int nslots, double omega, int* rec,
                           int* hdone) {
  TailEll te;
  bool any = false;
  for (int k = 0; k < kTailEll; ++k) {
    const int c = ct + k;
    te.eoff[k] = Lh.ell_width(c) ? Lh.ecoff[c] : -1;
    any = any || te.eoff[k] >= 0;
  }
  switch (any ? Lh.ew : 0) {
    case 4: gs_tail_launch<VT, 4>(Lh, L, ct, s, xa, xb, W, nslots, omega, rec, hdone, te); break;
    case 8: gs_tail_launch<VT, 8>(Lh, L, ct, s, xa, xb, W, nslots, omega, rec, hdone, te); break;
    case 12: gs_tail_launch<VT, 12>(Lh, L, ct, s, xa, xb, W, nslots, omega, rec, hdone, te); break;
    case 16: gs_tail_launch<VT, 16>(Lh, L, ct, s, xa, xb, W, nslots, omega, rec, hdone, te); break;
    case 20: gs_tail_launch<VT, 20>(Lh, L, ct, s, xa, xb, W, nslots, omega, rec, hdone, te); break;
    case 24: gs_tail_launch<VT, 24>(Lh, L, ct, s, xa, xb, W, nslots, omega, rec, hdone, te); break;
    case 28: gs_tail_launch<VT, 28>(Lh, L, ct, s, xa, xb, W, nslots, omega, rec, hdone, te); break;
    case 32: gs_tail_launch<VT, 32>(Lh, L, ct, s, xa, xb, W, nslots, omega, rec, hdone, te); break;
    default: gs_tail_launch<VT, 0>(Lh, L, ct, s, xa, xb, W, nslots, omega, rec, hdone, te);
  }
}

// Enqueues one smoothing (gs) or power phase: `forced` steps exactly when it
// is not negative, else up to `cap` steps with the cosine test.  The step
// count lands in *rec on the device.  before_wait, when given, runs once
// after the first chunk is enqueued and before any flag is awaited; it
// returns true when the phase is moot (the finest residual already met its
// tolerance), and the phase then ends without further launches.
template <class VT, class BeforeWait>
static bool run_phase_multi(bool gs, const Level& Lh, const LevelDesc& L, const Workspace& W,
                            int forced, int cap, double tol, double omega, hipStream_t s,
                            HostSync& hs, int* rec, bool use_halt, BeforeWait before_wait,
                            LaunchTimer* timer = nullptr) {
  const int lim = forced >= 0 ? forced : cap;
  k_phase_begin<<<1, 1, 0, s>>>(W.st, lim, forced >= 0 ? 1 : 0, tol, use_halt ? 1 : 0, rec,
                                hs.hdone_dev);
  VT* xa = static_cast<VT*>(W.xa);
  VT* xb = static_cast<VT*>(W.xb);
  // Trailing colours with at most kTailRows rows in all are swept by the
  // finishing block (k_finish_gs_tail) instead of one launch each.
  int ct = L.ncol;
  while (ct > 1 && Lh.cptr_h[L.ncol] - Lh.cptr_h[ct - 1] <= kTailRows) --ct;
  std::vector<int> nbs(L.ncol), rpt(L.ncol);
  int nslots = 0;
  for (int c = 0; c < ct; ++c) {
    const int rows = Lh.cptr_h[c + 1] - Lh.cptr_h[c];
    rpt[c] = tile_rpt<VT>(rows, Lh.cnnz_h[c + 1] - Lh.cnnz_h[c]);
    nbs[c] = nblk(rows, kBlock * rpt[c]);
    nslots += nbs[c];
  }
  const int pi_rpt = tile_rpt<VT>(L.n, L.m);
  const int pi_nb = nblk(L.n, kBlock * pi_rpt);
  // A level of more tiles than one round of resident blocks takes the power
  // step as a loop of tiles per block (one round of blocks).
  const int pi_grid = std::min(pi_nb, resident_tiles<VT>(pi_rpt));
  const bool pi_loop = pi_nb > pi_grid;
  if (nslots > W.stride) throw Error(FV_E_DEVICE, "partial-sum slots exceeded");
  auto enqueue = [&](int k) {
    for (int it = 0; it < k; ++it) {
      if (gs) {
        int base = 0;
        for (int c = 0; c < ct; ++c) {
          const int r0 = Lh.cptr_h[c], r1 = Lh.cptr_h[c + 1];
          hipEvent_t* ev = timer ? timer->pair() : nullptr;
          if (ev) FV_HIP(hipEventRecord(ev[0], s));
          if (launch_gs_ell<VT>(Lh, c, rpt[c], nbs[c], s, r0, r1, xa, xb, W, base, omega)) {
            // swept from the colour's ELL block
          } else if (rpt[c] == 2) {
            k_gs_tile<VT, 2><<<nbs[c], kBlock, 0, s>>>(L, r0, r1, xa, xb, W.st, W.part, W.stride,
                                                       base, omega);
          } else {
            k_gs_tile<VT, 1><<<nbs[c], kBlock, 0, s>>>(L, r0, r1, xa, xb, W.st, W.part, W.stride,
                                                       base, omega);
          }
          if (ev) {
            FV_HIP(hipEventRecord(ev[1], s));
            timer->bytes.push_back(pass_bytes(r1 - r0, Lh.cnnz_h[c + 1] - Lh.cnnz_h[c],
                                              sizeof(VT) == 4 ? FV_PREC_FP32_MIXED
                                                              : FV_PREC_FP64));
            ++timer->used;
          }
          base += nbs[c];
        }
        if (ct < L.ncol)
          launch_gs_tail<VT>(Lh, L, ct, s, xa, xb, W, nslots, omega, rec, hs.hdone_dev);
        else
          k_finish<<<1, kBlock, 0, s>>>(W.st, W.part, W.stride, nslots, L.n, kFinGS, rec,
                                        hs.hdone_dev);
      } else if (pi_loop) {
        if (pi_rpt == 2)
          k_pi_tile_loop<VT, 2><<<pi_grid, kBlock, 0, s>>>(L, xa, xb, W.st, W.part, W.stride,
                                                           pi_nb);
        else
          k_pi_tile_loop<VT, 1><<<pi_grid, kBlock, 0, s>>>(L, xa, xb, W.st, W.part, W.stride,
                                                           pi_nb);
        k_finish<<<1, kBlock, 0, s>>>(W.st, W.part, W.stride, pi_grid, L.n, kFinPI, rec,
                                      hs.hdone_dev);
      } else {
        if (pi_rpt == 2)
          k_pi_tile<VT, 2><<<pi_nb, kBlock, 0, s>>>(L, xa, xb, W.st, W.part, W.stride);
        else
          k_pi_tile<VT, 1><<<pi_nb, kBlock, 0, s>>>(L, xa, xb, W.st, W.part, W.stride);
        k_finish<<<1, kBlock, 0, s>>>(W.st, W.part, W.stride, pi_nb, L.n, kFinPI, rec,
                                      hs.hdone_dev);
      }
    }
    FV_HIP(hipGetLastError());
  };
  if (forced >= 0) {
    enqueue(forced);
    return before_wait();
  }
  int enq = 0, prev = -1, slot = 0;
  bool first = true;
  for (;;) {
    const int k = std::min(kChunk, lim - enq);
    enqueue(k);
    enq += k;
    const bool more = enq < lim;
    if (more) FV_HIP(hipEventRecord(hs.ev[slot], s));
    if (first) {
      first = false;
      if (before_wait()) return true;
    }
    if (!more) break;
    if (prev >= 0) {
      FV_HIP(hipEventSynchronize(hs.ev[prev]));
      if (*hs.hdone) break;
    }
    prev = slot;
    slot ^= 1;
  }
  return false;
}

static LevelDesc host_desc(const Level& F) { return desc_of(F); }

static void fill_task(GraphTask& T, const fv_hierarchy* h, const fv_solve_opts* o, int stop,
                      void* xa, void* xb, double* lx, double* x_out, DevState* st,
                      const int* replay, int replay_len, int* sched, int* sched_len) {
  std::memset(&T, 0, sizeof(T));
  T.lv = h->d_desc;
  T.J = h->levels - 1;
  T.stop = stop;
  T.prec = o->prec;
  T.finalize = stop == 0 ? 1 : 0;
  T.xa = xa;
  T.xb = xb;
  T.lx = lx;
  T.x_out = x_out;
  T.st = st;
  T.replay = replay;
  T.replay_len = replay_len;
  T.sched = sched;
  T.sched_len = sched_len;
  T.seed = o->seed;
  T.tol_cos = o->tol_cos;
  T.tol_res = o->tol_res;
  T.omega = o->omega;
  T.max_gs = o->max_gs;
  T.max_pi = o->max_pi;
  T.max_outer = o->max_outer;
  T.early_exit = o->early_exit ? 1 : 0;
  T.max_coarsest = o->max_coarsest;
  T.tol_coarse = o->tol_coarse;
}

static long long schedule_bytes(const fv_hierarchy* h, const int* sched, int len, int prec) {
  const int J = h->levels - 1;
  long long b = 0;
  int k = 1;
  for (int l = J - 1; l >= 0 && k + 1 < len; --l, k += 2) {
    const Level& F = h->lv[l];
    b += (long long)(sched[k] + sched[k + 1] + 1) * pass_bytes(F.n, F.m, prec);
  }
  const Level& F0 = h->lv[0];
  for (; k + 1 < len; k += 2)
    b += (long long)(sched[k] + sched[k + 1]) * pass_bytes(F0.n, F0.m, prec);
  return b;
}

static void release_scratch_device(fv_context* ctx, SolveScratch& sc) {
  if (sc.ws) dev_free(ctx, sc.ws, sc.ws_bytes, nullptr);
  sc.ws = nullptr;
  sc.ws_bytes = 0;
}

// Frees a workspace; the streams that used it must have been synchronised.
void release_scratch(fv_context* ctx, SolveScratch& sc) {
  release_scratch_device(ctx, sc);
  if (sc.pinned) (void)hipHostFree(sc.pinned);
  sc.pinned = nullptr;
  if (sc.hflags) (void)hipHostFree(sc.hflags);
  sc.hflags = nullptr;
  sc.hflags_dev = nullptr;
  for (hipEvent_t* e : {&sc.ev_t0, &sc.ev_t1, &sc.ev_chunk[0], &sc.ev_chunk[1], &sc.ev_res}) {
    if (*e) (void)hipEventDestroy(*e);
    *e = nullptr;
  }
  for (hipEvent_t e : sc.tev) (void)hipEventDestroy(e);
  sc.tev.clear();
}

void scratch_host_init(SolveScratch& sc) {
  if (!sc.pinned)
    FV_HIP(hipHostMalloc(reinterpret_cast<void**>(&sc.pinned), 256, hipHostMallocDefault));
  if (!sc.hflags) {
    FV_HIP(hipHostMalloc(reinterpret_cast<void**>(&sc.hflags), 256,
                         hipHostMallocMapped | hipHostMallocCoherent));
    FV_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&sc.hflags_dev), sc.hflags, 0));
  }
  if (!sc.ev_t0) FV_HIP(hipEventCreate(&sc.ev_t0));
  if (!sc.ev_t1) FV_HIP(hipEventCreate(&sc.ev_t1));
  for (hipEvent_t* e : {&sc.ev_chunk[0], &sc.ev_chunk[1], &sc.ev_res})
    if (!*e) FV_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
}

// The solve proper on the workspace ws (at least solve_workspace_bytes of the
// hierarchy) with the host buffers and events of sc (scratch_host_init done).
template <class VT>
static fv_status solve_one_t(fv_context* ctx, SolveScratch& sc, void* ws, const fv_hierarchy* h,
                             const fv_solve_opts* o, double* x_out, int x_on_device,
                             double* lambda_out, fv_solve_stats* stats, hipStream_t s) {
  (void)ctx;
  const int J = h->levels - 1;
  const size_t nmax = hierarchy_nmax(h);
  int maxcol = 1;
  for (int l = 0; l < h->levels; ++l) maxcol = std::max(maxcol, h->lv[l].ncol);
  Workspace W = carve(ws, nmax, maxcol);
  int* pinned = sc.pinned;

  // Split: levels whose vector fits the engine's LDS go to the one-workgroup
  // engine; the rest to multi-workgroup passes.
  const int lds_cap = (int)(kSoloLds / sizeof(VT));
  static const int engine_max = [] {
    const char* e = std::getenv("FV_ENGINE_MAX_N");
    return e ? std::atoi(e) : 8192;
  }();
  const int split = std::min(lds_cap, engine_max);
  int t = J;
  while (t > 0 && h->lv[t - 1].n <= split) --t;

  int replay_len = 0;
  if (o->replay) {
    replay_len = std::min(o->replay_len, FV_SCHEDULE_CAP);
    FV_HIP(hipMemcpyAsync(W.replay, o->replay, sizeof(int) * replay_len, hipMemcpyHostToDevice, s));
  }
  // Output staging for a host x_out: lx, free once the residual is done.
  double* out_dev = x_on_device ? x_out : W.lx;
  hipEvent_t e0 = sc.ev_t0, e1 = sc.ev_t1;
  LaunchTimer timer;
  if (o->time_finest) timer.pool = &sc.tev;
  LaunchTimer* tptr = timer.on() ? &timer : nullptr;
  FV_HIP(hipEventRecord(e0, s));

  GraphTask T;
  // The engine gets the replay prefix covering its levels.
  const int eng_len = !o->replay ? 0 : (t == 0 ? replay_len : std::min(replay_len, 1 + 2 * (J - t)));
  fill_task(T, h, o, t, W.xa, W.xb, W.lx, t == 0 ? out_dev : nullptr, W.st,
            o->replay ? W.replay : nullptr, eng_len, W.sched, W.sched_len);
  FV_HIP(hipMemcpyAsync(W.task, &T, sizeof(T), hipMemcpyHostToDevice, s));
  FV_HIP(hipMemsetAsync(W.queue, 0, sizeof(unsigned), s));
  FV_HIP(hipMemsetAsync(&W.st->counter, 0, sizeof(unsigned), s));
  enable_engine_lds<VT, kWGSolo>(kSoloLds);
  k_engine<VT, kWGSolo><<<1, kWGSolo, kSoloLds, s>>>(W.task, 1, W.queue, lds_cap);
  FV_HIP(hipGetLastError());

  std::vector<int> sched;
  fv_status status = FV_OK;
  double lam = 0.0, res = 0.0, fcos = 0.0;
  if (t == 0) {
    FV_HIP(hipEventRecord(e1, s));
    int slen = 0;
    FV_HIP(hipMemcpyAsync(pinned, W.sched_len, sizeof(int), hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    slen = std::min(pinned[0], FV_SCHEDULE_CAP);
    sched.resize(slen);
    DevState hs;
    FV_HIP(hipMemcpyAsync(sched.data(), W.sched, sizeof(int) * slen, hipMemcpyDeviceToHost, s));
    FV_HIP(hipMemcpyAsync(&hs, W.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    if (!x_on_device)
      FV_HIP(hipMemcpyAsync(x_out, W.lx, sizeof(double) * h->lv[0].n, hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    lam = hs.lambda;
    res = hs.res;
    fcos = hs.cos;
    if (hs.err) status = FV_E_NOT_CONVERGED;
  } else {
    // The engine records the coarsest count and one (smoothing, power) pair
    // per level it ran; the replay cursor continues after those.  Nothing is
    // read back until the end of the solve.
    const int elen = std::min(1 + 2 * (J - t), FV_SCHEDULE_CAP);
    int ri = elen;
    auto next_forced = [&]() -> int { return (o->replay && ri < replay_len) ? o->replay[ri++] : -1; };
    HostSync hsync;
    hsync.hdone = sc.hflags;
    hsync.hres = reinterpret_cast<volatile double*>(sc.hflags + 8);
    hsync.hdone_dev = sc.hflags_dev;
    hsync.hres_dev = reinterpret_cast<double*>(sc.hflags_dev + 8);
    hsync.ev[0] = sc.ev_chunk[0];
    hsync.ev[1] = sc.ev_chunk[1];
    hsync.ev_res = sc.ev_res;
    int nrec = 0;  // phases recorded in W.rec; the spare slot takes any overflow
    auto rec_slot = [&]() { return W.rec + std::min(nrec++, FV_SCHEDULE_CAP); };
    auto no_wait = [] { return false; };
    // Multi-workgroup levels t-1 .. 0.
    for (int l = t - 1; l >= 0; --l) {
      const Level& F = h->lv[l];
      const LevelDesc L = host_desc(F);
      // (from the FP64 coarsest vector: one row per thread)
      const int prpt = l == J - 1 ? 1 : tile_rpt<VT>(F.n, F.m);
      const int nb = nblk(F.n, kBlock * prpt);
      if (l == J - 1) {
        k_prolong_tile<double, VT, 1><<<nb, kBlock, 0, s>>>(
            L, static_cast<const double*>(W.xa), static_cast<const double*>(W.xb),
            static_cast<VT*>(W.xa), static_cast<VT*>(W.xb), W.st, W.part, W.stride);
      } else if (prpt == 2) {
        k_prolong_tile<VT, VT, 2><<<nb, kBlock, 0, s>>>(
            L, static_cast<const VT*>(W.xa), static_cast<const VT*>(W.xb), static_cast<VT*>(W.xa),
            static_cast<VT*>(W.xb), W.st, W.part, W.stride);
      } else {
        k_prolong_tile<VT, VT, 1><<<nb, kBlock, 0, s>>>(
            L, static_cast<const VT*>(W.xa), static_cast<const VT*>(W.xb), static_cast<VT*>(W.xa),
            static_cast<VT*>(W.xb), W.st, W.part, W.stride);
      }
      k_finish<<<1, kBlock, 0, s>>>(W.st, W.part, W.stride, nb, F.n, kFinProlong, nullptr,
                                    nullptr);
      FV_HIP(hipGetLastError());
      run_phase_multi<VT>(true, F, L, W, next_forced(), o->max_gs, o->tol_cos, o->omega, s, hsync,
                          rec_slot(), false, no_wait, l == 0 ? tptr : nullptr);
      run_phase_multi<VT>(false, F, L, W, next_forced(), o->max_pi, o->tol_cos, o->omega, s,
                          hsync, rec_slot(), false, no_wait);
    }
    const Level& F0 = h->lv[0];
    const LevelDesc L0 = host_desc(F0);
    // Under the residual test the last residual pass raises the device's halt
    // flag itself, so a round enqueued before the host has read it is void.
    const double tol_halt = o->replay ? 0.0 : o->tol_res;
    // early_left: with early exit, the rounds max_outer leaves after the
    // round this pass follows (-1: none, or no early exit).
    auto rq_res = [&](int early_left) {
      const int nb = nblk(F0.n);
      const VT* xa = static_cast<const VT*>(W.xa);
      const VT* xb = static_cast<const VT*>(W.xb);
      k_rq_tile<VT><<<nb, kBlock, 0, s>>>(L0, xa, xb, W.st, W.lx, W.part, W.stride);
      k_finish<<<1, kBlock, 0, s>>>(W.st, W.part, W.stride, nb, F0.n, kFinRQ, nullptr, nullptr);
      k_res_tile<VT><<<nb, kBlock, 0, s>>>(L0, xa, xb, W.st, W.lx, W.part, W.ipart);
      k_finish_res<VT><<<1, kBlock, 0, s>>>(L0, xa, xb, W.st, W.part, W.ipart, nb, tol_halt,
                                            early_left, hsync.hres_dev);
      FV_HIP(hipGetLastError());
    };
    rq_res(-1);
    const bool early = o->early_exit && !o->replay;
    double last_res = 0.0;  // the residual the host read before the current one
    int outer = 0;
    for (;;) {
      int fg, fp;
      bool spec = false;
      if (o->replay) {
        if (ri >= replay_len) break;
        fg = next_forced();
        fp = next_forced();
      } else {
        if (!(o->tol_res > 0.0) || outer >= o->max_outer) break;
        FV_HIP(hipEventRecord(hsync.ev_res, s));
        fg = fp = -1;
        spec = true;
      }
      // The round's first chunk is enqueued before the last residual is read.
      // With early exit it also ends the rounds when the residual cannot reach
      // tol_res in the rounds left, the test the residual pass made on the device.
      auto residual_met = [&]() -> bool {
        if (!spec) return false;
        FV_HIP(hipEventSynchronize(hsync.ev_res));
        const double r = *hsync.hres;
        const bool stop = r <= o->tol_res ||
                          (early && outer > 0 && !can_reach(r, last_res, o->tol_res,
                                                            o->max_outer - outer));
        last_res = r;
        return stop;
      };
      if (run_phase_multi<VT>(true, F0, L0, W, fg, o->max_gs, o->tol_cos, o->omega, s, hsync,
                              rec_slot(), spec, residual_met, tptr)) {
        --nrec;  // the void round is not part of the schedule
        break;
      }
      run_phase_multi<VT>(false, F0, L0, W, fp, o->max_pi, o->tol_cos, o->omega, s, hsync,
                          rec_slot(), spec, no_wait);
      ++outer;
      rq_res(early ? o->max_outer - outer : -1);
    }
    k_output<VT><<<nblk(F0.n), kBlock, 0, s>>>(L0, static_cast<const VT*>(W.xa),
                                               static_cast<const VT*>(W.xb), W.st, out_dev);
    FV_HIP(hipGetLastError());
    FV_HIP(hipEventRecord(e1, s));
    if (!x_on_device)
      FV_HIP(hipMemcpyAsync(x_out, W.lx, sizeof(double) * F0.n, hipMemcpyDeviceToHost, s));
    DevState hs;
    FV_HIP(hipMemcpyAsync(&hs, W.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    sched.resize(elen);
    FV_HIP(hipMemcpyAsync(sched.data(), W.sched, sizeof(int) * elen, hipMemcpyDeviceToHost, s));
    const int nr = std::min(nrec, FV_SCHEDULE_CAP);
    std::vector<int> recs(nr);
    if (nr > 0)
      FV_HIP(hipMemcpyAsync(recs.data(), W.rec, sizeof(int) * nr, hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    sched.insert(sched.end(), recs.begin(), recs.end());
    lam = hs.lambda;
    res = hs.res;
    fcos = hs.cos;
    if (hs.err) status = FV_E_NOT_CONVERGED;
    if (!o->replay && o->tol_res > 0.0 && res > o->tol_res) status = FV_E_NOT_CONVERGED;
  }
  float ms = 0.0f;
  FV_HIP(hipEventElapsedTime(&ms, e0, e1));
  if (lambda_out) *lambda_out = lam;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->levels = h->levels;
    for (int l = 0; l < h->levels; ++l) {
      stats->n[l] = h->lv[l].n;
      stats->nnz[l] = h->lv[l].m;
      stats->colours[l] = l == J ? 0 : h->lv[l].ncol;
    }
    stats->schedule_len = (int)std::min<size_t>(sched.size(), FV_SCHEDULE_CAP);
    for (int k = 0; k < stats->schedule_len; ++k) stats->schedule[k] = sched[k];
    stats->lambda = lam;
    stats->residual = res;
    stats->final_cos = fcos;
    stats->t_solve_ms = ms;
    stats->alg_bytes = schedule_bytes(h, sched.data(), (int)sched.size(), o->prec);
    double tsum = 0.0;
    long long bsum = 0;
    for (int k = 0; k < timer.used; ++k) {
      float t = 0.0f;
      FV_HIP(hipEventElapsedTime(&t, timer.pool->at(2 * k), timer.pool->at(2 * k + 1)));
      tsum += t;
      bsum += timer.bytes[k];
    }
    stats->n_finest_gs = timer.used;
    stats->t_finest_gs_ms = tsum;
    stats->finest_gs_bytes = bsum;
  }
  return status;
}

static size_t workspace_need(const fv_hierarchy* h) {
  int maxcol = 1;
  for (int l = 0; l < h->levels; ++l) maxcol = std::max(maxcol, h->lv[l].ncol);
  return solve_workspace_bytes(hierarchy_nmax(h), maxcol);
}

fv_status solve_one_with(fv_context* ctx, SolveScratch& sc, const fv_hierarchy* h,
                         const fv_solve_opts* o, double* x_out, int x_on_device,
                         double* lambda_out, fv_solve_stats* stats, hipStream_t s) {
  const size_t need = workspace_need(h);
  if (sc.ws_bytes < need) {
    // The old workspace may still be read by work queued on s.
    FV_HIP(hipStreamSynchronize(s));
    release_scratch_device(ctx, sc);
    sc.ws = dev_alloc(ctx, need, nullptr);
    sc.ws_bytes = need;
  }
  scratch_host_init(sc);
  if (o->prec == FV_PREC_FP32_MIXED)
    return solve_one_t<float>(ctx, sc, sc.ws, h, o, x_out, x_on_device, lambda_out, stats, s);
  return solve_one_t<double>(ctx, sc, sc.ws, h, o, x_out, x_on_device, lambda_out, stats, s);
}

// ---------------------------------------------------------------------------
// Allocation-free solve: the workspace is a fixed device array of this file.
// Each device holds its own copy from the first use of the library on it
// until the process ends.  Host code never passes the array's name to a
// kernel or a copy: that name is a host-side stand-in, not a device address.
// The address comes from hipGetSymbolAddress, once per device, with that
// device current.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[FV_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;

void* noalloc_scratch_init(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) return it->second;
  void* p = nullptr;
  FV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Error(FV_E_DEVICE, "no device address for the fixed scratch");
  g_scratch_ptr[device] = p;
  return p;
}

fv_status solve_noalloc(fv_context* ctx, const fv_hierarchy* h, const fv_solve_opts* o,
                        double* x_out, int x_on_device, double* lambda_out,
                        fv_solve_stats* stats) {
  if (workspace_need(h) > (size_t)FV_NOALLOC_SCRATCH_BYTES) return FV_E_SCRATCH;
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(ctx->device);
    if (it != g_scratch_ptr.end()) ws = it->second;
  }
  SolveScratch& sc = ctx->scratch;
  // Both were set up by fv_context_create; nothing is created here.
  if (!ws || !sc.pinned || !sc.hflags || !sc.ev_t0 || !sc.ev_res)
    throw Error(FV_E_DEVICE, "context set-up incomplete");
  hipStream_t s = o->stream ? static_cast<hipStream_t>(o->stream) : ctx->stream;
  fv_solve_opts oo = *o;
  oo.time_finest = 0;  // the timing's events are created on first use: not here
  if (o->prec == FV_PREC_FP32_MIXED)
    return solve_one_t<float>(ctx, sc, ws, h, &oo, x_out, x_on_device, lambda_out, stats, s);
  return solve_one_t<double>(ctx, sc, ws, h, &oo, x_out, x_on_device, lambda_out, stats, s);
}

fv_status solve_one(fv_context* ctx, const fv_hierarchy* h, const fv_solve_opts* o,
                    double* x_out, int x_on_device, double* lambda_out, fv_solve_stats* stats) {
  hipStream_t s = o->stream ? static_cast<hipStream_t>(o->stream) : ctx->stream;
  return solve_one_with(ctx, ctx->scratch, h, o, x_out, x_on_device, lambda_out, stats, s);
}

// ---------------------------------------------------------------------------
// Batch: one persistent launch, one workgroup per graph, largest first.
//
// Launch configuration: the dynamic LDS each workgroup gets (a graph's level
// vector and, when they fit, its staged CSRs) and, following from it, how many
// workgroups stay resident per CU.  More LDS keeps more levels on chip; less
// lets more graphs run at once.  The engine's arithmetic is the same whichever
// memory a level sits in, and a graph's result does not depend on which
// workgroup takes it, so every configuration gives bitwise the same results:
// the autotuner below may pick any of them.
// ---------------------------------------------------------------------------
static const size_t kBatchLdsCand[] = {32u << 10, 48u << 10, 64u << 10, 96u << 10, 144u << 10};
constexpr size_t kBatchLdsMax = 144u << 10;

__global__ void k_batch_reset(unsigned* queue) { *queue = 0; }

template <class VT>
static int batch_grid(int count, size_t lds) {
  enable_engine_lds<VT, kWGBatch>(kBatchLdsMax);
  int dev = 0, ncu = 256, per_cu = 1;
  FV_HIP(hipGetDevice(&dev));
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void*>(&k_engine<VT, kWGBatch>), kWGBatch, lds);
  return std::min(count, std::max(1, ncu * std::max(per_cu, 1)));
}

// The autotuner's cache key: precision and the size class of a batch (log2 of
// the median and largest finest level, log2 of the count, mean degree rounded
// to a half), process-wide.
struct TuneKey {
  int prec, med, mx, cnt, deg;
  bool operator<(const TuneKey& o) const {
    return std::tie(prec, med, mx, cnt, deg) < std::tie(o.prec, o.med, o.mx, o.cnt, o.deg);
  }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, size_t> g_tune;

static int ilog2(long long v) {
  int k = 0;
  while (v > 1) {
    v >>= 1;
    ++k;
  }
  return k;
}

static TuneKey tune_key(int count, const fv_hierarchy* const* hs, int prec) {
  std::vector<long long> ns(count);
  long long nn = 0, mm = 0;
  for (int k = 0; k < count; ++k) {
    ns[k] = hs[k]->lv[0].n;
    nn += hs[k]->lv[0].n;
    mm += hs[k]->lv[0].m;
  }
  std::nth_element(ns.begin(), ns.begin() + count / 2, ns.end());
  const long long med = ns[count / 2];
  const long long mx = *std::max_element(ns.begin(), ns.end());
  return TuneKey{prec, ilog2(med), ilog2(mx), ilog2(count), (int)(2.0 * mm / std::max(nn, 1LL))};
}

// The device and pinned memory of one batch: per-item vectors, outputs,
// states, schedules, the task table, the queue, and pinned mirrors of the
// task table and of the read-backs.
struct BatchBufs {
  fv_context* ctx = nullptr;
  void* dev = nullptr;
  size_t dev_bytes = 0;
  void* pin = nullptr;
  size_t pin_bytes = 0;
  size_t o_out = 0, o_st = 0, o_sched = 0, o_slen = 0, o_tasks = 0, o_queue = 0;
  size_t p_tasks = 0, p_st = 0, p_slen = 0, p_sched = 0, p_out = 0;
  void release() {
    if (dev) {
      block_put(ctx, dev);
      budget_release(ctx, dev_bytes);
    }
    if (pin) (void)hipHostFree(pin);
    dev = pin = nullptr;
    dev_bytes = pin_bytes = 0;
  }
};

// A captured launch sequence, kept by the context for the next batch call
// with the same task table and configuration.
struct BatchGraph {
  std::vector<unsigned char> key;
  BatchBufs bufs;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    bufs.release();
    key.clear();
  }
};

void release_batch_graph(fv_context* ctx) {
  if (!ctx->bgraph) return;
  static_cast<BatchGraph*>(ctx->bgraph)->release();
  delete static_cast<BatchGraph*>(ctx->bgraph);
  ctx->bgraph = nullptr;
}

// Enqueues the batch's launch sequence on s: task table upload (from the
// pinned mirror), queue reset, the engine, and the read-backs into the pinned
// mirrors.  No memset node: the reset is a kernel, so the sequence can be
// captured and replayed.
template <class VT>
static void enqueue_batch(const BatchBufs& B, int count, size_t lds, int grid, bool want_sched,
                          size_t nout, hipStream_t s) {
  char* base = static_cast<char*>(B.dev);
  char* pin = static_cast<char*>(B.pin);
  GraphTask* d_tasks = reinterpret_cast<GraphTask*>(base + B.o_tasks);
  unsigned* queue = reinterpret_cast<unsigned*>(base + B.o_queue);
  FV_HIP(hipMemcpyAsync(d_tasks, pin + B.p_tasks, sizeof(GraphTask) * count,
                        hipMemcpyHostToDevice, s));
  k_batch_reset<<<1, 1, 0, s>>>(queue);
  k_engine<VT, kWGBatch><<<grid, kWGBatch, lds, s>>>(d_tasks, count, queue,
                                                     (int)(lds / sizeof(VT)));
  FV_HIP(hipGetLastError());
  FV_HIP(hipMemcpyAsync(pin + B.p_st, base + B.o_st, sizeof(DevState) * count,
                        hipMemcpyDeviceToHost, s));
  FV_HIP(hipMemcpyAsync(pin + B.p_slen, base + B.o_slen, sizeof(int) * count,
                        hipMemcpyDeviceToHost, s));
  if (want_sched)
    FV_HIP(hipMemcpyAsync(pin + B.p_sched, base + B.o_sched,
                          sizeof(int) * FV_SCHEDULE_CAP * count, hipMemcpyDeviceToHost, s));
  if (nout)
    FV_HIP(hipMemcpyAsync(pin + B.p_out, base + B.o_out, sizeof(double) * nout,
                          hipMemcpyDeviceToHost, s));
}

template <class VT>
static fv_status solve_batch_t(fv_context* ctx, int count, const fv_hierarchy* const* hs,
                               const fv_solve_opts* o, fv_batch_opts* bo, double* const* x_out,
                               int x_on_device, double* lambda_out, fv_solve_stats* stats,
                               fv_status* item_status, hipStream_t s) {
  // Per-item device memory: xa, xb, lx (8 bytes each per vertex) and, for
  // host outputs, the FP64 result.  States, schedules and schedule lengths of
  // all items are contiguous so that one copy each reads them back.
  std::vector<size_t> off(count + 1, 0), xoff(count + 1, 0);
  for (int k = 0; k < count; ++k) {
    const size_t n = hierarchy_nmax(hs[k]);
    off[k + 1] = off[k] + align_up(8 * n) * 3;
    xoff[k + 1] = xoff[k] + (x_on_device ? 0 : n);
  }
  const size_t nout = xoff[count];
  BatchBufs B;
  B.ctx = ctx;
  B.o_out = off[count];
  B.o_st = B.o_out + align_up(8 * nout);
  B.o_sched = B.o_st + align_up(sizeof(DevState) * count);
  B.o_slen = B.o_sched + align_up(sizeof(int) * FV_SCHEDULE_CAP * count);
  B.o_tasks = B.o_slen + align_up(sizeof(int) * count);
  B.o_queue = B.o_tasks + align_up(sizeof(GraphTask) * count);
  const size_t dev_bytes = B.o_queue + 256;
  B.p_tasks = 0;
  B.p_st = align_up(sizeof(GraphTask) * count);
  B.p_slen = B.p_st + align_up(sizeof(DevState) * count);
  B.p_sched = B.p_slen + align_up(sizeof(int) * count);
  B.p_out = B.p_sched + (stats ? align_up(sizeof(int) * FV_SCHEDULE_CAP * count) : 0);
  const size_t pin_bytes = B.p_out + align_up(8 * nout);

  // Task table (largest first), addresses relative to a workspace base that
  // is filled in below, once the workspace is known.
  std::vector<long long> work(count);
  std::vector<int> order(count);
  for (int k = 0; k < count; ++k) {
    long long w = 0;
    for (int l = 0; l < hs[k]->levels; ++l) w += hs[k]->lv[l].m + hs[k]->lv[l].n;
    work[k] = w;
    order[k] = k;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  auto make_tasks = [&](char* base, std::vector<GraphTask>& sorted) {
    DevState* d_st = reinterpret_cast<DevState*>(base + B.o_st);
    int* d_sched = reinterpret_cast<int*>(base + B.o_sched);
    int* d_slen = reinterpret_cast<int*>(base + B.o_slen);
    double* d_out = reinterpret_cast<double*>(base + B.o_out);
    sorted.resize(count);
    for (int j = 0; j < count; ++j) {
      const int k = order[j];
      char* p = base + off[k];
      const size_t n = hierarchy_nmax(hs[k]);
      double* xo = x_on_device ? x_out[k] : d_out + xoff[k];
      fill_task(sorted[j], hs[k], o, 0, p, p + align_up(8 * n),
                reinterpret_cast<double*>(p + 2 * align_up(8 * n)), xo, d_st + k, nullptr, 0,
                d_sched + (size_t)k * FV_SCHEDULE_CAP, d_slen + k);
      sorted[j].work = work[k];
    }
  };

  // Launch configuration: forced, the autotuner's cached choice, a tuning
  // run, or the default.
  size_t lds = kBatchLds;
  int tuned = 0;
  const TuneKey key = tune_key(count, hs, o->prec);
  if (bo && bo->lds_bytes > 0) {
    lds = std::min<size_t>((size_t)bo->lds_bytes, kBatchLdsMax);
  } else if (bo && bo->autotune) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      lds = it->second;
      tuned = 1;
    }
  }
  const bool tune_now = bo && bo->autotune == 1 && bo->lds_bytes <= 0 && !tuned;
  struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  FV_HIP(hipEventCreate(&ev.a));
  FV_HIP(hipEventCreate(&ev.b));

  // The captured graph of the previous call, if this call repeats it.
  BatchGraph* bg = (bo && bo->graph) ? static_cast<BatchGraph*>(ctx->bgraph) : nullptr;
  std::vector<unsigned char> gkey;
  if (bo && bo->graph) {
    // what determines the captured sequence: every task's inputs and
    // outputs (by their hierarchy and output pointers), the options, the
    // configuration
    auto put = [&](const void* p, size_t n) {
      const unsigned char* c = static_cast<const unsigned char*>(p);
      gkey.insert(gkey.end(), c, c + n);
    };
    put(&count, sizeof(count));
    put(&x_on_device, sizeof(x_on_device));
    put(o, sizeof(*o));
    put(&lds, sizeof(lds));
    const int ws = stats ? 1 : 0;
    put(&ws, sizeof(ws));
    for (int k = 0; k < count; ++k) {
      put(&hs[k]->serial, sizeof(hs[k]->serial));  // a rebuilt hierarchy never matches
      // device outputs are written by the captured launch itself; host
      // outputs are copied from the pinned mirror after it, wherever they are
      if (x_on_device) put(&x_out[k], sizeof(x_out[k]));
    }
  }
  const bool replay = bg && !tune_now && bg->exec && bg->key == gkey;

  BatchBufs local;
  BatchBufs* buf = &local;
  if (replay) {
    buf = &bg->bufs;
  } else {
    local = B;
    budget_reserve(ctx, dev_bytes);
    try {
      local.dev = block_get(ctx, dev_bytes);
    } catch (...) {
      budget_release(ctx, dev_bytes);
      throw;
    }
    local.dev_bytes = dev_bytes;
    if (hipHostMalloc(&local.pin, pin_bytes, hipHostMallocDefault) != hipSuccess) {
      local.pin = nullptr;
      local.release();
      throw Error(FV_E_NOMEM, "pinned staging of the batch");
    }
    local.pin_bytes = pin_bytes;
    std::vector<GraphTask> sorted;
    make_tasks(static_cast<char*>(local.dev), sorted);
    std::memcpy(local.pin, sorted.data(), sizeof(GraphTask) * count);
  }
  struct Guard {
    BatchBufs* b;
    hipStream_t s;
    bool own;
    ~Guard() {
      if (!own) return;
      (void)hipStreamSynchronize(s);
      b->release();
    }
  } guard{&local, s, !replay};

  if (tune_now) {
    // Autotuning: each candidate configuration runs a size-stratified sample
    // of the batch (every 4th graph in the largest-first order, the whole
    // batch below 1,024 graphs, at most 2,048), enough graphs per workgroup
    // that the sample's time measures throughput and not the slowest graph
    // alone, on this batch's own buffers; the fastest is cached for the size
    // class.  One untimed launch of the sample's smallest graphs first pays
    // the first use of the engine.  The sample's results are overwritten by
    // the full launch below.
    const int stride = count < 1024 ? 1 : 4;
    std::vector<GraphTask> all(count), samp;
    std::memcpy(all.data(), local.pin, sizeof(GraphTask) * count);
    for (int j = 0; j < count && (int)samp.size() < 2048; j += stride) samp.push_back(all[j]);
    const int ns = (int)samp.size();
    const int nw = std::min(ns, 8);
    std::memcpy(local.pin, samp.data() + (ns - nw), sizeof(GraphTask) * nw);
    enqueue_batch<VT>(local, nw, kBatchLdsCand[0], batch_grid<VT>(nw, kBatchLdsCand[0]), false, 0,
                      s);
    FV_HIP(hipStreamSynchronize(s));  // its task copy has left the pinned buffer
    std::memcpy(local.pin, samp.data(), sizeof(GraphTask) * ns);
    hipEvent_t a = ev.a, b = ev.b;
    float best_ms = 0.0f;
    size_t best = lds;
    bool first = true;
    for (size_t cand : kBatchLdsCand) {
      const int grid = batch_grid<VT>(ns, cand);
      FV_HIP(hipEventRecord(a, s));
      enqueue_batch<VT>(local, ns, cand, grid, false, 0, s);
      FV_HIP(hipEventRecord(b, s));
      FV_HIP(hipEventSynchronize(b));
      float ms = 0.0f;
      FV_HIP(hipEventElapsedTime(&ms, a, b));
      if (first || ms < best_ms) {
        best_ms = ms;
        best = cand;
        first = false;
      }
    }
    lds = best;
    tuned = 1;
    {
      std::lock_guard<std::mutex> g(g_tune_mu);
      g_tune[key] = lds;
    }
    std::memcpy(local.pin, all.data(), sizeof(GraphTask) * count);
  }
  const int grid = batch_grid<VT>(count, lds);

  hipEvent_t e0 = ev.a, e1 = ev.b;
  if (replay) {
    FV_HIP(hipEventRecord(e0, s));
    FV_HIP(hipGraphLaunch(bg->exec, s));
    FV_HIP(hipEventRecord(e1, s));
  } else if (bo && bo->graph && !gkey.empty()) {
    // Capture the sequence, keep it (with its buffers) for a repeat of this
    // call, and run it.
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    FV_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      enqueue_batch<VT>(local, count, lds, grid, stats != nullptr, nout, s);
    } catch (...) {
      (void)hipStreamEndCapture(s, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    FV_HIP(hipStreamEndCapture(s, &graph));
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      throw Error(FV_E_DEVICE, "hipGraphInstantiate");
    }
    if (!ctx->bgraph) ctx->bgraph = new BatchGraph();
    bg = static_cast<BatchGraph*>(ctx->bgraph);
    FV_HIP(hipStreamSynchronize(s));  // the old graph's buffers are idle
    bg->release();
    bg->graph = graph;
    bg->exec = exec;
    bg->key = gkey;
    bg->bufs = local;
    guard.own = false;
    buf = &bg->bufs;
    FV_HIP(hipEventRecord(e0, s));
    FV_HIP(hipGraphLaunch(exec, s));
    FV_HIP(hipEventRecord(e1, s));
  } else {
    FV_HIP(hipEventRecord(e0, s));
    enqueue_batch<VT>(local, count, lds, grid, stats != nullptr, nout, s);
    FV_HIP(hipEventRecord(e1, s));
  }
  FV_HIP(hipStreamSynchronize(s));
  float ms = 0.0f;
  FV_HIP(hipEventElapsedTime(&ms, e0, e1));
  const char* pin = static_cast<const char*>(buf->pin);
  const DevState* hst = reinterpret_cast<const DevState*>(pin + buf->p_st);
  const int* hslen = reinterpret_cast<const int*>(pin + buf->p_slen);
  const int* hsched = reinterpret_cast<const int*>(pin + buf->p_sched);
  const double* hout = reinterpret_cast<const double*>(pin + buf->p_out);
  if (!x_on_device)
    for (int k = 0; k < count; ++k)
      std::memcpy(x_out[k], hout + xoff[k], sizeof(double) * (xoff[k + 1] - xoff[k]));
  for (int k = 0; k < count; ++k) {
    if (lambda_out) lambda_out[k] = hst[k].lambda;
    if (item_status) item_status[k] = hst[k].err ? FV_E_NOT_CONVERGED : FV_OK;
    if (stats) {
      fv_solve_stats& S = stats[k];
      std::memset(&S, 0, sizeof(S));
      const fv_hierarchy* h = hs[k];
      S.levels = h->levels;
      for (int l = 0; l < h->levels; ++l) {
        S.n[l] = h->lv[l].n;
        S.nnz[l] = h->lv[l].m;
        S.colours[l] = l == h->levels - 1 ? 0 : h->lv[l].ncol;
      }
      S.schedule_len = std::min(hslen[k], FV_SCHEDULE_CAP);
      for (int i = 0; i < S.schedule_len; ++i) S.schedule[i] = hsched[(size_t)k * FV_SCHEDULE_CAP + i];
      S.lambda = hst[k].lambda;
      S.residual = hst[k].res;
      S.final_cos = hst[k].cos;
      S.t_solve_ms = ms;  // the whole launch
      S.alg_bytes = schedule_bytes(h, S.schedule, S.schedule_len, o->prec);
    }
  }
  if (bo) {
    bo->lds_bytes_used = (int64_t)lds;
    bo->grid = grid;
    bo->tuned = tuned;
    bo->replayed = replay ? 1 : 0;
    bo->launch_ms = ms;
  }
  return FV_OK;
}

fv_status solve_batch(fv_context* ctx, int count, const fv_hierarchy* const* hs,
                      const fv_solve_opts* o, fv_batch_opts* bo, double* const* x_out,
                      int x_on_device, double* lambda_out, fv_solve_stats* stats,
                      fv_status* item_status, hipStream_t s) {
  if (count <= 0) return FV_OK;
  if (o->prec == FV_PREC_FP32_MIXED)
    return solve_batch_t<float>(ctx, count, hs, o, bo, x_out, x_on_device, lambda_out, stats,
                                item_status, s);
  return solve_batch_t<double>(ctx, count, hs, o, bo, x_out, x_on_device, lambda_out, stats,
                               item_status, s);
}

}  // namespace fv
