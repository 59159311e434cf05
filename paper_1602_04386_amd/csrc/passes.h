// Multi-workgroup passes over one large level (included by solve.hip after the
// per-row arithmetic).
//
// Each pass kernel handles tiles of kBlock consecutive rows (solve order).  A
// tile first stages its row pointers in LDS, then walks its rows in chunks
// whose CSR slice fits the tile's LDS capacity: the chunk's column indices, weights
// and the neighbour values those columns gather are staged in LDS with
// unit-stride loads and all gathers of the chunk in flight together, and each
// thread then reduces its own row from LDS in CSR order, the same arithmetic
// as the direct row functions.  Usually the whole tile is one chunk; dense
// tiles (irregular graphs put their high-degree vertices in the last colours)
// take two, and a single row longer than the capacity uses direct loads.
//
// A pass writes one partial-sum slot per block; a one-block finishing kernel
// reduces the slots in a fixed order and updates the device state.  The
// kernel boundary makes the partials visible, so no block needs a
// device-scope fence.
#pragma once

// Entries a tile stages at once.  2048 keeps an FP32 tile at 25 KB of LDS
// (six blocks per CU); 4096 entries made the level-0 sweeps 15 % slower
// through the lost occupancy.
template <class WT, class XT>
constexpr int tile_cap() { return 2048; }
constexpr int kStageU = 8;  // staging slots per thread: kStageU * kBlock = the tile capacity

// Waves per SIMD that a tile kernel's LDS leaves room for: six FP32 tiles of
// one row per thread (26 KB each), five of two rows per thread (27 KB), or
// three FP64 tiles fit a CU.  The kernels ask the compiler for that many so
// that registers never cut the occupancy below what LDS allows (at 86
// registers the one-row FP32 sweep ran five blocks per CU, and the 1,488-block
// colours of the 1024 x 1000 grid then needed a second round of blocks).
template <class VT, int RPT = 1>
constexpr int tile_waves() { return sizeof(VT) == 4 ? (RPT == 1 ? 6 : 5) : 3; }

// A tile is RPT * kBlock consecutive rows, RPT per thread (rows t, t + kBlock,
// ...).  Two rows per thread let a colour of up to twice as many rows run in
// one round of resident blocks, so that its blocks' dependent load phases are
// paid once (a second, partial round pays them again).
template <class WT, class XT, int RPT = 1>
struct TileLds {
  static constexpr int kRows = RPT * kBlock;
  static constexpr int kCap = tile_cap<WT, XT>();
  int rp[kRows + 1];
  int col[kCap];
  WT w[kCap];
  XT x[kCap];
};

// Stages a chunk of cnt <= U * kBlock entries starting at CSR position p_lo:
// thread t takes entries u * kBlock + t (u < U).  Every load and LDS store is
// unconditional (positions past the chunk repeat its last entry and land in
// LDS slots that no row reads), and all index and weight loads come before
// all gathers: the chunk costs two memory round trips.  With loads or stores
// under per-entry conditions the compiler moves loads next to their
// conditional use and waits for each before issuing the next.
template <int U, class WT, class XT, int RPT, class G>
__device__ __forceinline__ void stage_chunk(const int* __restrict__ col,
                                            const WT* __restrict__ w, int p_lo, int cnt,
                                            TileLds<WT, XT, RPT>& T, G gather) {
  static_assert(U * kBlock <= TileLds<WT, XT, RPT>::kCap, "staging slots exceed the tile");
  const int t = threadIdx.x;
  int cc[U];
  WT ww[U];
  XT xx[U];
#pragma unroll
  for (int u = 0; u < U; ++u) cc[u] = col[p_lo + min(u * kBlock + t, cnt - 1)];
#pragma unroll
  for (int u = 0; u < U; ++u) ww[u] = w[p_lo + min(u * kBlock + t, cnt - 1)];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < U; ++u) xx[u] = gather(cc[u]);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    T.col[u * kBlock + t] = cc[u];
    T.w[u * kBlock + t] = ww[u];
    T.x[u * kBlock + t] = xx[u];
  }
}

// A tile's row pointers as for_tile_chunks_from stages them: thread t holds those
// of rows t + k kBlock (k < RPT) and thread 0 the one past a full tile.
template <int RPT>
struct TileRp {
  int a[RPT];
  int b;
};

template <int RPT>
__device__ inline TileRp<RPT> load_tile_rp(const LevelDesc& L, int rs, int re) {
  constexpr int kRows = RPT * kBlock;
  const int nr = re - rs;
  const int t = threadIdx.x;
  TileRp<RPT> r;
#pragma unroll
  for (int k = 0; k < RPT; ++k) r.a[k] = t + k * kBlock <= nr ? L.rp[rs + t + k * kBlock] : 0;
  r.b = (t == 0 && nr == kRows) ? L.rp[rs + kRows] : 0;
  return r;
}

// Walks the rows [rs, re) (re - rs <= T.kRows) of a tile chunk by chunk.  For
// each chunk it stages the CSR slice and gather(col) in LDS, then calls
// body(tt, k, a, e) for every row rs + tt of the chunk in the thread that owns
// it (tt = threadIdx.x + k kBlock, k < RPT a compile-time index after
// unrolling), [a, e) being that row's entries in T.  A row longer than
// T.kCap is passed to direct(tt) instead.  Every thread of the block must
// call; the rows of one tile never read values that the body writes.
// skip (the phase's stop flag, loaded by the caller before this call) is
// tested only after the row pointers are requested, so that both loads are in
// flight together; when set, nothing else happens and false is returned.
// pre() runs in every thread once the row pointer loads are issued and before
// their values are used: the loads a thread issues there (its own rows'
// values) travel alongside the CSR staging instead of after it.  The block has
// kBlock threads.
// The tile's row pointers come already requested (rpl, from load_tile_rp),
// so that a loop over tiles can request the next tile's while this one runs.
template <class WT, class XT, int RPT, class P, class G, class B, class D>
__device__ inline bool for_tile_chunks_from(const LevelDesc& L, const WT* __restrict__ w, int rs,
                                            int re, TileLds<WT, XT, RPT>& T, int skip,
                                            const TileRp<RPT>& rpl, P pre, G gather, B body,
                                            D direct) {
  constexpr int kRows = TileLds<WT, XT, RPT>::kRows;
  const int nr = re - rs;
  const int t = threadIdx.x;
  const bool extra = t == 0 && nr == kRows;  // the pointer past a full tile
  int rp_a[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) rp_a[k] = rpl.a[k];
  const int rp_b = rpl.b;
  pre();
#pragma unroll
  for (int k = 0; k < RPT; ++k)
    if (t + k * kBlock <= nr) T.rp[t + k * kBlock] = rp_a[k];
  if (extra) T.rp[kRows] = rp_b;
  __syncthreads();
  if (skip) return false;
  const int* __restrict__ col = L.col;
  int lo = 0;
  while (lo < nr) {  // uniform: every bound comes from T.rp
    const int p_lo = T.rp[lo];
    if (T.rp[lo + 1] - p_lo > T.kCap) {
      if (t == lo % kBlock) direct(lo);
      ++lo;
      continue;
    }
    int a = lo + 1, b = nr;  // last row boundary whose slice still fits
    while (a < b) {
      const int mid = (a + b + 1) >> 1;
      if (T.rp[mid] - p_lo <= T.kCap) a = mid; else b = mid - 1;
    }
    const int hi = a, cnt = T.rp[hi] - p_lo;
    // A chunk with at most half the slots filled takes the narrow form, so no
    // load is wasted on the common short tiles.
    if (cnt <= 0) {
      // rows without entries: nothing to stage
    } else if (cnt <= (kStageU / 2) * kBlock) {
      stage_chunk<kStageU / 2>(col, w, p_lo, cnt, T, gather);
    } else {
      stage_chunk<kStageU>(col, w, p_lo, cnt, T, gather);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int tt = t + k * kBlock;
      if (tt >= lo && tt < hi) body(tt, k, T.rp[tt] - p_lo, T.rp[tt + 1] - p_lo);
    }
    __syncthreads();
    lo = hi;
  }
  return true;
}

// for_tile_chunks_from with the tile's own row pointers requested first.
template <class WT, class XT, int RPT, class P, class G, class B, class D>
__device__ inline bool for_tile_chunks(const LevelDesc& L, const WT* __restrict__ w, int rs,
                                       int re, TileLds<WT, XT, RPT>& T, int skip, P pre,
                                       G gather, B body, D direct) {
  const TileRp<RPT> rpl = load_tile_rp<RPT>(L, rs, re);
  return for_tile_chunks_from<WT, XT, RPT>(L, w, rs, re, T, skip, rpl, pre, gather, body, direct);
}

// Opens a phase.  With use_halt set, a phase enqueued after the finest
// residual met its tolerance starts finished, so the host may enqueue the next
// finest round before it has read that residual.  *rec receives the phase's
// step count (the finishing kernels keep it current); *hdone, in mapped host
// memory, the phase's stop flag (likewise kept current).
__global__ void k_phase_begin(DevState* st, int cap, int forced, double tol, int use_halt,
                              int* rec, int* hdone) {
  const int done = (cap <= 0 || (use_halt && st->halt)) ? 1 : 0;
  st->done = done;
  *hdone = done;  // the finishing kernels only ever raise it
  *rec = 0;
  st->iters = 0;
  st->cap = cap;
  st->forced = forced;
  st->tol = tol;
}

// Reduces a block's kNP sums and writes them to partial slot `slot`; threads
// 0 .. kNP-1 store one value each.
__device__ inline void store_block_sum(double (&S)[kNP], double* lds, double* part, int stride,
                                       int slot) {
  const double t = block_sum_spread<kNP>(S, lds);
  if (threadIdx.x < kNP) part[threadIdx.x * stride + slot] = t;
}

// ---- finishing kernels (one block) -----------------------------------------

enum FinishMode { kFinGS = 0, kFinPI = 1, kFinProlong = 2, kFinRQ = 3 };

// Adds the partial-slot rows 0 .. NR-1 of slots threadIdx.x, + blockDim.x, ...
// into S in that order.  The loads of kSlotU consecutive slots are issued
// before any of their additions, so a large level's thousands of slots cost a
// few memory round trips per thread instead of one per slot.
constexpr int kSlotU = 8;

template <int NR>
__device__ inline void sum_slots(const double* part, int stride, int nslots, double (&S)[kNP]) {
  for (int s0 = threadIdx.x; s0 < nslots; s0 += blockDim.x * kSlotU) {
    double v[kSlotU][NR];
#pragma unroll
    for (int u = 0; u < kSlotU; ++u) {
      const int s = s0 + u * blockDim.x;
#pragma unroll
      for (int k = 0; k < NR; ++k) v[u][k] = s < nslots ? part[k * stride + s] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kSlotU; ++u)
#pragma unroll
      for (int k = 0; k < NR; ++k) S[k] += v[u][k];
  }
}


// State update that closes a smoothing sweep (S: the sweep's sums, in wave 0
// lane 0): next pending normalisation and shift, cosine, step count and the
// stop decision.
__device__ inline void close_gs_sweep(DevState* st, const double (&S)[kNP], int n, int* rec,
                                      int* hdone) {
  const Scal r = after_gs(S, n);
  st->mu = r.mu;
  st->inv_s = r.inv_s;
  st->cos = r.cos;
  st->rho = r.rho;
  const int it = st->iters + 1;
  st->iters = it;
  *rec = it;
  const int done =
      (it >= st->cap || (!st->forced && st->tol > 0.0 && r.cos > 1.0 - st->tol)) ? 1 : 0;
  st->done = done;
  // The host copy only ever goes from 0 (set when the phase opens) to 1: a
  // write across the bus on every step would hold up the kernel's end.
  if (done) *hdone = 1;
}

// ---- smoothing sweep, one colour -------------------------------------------

// The rows [rs, re) of colour [r0, r1) as one tile, their row pointers
// already requested (rpl): each row relaxed in place, its sums added to acc.
// False, with nothing done, when the phase has ended (skip).
template <class VT, int RPT>
__device__ inline bool gs_tile_rows(const LevelDesc& L, int r0, int rs, int re,
                                    TileLds<VT, VT, RPT>& T, int skip, const TileRp<RPT>& rpl,
                                    VT* x, double mu, double inv_s, double rho, double omega,
                                    double (&acc)[kNP]) {
  const auto* w = WSel<VT>::w(L);
  VT xown[RPT];
  return for_tile_chunks_from<VT, VT, RPT>(
      L, w, rs, re, T, skip, rpl,
      [&] {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int i = rs + (int)threadIdx.x + k * kBlock;
          xown[k] = i < re ? x[i] : VT(0);
        }
      },
      [&](int c) { return x[c]; },
      [&](int t, int kk, int a, int e) {
        const int i = rs + t;
        const double xo = ((double)xown[kk] - mu) * inv_s;
        double num = 0.0, den = 0.0;
        for (int k = a; k < e; ++k)
          gs_entry(num, den, (double)T.w[k], (double)T.x[k], T.col[k] < r0, mu, inv_s);
        const VT us = (VT)gs_relax(num, den, xo, rho, omega);
        x[i] = us;
        const double ud = (double)us;
        double en = 0.0;
        for (int k = a; k < e; ++k)
          if (T.col[k] < r0) gs_energy(en, (double)T.w[k], ud, (double)T.x[k]);
        gs_sums(acc, ud, xo, en);
      },
      [&](int t) { row_gs<VT>(rs + t, L, x, r0, mu, inv_s, rho, omega, acc); });
}

// One tile of a colour per block (tile b, in XCD order); its sums go to
// partial slot slot_base + blockIdx.x.
template <class VT, int RPT>
__global__ __launch_bounds__(kBlock, (tile_waves<VT, RPT>())) void k_gs_tile(LevelDesc L, int r0, int r1, VT* xa, VT* xb,
                                                  const DevState* st, double* part, int stride,
                                                  int slot_base, double omega) {
  __shared__ TileLds<VT, VT, RPT> T;
  __shared__ double lds[block_sum_lds(kBlock)];
  const int done = st->done;
  VT* x = st->cur ? xb : xa;
  const double mu = st->mu, inv_s = st->inv_s, rho = st->rho;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int rs = r0 + b * T.kRows, re = min(rs + T.kRows, r1);
  double acc[kNP] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (!gs_tile_rows<VT, RPT>(L, r0, rs, re, T, done, load_tile_rp<RPT>(L, rs, re), x, mu, inv_s,
                             rho, omega, acc))
    return;
  store_block_sum(acc, lds, part, stride, slot_base + blockIdx.x);
}

// ---- smoothing sweep, one colour, from the level's ELL copy ----------------

// The rows, block-to-slot mapping, arithmetic and summation order of
// k_gs_tile<VT, RPT>, so the two give bitwise-equal sweeps; the row's entries
// come from the colour's slot-major block (ec, ev: entry k of row r0 + i at
// k * (r1 - r0) + i; EW slots, column -1 past the row's end) straight into
// registers.  Entry k of the rows of a wave are consecutive
// words, so the loads are coalesced and need no row pointers.  Two load
// phases: the column indices (with the phase state), then the weights, the
// row's own values and the gathers of the neighbour values together.  No LDS
// staging and no barrier before the block's sum.
// Waves per SIMD the ELL sweep asks the compiler to leave room for: those of
// the tile sweep of the same rows per thread (the same block counts then run
// in one round), four for rows of 12 or 16 slots and two for wider rows
// (their registers: an index, a weight and a gathered value per slot), which
// only smaller colours have.
template <class VT, int EW, int RPT>
constexpr int ell_waves() { return EW <= 8 ? tile_waves<VT, RPT>() : EW <= 16 ? 4 : 2; }

template <class VT, int EW, int RPT>
__global__ __launch_bounds__(kBlock, (ell_waves<VT, EW, RPT>())) void k_gs_ell(
    int r0, int r1, const int* __restrict__ ec, const VT* __restrict__ ev, VT* xa, VT* xb,
    const DevState* st, double* part, int stride, int slot_base, double omega) {
  __shared__ double lds[block_sum_lds(kBlock)];
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int rs = r0 + b * RPT * kBlock;
  const int rows = r1 - r0;
  int done = st->done, cur = st->cur;
  double mu = st->mu, inv_s = st->inv_s, rho = st->rho;
  int row[RPT];
  int cc[RPT][EW];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    // rows past the colour repeat its last row (loaded, never written)
    row[k] = min(rs + (int)threadIdx.x + k * kBlock, r1 - 1);
#pragma unroll
    for (int j = 0; j < EW; ++j) cc[k][j] = ec[j * rows + row[k] - r0];
  }
  // The index loads and the phase state complete together here, before the
  // stop flag is tested: the compiler would otherwise test the flag first and
  // issue the index loads after it, and load the state after the flag, each a
  // memory round trip of its own.  A launch after the phase has ended reads
  // the indices and returns.
#pragma unroll
  for (int k = 0; k < RPT; ++k)
#pragma unroll
    for (int j = 0; j < EW; ++j) asm volatile("" : "+v"(cc[k][j]));
  asm volatile("" : "+s"(done), "+s"(cur), "+s"(mu), "+s"(inv_s), "+s"(rho));
  if (done) return;
  VT* x = cur ? xb : xa;
  VT ww[RPT][EW];
  VT xown[RPT];
  VT xg[RPT][EW];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
#pragma unroll
    for (int j = 0; j < EW; ++j) ww[k][j] = ev[j * rows + row[k] - r0];
    xown[k] = x[row[k]];
#pragma unroll
    for (int j = 0; j < EW; ++j) xg[k][j] = x[cc[k][j] >= 0 ? cc[k][j] : row[k]];
  }
  double acc[kNP] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int i = rs + (int)threadIdx.x + k * kBlock;
    if (i >= r1) continue;
    const double xo = ((double)xown[k] - mu) * inv_s;
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int j = 0; j < EW; ++j)
      if (cc[k][j] >= 0)
        gs_entry(num, den, (double)ww[k][j], (double)xg[k][j], cc[k][j] < r0, mu, inv_s);
    const VT us = (VT)gs_relax(num, den, xo, rho, omega);
    x[i] = us;
    const double ud = (double)us;
    double en = 0.0;
#pragma unroll
    for (int j = 0; j < EW; ++j)
      if (cc[k][j] >= 0 && cc[k][j] < r0) gs_energy(en, (double)ww[k][j], ud, (double)xg[k][j]);
    gs_sums(acc, ud, xo, en);
  }
  store_block_sum(acc, lds, part, stride, slot_base + blockIdx.x);
}

// ---- power step ------------------------------------------------------------

// The rows [rs, re) as one tile of the power step, their row pointers already
// requested (rpl): y = (sigma I - L) x over the normalised x, the sums added to
// acc.  False, with nothing done, when the phase has ended (skip).
template <class VT, int RPT>
__device__ inline bool pi_tile_rows(const LevelDesc& L, int rs, int re, TileLds<VT, VT, RPT>& T,
                                    int skip, const TileRp<RPT>& rpl, const VT* x, VT* y,
                                    double mu, double inv_s, double (&acc)[kNP]) {
  const auto* w = WSel<VT>::w(L);
  const double sigma = L.sigma;
  VT xown[RPT];
  return for_tile_chunks_from<VT, VT, RPT>(
      L, w, rs, re, T, skip, rpl,
      [&] {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int i = rs + (int)threadIdx.x + k * kBlock;
          xown[k] = i < re ? x[i] : VT(0);
        }
      },
      [&](int c) { return x[c]; },
      [&](int t, int kk, int a, int e) {
        const int i = rs + t;
        const double xi = (double)xown[kk];
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
      },
      [&](int t) { row_pi<VT>(rs + t, L, x, y, mu, inv_s, sigma, acc); });
}

template <class VT, int RPT>
__global__ __launch_bounds__(kBlock, (tile_waves<VT, RPT>())) void k_pi_tile(LevelDesc L, VT* xa, VT* xb,
                                                  const DevState* st, double* part, int stride) {
  __shared__ TileLds<VT, VT, RPT> T;
  __shared__ double lds[block_sum_lds(kBlock)];
  const int done = st->done;
  const int cur = st->cur;
  const VT* x = cur ? xb : xa;
  VT* y = cur ? xa : xb;
  const double mu = st->mu, inv_s = st->inv_s;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int rs = b * T.kRows, re = min(rs + T.kRows, L.n);
  double acc[kNP] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (!pi_tile_rows<VT, RPT>(L, rs, re, T, done, load_tile_rp<RPT>(L, rs, re), x, y, mu, inv_s,
                             acc))
    return;
  store_block_sum(acc, lds, part, stride, blockIdx.x);
}

// The power step over a level of more tiles than one round of resident
// blocks: each of the grid's blocks takes tiles b, b + G, b + 2G, ... (G the
// grid; b in XCD order) and requests the next tile's row pointers before it
// stages the current one, so that their round trip overlaps the current
// tile's loads and arithmetic.  The block adds all its tiles' sums into one
// partial slot.
template <class VT, int RPT>
__global__ __launch_bounds__(kBlock, (tile_waves<VT, RPT>())) void k_pi_tile_loop(
    LevelDesc L, VT* xa, VT* xb, const DevState* st, double* part, int stride, int ntiles) {
  __shared__ TileLds<VT, VT, RPT> T;
  __shared__ double lds[block_sum_lds(kBlock)];
  const int done = st->done;
  const int cur = st->cur;
  const VT* x = cur ? xb : xa;
  VT* y = cur ? xa : xb;
  const double mu = st->mu, inv_s = st->inv_s;
  const int G = gridDim.x;
  double acc[kNP] = {0.0, 0.0, 0.0, 0.0, 0.0};
  int tile = xcd_block(blockIdx.x, G);
  int rs = tile * T.kRows, re = min(rs + T.kRows, L.n);
  TileRp<RPT> rpl = load_tile_rp<RPT>(L, rs, re);
  for (; tile < ntiles; tile += G) {
    const int ns = rs + G * T.kRows;
    TileRp<RPT> next = rpl;
    if (tile + G < ntiles) next = load_tile_rp<RPT>(L, ns, min(ns + T.kRows, L.n));
    if (!pi_tile_rows<VT, RPT>(L, rs, re, T, done, rpl, x, y, mu, inv_s, acc)) return;
    __syncthreads();  // the tile's LDS is read before the next tile stages into it
    rs = ns;
    re = min(rs + T.kRows, L.n);
    rpl = next;
  }
  store_block_sum(acc, lds, part, stride, blockIdx.x);
}

// ---- prolongation ----------------------------------------------------------

template <class SRC, class VT, int RPT>
__global__ __launch_bounds__(kBlock, (tile_waves<VT, RPT>())) void k_prolong_tile(LevelDesc L, const SRC* xc_a,
                                                       const SRC* xc_b, VT* xf_a, VT* xf_b,
                                                       const DevState* st, double* part,
                                                       int stride) {
  __shared__ TileLds<VT, VT, RPT> T;
  __shared__ double lds[block_sum_lds(kBlock)];
  const int cur = st->cur;
  const SRC* xc = cur ? xc_b : xc_a;
  VT* xf = cur ? xf_a : xf_b;
  const double mu = st->mu, inv_s = st->inv_s;
  const int* __restrict__ qs = L.qs;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int rs = b * T.kRows, re = min(rs + T.kRows, L.n);
  const auto* w = WSel<VT>::w(L);
  double acc[kNP] = {0.0, 0.0, 0.0, 0.0, 0.0};
  SRC cown[RPT];
  for_tile_chunks<VT, VT, RPT>(
      L, w, rs, re, T, 0,
      [&] {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int i = rs + (int)threadIdx.x + k * kBlock;
          cown[k] = i < re ? xc[qs[i]] : SRC(0);
        }
      },
      [&](int c) { return (VT)(((double)xc[qs[c]] - mu) * inv_s); },
      [&](int t, int kk, int a, int e) {
        const int i = rs + t;
        const VT vs = (VT)(((double)cown[kk] - mu) * inv_s);
        xf[i] = vs;
        const double v = (double)vs;
        double en = 0.0;
        for (int k = a; k < e; ++k) {
          const double d = v - (double)T.x[k];
          en += (double)T.w[k] * d * d;
        }
        acc[0] += v;
        acc[1] += v * v;
        acc[4] += 0.5 * en;
      },
      [&](int t) { row_prolong<SRC, VT>(rs + t, L, xc, xf, mu, inv_s, acc); });
  store_block_sum(acc, lds, part, stride, blockIdx.x);
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
  VT xown = VT(0);
  for_tile_chunks<double, VT, 1>(
      L, L.w64, rs, re, T, 0,
      [&] {
        if (rs + (int)threadIdx.x < re) xown = x[rs + threadIdx.x];
      },
      [&](int c) { return x[c]; },
      [&](int t, int, int a, int e) {
        const int i = rs + t;
        const double xi = ((double)xown - mu) * inv_s;
        double lx = 0.0, en = 0.0;
        for (int k = a; k < e; ++k) {
          const double d = xi - ((double)T.x[k] - mu) * inv_s;
          lx += T.w[k] * d;
          en += T.w[k] * d * d;
        }
        lxo[i] = lx;
        a3[0] += xi * xi;
        a3[1] += 0.5 * en;
        a3[2] = fmax(a3[2], fabs(xi));
      },
      [&](int t) { row_rq<VT>(rs + t, L, x, mu, inv_s, lxo, a3); });
  const double mx = block_max(a3[2], lds);
  double t2[2] = {a3[0], a3[1]};
  const double t = block_sum_spread<2>(t2, lds);
  if (threadIdx.x < 2) part[threadIdx.x * stride + blockIdx.x] = t;
  if (threadIdx.x == 2) part[2 * stride + blockIdx.x] = mx;
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

__global__ __launch_bounds__(kBlock) void k_finish(DevState* st, const double* part, int stride,
                                                 int nslots, int n, int mode, int* rec,
                                                 int* hdone) {
  __shared__ double lds[block_sum_lds(kBlock)];
  if ((mode == kFinGS || mode == kFinPI) && st->done) return;
  double S[kNP] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double mx = 0.0;
  if (mode == kFinRQ) {
    for (int s = threadIdx.x; s < nslots; s += blockDim.x) {
      S[0] += part[s];
      S[1] += part[stride + s];
      mx = fmax(mx, part[2 * stride + s]);
    }
  } else {
    sum_slots<kNP>(part, stride, nslots, S);
  }
  const double t = block_sum_spread<kNP>(S, lds);
  if (mode == kFinRQ) {
    __syncthreads();  // the row sums in lds are read before block_max reuses it
    mx = block_max(mx, lds);
  }
  if (threadIdx.x >= 64) return;
  wave0_collect<kNP>(t, S);
  if (threadIdx.x != 0) return;
  if (mode == kFinRQ) {
    st->sumsq = S[0];
    st->lambda = S[1] / S[0];
    st->xmax = mx;
    st->rho = st->lambda;
    return;
  }
  if (mode == kFinGS) {
    close_gs_sweep(st, S, n, rec, hdone);
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
  *rec = it;
  const int done =
      (it >= st->cap || (!st->forced && st->tol > 0.0 && r.cos > 1.0 - st->tol)) ? 1 : 0;
  st->done = done;
  if (done) *hdone = 1;
}

// Finishing kernel of a sweep whose last colours are small: the block first
// sweeps the rows of colours c0 .. ncol-1 itself (colour by colour, the
// barrier ordering them), adding their sums to the partial slots of the
// colours the tile kernels did, then finishes as k_finish does.  One launch
// instead of one per small trailing colour (first-fit colourings leave a few
// colours with a handful of rows each).  A tail colour with an ELL block
// (eoff[c - c0] >= 0, EW > 0 slots a row) is swept from it: two dependent
// load phases instead of a row-pointer phase and one pair per batch of eight
// entries (the dense last colours of irregular levels hold 15 to 20).
constexpr int kTailBlock = 512;
constexpr int kTailRows = 512;  // one row per thread: the tail adds one dependent row pass
constexpr int kTailEll = 8;     // tail colours that may have ELL blocks

struct TailEll {
  long long eoff[kTailEll];  // slot offset of tail colour c0 + k's block, or -1
};

// Shifted sweep update of row i (of a colour with rows [r0, r0 + rows)) from
// the colour's ELL block at ec / ev: the arithmetic of row_gs_batched.
template <class VT, int EW>
__device__ inline void row_gs_ell(int i, int r0, int rows, const int* __restrict__ ec,
                                  const VT* __restrict__ ev, VT* __restrict__ x, double mu,
                                  double inv_s, double rho, double omega, double (&acc)[kNP]) {
  const int li = i - r0;
  int cc[EW];
  VT ww[EW], xg[EW];
#pragma unroll
  for (int j = 0; j < EW; ++j) cc[j] = ec[j * rows + li];
#pragma unroll
  for (int j = 0; j < EW; ++j) ww[j] = ev[j * rows + li];
  const VT xv = x[i];
#pragma unroll
  for (int j = 0; j < EW; ++j) xg[j] = x[cc[j] >= 0 ? cc[j] : i];
  const double xo = ((double)xv - mu) * inv_s;
  double num = 0.0, den = 0.0;
#pragma unroll
  for (int j = 0; j < EW; ++j)
    if (cc[j] >= 0) gs_entry(num, den, (double)ww[j], (double)xg[j], cc[j] < r0, mu, inv_s);
  const VT us = (VT)gs_relax(num, den, xo, rho, omega);
  x[i] = us;
  const double ud = (double)us;
  double e = 0.0;
#pragma unroll
  for (int j = 0; j < EW; ++j)
    if (cc[j] >= 0 && cc[j] < r0) gs_energy(e, (double)ww[j], ud, (double)xg[j]);
  gs_sums(acc, ud, xo, e);
}

template <class VT, int EW>
__global__ __launch_bounds__(kTailBlock) void k_finish_gs_tail(LevelDesc L, VT* xa, VT* xb,
                                                             DevState* st, const double* part,
                                                             int stride, int nslots, int c0,
                                                             int tr0, int tr1, double omega,
                                                             TailEll te, int* rec, int* hdone) {
  __shared__ double lds[block_sum_lds(kTailBlock)];
  if (st->done) return;
  VT* x = st->cur ? xb : xa;
  const double mu = st->mu, inv_s = st->inv_s, rho = st->rho;
  const VT* ev0 = nullptr;
  if constexpr (EW > 0)
    ev0 = sizeof(VT) == 4 ? reinterpret_cast<const VT*>(L.ew32) : reinterpret_cast<const VT*>(L.ew64);
  auto ell_of = [&](int c) -> long long {
    return EW > 0 && c - c0 < kTailEll ? te.eoff[c - c0] : -1;
  };
  // The first tail colour holds rows [tr0, tr1) (at most kTailRows, one per
  // thread); its row pointers are requested before the partial slots are
  // added, so that the two round trips overlap.
  const int i0 = tr0 + threadIdx.x;
  const long long e0 = ell_of(c0);
  int p0 = 0, p1 = 0;
  if (i0 < tr1 && e0 < 0) {
    p0 = L.rp[i0];
    p1 = L.rp[i0 + 1];
  }
  double S[kNP] = {0.0, 0.0, 0.0, 0.0, 0.0};
  sum_slots<kNP>(part, stride, nslots, S);
  if (i0 < tr1) {
    if constexpr (EW > 0) {
      if (e0 >= 0)
        row_gs_ell<VT, EW>(i0, tr0, tr1 - tr0, L.ecol + e0, ev0 + e0, x, mu, inv_s, rho, omega, S);
      else
        row_gs_batched<VT>(i0, p0, p1, L, x, tr0, mu, inv_s, rho, omega, S);
    } else {
      row_gs_batched<VT>(i0, p0, p1, L, x, tr0, mu, inv_s, rho, omega, S);
    }
  }
  __syncthreads();  // the next colour reads this colour's new values
  for (int c = c0 + 1; c < L.ncol; ++c) {
    const int r0 = L.cptr[c], r1 = L.cptr[c + 1];
    const long long ec = ell_of(c);
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
      if constexpr (EW > 0) {
        if (ec >= 0) {
          row_gs_ell<VT, EW>(i, r0, r1 - r0, L.ecol + ec, ev0 + ec, x, mu, inv_s, rho, omega, S);
          continue;
        }
      }
      row_gs_batched<VT>(i, L.rp[i], L.rp[i + 1], L, x, r0, mu, inv_s, rho, omega, S);
    }
    __syncthreads();
  }
  const double t = block_sum_spread<kNP>(S, lds);
  if (threadIdx.x >= 64) return;
  wave0_collect<kNP>(t, S);
  if (threadIdx.x != 0) return;
  const Scal r = after_gs(S, L.n);
  st->mu = r.mu;
  st->inv_s = r.inv_s;
  st->cos = r.cos;
  st->rho = r.rho;
  const int it = st->iters + 1;
  st->iters = it;
  *rec = it;
  const int done =
      (it >= st->cap || (!st->forced && st->tol > 0.0 && r.cos > 1.0 - st->tol)) ? 1 : 0;
  st->done = done;
  if (done) *hdone = 1;
}

// Finishes the finest residual pass.  The halt flag (later phases do
// nothing) goes up when the residual meets tol_halt or, with early exit
// (early_left >= 0: rounds max_outer leaves after this pass, which follows
// at least one finest round), when it cannot reach tol_halt in those rounds.
template <class VT>
__global__ __launch_bounds__(kBlock) void k_finish_res(LevelDesc L, const VT* xa, const VT* xb,
                                                     DevState* st, const double* part,
                                                     const int* ipart, int nslots,
                                                     double tol_halt, int early_left,
                                                     double* hres) {
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
  const double res = sqrt(s[0] / st->sumsq);
  const double res_prev = st->res;
  st->res = res;
  *hres = res;
  st->halt = (tol_halt > 0.0 && (res <= tol_halt ||
                                 (early_left >= 0 && !can_reach(res, res_prev, tol_halt,
                                                                early_left))))
                 ? 1
                 : 0;
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
