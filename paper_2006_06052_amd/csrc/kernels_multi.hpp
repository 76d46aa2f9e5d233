// gfx950 kernels for K <= 32 right-hand sides solved together.
//
// Vectors are [n][K] row-major (the K right-hand sides of one scalar row are
// contiguous).  In the matrix kernels a workgroup of 256 lanes covers 8 block
// rows, 32 lanes per row, and lane k < K computes every scalar row of its block
// row for right-hand side k.  The workgroup first copies its rows' column indices
// and block values (a contiguous range) into LDS with coalesced loads; each lane
// then reads them from LDS, so a stored block is fetched from HBM once, and reads
// each x block as b coalesced K-element rows.
//
// The products are HBM-bound (about 2 flop per byte of matrix per right-hand
// side), so vector FMA is used, not MFMA.  Each output sums its blocks in
// ascending order with explicit FMAs.
#pragma once
#include <type_traits>

#include "kernels.hpp"

namespace mgk {

constexpr int KL = 32;                 // max right-hand sides (lanes per half-wavefront)
constexpr int MROWS = WG / KL;         // block rows (row slots) per workgroup

// Matrix kernels: the 8 half-wavefront slots of a workgroup hold 8 >> qs block rows, each
// cut into Q = 1 << qs slices of its blocks (long rows: the slices of a row are summed in
// slice order at the end); slot s takes slice s % Q of row s / Q, and lane k = lane & 31 is
// the right-hand side.  With Q = 1 a wavefront owns two rows, i0 (lanes 0-31) and i0 + 1
// (lanes 32-63); with Q > 1 both halves of a wavefront hold slices of one row i0.  i0 is
// uniform over the wavefront (the smoother's diagonal blocks arrive through scalar loads
// and each half selects its own).
struct MRow {
  int i0;  // first row of the wavefront (uniform)
  int h;   // 0: row i0, 1: row i0 + 1
  int i;   // i0 + h
  int k;   // right-hand side
  int q;   // slice of the row
};

__device__ __forceinline__ MRow mrow(int lw, int qs = 0) {
  const int slot = threadIdx.x >> 5;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int r0 = lw * (MROWS >> qs);
  MRow m;
  m.i0 = r0 + ((2 * wave) >> qs);
  m.h = qs ? 0 : slot & 1;
  m.i = r0 + (slot >> qs);
  m.q = slot & ((1 << qs) - 1);
  m.k = threadIdx.x & 31;
  return m;
}

// Order in which the workgroups of a product over a structured-grid operator take their
// 8-row blocks.  With the largest block-diagonal offset P (a grid plane: rows i and i +- P
// read the same x rows), the linear order reuses an x row only after about P further rows,
// which for K right-hand sides of FP64 is far more than one XCD's L2 holds, so x would be
// fetched three times.  Instead the rows of every plane are cut into 8 tiles of tb blocks,
// and XCD t takes tile t of plane 0, 1, 2, ... in turn: a row's z-neighbours are read a few
// hundred rows apart.  pb = P / 8 blocks per plane, np planes; tb = 0 keeps the linear
// order.  Only the schedule changes: each row's sums and the per-block dot partials (stored
// by block index) are the same.
struct MSched {
  int pb, tb, np;
};

// Row block of logical workgroup lw (after the XCD remap over the 8 * np * tb workgroups,
// XCD t holds the contiguous range of tile t), or -1 for a slot past a plane's last tile.
__device__ __forceinline__ int msched_block(int lw, const MSched& ms) {
  if (ms.tb == 0) return lw;
  const int per = ms.np * ms.tb;
  const int t = lw / per, rem = lw - t * per;
  const int p = rem / ms.tb, u = rem - p * ms.tb;
  const int q = t * ms.tb + u;
  return q < ms.pb ? p * ms.pb + q : -1;
}

template <int B, class TV, class TA>
__device__ __forceinline__ void load_block(const TV* __restrict__ p, TA* out) {
  if constexpr (sizeof(TV) == 2) {
    const uint16_t* q = reinterpret_cast<const uint16_t*>(p);
#pragma unroll
    for (int e = 0; e < B * B; ++e) out[e] = (TA)bf16_to_f32(q[e]);
  } else {
#pragma unroll
    for (int e = 0; e < B * B; ++e) out[e] = (TA)p[e];
  }
}

template <int BR, int BC, class TV, class TA>
__device__ __forceinline__ void load_rect(const TV* __restrict__ p, TA* out) {
  if constexpr (BR == BC) {
    load_block<BR, TV, TA>(p, out);
  } else {
#pragma unroll
    for (int e = 0; e < BR * BC; ++e) {
      if constexpr (sizeof(TV) == 2)
        out[e] = (TA)bf16_to_f32(reinterpret_cast<const uint16_t*>(p)[e]);
      else
        out[e] = (TA)p[e];
    }
  }
}

// Matrix values and column indices staged in LDS per pass (at most 16 KB of
// values): the workgroup's 8 rows own the contiguous block range
// [ptr[r0], ptr[r0 + 8]), which is copied with coalesced loads, so no lane waits
// on a column index or a block from HBM one block at a time.
template <int BR, int BC, class TV>
constexpr int mstage_cap() { return 16384 / (BR * BC * (int)sizeof(TV)); }

// x rows requested together per step of a lane's walk over its row.
constexpr int MU = 4;

// acc[r] = sum over blocks (i, j) of sum_c A_ij[r][c] X[j*BC + c][k]  (r < BR) for
// row i of the workgroup whose 8 >> qs rows start at r0 (on: the lane has a row and a
// right-hand side; q: its slice of the row).  Every lane of the workgroup must call this
// (it holds barriers).  A slice sums its blocks in ascending order: passes ascend, and
// within a pass the lane walks its slice's blocks in order; steps past the slice's end
// re-read an in-bounds block and are skipped at the FMA.  With qs > 0 the row's 1 << qs
// contiguous slices (slice q: blocks [k0 + len*q/Q, k0 + len*(q+1)/Q)) are then added in
// slice order, and the sum is in the q = 0 lanes.
// SMALL: a stage of at most 128 blocks per pass (at least what the slice sums need), for
// operators whose workgroups own few blocks (prolongators, sliced coarse rows): every lane
// then holds far fewer staging registers, so more wavefronts fit on a CU.
template <int BR, int BC, class TV, class TX, class TA, bool SMALL = false>
__device__ __forceinline__ void block_rows_staged(int r0, int nbr, int i, bool on, int k, int K,
                                                  const int* __restrict__ ptr,
                                                  const int* __restrict__ col,
                                                  const TV* __restrict__ val,
                                                  const TX* __restrict__ X, TA* acc,
                                                  int qs = 0, int q = 0) {
  constexpr int BB = BR * BC;
  typedef typename std::conditional<sizeof(TV) == 2, uint16_t, TV>::type TS;
  constexpr int CAPF = mstage_cap<BR, BC, TV>();
  constexpr int CAPR = (int)((sizeof(TA) * BR * WG + BB * sizeof(TS) - 1) / (BB * sizeof(TS)));
  constexpr int CAPS = CAPF < 128 ? CAPF : (CAPR > 128 ? CAPR : 128);
  constexpr int CAP = SMALL ? CAPS : CAPF;
  __shared__ int s_col[CAP];
  __shared__ alignas(16) TS s_val[CAP * BB];
  static_assert(sizeof(TS) * CAP * BB >= sizeof(TA) * BR * WG, "slice sums fit the stage");
#pragma unroll
  for (int r = 0; r < BR; ++r) acc[r] = 0;
  const TS* gval = reinterpret_cast<const TS*>(val);
  const int c_begin = ptr[r0], c_end = ptr[min(r0 + (MROWS >> qs), nbr)];
  int k0 = on ? ptr[i] : 0, k1 = on ? ptr[i + 1] : 0;
  if (qs) {
    const int len = k1 - k0;
    k1 = k0 + ((len * (q + 1)) >> qs);
    k0 = k0 + ((len * q) >> qs);
  }
  for (int c = c_begin; c < c_end; c += CAP) {
    const int cn = min(CAP, c_end - c);
    // every load of the pass is issued before the first LDS write
    constexpr int NC = (CAP + WG - 1) / WG, NV = (CAP * BB + WG - 1) / WG;
    int tc[NC];
    TS tv[NV];
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const int q = threadIdx.x + u * WG;
      if (q < cn) tc[u] = col[c + q];
    }
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int q = threadIdx.x + u * WG;
      if (q < cn * BB) tv[u] = gval[(size_t)c * BB + q];
    }
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const int q = threadIdx.x + u * WG;
      if (q < cn) s_col[q] = tc[u];
    }
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int q = threadIdx.x + u * WG;
      if (q < cn * BB) s_val[q] = tv[u];
    }
    __syncthreads();
    const int lo = max(k0, c), hi = min(k1, c + cn);
    for (int kb = lo; kb < hi; kb += MU) {
      int q[MU];
      TA xv[MU][BC];
#pragma unroll
      for (int u = 0; u < MU; ++u) {
        q[u] = min(kb + u, hi - 1) - c;
        const int j = s_col[q[u]];
#pragma unroll
        for (int cc = 0; cc < BC; ++cc) xv[u][cc] = (TA)X[((size_t)j * BC + cc) * K + k];
      }
#pragma unroll
      for (int u = 0; u < MU; ++u) {
        TA a[BB];
        load_rect<BR, BC, TV, TA>(reinterpret_cast<const TV*>(s_val + q[u] * BB), a);
        const bool in_row = kb + u < hi;
#pragma unroll
        for (int r = 0; r < BR; ++r) {
          TA t = acc[r];
#pragma unroll
          for (int cc = 0; cc < BC; ++cc) t = fma_(a[r * BC + cc], xv[u][cc], t);
          acc[r] = in_row ? t : acc[r];
        }
      }
    }
    __syncthreads();
  }
  if (qs) {
    // slice q of a row sits 32 q lanes after its slice 0; the stage is free again (the
    // last pass ended with a barrier)
    TA* s_red = reinterpret_cast<TA*>(s_val);
#pragma unroll
    for (int r = 0; r < BR; ++r) s_red[r * WG + threadIdx.x] = acc[r];
    __syncthreads();
    if (q == 0) {
#pragma unroll
      for (int r = 0; r < BR; ++r) {
        TA t = s_red[r * WG + threadIdx.x];
        for (int j = 1; j < (1 << qs); ++j) t += s_red[r * WG + threadIdx.x + j * KL];
        acc[r] = t;
      }
    }
  }
}

// The same product on the diagonal layout (DiaOffs; val holds n_brows x of.k blocks).
// The workgroup's 8 rows own one contiguous range of of.k blocks per row, staged in LDS.
// Every load is issued up front and unconditionally, in this order: the row's stored-slot
// mask, the values, the x rows of all DIA_MAX slots (the column i + o[d] is known without
// reading anything; a slot past the row's count or the matrix edge reads row i's own x),
// then the caller's epilogue operands (pre()).  Memory results return in issue order, so
// the wait that lets the values reach LDS leaves every x and epilogue load in flight.  A
// slot the row does not store is skipped at the FMA, so the row sums its stored blocks in
// ascending column order, as the walk over its BSR row does: the two are bitwise equal.
template <int BR, class TV, class TX, class TA, class Pre>
__device__ __forceinline__ void block_rows_dia(int r0, int nbr, int i, bool on, int k, int K,
                                               const DiaOffs& of, const TV* __restrict__ val,
                                               const TX* __restrict__ X, TA* acc, Pre&& pre) {
  constexpr int BB = BR * BR;
  constexpr int CAP = MROWS * DIA_MAX * BB;
  constexpr int NV = (CAP + WG - 1) / WG;
  typedef typename std::conditional<sizeof(TV) == 2, uint16_t, TV>::type TS;
  // every lane stores all NV of its loads (entries past the range hold copies of entry 0
  // and are never read), so no load is sunk into a branch after the x loads
  __shared__ TS s_val[NV * WG];
  const int kd = of.k;
  const int ic = i < nbr ? i : nbr - 1;
  const int kk = k < K ? k : 0;
  const int nrow = min(MROWS, nbr - r0);
  const int cnt = nrow * kd * BB;
  const TS* g = reinterpret_cast<const TS*>(val) + (size_t)r0 * kd * BB;
  // with no mask every row stores every slot; the byte is then read from the values
  const uint8_t* mp = of.mask ? of.mask + ic : reinterpret_cast<const uint8_t*>(g);
  const unsigned mbyte = *mp;
  TS tv[NV];
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const int q = threadIdx.x + u * WG;
    tv[u] = g[q < cnt ? q : 0];
  }
  __builtin_amdgcn_sched_barrier(0);
  TX xr[DIA_MAX][BR];
#pragma unroll
  for (int d = 0; d < DIA_MAX; ++d) {
    const int j = ic + of.o[d];
    const int jc = (d < kd && j >= 0 && j < nbr) ? j : ic;
#pragma unroll
    for (int c = 0; c < BR; ++c) xr[d][c] = X[((size_t)jc * BR + c) * K + kk];
  }
  pre();
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < NV; ++u) s_val[threadIdx.x + u * WG] = tv[u];
  __syncthreads();
  const unsigned present = of.mask ? mbyte : 0xffu;
#pragma unroll
  for (int r = 0; r < BR; ++r) acc[r] = 0;
  const TS* rowv = s_val + (i - r0 < nrow ? i - r0 : 0) * kd * BB;
#pragma unroll
  for (int d = 0; d < DIA_MAX; ++d) {
    if (d < kd) {
      TA a[BB];
      load_block<BR, TV, TA>(reinterpret_cast<const TV*>(rowv + d * BB), a);
      const bool use = on && ((present >> d) & 1u);
#pragma unroll
      for (int r = 0; r < BR; ++r) {
        TA t = acc[r];
#pragma unroll
        for (int c = 0; c < BR; ++c) t = fma_(a[r * BR + c], (TA)xr[d][c], t);
        acc[r] = use ? t : acc[r];
      }
    }
  }
}

// Row product of a square operator in either layout (DIA: val is the diagonal layout's);
// pre() issues the caller's epilogue loads (first for the BSR walk, whose x loads wait for
// column indices anyway; after the x loads on the diagonal layout).
template <int B, class TV, class TX, class TA, bool DIA, bool SMALL = false, class Pre>
__device__ __forceinline__ void block_rows(int r0, int nbr, int i, bool on, int k, int K,
                                           const int* __restrict__ ptr,
                                           const int* __restrict__ col,
                                           const TV* __restrict__ val, const DiaOffs& of,
                                           const TX* __restrict__ X, TA* acc, Pre&& pre,
                                           int qs = 0, int q = 0) {
  if constexpr (DIA) {
    block_rows_dia<B, TV, TX, TA>(r0, nbr, i, on, k, K, of, val, X, acc, pre);
  } else {
    pre();
    block_rows_staged<B, B, TV, TX, TA, SMALL>(r0, nbr, i, on, k, K, ptr, col, val, X, acc, qs,
                                               q);
  }
}

// The lane's B entries p[(i*B + r)*K + k] (r < B) of an [n][K] operand, loaded ahead of
// the row product by every lane (a lane past the last row or right-hand side reads the
// last row's or column 0's entries: no branch and no constant address, so no wait for
// these loads is put before the product's loads).
template <int B, class T>
__device__ __forceinline__ void load_rows_ahead(const T* __restrict__ p, int nbr, int i, int k,
                                                int K, T (&out)[B]) {
  const int ic = i < nbr ? i : nbr - 1;
  const int kk = k < K ? k : 0;
#pragma unroll
  for (int r = 0; r < B; ++r) out[r] = p[((size_t)ic * B + r) * K + kk];
}

// Block M_i of a block-diagonal matrix for the lane's row, both rows' blocks
// fetched through scalar loads.
template <int B, class TM, class TA>
__device__ __forceinline__ void diag_block(const MRow& m, bool has_b, const TM* __restrict__ M,
                                           TA* out) {
  TA va[B * B], vb[B * B];
  load_block<B, TM, TA>(M + (size_t)m.i0 * B * B, va);
  load_block<B, TM, TA>(M + (size_t)(has_b ? m.i0 + 1 : m.i0) * B * B, vb);
#pragma unroll
  for (int e = 0; e < B * B; ++e) out[e] = m.h ? vb[e] : va[e];
}

// Y = alpha A X + beta Y.
template <int BR, int BC, class TV, class TX, class TY, class TA, bool SMALL>
__global__ __launch_bounds__(WG) void k_spmm(int nbr, int K, const int* __restrict__ ptr,
                                             const int* __restrict__ col,
                                             const TV* __restrict__ val,
                                             const TX* __restrict__ X, TY* __restrict__ Y,
                                             TA alpha, TA beta, int qs) {
  const int lw = xcd_remap(blockIdx.x, gridDim.x);
  const MRow m = mrow(lw, qs);
  const int i = m.i, k = m.k;
  const bool on = i < nbr && k < K;
  TY yr[BR];
  if (beta != TA(0)) load_rows_ahead<BR>(Y, nbr, i, k, K, yr);
  TA acc[BR];
  block_rows_staged<BR, BC, TV, TX, TA, SMALL>(lw * (MROWS >> qs), nbr, i, on, k, K, ptr, col,
                                               val, X, acc, qs, m.q);
  if (!on || m.q) return;
#pragma unroll
  for (int r = 0; r < BR; ++r) {
    const size_t e = ((size_t)i * BR + r) * K + k;
    TA out = alpha * acc[r];
    if (beta != TA(0)) out = fma_(beta, (TA)yr[r], out);
    Y[e] = (TY)out;
  }
}

// Restriction fused with the coarse level's pre-smoothing from a zero guess: Y = A X and
// Z = M Y, M holding one BR x BR smoother block per block row of Y.  The lane that writes
// column k of a block row holds all BR of its outputs; it multiplies them (rounded to TY, as
// stored in Y) by the row's M block in the order of k_block_diag_m, so Z is bitwise the
// same as that two-kernel sequence.
template <int BR, int BC, class TV, class TX, class TY, class TA, class TM, bool SMALL>
__global__ __launch_bounds__(WG) void k_spmm_bd(int nbr, int K, const int* __restrict__ ptr,
                                                const int* __restrict__ col,
                                                const TV* __restrict__ val,
                                                const TX* __restrict__ X, TY* __restrict__ Y,
                                                const TM* __restrict__ M, TY* __restrict__ Z,
                                                int qs) {
  const int lw = xcd_remap(blockIdx.x, gridDim.x);
  const MRow m = mrow(lw, qs);
  const int i = m.i, k = m.k;
  const bool on = i < nbr && k < K;
  TA acc[BR];
  block_rows_staged<BR, BC, TV, TX, TA, SMALL>(lw * (MROWS >> qs), nbr, i, on, k, K, ptr, col,
                                               val, X, acc, qs, m.q);
  if (!on || m.q) return;
  TA mb[BR * BR];
  load_block<BR, TM, TA>(M + (size_t)i * BR * BR, mb);
  TA y[BR];
#pragma unroll
  for (int r = 0; r < BR; ++r) {
    const TY yo = (TY)acc[r];
    Y[((size_t)i * BR + r) * K + k] = yo;
    y[r] = (TA)yo;
  }
#pragma unroll
  for (int r = 0; r < BR; ++r) {
    TA out = 0;
#pragma unroll
    for (int c = 0; c < BR; ++c) out = fma_(mb[r * BR + c], y[c], out);
    Z[((size_t)i * BR + r) * K + k] = (TY)out;
  }
}

// Y = A X (FP64) with per-column partials of <W1_k, Y_k> and (two) <Y_k, Y_k>:
// part[w * KL + k] and part[(G + w) * KL + k] for row block w of G = ceil(nbr / 8) (the
// block's 8 rows summed in order).
template <int B, bool DIA>
__global__ __launch_bounds__(WG) void k_spmm_dot(int nbr, int K, const int* __restrict__ ptr,
                                                 const int* __restrict__ col,
                                                 const double* __restrict__ val,
                                                 const double* __restrict__ X,
                                                 double* __restrict__ Y, int two,
                                                 const double* __restrict__ W1,
                                                 double* __restrict__ part, DiaOffs of,
                                                 MSched ms) {
  const int lw = msched_block(xcd_remap(blockIdx.x, gridDim.x), ms);
  if (lw < 0 || lw * MROWS >= nbr) return;
  const int G = (nbr + MROWS - 1) / MROWS;
  const MRow m = mrow(lw);
  const bool on = m.i < nbr && m.k < K;
  double d1 = 0.0, d2 = 0.0;
  double w[B];
  double acc[B];
  block_rows<B, double, double, double, DIA>(lw * MROWS, nbr, m.i, on, m.k, K, ptr, col, val,
                                             of, X, acc,
                                             [&] { load_rows_ahead<B>(W1, nbr, m.i, m.k, K, w); });
  if (on) {
#pragma unroll
    for (int r = 0; r < B; ++r) {
      const size_t e = ((size_t)m.i * B + r) * K + m.k;
      Y[e] = acc[r];
      d1 = fma_(w[r], acc[r], d1);
      d2 = fma_(acc[r], acc[r], d2);
    }
  }
  // lane (w, h, k) holds row lw * 8 + 2 w + h = lw * 8 + threadIdx.x / 32
  __shared__ double sa[WG], sb[WG];
  sa[threadIdx.x] = d1;
  sb[threadIdx.x] = d2;
  __syncthreads();
  if (threadIdx.x < KL) {
    double x = 0.0, y = 0.0;
    for (int q = 0; q < MROWS; ++q) {
      x += sa[q * KL + threadIdx.x];
      y += sb[q * KL + threadIdx.x];
    }
    part[(size_t)lw * KL + threadIdx.x] = x;
    if (two) part[(size_t)(G + lw) * KL + threadIdx.x] = y;
  }
}

// First reduction stage for per-column partials: workgroup b sums partial rows
// [b*128, (b+1)*128) of one or two arrays of `count` rows (32 lanes per column,
// 8 row slots each summing 16 rows in ascending order with every load issued first,
// then the 8 slots in order).
constexpr int MRED_CHUNK = 128;

static __global__ __launch_bounds__(WG) void k_reduce_stage_m(const double* __restrict__ part, int count,
                                                       int two, double* __restrict__ out) {
  constexpr int PER = MRED_CHUNK / MROWS;
  const int k = threadIdx.x % KL, q0 = threadIdx.x / KL;
  const int b0 = blockIdx.x * MRED_CHUNK;
  double va[PER], vc[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = b0 + q0 + u * MROWS;
    va[u] = q < count ? part[(size_t)q * KL + k] : 0.0;
    vc[u] = (two && q < count) ? part[(size_t)(count + q) * KL + k] : 0.0;
  }
  double a = 0.0, c = 0.0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    if (b0 + q0 + u * MROWS < count) {
      a += va[u];
      c += vc[u];
    }
  }
  __shared__ double sa[WG], sb[WG];
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x < KL) {
    double x = 0.0, y = 0.0;
    for (int q = 0; q < MROWS; ++q) {
      x += sa[q * KL + threadIdx.x];
      y += sb[q * KL + threadIdx.x];
    }
    out[(size_t)blockIdx.x * KL + threadIdx.x] = x;
    if (two) out[(size_t)(gridDim.x + blockIdx.x) * KL + threadIdx.x] = y;
  }
}

// T = F - A Z.
template <int B, class TV, class TX, class TF, class TA, bool DIA, bool SMALL = false>
__global__ __launch_bounds__(WG) void k_residual_m(int nbr, int K, const int* __restrict__ ptr,
                                                   const int* __restrict__ col,
                                                   const TV* __restrict__ val,
                                                   const TF* __restrict__ F,
                                                   const TX* __restrict__ Z,
                                                   TX* __restrict__ T, DiaOffs of, MSched ms,
                                                   int qs) {
  const int lw = msched_block(xcd_remap(blockIdx.x, gridDim.x), ms);
  if (lw < 0 || lw * (MROWS >> qs) >= nbr) return;
  const MRow m = mrow(lw, qs);
  const int i = m.i, k = m.k;
  const bool on = i < nbr && k < K;
  TF fr[B];
  TA acc[B];
  block_rows<B, TV, TX, TA, DIA, SMALL>(lw * (MROWS >> qs), nbr, i, on, k, K, ptr, col, val, of,
                                        Z, acc, [&] { load_rows_ahead<B>(F, nbr, i, k, K, fr); },
                                        qs, m.q);
  if (!on || m.q) return;
#pragma unroll
  for (int r = 0; r < B; ++r) {
    const size_t e = ((size_t)i * B + r) * K + k;
    T[e] = (TX)((TA)fr[r] - acc[r]);
  }
}

// Zout = Z + M (F - A Z), M block diagonal.
template <int B, class TV, class TX, class TF, class TO, class TM, class TA, bool DIA,
          bool SMALL = false>
__global__ __launch_bounds__(WG) void k_smooth_m(int nbr, int K, const int* __restrict__ ptr,
                                                 const int* __restrict__ col,
                                                 const TV* __restrict__ val,
                                                 const TM* __restrict__ M,
                                                 const TF* __restrict__ F,
                                                 const TX* __restrict__ Z,
                                                 TO* __restrict__ Zout, DiaOffs of, MSched ms,
                                                 int qs) {
  const int lw = msched_block(xcd_remap(blockIdx.x, gridDim.x), ms);
  if (lw < 0 || lw * (MROWS >> qs) >= nbr) return;
  const MRow m = mrow(lw, qs);
  const int i = m.i, k = m.k;
  const bool on = i < nbr && k < K;
  TF fr[B];
  TX zr[B];
  // M blocks (scalar loads) ahead of the product too; a wavefront whose rows lie past nbr
  // reads row 0's
  MRow mc = m;
  if (mc.i0 >= nbr) mc.i0 = 0;
  TA mb[B * B];
  diag_block<B, TM, TA>(mc, mc.i0 + 1 < nbr, M, mb);
  TA acc[B];
  block_rows<B, TV, TX, TA, DIA, SMALL>(
      lw * (MROWS >> qs), nbr, i, on, k, K, ptr, col, val, of, Z, acc,
      [&] {
        load_rows_ahead<B>(F, nbr, i, k, K, fr);
        load_rows_ahead<B>(Z, nbr, i, k, K, zr);
      },
      qs, m.q);
  if (!on || m.q) return;
  TA res[B];
#pragma unroll
  for (int r = 0; r < B; ++r) res[r] = (TA)fr[r] - acc[r];
#pragma unroll
  for (int r = 0; r < B; ++r) {
    const size_t e = ((size_t)i * B + r) * K + k;
    TA out = (TA)zr[r];
#pragma unroll
    for (int c = 0; c < B; ++c) out = fma_(mb[r * B + c], res[c], out);
    Zout[e] = (TO)out;
  }
}

// Z = M F.
template <int B, class TM, class TF, class TX, class TA>
__global__ __launch_bounds__(WG) void k_block_diag_m(int nbr, int K, const TM* __restrict__ M,
                                                     const TF* __restrict__ F,
                                                     TX* __restrict__ Z) {
  const MRow m = mrow(blockIdx.x);
  if (m.i0 >= nbr) return;
  TA mb[B * B];
  diag_block<B, TM, TA>(m, m.i0 + 1 < nbr, M, mb);
  const int i = m.i, k = m.k;
  if (i >= nbr || k >= K) return;
  TA f[B];
#pragma unroll
  for (int c = 0; c < B; ++c) f[c] = (TA)F[((size_t)i * B + c) * K + k];
#pragma unroll
  for (int r = 0; r < B; ++r) {
    TA acc = 0;
#pragma unroll
    for (int c = 0; c < B; ++c) acc = fma_(mb[r * B + c], f[c], acc);
    Z[((size_t)i * B + r) * K + k] = (TX)acc;
  }
}

// Z = Cinv R for the dense FP64 coarsest inverse (n x n), R and Z [n][K]: one
// workgroup per row i of Z.  Half-wavefront q of 8 takes the contiguous slice
// [q c, (q + 1) c) of the row (c = ceil(n / 8)) and sums it in ascending order for
// right-hand side k = lane & 31, eight entries' loads issued per step; the 8 slice
// sums are then added in slice order.
template <class TI, class TO>
__global__ __launch_bounds__(WG) void k_coarse_gemm(int n, int K, const double* __restrict__ Cinv,
                                                    const TI* __restrict__ R,
                                                    TO* __restrict__ Z) {
  constexpr int U = 8;
  const int i = blockIdx.x;
  const int k = threadIdx.x % KL, q = threadIdx.x / KL;
  const int kk = k < K ? k : 0;
  const int c = (n + MROWS - 1) / MROWS;
  const int j0 = min(n, q * c), j1 = min(n, j0 + c);
  const double* a = Cinv + (size_t)i * n;
  double acc = 0.0;
  int j = j0;
  for (; j + U <= j1; j += U) {
    double av[U], rv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      av[u] = a[j + u];
      rv[u] = (double)R[(size_t)(j + u) * K + kk];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc = fma_(av[u], rv[u], acc);
  }
  for (; j < j1; ++j) acc = fma_(a[j], (double)R[(size_t)j * K + kk], acc);
  __shared__ double sq[WG];
  sq[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < KL && k < K) {
    double z = 0.0;
    for (int t = 0; t < MROWS; ++t) z += sq[t * KL + threadIdx.x];
    Z[(size_t)i * K + k] = (TO)z;
  }
}

// ---- per-column Krylov kernels (FP64) ----------------------------------------
//
// Per-column scalars live in scm[idx * KL + k].  A thread handles column
// k = tid % 32 of rows tid / 32, tid / 32 + 8, ... of its grid-stride range; the
// per-column partials of a workgroup are combined over its 8 row slots in LDS
// in a fixed order.

enum ScM { SM_RHO = 0, SM_RHO1, SM_ALPHA, SM_OMEGA, SM_RV, SM_SS, SM_TS, SM_TT, SM_RR, SM_NB,
           SM_COUNT };

#define MROW_STRIDE(row, n) \
  for (size_t row = (size_t)blockIdx.x * MROWS + threadIdx.x / KL; row < (size_t)(n); \
       row += (size_t)gridDim.x * MROWS)

__device__ __forceinline__ void col_sum2(double a, double b, int two, double* __restrict__ part,
                                         int slot, int nslots) {
  __shared__ double sa[WG], sb[WG];
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  if (threadIdx.x < KL) {
    double x = 0.0, y = 0.0;
    for (int q = 0; q < MROWS; ++q) {
      x += sa[q * KL + threadIdx.x];
      y += sb[q * KL + threadIdx.x];
    }
    part[(size_t)slot * KL + threadIdx.x] = x;
    if (two) part[(size_t)(nslots + slot) * KL + threadIdx.x] = y;
  }
}

// Per-column <A_k, B_k> and (optionally) <C_k, D_k> partials.
static __global__ __launch_bounds__(WG) void k_dot_m(size_t n, int K, const double* __restrict__ A,
                                              const double* __restrict__ Bv,
                                              const double* __restrict__ C,
                                              const double* __restrict__ D,
                                              double* __restrict__ part) {
  const int k = threadIdx.x % KL;
  double s1 = 0.0, s2 = 0.0;
  if (k < K) {
    MROW_STRIDE(row, n) {
      const size_t e = row * K + k;
      s1 = fma_(A[e], Bv[e], s1);
      if (C) s2 = fma_(C[e], D[e], s2);
    }
  }
  col_sum2(s1, s2, C != nullptr, part, blockIdx.x, gridDim.x);
}

enum FinM { FINM_STORE1 = 0, FINM_STORE2, FINM_ALPHA, FINM_OMEGA, FINM_RHO };

static __global__ __launch_bounds__(WG) void k_finalize_m(const double* __restrict__ part, int count,
                                                   int two, int op, int i0, int i1, int K,
                                                   const int* __restrict__ active,
                                                   double* __restrict__ scm) {
  // one workgroup per column: strided partial sums, then the fixed workgroup tree
  const int k = blockIdx.x;
  if (k >= K) return;
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < count; q += WG) {
    a += part[(size_t)q * KL + k];
    if (two) b += part[(size_t)(count + q) * KL + k];
  }
  wg_sum2(a, b);
  if (threadIdx.x != 0) return;
  if (!active[k] && op != FINM_STORE1 && op != FINM_STORE2) return;
  double* s = scm;
  switch (op) {
    case FINM_STORE1: s[i0 * KL + k] = a; break;
    case FINM_STORE2: s[i0 * KL + k] = a; s[i1 * KL + k] = b; break;
    case FINM_ALPHA: s[SM_RV * KL + k] = a; s[SM_ALPHA * KL + k] = s[SM_RHO1 * KL + k] / a; break;
    case FINM_OMEGA:
      s[SM_TS * KL + k] = a;
      s[SM_TT * KL + k] = b;
      s[SM_OMEGA * KL + k] = b != 0.0 ? a / b : 0.0;
      break;
    case FINM_RHO:
      s[SM_RR * KL + k] = a;
      s[SM_RHO * KL + k] = s[SM_RHO1 * KL + k];
      s[SM_RHO1 * KL + k] = b;
      break;
  }
}

// p = r + beta (p - omega v) for active columns.
static __global__ __launch_bounds__(WG) void k_bicg_p_m(size_t n, int K, const int* __restrict__ active,
                                                 const double* __restrict__ scm,
                                                 const double* __restrict__ r,
                                                 const double* __restrict__ v,
                                                 double* __restrict__ p) {
  const int k = threadIdx.x % KL;
  if (k >= K || !active[k]) return;
  const double beta = (scm[SM_RHO1 * KL + k] / scm[SM_RHO * KL + k]) *
                      (scm[SM_ALPHA * KL + k] / scm[SM_OMEGA * KL + k]);
  const double om = scm[SM_OMEGA * KL + k];
  MROW_STRIDE(row, n) {
    const size_t e = row * K + k;
    p[e] = r[e] + beta * (p[e] - om * v[e]);
  }
}

// s = r - alpha v (active columns); partials of ||s||^2.  (x += alpha phat is deferred to
// k_bicg_xr_m, or to k_bicg_x_m for the columns that stop at s.)
static __global__ __launch_bounds__(WG) void k_bicg_s_m(size_t n, int K, const int* __restrict__ active,
                                                 const double* __restrict__ scm,
                                                 const double* __restrict__ r,
                                                 const double* __restrict__ v,
                                                 double* __restrict__ s,
                                                 double* __restrict__ part) {
  const int k = threadIdx.x % KL;
  double ss = 0.0;
  if (k < K && active[k]) {
    const double al = scm[SM_ALPHA * KL + k];
    MROW_STRIDE(row, n) {
      const size_t e = row * K + k;
      const double si = r[e] - al * v[e];
      s[e] = si;
      ss = fma_(si, si, ss);
    }
  }
  col_sum2(ss, 0.0, 0, part, blockIdx.x, gridDim.x);
}

// x += alpha phat for the columns flagged in mask (they stopped at s).
static __global__ __launch_bounds__(WG) void k_bicg_x_m(size_t n, int K, const int* __restrict__ mask,
                                                 const double* __restrict__ scm,
                                                 const double* __restrict__ ph,
                                                 double* __restrict__ x) {
  const int k = threadIdx.x % KL;
  if (k >= K || !mask[k]) return;
  const double al = scm[SM_ALPHA * KL + k];
  MROW_STRIDE(row, n) {
    const size_t e = row * K + k;
    x[e] += al * ph[e];
  }
}

// x = (x + alpha phat) + omega shat; r = s - omega t; partials of ||r||^2 and (rhat, r).
// One pass over x per iteration, with the two additions in the order of the two updates.
static __global__ __launch_bounds__(WG) void k_bicg_xr_m(size_t n, int K, const int* __restrict__ active,
                                                  const double* __restrict__ scm,
                                                  const double* __restrict__ s,
                                                  const double* __restrict__ t,
                                                  const double* __restrict__ ph,
                                                  const double* __restrict__ sh,
                                                  const double* __restrict__ rh,
                                                  double* __restrict__ x, double* __restrict__ r,
                                                  double* __restrict__ part) {
  const int k = threadIdx.x % KL;
  double rr = 0.0, rho = 0.0;
  if (k < K && active[k]) {
    const double al = scm[SM_ALPHA * KL + k], om = scm[SM_OMEGA * KL + k];
    MROW_STRIDE(row, n) {
      const size_t e = row * K + k;
      x[e] = (x[e] + al * ph[e]) + om * sh[e];
      const double ri = s[e] - om * t[e];
      r[e] = ri;
      rr = fma_(ri, ri, rr);
      rho = fma_(rh[e], ri, rho);
    }
  }
  col_sum2(rr, rho, 1, part, blockIdx.x, gridDim.x);
}

// Restart the columns flagged in mask: rhat = r, p = v = 0 (scalars set by the host).
static __global__ __launch_bounds__(WG) void k_restart_m(size_t n, int K, const int* __restrict__ mask,
                                                  const double* __restrict__ r,
                                                  double* __restrict__ rh, double* __restrict__ p,
                                                  double* __restrict__ v) {
  const int k = threadIdx.x % KL;
  if (k >= K || !mask[k]) return;
  MROW_STRIDE(row, n) {
    const size_t e = row * K + k;
    rh[e] = r[e];
    p[e] = 0.0;
    v[e] = 0.0;
  }
}

}  // namespace mgk
