// Grouped (work-list) kernels for several independent systems of uneven size.
//
// One launch processes one stage of the solve (a smoother, a residual, a
// transfer, a coarse solve or a Krylov vector update) for every system that
// takes part in it.  The stage's work list is an array of items (one per
// system: its operator, vectors and first tile in the launch's tile space);
// a persistent grid of workgroups walks the tile space with a grid stride and
// each tile finds its item by a scan of the (few) item starts.  Tiles of a
// system whose iteration has stopped are skipped.  Row products use the same
// block-row engine and summation order as the single-system kernels, so a
// system gives the same result alone or in a batch.
#pragma once
#include "kernels.hpp"

namespace mgk {

struct GItem {
  const int* ptr;
  const int* col;
  const void* val;
  const void* M;      // smoother blocks, or the coarse inverse (double)
  const void* in;     // x of y = A x, z of t = f - A z, f of z = M f, r of the coarse solve
  const void* f;      // right-hand side of residual / smoother
  void* out;          // y, t, z or z_out
  int nbr;            // block rows (coarse: scalar rows)
  int tile0;          // first tile of this item
  int sys;            // system index
  int pad;
  DiaOffs dia;        // diagonal layout of a square operator (val then holds its blocks)
};

__device__ __forceinline__ int find_item(const GItem* __restrict__ items, int nitems, int w) {
  int it = 0;
  for (int q = 1; q < nitems; ++q)
    if (items[q].tile0 <= w) it = q;
  return it;
}

// A pointer read from memory is a generic (flat) address to the compiler, and flat loads
// count against both the vector-memory and the scalar-memory counters, so every wait for a
// scalar load would also wait for them.  The item lists are written by the host before the
// launch and only read by the kernels, so they are read through the constant address
// space: the pointers read from it are known to be global, and their loads are global ones.
#define MGK_CONST const __attribute__((address_space(4)))

// The item of tile w, copied member by member through the constant address space.
__device__ __forceinline__ GItem item_of(const GItem* __restrict__ items, int nitems, int w) {
  MGK_CONST GItem* q = (MGK_CONST GItem*)items + find_item(items, nitems, w);
  GItem g;
  g.ptr = q->ptr;
  g.col = q->col;
  g.val = q->val;
  g.M = q->M;
  g.in = q->in;
  g.f = q->f;
  g.out = q->out;
  g.nbr = q->nbr;
  g.tile0 = q->tile0;
  g.sys = q->sys;
  g.pad = 0;
  g.dia.k = q->dia.k;
#pragma unroll
  for (int d = 0; d < DIA_MAX; ++d) g.dia.o[d] = q->dia.o[d];
  g.dia.mask = q->dia.mask;
  return g;
}

// Tile walk of a grouped launch.  gridDim.x >= total: one tile per workgroup,
// remapped so that each XCD takes one contiguous range of tiles; gridDim.x <
// total: a persistent grid striding through the tile space.
#define GROUP_TILES(w, total)                                                         \
  for (int w = (int)gridDim.x >= (total) ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x; \
       w < (total); w += (int)gridDim.x)

// Row product of item g for lane L, in the diagonal layout when DIA (every item of the
// launch then has one); the row range is loaded first, as in the single-system kernels.
template <int BR, int BC, int S, int U, class TV, class TX, class TA, bool CACHED, bool DIA,
          class Pre>
__device__ __forceinline__ TA g_row_product(const LaneInfo& L, const GItem& g, const TX* x,
                                            Pre&& pre) {
  const RowRange rr = row_range<DIA>(g.ptr, g.dia, L.i, g.nbr);
  __builtin_amdgcn_sched_barrier(0);
  pre();
  TA acc[1];
  row_product_r<BR, BC, S, U, false, TV, TX, TA, 1, CACHED, DIA, const TX*, true>(
      L, g.nbr, g.ptr, g.col, nullptr, (const TV*)g.val, x, acc, g.dia, rr);
  return acc[0];
}

// y = A x + beta y
template <int BR, int BC, int S, int U, class TV, class TX, class TY, class TA,
          bool CACHED = false, bool DIA = false>
__global__ __launch_bounds__(WG) void k_g_spmv(const GItem* __restrict__ items, int nitems,
                                               int total, const int* __restrict__ active,
                                               TA beta) {
  GROUP_TILES(w, total) {
    const GItem g = item_of(items, nitems, w);
    if (!active[g.sys]) continue;
    const LaneInfo L = lane_info<BR, S>(w - g.tile0);
    const bool own = L.active && L.s == 0 && L.i < g.nbr;
    const size_t row = (size_t)L.i * BR + L.r;
    TY* y = (TY*)g.out;
    TY yr[1];
    const TA acc = g_row_product<BR, BC, S, U, TV, TX, TA, CACHED, DIA>(
        L, g, (const TX*)g.in, [&] {
          if (beta != TA(0)) load_ahead<1>(y, row, own, yr);
        });
    if (own) {
      TA out = acc;
      if (beta != TA(0)) out = fma_(beta, (TA)yr[0], out);
      y[row] = (TY)out;
    }
  }
}

// t = f - A z
template <int B, int S, int U, class TV, class TX, class TF, class TA, bool CACHED = false,
          bool DIA = false>
__global__ __launch_bounds__(WG) void k_g_residual(const GItem* __restrict__ items, int nitems,
                                                   int total, const int* __restrict__ active) {
  GROUP_TILES(w, total) {
    const GItem g = item_of(items, nitems, w);
    if (!active[g.sys]) continue;
    const LaneInfo L = lane_info<B, S>(w - g.tile0);
    const bool own = L.active && L.s == 0 && L.i < g.nbr;
    const size_t row = (size_t)L.i * B + L.r;
    TF fr[1];   // ahead of the row product
    const TA acc = g_row_product<B, B, S, U, TV, TX, TA, CACHED, DIA>(
        L, g, (const TX*)g.in, [&] { load_ahead<1>((const TF*)g.f, row, own, fr); });
    if (own) ((TX*)g.out)[row] = (TX)((TA)fr[0] - acc);
  }
}

// z_out = z + M (f - A z)
template <int B, int S, int U, class TV, class TX, class TF, class TO, class TM, class TA,
          bool CACHED = false, bool DIA = false>
__global__ __launch_bounds__(WG) void k_g_smooth(const GItem* __restrict__ items, int nitems,
                                                 int total, const int* __restrict__ active) {
  GROUP_TILES(w, total) {
    const GItem g = item_of(items, nitems, w);
    if (!active[g.sys]) continue;   // uniform per workgroup: the whole tile skips
    const LaneInfo L = lane_info<B, S>(w - g.tile0);
    const TX* z = (const TX*)g.in;
    const bool own = L.active && L.s == 0 && L.i < g.nbr;
    const size_t row = (size_t)L.i * B + L.r;
    // f, z and the row of M are loaded ahead of the row product
    TF fr[1];
    TX zr[1];
    TM mr[B];
    const TA acc = g_row_product<B, B, S, U, TV, TX, TA, CACHED, DIA>(L, g, z, [&] {
      load_ahead<1>((const TF*)g.f, row, own, fr);
      load_ahead<1>(z, row, own, zr);
      load_ahead<B>((const TM*)g.M, ((size_t)L.i * B + L.r) * B, own, mr);
    });
    const TA res = own ? (TA)fr[0] - acc : TA(0);
    const TA zv = (TA)zr[0];
    TA mv[B];
#pragma unroll
    for (int c = 0; c < B; ++c) mv[c] = to_acc<TA>(mr[c]);
    TA rv[B];
#pragma unroll
    for (int c = 0; c < B; ++c) rv[c] = __shfl(res, L.gbase + c, WAVE);
    if (own) {
      TA out = zv;
#pragma unroll
      for (int c = 0; c < B; ++c) out = fma_(mv[c], rv[c], out);
      ((TO*)g.out)[row] = (TO)out;
    }
  }
}

// z = M f, one tile = WG scalar rows
template <int B, class TM, class TF, class TX, class TA>
__global__ __launch_bounds__(WG) void k_g_block_diag(const GItem* __restrict__ items, int nitems,
                                                     int total, const int* __restrict__ active) {
  GROUP_TILES(w, total) {
    const GItem g = item_of(items, nitems, w);
    if (!active[g.sys]) continue;
    const size_t row = (size_t)(w - g.tile0) * WG + threadIdx.x;
    if (row >= (size_t)g.nbr * B) continue;
    const size_t i = row / B;
    const int r = (int)(row - i * B);
    const TM* m = (const TM*)g.M + i * B * B;
    TA fv[B], mv[B];
    load_x<B, TF, TA>((const TF*)g.in + i * B, fv);
    if constexpr (B == 4) {
      load_vals<B, TM, TA, true>(m + r * B, mv);
    } else {
#pragma unroll
      for (int c = 0; c < B; ++c) mv[c] = to_acc<TA>(m[r * B + c]);
    }
    TA acc = 0;
#pragma unroll
    for (int c = 0; c < B; ++c) acc = fma_(mv[c], fv[c], acc);
    ((TX*)g.out)[row] = (TX)acc;
  }
}

// coarse z = Cinv r: one tile = one row of one system's dense inverse
template <class TI, class TO>
__global__ __launch_bounds__(WG) void k_g_coarse(const GItem* __restrict__ items, int nitems,
                                                 int total, const int* __restrict__ active) {
  GROUP_TILES(w, total) {
    const GItem g = item_of(items, nitems, w);
    const int i = w - g.tile0;
    double s = 0.0, dummy = 0.0;
    const bool on = active[g.sys] != 0;   // uniform per workgroup
    if (on) {
      const double* a = (const double*)g.M + (size_t)i * g.nbr;
      const TI* r = (const TI*)g.in;
      for (int j = threadIdx.x; j < g.nbr; j += WG) s = fma_(a[j], (double)r[j], s);
    }
    wg_sum2(s, dummy);
    if (on && threadIdx.x == 0) ((TO*)g.out)[i] = (TO)s;
    __syncthreads();
  }
}

// ---- grouped FP64 Krylov vector kernels --------------------------------------

constexpr int VTILE = 16 * WG;   // elements per vector tile

struct GVec {
  double* a[7];
  long long n;
  int tile0, ntiles, sys, pad;
};

__device__ __forceinline__ int find_vec(const GVec* __restrict__ v, int nv, int w) {
  int it = 0;
  for (int q = 1; q < nv; ++q)
    if (v[q].tile0 <= w) it = q;
  return it;
}

enum GVOp {
  GV_DOT = 0,    // part = <a0, a1>, part2 = <a2, a3> (a2 may be null)
  GV_P = 1,      // a2 (p) = a0 (r) + beta (p - omega a1 (v))
  GV_S = 2,      // a3 (s) = a0 (r) - alpha a1 (v); part = ||s||^2
  GV_XR = 3,     // a4 (x) = (x + alpha a6 (ph)) + omega a2 (sh); a5 (r) = a0 (s) - omega a1 (t);
                 // part = ||r||^2, part2 = (a3 rh, r): one pass over x per iteration, the
                 // two additions in the order of the two updates
  GV_COPY = 4,   // a1 = a0
  GV_ZERO = 5,   // a0 = 0
  GV_X = 6       // a4 (x) += alpha a2 (ph) (the iteration stopped at s)
};

__global__ __launch_bounds__(WG) void k_g_vec(const GVec* __restrict__ vs, int nv, int total,
                                              int op, const int* __restrict__ active,
                                              const double* __restrict__ scb,
                                              double* __restrict__ part) {
  GROUP_TILES(w, total) {
    MGK_CONST GVec* vq = (MGK_CONST GVec*)vs + find_vec(vs, nv, w);
    GVec v;
#pragma unroll
    for (int q = 0; q < 7; ++q) v.a[q] = vq->a[q];
    v.n = vq->n;
    v.tile0 = vq->tile0;
    v.sys = vq->sys;
    double d1 = 0.0, d2 = 0.0;
    const bool on = active[v.sys] != 0;
    if (on) {
      const double* sc = scb + (size_t)v.sys * SC_COUNT;
      const long long e0 = (long long)(w - v.tile0) * VTILE;
      const long long e1 = e0 + VTILE < v.n ? e0 + VTILE : v.n;
      if (op == GV_DOT) {
        for (long long e = e0 + threadIdx.x; e < e1; e += WG) {
          d1 = fma_(v.a[0][e], v.a[1][e], d1);
          if (v.a[2]) d2 = fma_(v.a[2][e], v.a[3][e], d2);
        }
      } else if (op == GV_P) {
        const double beta = (sc[SC_RHO1] / sc[SC_RHO]) * (sc[SC_ALPHA] / sc[SC_OMEGA]);
        const double om = sc[SC_OMEGA];
        for (long long e = e0 + threadIdx.x; e < e1; e += WG)
          v.a[2][e] = v.a[0][e] + beta * (v.a[2][e] - om * v.a[1][e]);
      } else if (op == GV_S) {
        const double al = sc[SC_ALPHA];
        for (long long e = e0 + threadIdx.x; e < e1; e += WG) {
          const double si = v.a[0][e] - al * v.a[1][e];
          v.a[3][e] = si;
          d1 = fma_(si, si, d1);
        }
      } else if (op == GV_X) {
        const double al = sc[SC_ALPHA];
        for (long long e = e0 + threadIdx.x; e < e1; e += WG) v.a[4][e] += al * v.a[2][e];
      } else if (op == GV_XR) {
        const double al = sc[SC_ALPHA], om = sc[SC_OMEGA];
        for (long long e = e0 + threadIdx.x; e < e1; e += WG) {
          v.a[4][e] = (v.a[4][e] + al * v.a[6][e]) + om * v.a[2][e];
          const double ri = v.a[0][e] - om * v.a[1][e];
          v.a[5][e] = ri;
          d1 = fma_(ri, ri, d1);
          d2 = fma_(v.a[3][e], ri, d2);
        }
      } else if (op == GV_COPY) {
        for (long long e = e0 + threadIdx.x; e < e1; e += WG) v.a[1][e] = v.a[0][e];
      } else {
        for (long long e = e0 + threadIdx.x; e < e1; e += WG) v.a[0][e] = 0.0;
      }
    }
    if (part) {
      wg_sum2(d1, d2);
      if (threadIdx.x == 0) {
        part[w] = d1;
        part[total + w] = d2;
      }
      __syncthreads();
    }
  }
}

enum GFin { GF_STORE1 = 0, GF_STORE2, GF_ALPHA, GF_OMEGA, GF_RHO };

// Per-system sums of the partials of tiles [tile0, tile0 + ntiles) of one or two
// partial arrays (each `total` long), in a fixed order; launched with one
// workgroup per system; partial source of GF_ALPHA /
// GF_OMEGA is the dot launch over (rhat, v) / (t, s), (t, t).
__global__ __launch_bounds__(WG) void k_g_finalize(const GVec* __restrict__ vs, int nv, int total,
                                                   const double* __restrict__ part, int op,
                                                   int i0, int i1, const int* __restrict__ active,
                                                   double* __restrict__ scb) {
  // one workgroup per system: strided partial sums, then the fixed workgroup tree
  const int q = blockIdx.x;
  if (q >= nv) return;
  const GVec& v = vs[q];
  double a = 0.0, b = 0.0;
  for (int t = threadIdx.x; t < v.ntiles; t += WG) {
    a += part[v.tile0 + t];
    b += part[total + v.tile0 + t];
  }
  wg_sum2(a, b);
  if (threadIdx.x != 0) return;
  double* sc = scb + (size_t)v.sys * SC_COUNT;
  if (op == GF_STORE1) { sc[i0] = a; return; }
  if (op == GF_STORE2) { sc[i0] = a; sc[i1] = b; return; }
  if (!active[v.sys]) return;
  if (op == GF_ALPHA) {
    sc[SC_RV] = a;
    sc[SC_ALPHA] = sc[SC_RHO1] / a;
  } else if (op == GF_OMEGA) {
    sc[SC_TS] = a;
    sc[SC_TT] = b;
    sc[SC_OMEGA] = b != 0.0 ? a / b : 0.0;
  } else if (op == GF_RHO) {
    sc[SC_RR] = a;
    sc[SC_RHO] = sc[SC_RHO1];
    sc[SC_RHO1] = b;
  }
}

}  // namespace mgk
