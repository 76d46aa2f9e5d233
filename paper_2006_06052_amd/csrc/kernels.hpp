// gfx950 kernels of the solve phase.
//
// The solve phase of the paper's solver is expressed in a handful of backend
// primitives: the sparse matrix-vector product inside the residual, inner
// products and linear combinations of vectors (Section 2.3), applied with
// small statically sized blocks as values (Section 2.4, Section 4 block-valued
// backend) and, for the nested preconditioner, in single precision (Section 4,
// mixed-precision variant: it pays because the solve is memory bound).
//
// Every kernel here streams HBM; none is a dense contraction, so none uses
// MFMA.  Layout and mapping choices for CDNA4:
//  - one block row of a BR x BC block matrix is owned by a group of BR*S lanes
//    of a 64-wide wavefront: lane (s, r) takes scalar row r of every S-th
//    block of the row, so BR adjacent lanes read one block row-contiguously
//    and S*BR adjacent lanes read S consecutive blocks; the S partial sums of
//    a row are combined with cross-lane shuffles;
//  - block values and column indices of the outer FP64 operator are read with
//    non-temporal loads (streamed once per product), which keeps the gathered x
//    vector resident in L2; the preconditioner's smaller operators, each used
//    several times per iteration, are read with ordinary cached loads (measured
//    faster for them);
//  - workgroup ids are remapped so that each of the 8 XCDs (each with its own
//    L2) processes one contiguous range of block rows, keeping the x windows of
//    neighbouring rows in the same L2;
//  - every reduction is two-stage with a fixed order (per-workgroup partials,
//    then one finalizing workgroup), so results are bitwise reproducible.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mgk {

struct bf16 {
  uint16_t u;
};

// Storage type of the smoother blocks M of a hierarchy whose values are of type TV: the
// same precision (FP64, FP32 or BF16).
template <class TV>
struct SmootherOf {
  using type = TV;
};

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef uint32_t u2v __attribute__((ext_vector_type(2)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));

constexpr int WG = 256;          // threads per workgroup (4 waves)
constexpr int WAVE = 64;

// Explicit fused multiply-add.  Device code is compiled without automatic
// contraction, so every rounding step is the one written here in every kernel
// instantiation (results do not depend on the kernel tile).
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

__device__ __forceinline__ float bf16_to_f32(uint16_t u) {
  return __uint_as_float(((uint32_t)u) << 16);
}

// A stored value as the accumulation type (BF16 widened exactly to FP32).
template <class TA, class T>
__device__ __forceinline__ TA to_acc(T v) {
  if constexpr (sizeof(T) == 2) return (TA)bf16_to_f32(reinterpret_cast<const uint16_t&>(v));
  else return (TA)v;
}

// ---- value loads -----------------------------------------------------------

// A matrix value or column-index load: streamed (non-temporal) by default, an
// ordinary cached load when CACHED (the launch chooses per operator: cached for the
// preconditioner's operators, streamed for the outer FP64 operator).
template <bool CACHED, class T>
__device__ __forceinline__ T ld_val(const T* p) {
  if constexpr (CACHED) return *p;
  else return __builtin_nontemporal_load(p);
}

// BC consecutive values of a stored block (one block row, or several adjacent
// block rows for the wide BF16 lanes).
template <int BC, class TV, class TA, bool CACHED = false>
__device__ __forceinline__ void load_vals(const TV* __restrict__ p, TA* out) {
  if constexpr (sizeof(TV) == 8 && BC % 2 == 0) {
    // 16-byte loads of two values each (one block row is two of them)
#pragma unroll
    for (int q = 0; q < BC / 2; ++q) {
      const d2v a = ld_val<CACHED>(reinterpret_cast<const d2v*>(p) + q);
      out[2 * q] = a.x;
      out[2 * q + 1] = a.y;
    }
  } else if constexpr (sizeof(TV) == 4 && BC % 4 == 0) {
#pragma unroll
    for (int q = 0; q < BC / 4; ++q) {
      const f4v a = ld_val<CACHED>(reinterpret_cast<const f4v*>(p) + q);
      out[4 * q] = a.x; out[4 * q + 1] = a.y; out[4 * q + 2] = a.z; out[4 * q + 3] = a.w;
    }
  } else if constexpr (sizeof(TV) == 2 && BC % 8 == 0) {
    // several consecutive block rows: 16-byte loads of eight values each
#pragma unroll
    for (int q = 0; q < BC / 8; ++q) {
      const u4v a = ld_val<CACHED>(reinterpret_cast<const u4v*>(p) + q);
      out[8 * q + 0] = __uint_as_float(a.x << 16);
      out[8 * q + 1] = __uint_as_float(a.x & 0xffff0000u);
      out[8 * q + 2] = __uint_as_float(a.y << 16);
      out[8 * q + 3] = __uint_as_float(a.y & 0xffff0000u);
      out[8 * q + 4] = __uint_as_float(a.z << 16);
      out[8 * q + 5] = __uint_as_float(a.z & 0xffff0000u);
      out[8 * q + 6] = __uint_as_float(a.w << 16);
      out[8 * q + 7] = __uint_as_float(a.w & 0xffff0000u);
    }
  } else if constexpr (sizeof(TV) == 2 && BC == 4) {
    const u2v a = ld_val<CACHED>(reinterpret_cast<const u2v*>(p));
    out[0] = __uint_as_float(a.x << 16);
    out[1] = __uint_as_float(a.x & 0xffff0000u);
    out[2] = __uint_as_float(a.y << 16);
    out[3] = __uint_as_float(a.y & 0xffff0000u);
  } else if constexpr (sizeof(TV) == 2) {
    const uint16_t* q = reinterpret_cast<const uint16_t*>(p);
#pragma unroll
    for (int c = 0; c < BC; ++c) out[c] = (TA)bf16_to_f32(ld_val<CACHED>(q + c));
  } else {
#pragma unroll
    for (int c = 0; c < BC; ++c) out[c] = (TA)ld_val<CACHED>(p + c);
  }
}

// N consecutive stored values as loaded, before any conversion: the row engine issues
// every load of a step into these and converts afterwards, so that no conversion sits
// between a load and the next block's loads (a conversion inside the branch that guards a
// block makes the compiler wait for that block's loads before issuing the next ones).
// FP32 / FP64: the values; BF16 in multiples of 4: packed pairs; other BF16: halves.
template <int N, class TV, bool PACKED = (sizeof(TV) == 2 && N % 4 == 0)>
struct VRaw {
  TV v[N];
};
template <int N, class TV>
struct VRaw<N, TV, true> {
  uint32_t w[N / 2];
};

template <int N, class TV, bool CACHED>
__device__ __forceinline__ void load_vals_raw(const TV* __restrict__ p, VRaw<N, TV>& r) {
  if constexpr (sizeof(TV) == 2 && N % 8 == 0) {
#pragma unroll
    for (int q = 0; q < N / 8; ++q) {
      const u4v a = ld_val<CACHED>(reinterpret_cast<const u4v*>(p) + q);
      r.w[4 * q] = a.x; r.w[4 * q + 1] = a.y; r.w[4 * q + 2] = a.z; r.w[4 * q + 3] = a.w;
    }
  } else if constexpr (sizeof(TV) == 2 && N % 4 == 0) {
#pragma unroll
    for (int q = 0; q < N / 4; ++q) {
      const u2v a = ld_val<CACHED>(reinterpret_cast<const u2v*>(p) + q);
      r.w[2 * q] = a.x; r.w[2 * q + 1] = a.y;
    }
  } else if constexpr (sizeof(TV) == 2) {
    const uint16_t* q = reinterpret_cast<const uint16_t*>(p);
#pragma unroll
    for (int c = 0; c < N; ++c) r.v[c].u = ld_val<CACHED>(q + c);
  } else if constexpr (sizeof(TV) == 8 && N % 2 == 0) {
#pragma unroll
    for (int q = 0; q < N / 2; ++q) {
      const d2v a = ld_val<CACHED>(reinterpret_cast<const d2v*>(p) + q);
      r.v[2 * q] = a.x; r.v[2 * q + 1] = a.y;
    }
  } else if constexpr (sizeof(TV) == 4 && N % 4 == 0) {
#pragma unroll
    for (int q = 0; q < N / 4; ++q) {
      const f4v a = ld_val<CACHED>(reinterpret_cast<const f4v*>(p) + q);
      r.v[4 * q] = a.x; r.v[4 * q + 1] = a.y; r.v[4 * q + 2] = a.z; r.v[4 * q + 3] = a.w;
    }
  } else {
#pragma unroll
    for (int c = 0; c < N; ++c) r.v[c] = ld_val<CACHED>(p + c);
  }
}

template <int N, class TV>
__device__ __forceinline__ void zero_raw(VRaw<N, TV>& r) {
  if constexpr (sizeof(TV) == 2 && N % 4 == 0) {
#pragma unroll
    for (int q = 0; q < N / 2; ++q) r.w[q] = 0u;
  } else if constexpr (sizeof(TV) == 2) {
#pragma unroll
    for (int c = 0; c < N; ++c) r.v[c].u = 0;
  } else {
#pragma unroll
    for (int c = 0; c < N; ++c) r.v[c] = TV(0);
  }
}

template <int N, class TV, class TA>
__device__ __forceinline__ void finish_vals(const VRaw<N, TV>& r, TA* out) {
  if constexpr (sizeof(TV) == 2 && N % 4 == 0) {
#pragma unroll
    for (int q = 0; q < N / 2; ++q) {
      out[2 * q] = (TA)__uint_as_float(r.w[q] << 16);
      out[2 * q + 1] = (TA)__uint_as_float(r.w[q] & 0xffff0000u);
    }
  } else {
#pragma unroll
    for (int c = 0; c < N; ++c) out[c] = to_acc<TA>(r.v[c]);
  }
}

// Single value (used by the transposed product, which reads block columns).
template <class TV, class TA>
__device__ __forceinline__ TA load_val(const TV* __restrict__ p) {
  if constexpr (sizeof(TV) == 2) {
    return (TA)bf16_to_f32(__builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p)));
  } else {
    return (TA)__builtin_nontemporal_load(p);
  }
}

// Block of x: BC consecutive entries (cached loads; x is gathered repeatedly).
template <int BC, class TX, class TA>
__device__ __forceinline__ void load_x(const TX* __restrict__ p, TA* out) {
  if constexpr (sizeof(TX) == 8 && BC == 4) {
    const d2v a = *reinterpret_cast<const d2v*>(p);
    const d2v b = *(reinterpret_cast<const d2v*>(p) + 1);
    out[0] = a.x; out[1] = a.y; out[2] = b.x; out[3] = b.y;
  } else if constexpr (sizeof(TX) == 4 && BC == 4) {
    const f4v a = *reinterpret_cast<const f4v*>(p);
    out[0] = a.x; out[1] = a.y; out[2] = a.z; out[3] = a.w;
  } else {
#pragma unroll
    for (int c = 0; c < BC; ++c) out[c] = (TA)p[c];
  }
}

// N consecutive vector entries p[e .. e+N-1] of a lane's own rows, read ahead of its row
// product.  Every lane issues the loads (lanes that own no rows read entries 0 .. N-1,
// which every vector holds, all at one address), so no branch separates them from the
// product's loads and the compiler places no wait for them before it; the caller
// converts the raw values after the product and uses them in its owning lanes only.
template <int N, bool NT = false, class T>
__device__ __forceinline__ void load_ahead(const T* __restrict__ p, size_t e, bool own,
                                           T (&raw)[N]) {
  const T* q = p + (own ? e : 0);
#pragma unroll
  for (int c = 0; c < N; ++c) {
    if constexpr (NT) raw[c] = __builtin_nontemporal_load(q + c);
    else raw[c] = q[c];
  }
}

// Logical workgroup id: XCD x (hardware places workgroup w on XCD w % 8)
// receives one contiguous range of logical ids.
__device__ __forceinline__ int xcd_remap(int w, int nwg) {
  const int q = nwg >> 3, rem = nwg & 7, x = w & 7;
  return x * q + min(x, rem) + (w >> 3);
}

// ---- block-row engine --------------------------------------------------------

// RPL: scalar rows of the block row owned by one lane (1, or 2 / 4 for the
// BF16 square blocks, whose single block row is only 8 bytes wide).
template <int BR, int S, int RPL = 1>
struct RowMap {
  static_assert(BR % RPL == 0, "rows per lane");
  static constexpr int LB = BR / RPL;           // lanes per block
  static constexpr int G = LB * S;              // lanes per block row
  static constexpr int GPW = WAVE / G;          // block rows per wave
  static constexpr int ROWS = GPW * (WG / WAVE);// block rows per workgroup
};

struct LaneInfo {
  int i;        // block row (may be >= nbr for idle groups)
  int r, s;     // first scalar row inside the block (RPL rows r, r+1, ...), split index
  int gbase;    // first lane of this group inside the wave
  bool active;  // lane belongs to a group
};

template <int BR, int S, int RPL = 1>
__device__ __forceinline__ LaneInfo lane_info(int logical_wg) {
  using M = RowMap<BR, S, RPL>;
  LaneInfo L;
  const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x >> 6;
  const int g = lane / M::G, w = lane - g * M::G;
  L.active = g < M::GPW;
  L.s = w / M::LB;
  L.r = (w - L.s * M::LB) * RPL;
  L.gbase = g * M::G;
  L.i = (logical_wg * (WG / WAVE) + wave) * M::GPW + g;
  return L;
}

// Diagonal layout of a square block operator whose blocks lie on at most DIA_MAX block
// diagonals: block row i has k slots, slot d holding A(i, i + o[d]) (o ascending, so a
// full row's slots are its stored blocks in ascending column order); a slot with no
// stored block holds zeros and is skipped by the row mask.  No row pointers and no
// column indices are read: the x gather no longer waits for them.
constexpr int DIA_MAX = 8;
struct DiaOffs {
  int k;
  int o[DIA_MAX];
  // bit d of mask[i]: block row i stores a block on diagonal d.  Absent blocks (zero
  // padding) are neither read nor multiplied; nullptr when every row stores all k.
  const uint8_t* mask;
};

// Offsets of the slots L.s + m*S (m < NSLOT) that one lane of an S-way split reads.  The
// offsets are kernel arguments; a lane-dependent index into them would be compiled into a
// memory load from the argument segment (one dependent load, with a full wait, per
// block), so each is first pinned to a scalar register and the lane's offsets are then
// selected by value, once per kernel.
template <int S, int NSLOT>
__device__ __forceinline__ void dia_lane_offsets(const DiaOffs& of, int s, int (&out)[NSLOT]) {
  int o[DIA_MAX];
#pragma unroll
  for (int q = 0; q < DIA_MAX; ++q) {
    o[q] = of.o[q];
    asm volatile("" : "+s"(o[q]));
  }
#pragma unroll
  for (int m = 0; m < NSLOT; ++m) {
    int v = o[m * S < DIA_MAX ? m * S : 0];
#pragma unroll
    for (int t = 1; t < S; ++t)
      if (m * S + t < DIA_MAX) v = s == t ? o[m * S + t] : v;
    out[m] = v;
  }
}

// x source of the row engine: fetch_raw issues a block's loads, finish_x converts after
// every load of the step is in flight.  A stored vector: block j is BC consecutive
// entries.
template <class XSrc, int BC>
struct XRaw;
template <class TX, int BC>
struct XRaw<const TX*, BC> {
  TX x[BC];
};

template <int BC, class TX>
__device__ __forceinline__ void fetch_raw(const TX* __restrict__ x, int j, XRaw<const TX*, BC>& r) {
  load_x<BC, TX, TX>(x + (size_t)j * BC, r.x);
}
template <int BC, class TX>
__device__ __forceinline__ void zero_xraw(const TX*, XRaw<const TX*, BC>& r) {
#pragma unroll
  for (int c = 0; c < BC; ++c) r.x[c] = TX(0);
}
template <int BC, class TA, class TX>
__device__ __forceinline__ void finish_x(const TX*, const XRaw<const TX*, BC>& r, TA* out) {
#pragma unroll
  for (int c = 0; c < BC; ++c) out[c] = (TA)r.x[c];
}

// A lane's block row as the row product walks it: blocks [k0, k1) (positions in the BSR
// arrays, or slots of the diagonal layout) and, for the diagonal layout, its stored-block
// bits (all bits without a row mask).
struct RowRange {
  int k0, k1;
  unsigned present;
};

// Kernels load the range before their own operands, and keep the scheduler from moving
// those loads above it (sched_barrier), so that the row product's wait for the range does
// not also wait for them (memory results arrive in issue order).  Lanes past the last row
// read an in-range row's entries (the row product skips them).
template <bool DIA>
__device__ __forceinline__ RowRange row_range(const int* __restrict__ ptr, const DiaOffs& of,
                                              int i, int nbr) {
  const int ic = i < nbr ? i : (nbr > 0 ? nbr - 1 : 0);
  if constexpr (DIA) return RowRange{ic * of.k, ic * of.k + of.k, of.mask ? (unsigned)of.mask[ic] : 0xffu};
  else return RowRange{ptr[ic], ptr[ic + 1], 0xffu};
}

// Rows r .. r+RPL-1 of block row i times x, for the lane (s, r) of a group of
// (BR/RPL)*S lanes.
//
// Summation order, identical for every tile (S, U, RPL): block kr (kr-th stored block of
// the row, or kr-th slot of the diagonal layout) is added, in ascending kr, to stripe
// kr mod NS (NS = 16, or 32 for scalar rows); the NS stripes are then combined by the
// fixed tree (q, q + NS/2), (q, q + NS/4), ..., (q, q + 1).  Lane s owns stripes
// s + S*t, t < T = NS/S: the upper tree levels are formed inside the lane and
// the last log2(S) levels across lanes with shuffles.  Results are therefore
// bitwise the same whatever tile the autotuner picks.
//
// U blocks are handled per step with every load issued before the first use,
// so each lane keeps U independent gathers in flight (the fine-level rows are
// short and would otherwise be bound by one dependent col -> x chain per
// block).  When T > U the stripe accumulators rotate by U after each step so
// that block u of a step always lands in accumulator u.
template <int BR, int BC, int S, int U, bool TRANS, class TV, class TX, class TA, int RPL,
          bool CACHED = false, bool DIA = false, class XSrc = const TX*, bool FENCE = false>
__device__ __forceinline__ void row_product_r(const LaneInfo& L, int nbr,
                                              const int* __restrict__ ptr,
                                              const int* __restrict__ col,
                                              const int* __restrict__ blk,
                                              const TV* __restrict__ val,
                                              XSrc x, TA (&out)[RPL],
                                              const DiaOffs& of, const RowRange& rr) {
  constexpr int NS = BR == 1 ? 32 : 16;
  constexpr int T = NS / S;
  constexpr int LB = BR / RPL;
  static_assert(S <= NS && (U % T == 0 || T % U == 0), "tile");
  static_assert(!TRANS || RPL == 1, "transposed products read block columns, one row per lane");
  TA acc[RPL][T];
#pragma unroll
  for (int q = 0; q < RPL; ++q)
#pragma unroll
    for (int t = 0; t < T; ++t) acc[q][t] = 0;
  if (L.active && L.i < nbr) {
    // diagonal layout: the row's blocks are slots i*k .. i*k + k - 1, columns implied
    const int k0 = rr.k0, k1 = rr.k1;
    const unsigned present = rr.present;
    int steps = 0;
    // One step: blocks kb + u*S (u < U) of the row; colof(u, k) is block k's column,
    // has(k) whether block k is stored, alt an in-range block of this row that is read
    // anyway (a slot that is past the row's end or absent reads that block's values, at an
    // address another lane fetches, and is masked out).  Every load of the step is issued
    // unconditionally, so no branch forces a wait between the blocks' loads; conversions
    // and products follow.
    auto step = [&](int kb, auto colof, auto has, int alt) {
      int j[U], kk[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = kb + u * S;
        ok[u] = k < k1 && has(k);
        const int kc = k < k1 ? k : alt;
        j[u] = colof(u, kc);
        kk[u] = TRANS ? __builtin_nontemporal_load(blk + kc) : (ok[u] ? k : alt);
      }
      VRaw<RPL * BC, TV> vr[U];
      XRaw<XSrc, BC> xr[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        fetch_raw<BC>(x, j[u], xr[u]);
        if constexpr (!TRANS) {
          load_vals_raw<RPL * BC, TV, CACHED>(val + (size_t)kk[u] * (BR * BC) + L.r * BC, vr[u]);
        } else {
          // Block kk of A (BC x BR) read by columns: (A^T)[r][c] = A_kk[c][r].
          const TV* b = val + (size_t)kk[u] * (BR * BC);
          if constexpr (sizeof(TV) == 2 && BC % 4 == 0) {
            const uint16_t* h = reinterpret_cast<const uint16_t*>(b);
#pragma unroll
            for (int c = 0; c < BC; c += 2)
              vr[u].w[c / 2] = (uint32_t)__builtin_nontemporal_load(h + c * BR + L.r) |
                               ((uint32_t)__builtin_nontemporal_load(h + (c + 1) * BR + L.r)
                                << 16);
          } else if constexpr (sizeof(TV) == 2) {
            const uint16_t* h = reinterpret_cast<const uint16_t*>(b);
#pragma unroll
            for (int c = 0; c < BC; ++c) vr[u].v[c].u = __builtin_nontemporal_load(h + c * BR + L.r);
          } else {
#pragma unroll
            for (int c = 0; c < BC; ++c) vr[u].v[c] = __builtin_nontemporal_load(b + c * BR + L.r);
          }
        }
      }
      // FENCE: the step's loads all leave before the first conversion or mask uses one of
      // them (a product inside a loop is otherwise free to interleave them)
      if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        TA v[RPL * BC], xv[BC];
        finish_vals<RPL * BC, TV, TA>(vr[u], v);
        finish_x<BC, TA>(x, xr[u], xv);
        // masked slots contribute fma(0, 0, a) = a, as a zero block would
#pragma unroll
        for (int c = 0; c < RPL * BC; ++c) v[c] = ok[u] ? v[c] : TA(0);
#pragma unroll
        for (int c = 0; c < BC; ++c) xv[c] = ok[u] ? xv[c] : TA(0);
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
          TA& a = acc[q][u % T];
#pragma unroll
          for (int c = 0; c < BC; ++c) a = fma_(v[q * BC + c], xv[c], a);
        }
      }
      if constexpr (T > U) {
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
          TA tmp[T];
#pragma unroll
          for (int t = 0; t < T; ++t) tmp[t] = acc[q][(t + U) % T];
#pragma unroll
          for (int t = 0; t < T; ++t) acc[q][t] = tmp[t];
        }
      }
    };
    if constexpr (DIA) {
      // slot d = L.s + m*S of the lane holds column i + o[d] (clamped; absent blocks
      // are zero); the steps are unrolled, so every slot's offset is a register
      constexpr int NSLOT = (DIA_MAX + S - 1) / S, NSTEP = (NSLOT + U - 1) / U;
      int loff[NSLOT];
      dia_lane_offsets<S, NSLOT>(of, L.s, loff);
      // absent slots read the row's first stored block (fetched by another lane anyway)
      const int alt = k0 + (present ? __builtin_ctz(present) : 0);
#pragma unroll
      for (int st = 0; st < NSTEP; ++st) {
        const int kb = k0 + L.s + st * S * U;
        if (kb >= k1) break;
        step(
            kb,
            [&](int u, int) {
              const int m = st * U + u;
              const int c = L.i + loff[m < NSLOT ? m : 0];
              return c < 0 ? 0 : (c >= nbr ? nbr - 1 : c);
            },
            [&](int k) { return ((present >> (k - k0)) & 1u) != 0; }, alt);
        ++steps;
      }
    } else {
      for (int kb = k0 + L.s; kb < k1; kb += S * U, ++steps)
        step(kb, [&](int, int k) { return ld_val<CACHED>(col + k); }, [](int) { return true; },
             k1 > k0 ? k1 - 1 : 0);
    }
    if constexpr (T > U) {
      // undo the rotations: acc[.][t] now holds stripe (t + steps*U) mod T
      for (int n = (T / U - steps % (T / U)) % (T / U); n > 0; --n)
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
          TA tmp[T];
#pragma unroll
          for (int t = 0; t < T; ++t) tmp[t] = acc[q][(t + U) % T];
#pragma unroll
          for (int t = 0; t < T; ++t) acc[q][t] = tmp[t];
        }
    }
  }
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
#pragma unroll
    for (int h = T / 2; h >= 1; h >>= 1)
#pragma unroll
      for (int t = 0; t < h; ++t) acc[q][t] += acc[q][t + h];
    TA a0 = acc[q][0];
#pragma unroll
    for (int m = S / 2; m >= 1; m >>= 1) a0 += __shfl_down(a0, LB * m, WAVE);
    out[q] = a0;
  }
}

template <int BR, int BC, int S, int U, bool TRANS, class TV, class TX, class TA,
          bool CACHED = false>
__device__ __forceinline__ TA row_product(const LaneInfo& L, int nbr, const int* __restrict__ ptr,
                                          const int* __restrict__ col, const int* __restrict__ blk,
                                          const TV* __restrict__ val, const TX* __restrict__ x) {
  TA out[1];
  const RowRange rr = row_range<false>(ptr, DiaOffs{}, L.i, nbr);
  row_product_r<BR, BC, S, U, TRANS, TV, TX, TA, 1, CACHED>(L, nbr, ptr, col, blk, val, x, out,
                                                             DiaOffs{}, rr);
  return out[0];
}

// Deterministic workgroup sum of up to two values; thread 0 returns them.
template <class T>
__device__ __forceinline__ void wg_sum2(T& a, T& b) {
  __shared__ T sa[WG / WAVE], sb[WG / WAVE];
#pragma unroll
  for (int m = WAVE / 2; m >= 1; m >>= 1) {
    a += __shfl_xor(a, m, WAVE);
    b += __shfl_xor(b, m, WAVE);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & (WAVE - 1)) == 0) {
    sa[wave] = a;
    sb[wave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = sa[0];
    b = sb[0];
#pragma unroll
    for (int w = 1; w < WG / WAVE; ++w) {
      a += sa[w];
      b += sb[w];
    }
  }
}

// ---- sparse kernels ------------------------------------------------------------

// y = alpha A x + beta y   (beta == 0: y is not read).
template <int BR, int BC, int S, int U, bool TRANS, class TV, class TX, class TY, class TA,
          int RPL = 1, bool CACHED = false, bool DIA = false>
__global__ __launch_bounds__(WG) void k_spmv(int nbr, const int* __restrict__ ptr,
                                             const int* __restrict__ col,
                                             const int* __restrict__ blk,
                                             const TV* __restrict__ val,
                                             const TX* __restrict__ x, TY* __restrict__ y,
                                             TA alpha, TA beta, DiaOffs of) {
  const int lw = xcd_remap(blockIdx.x, gridDim.x);
  const LaneInfo L = lane_info<BR, S, RPL>(lw);
  const bool own = L.active && L.s == 0 && L.i < nbr;
  const size_t row0 = (size_t)L.i * BR + L.r;
  const RowRange rr = row_range<DIA>(ptr, of, L.i, nbr);
  __builtin_amdgcn_sched_barrier(0);
  // epilogue operands are loaded before the row product so their latency overlaps it
  TY yr[RPL];
  if (beta != TA(0)) load_ahead<RPL>(y, row0, own, yr);
  TA acc[RPL];
  row_product_r<BR, BC, S, U, TRANS, TV, TX, TA, RPL, CACHED, DIA>(L, nbr, ptr, col, blk, val,
                                                                    x, acc, of, rr);
  if (own) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      TA out = alpha * acc[q];
      if (beta != TA(0)) out += beta * (TA)yr[q];
      y[row0 + q] = (TY)out;
    }
  }
}

// Restriction fused with the coarse level's pre-smoothing from a zero guess: y = A x and
// z = M y, M holding one BR x BR smoother block per block row of y.  Each lane gathers its
// block row's BR outputs (rounded to TY, as stored in y) from the s == 0 lanes and sums
// them against its rows of M in ascending order from zero, as the block-diagonal kernel
// does when it reads y back, so z is bitwise the same as that two-kernel sequence.
template <int BR, int BC, int S, int U, class TV, class TX, class TY, class TA, class TM,
          int RPL = 1, bool CACHED = false>
__global__ __launch_bounds__(WG) void k_spmv_bd(int nbr, const int* __restrict__ ptr,
                                                const int* __restrict__ col,
                                                const TV* __restrict__ val,
                                                const TX* __restrict__ x, TY* __restrict__ y,
                                                const TM* __restrict__ M, TY* __restrict__ z) {
  const int lw = xcd_remap(blockIdx.x, gridDim.x);
  const LaneInfo L = lane_info<BR, S, RPL>(lw);
  const bool own = L.active && L.s == 0 && L.i < nbr;
  const size_t row0 = (size_t)L.i * BR + L.r;
  const RowRange rr = row_range<false>(ptr, DiaOffs{}, L.i, nbr);
  __builtin_amdgcn_sched_barrier(0);
  // the lane's rows of M are loaded ahead of the row product
  TM mr[RPL * BR];
  const TM* m = M + (own ? (size_t)L.i * BR * BR : 0);
  if constexpr (BR == 4 && sizeof(TM) >= 4)
    load_vals<RPL * BR, TM, TM, true>(m + (own ? L.r * BR : 0), mr);
  else
    load_ahead<RPL * BR>(m, own ? L.r * BR : 0, true, mr);
  TA acc[RPL];
  row_product_r<BR, BC, S, U, false, TV, TX, TA, RPL, CACHED>(L, nbr, ptr, col, nullptr, val, x,
                                                              acc, DiaOffs{}, rr);
  TY yo[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) yo[q] = (TY)acc[q];
  // row c of the block row is entry c % RPL of lane c / RPL of the group
  TA yv[BR];
#pragma unroll
  for (int c = 0; c < BR; ++c) yv[c] = (TA)__shfl(yo[c % RPL], L.gbase + c / RPL, WAVE);
  if (own) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      y[row0 + q] = yo[q];
      TA out = 0;
#pragma unroll
      for (int c = 0; c < BR; ++c) out = fma_(to_acc<TA>(mr[q * BR + c]), yv[c], out);
      z[row0 + q] = (TY)out;
    }
  }
}

// y = A x fused with the partial dot products <w1, y> and (two) <y, y> of the
// Krylov iteration (FP64 outer operator).  The partials have a fixed partition
// whatever the tile: one per group of DOT_ROWS consecutive block rows, summed over
// the group's scalar rows staged in LDS by one fixed tree, so the partials (and the
// whole solve) do not depend on the tile.  A workgroup covers max(DOT_ROWS, rows per
// pass of its tile) block rows, i.e. one or several groups, and writes one partial per
// group.  16 block rows are one pass of the four-lane split (S = 4) tile that suits
// short 3x3 / 4x4 block rows; scalar rows use 64.
template <int BR>
constexpr int dot_rows() {
  return BR == 1 ? 64 : 16;
}

// Block rows per workgroup of the fused kernel for a tile: whole groups covering at
// least one pass of the tile.
template <int BR, int S, int RPL>
constexpr int dot_wg_rows() {
  constexpr int D = dot_rows<BR>(), R = RowMap<BR, S, RPL>::ROWS;
  return D * ((R + D - 1) / D);
}

template <int BR, int BC, int S, int U, bool TRANS, class TV, class TX, int RPL = 1,
          bool CACHED = false, bool DIA = false>
__global__ __launch_bounds__(WG) void k_spmv_dot(int nbr, const int* __restrict__ ptr,
                                                 const int* __restrict__ col,
                                                 const int* __restrict__ blk,
                                                 const TV* __restrict__ val,
                                                 const TX* __restrict__ x,
                                                 double* __restrict__ y, int two,
                                                 const double* __restrict__ w1,
                                                 double* __restrict__ part, DiaOffs of) {
  using M = RowMap<BR, S, RPL>;
  constexpr int DOT_ROWS = dot_rows<BR>();
  constexpr int WROWS = dot_wg_rows<BR, S, RPL>();   // block rows of the workgroup
  constexpr int NG = WROWS / DOT_ROWS;                // partial groups of the workgroup
  constexpr int GR = DOT_ROWS * BR;                   // scalar rows of a group
  constexpr int NR = GR < 64 ? 64 : (GR <= 128 ? 128 : 256);   // slots per group
  static_assert(WROWS % DOT_ROWS == 0 && GR <= NR, "dot staging");
  __shared__ double sd1[NG * NR], sd2[NG * NR];
  for (int t = threadIdx.x; t < NG * NR; t += WG) {
    sd1[t] = 0.0;
    sd2[t] = 0.0;
  }
  __syncthreads();
  const int lw = xcd_remap(blockIdx.x, gridDim.x);
  const int rb0 = lw * WROWS, rb1 = min(nbr, rb0 + WROWS);
  const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x >> 6;
  for (int base = rb0; base < rb1; base += M::ROWS) {
    LaneInfo L;
    const int g = lane / M::G, w = lane - g * M::G;
    L.active = g < M::GPW;
    L.s = w / M::LB;
    L.r = (w - L.s * M::LB) * RPL;
    L.gbase = g * M::G;
    L.i = base + wave * M::GPW + g;
    const int lim = L.i < rb1 ? nbr : 0;   // rows past this workgroup's range idle
    const bool own = L.active && L.s == 0 && L.i < rb1;
    const size_t row = (size_t)L.i * BR + L.r;
    const RowRange rr = row_range<DIA>(ptr, of, L.i, lim);
    __builtin_amdgcn_sched_barrier(0);
    double wv[RPL];   // ahead of the product
    load_ahead<RPL, true>(w1, row, own, wv);
    double acc[RPL];
    row_product_r<BR, BC, S, U, TRANS, TV, TX, double, RPL, CACHED, DIA>(L, lim, ptr, col, blk,
                                                                          val, x, acc, of, rr);
    if (own) {
      const int rl = L.i - rb0;
      const int q0 = (rl / DOT_ROWS) * NR + (rl % DOT_ROWS) * BR + L.r;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        __builtin_nontemporal_store(acc[q], y + row + q);
        sd1[q0 + q] = wv[q] * acc[q];
        sd2[q0 + q] = acc[q] * acc[q];
      }
    }
  }
  __syncthreads();
  for (int h = NR / 2; h >= 1; h >>= 1) {   // NR is a power of two; every group alike
    for (int t = threadIdx.x; t < NG * h; t += WG) {
      const int q = (t / h) * NR + t % h;
      sd1[q] += sd1[q + h];
      sd2[q] += sd2[q + h];
    }
    __syncthreads();
  }
  const int ngroups = (nbr + DOT_ROWS - 1) / DOT_ROWS;
  if (threadIdx.x < NG) {
    const int gi = lw * NG + threadIdx.x;
    if (gi < ngroups) {
      part[gi] = sd1[threadIdx.x * NR];
      if (two) part[ngroups + gi] = sd2[threadIdx.x * NR];
    }
  }
}

// t = f - A z  (A may be rectangular: BR x BC blocks).
template <int BR, int BC, int S, int U, bool TRANS, class TV, class TX, class TF, class TA,
          int RPL = 1, bool CACHED = false, bool DIA = false>
__global__ __launch_bounds__(WG) void k_residual(int nbr, const int* __restrict__ ptr,
                                                 const int* __restrict__ col,
                                                 const int* __restrict__ blk,
                                                 const TV* __restrict__ val,
                                                 const TF* __restrict__ f,
                                                 const TX* __restrict__ z, TX* __restrict__ t,
                                                 DiaOffs of) {
  const int lw = xcd_remap(blockIdx.x, gridDim.x);
  const LaneInfo L = lane_info<BR, S, RPL>(lw);
  const bool own = L.active && L.s == 0 && L.i < nbr;
  const size_t row0 = (size_t)L.i * BR + L.r;
  const RowRange rr = row_range<DIA>(ptr, of, L.i, nbr);
  __builtin_amdgcn_sched_barrier(0);
  TF fr[RPL];   // loaded ahead of the row product
  load_ahead<RPL>(f, row0, own, fr);
  TA acc[RPL];
  row_product_r<BR, BC, S, U, TRANS, TV, TX, TA, RPL, CACHED, DIA>(L, nbr, ptr, col, blk, val,
                                                                    z, acc, of, rr);
  if (own) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) t[row0 + q] = (TX)((TA)fr[q] - acc[q]);
  }
}

// Post-smoothing: zout = z + M (f - A z), M block diagonal (M^T when TRANS).
template <int BR, int S, int U, bool TRANS, class TV, class TX, class TF, class TO, class TM,
          class TA, int RPL = 1, bool CACHED = false, bool DIA = false>
static __global__ __launch_bounds__(WG) void k_smooth(int nbr, const int* __restrict__ ptr,
                                               const int* __restrict__ col,
                                               const int* __restrict__ blk,
                                               const TV* __restrict__ val,
                                               const TM* __restrict__ M,
                                               const TF* __restrict__ f,
                                               const TX* __restrict__ z, TO* __restrict__ zout,
                                               DiaOffs of) {
  const int lw = xcd_remap(blockIdx.x, gridDim.x);
  const LaneInfo L = lane_info<BR, S, RPL>(lw);
  const bool own = L.active && L.s == 0 && L.i < nbr;
  const size_t row0 = (size_t)L.i * BR + L.r;
  const RowRange rr = row_range<DIA>(ptr, of, L.i, nbr);
  __builtin_amdgcn_sched_barrier(0);
  // f, z and the lane's rows of M are loaded ahead of the row product
  TF fr[RPL];
  TX zr[RPL];
  TM mr[RPL * BR];
  load_ahead<RPL>(f, row0, own, fr);
  load_ahead<RPL>(z, row0, own, zr);
  const TM* m = M + (own ? (size_t)L.i * BR * BR : 0);
  if constexpr (TRANS) {
    // rows r of M^T are columns of M (one row per lane)
#pragma unroll
    for (int c = 0; c < BR; ++c) mr[c] = m[c * BR + L.r];
  } else if constexpr (BR == 4 && sizeof(TM) >= 4) {
    // the lane's RPL rows of a 4x4 block are contiguous and 16-byte aligned
    load_vals<RPL * BR, TM, TM, true>(m + (own ? L.r * BR : 0), mr);
  } else {
    load_ahead<RPL * BR>(m, own ? L.r * BR : 0, true, mr);
  }
  TA acc[RPL];
  row_product_r<BR, BR, S, U, TRANS, TV, TX, TA, RPL, CACHED, DIA>(L, nbr, ptr, col, blk, val,
                                                                    z, acc, of, rr);
  TA res[RPL], zv[RPL], mv[RPL][BR];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    res[q] = own ? (TA)fr[q] - acc[q] : TA(0);
    zv[q] = (TA)zr[q];
#pragma unroll
    for (int c = 0; c < BR; ++c) mv[q][c] = to_acc<TA>(mr[q * BR + c]);
  }
  // Gather the BR residuals of the block row from the s == 0 lanes (row c is
  // entry c % RPL of lane c / RPL of the group).
  TA rv[BR];
#pragma unroll
  for (int c = 0; c < BR; ++c) rv[c] = __shfl(res[c % RPL], L.gbase + c / RPL, WAVE);
  if (own) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      TA out = zv[q];
#pragma unroll
      for (int c = 0; c < BR; ++c) out = fma_(mv[q][c], rv[c], out);
      zout[row0 + q] = (TO)out;
    }
  }
}

// Pre-smoothing from a zero guess: z = M f (block diagonal; M^T when trans).
template <int B, class TM, class TF, class TX, class TA>
__global__ __launch_bounds__(WG) void k_block_diag(int nbr, int trans, const TM* __restrict__ M,
                                                   const TF* __restrict__ f,
                                                   TX* __restrict__ z) {
  const size_t row = (size_t)blockIdx.x * WG + threadIdx.x;
  if (row >= (size_t)nbr * B) return;
  const size_t i = row / B;
  const int r = (int)(row - i * B);
  const TM* m = M + i * B * B;
  TA fv[B], mv[B];
  load_x<B, TF, TA>(f + i * B, fv);
  if (trans) {
#pragma unroll
    for (int c = 0; c < B; ++c) mv[c] = to_acc<TA>(m[c * B + r]);
  } else if constexpr (B == 4) {
    load_vals<B, TM, TA, true>(m + r * B, mv);   // the row, one vector load
  } else {
#pragma unroll
    for (int c = 0; c < B; ++c) mv[c] = to_acc<TA>(m[r * B + c]);
  }
  TA acc = 0;
#pragma unroll
  for (int c = 0; c < B; ++c) acc = fma_(mv[c], fv[c], acc);
  z[row] = (TX)acc;
}

// ---- dense coarsest-level solve -------------------------------------------------

// z = Cinv r, Cinv n x n FP64 row-major; one workgroup per row.
template <class TI, class TO>
__global__ __launch_bounds__(WG) void k_coarse_gemv(int n, const double* __restrict__ Cinv,
                                                    const TI* __restrict__ r,
                                                    TO* __restrict__ z) {
  const int i = blockIdx.x;
  const double* a = Cinv + (size_t)i * n;
  double s = 0.0, dummy = 0.0;
  int j = threadIdx.x;
  // four row entries per step with every load issued first; the products are added in
  // the same order as one entry per step
  for (; j + 3 * WG < n; j += 4 * WG) {
    double av[4], rv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      av[q] = a[j + q * WG];
      rv[q] = (double)r[j + q * WG];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) s = fma_(av[q], rv[q], s);
  }
  for (; j < n; j += WG) s = fma_(a[j], (double)r[j], s);
  wg_sum2(s, dummy);
  if (threadIdx.x == 0) z[i] = (TO)s;
}

// ---- vector kernels (FP64 Krylov) --------------------------------------------

// Grid-stride loop bounds shared by the reductions: the grid has a fixed size
// per vector length, so partial counts are fixed and sums reproducible.
#define GRID_STRIDE(i, n) \
  for (size_t i = (size_t)blockIdx.x * WG + threadIdx.x; i < (size_t)(n); i += (size_t)gridDim.x * WG)

// part[blk] = <a,b>, part[grid + blk] = <c,d> (second dot optional).
static __global__ __launch_bounds__(WG) void k_dot2(size_t n, const double* __restrict__ a,
                                             const double* __restrict__ b,
                                             const double* __restrict__ c,
                                             const double* __restrict__ d,
                                             double* __restrict__ part) {
  double s1 = 0.0, s2 = 0.0;
  GRID_STRIDE(i, n) {
    s1 += a[i] * b[i];
    if (c) s2 += c[i] * d[i];
  }
  wg_sum2(s1, s2);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1;
    if (c) part[gridDim.x + blockIdx.x] = s2;
  }
}

// Device-resident scalars of the Krylov iteration.
enum Sc {
  SC_RHO = 0,    // rho of the previous iteration
  SC_RHO1 = 1,   // (rhat, r) of the current iteration
  SC_ALPHA = 2,
  SC_OMEGA = 3,
  SC_RV = 4,     // (rhat, v)
  SC_SS = 5,     // ||s||^2
  SC_TS = 6,
  SC_TT = 7,
  SC_RR = 8,     // ||r||^2
  SC_TMP = 9,
  SC_TMP2 = 10,
  SC_COUNT = 16
};

enum FinOp {
  FIN_STORE1 = 0,   // sc[i0] = sum part0
  FIN_STORE2 = 1,   // sc[i0] = sum part0, sc[i1] = sum part1
  FIN_ALPHA = 2,    // sc[RV] = sum; alpha = rho1 / rv
  FIN_OMEGA = 3,    // ts, tt -> omega = ts / tt (0 if tt == 0)
  FIN_RHO = 4       // rr, rho1' -> rho = rho1, rho1 = rho1'
};

// First stage of a fixed-order reduction over many partials: workgroup b sums
// partials [b*RED_CHUNK, (b+1)*RED_CHUNK) of one or two arrays of length count.
constexpr int RED_CHUNK = 4096;

// Sums of part[b0 .. b1) (and of part[count + b0 .. count + b1) when two) by the fixed
// per-thread partition: thread t adds entries b0 + t + WG*(q + 4*it) into a[q], in
// ascending it.  b1 - b0 <= RED_CHUNK, so every load (at most 16 per array) is issued
// before the first addition (an out-of-range entry reads a clamped in-range one and is
// not added).
__device__ __forceinline__ void chunk_sums(const double* __restrict__ part, int count, int two,
                                           int b0, int b1, double (&a)[4], double (&c)[4]) {
  constexpr int IT = RED_CHUNK / (4 * WG);
  double va[IT][4], vc[IT][4];
  const int last = b1 > b0 ? b1 - 1 : b0;
#pragma unroll
  for (int it = 0; it < IT; ++it)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kq = min(b0 + (int)threadIdx.x + (4 * it + q) * WG, last);
      va[it][q] = part[kq];
      vc[it][q] = two ? part[count + kq] : 0.0;
    }
#pragma unroll
  for (int it = 0; it < IT; ++it)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (b0 + (int)threadIdx.x + (4 * it + q) * WG < b1) {
        a[q] += va[it][q];
        c[q] += vc[it][q];
      }
}

static __global__ __launch_bounds__(WG) void k_reduce_stage(const double* __restrict__ part, int count,
                                                     int two, double* __restrict__ out) {
  const int b0 = blockIdx.x * RED_CHUNK, b1 = min(count, b0 + RED_CHUNK);
  double a[4] = {0.0, 0.0, 0.0, 0.0}, c[4] = {0.0, 0.0, 0.0, 0.0};
  chunk_sums(part, count, two, b0, b1, a, c);
  double sa = (a[0] + a[1]) + (a[2] + a[3]), sc = (c[0] + c[1]) + (c[2] + c[3]);
  wg_sum2(sa, sc);
  if (threadIdx.x == 0) {
    out[blockIdx.x] = sa;
    if (two) out[gridDim.x + blockIdx.x] = sc;
  }
}

static __global__ __launch_bounds__(WG) void k_finalize(const double* __restrict__ part, int count,
                                                 int two, int op, int i0, int i1,
                                                 double* __restrict__ sc) {
  double a[4] = {0.0, 0.0, 0.0, 0.0}, b[4] = {0.0, 0.0, 0.0, 0.0};
  chunk_sums(part, count, two, 0, count, a, b);   // count <= RED_CHUNK
  double sa = (a[0] + a[1]) + (a[2] + a[3]), sb = (b[0] + b[1]) + (b[2] + b[3]);
  wg_sum2(sa, sb);
  if (threadIdx.x != 0) return;
  const double a0 = sa, b0 = sb;
  switch (op) {
    case FIN_STORE1: sc[i0] = a0; break;
    case FIN_STORE2: sc[i0] = a0; sc[i1] = b0; break;
    case FIN_ALPHA: sc[SC_RV] = a0; sc[SC_ALPHA] = sc[SC_RHO1] / a0; break;
    case FIN_OMEGA:
      sc[SC_TS] = a0;
      sc[SC_TT] = b0;
      sc[SC_OMEGA] = b0 != 0.0 ? a0 / b0 : 0.0;
      break;
    case FIN_RHO:
      sc[SC_RR] = a0;
      sc[SC_RHO] = sc[SC_RHO1];
      sc[SC_RHO1] = b0;
      break;
  }
}

// p = r + beta (p - omega v), beta = (rho1 / rho) (alpha / omega); p32 (if given) = p
// rounded to FP32, the input of an FP32-accumulating V-cycle (which rounds its FP64 input
// to FP32 on reading, so it gives the same result from the copy).
static __global__ __launch_bounds__(WG) void k_bicg_p(size_t n, const double* __restrict__ sc,
                                               const double* __restrict__ r,
                                               const double* __restrict__ v,
                                               double* __restrict__ p,
                                               float* __restrict__ p32) {
  const double beta = (sc[SC_RHO1] / sc[SC_RHO]) * (sc[SC_ALPHA] / sc[SC_OMEGA]);
  const double om = sc[SC_OMEGA];
  if (p32) {
    GRID_STRIDE(i, n) {
      const double pi = r[i] + beta * (p[i] - om * v[i]);
      p[i] = pi;
      p32[i] = (float)pi;
    }
  } else {
    GRID_STRIDE(i, n) p[i] = r[i] + beta * (p[i] - om * v[i]);
  }
}

// s = r - alpha v; partials of ||s||^2; s32 (if given) = s rounded to FP32, as for p.
// (x += alpha phat is deferred to k_bicg_xr, or to k_bicg_x when the iteration stops at s.)
static __global__ __launch_bounds__(WG) void k_bicg_s(size_t n, const double* __restrict__ sc,
                                               const double* __restrict__ r,
                                               const double* __restrict__ v,
                                               double* __restrict__ s,
                                               float* __restrict__ s32,
                                               double* __restrict__ part) {
  const double al = sc[SC_ALPHA];
  double ss = 0.0, dummy = 0.0;
  GRID_STRIDE(i, n) {
    const double si = r[i] - al * v[i];
    s[i] = si;
    if (s32) s32[i] = (float)si;
    ss += si * si;
  }
  wg_sum2(ss, dummy);
  if (threadIdx.x == 0) part[blockIdx.x] = ss;
}

// x += alpha phat (the iteration stopped at s).
static __global__ __launch_bounds__(WG) void k_bicg_x(size_t n, const double* __restrict__ sc,
                                               const double* __restrict__ ph,
                                               double* __restrict__ x) {
  const double al = sc[SC_ALPHA];
  GRID_STRIDE(i, n) x[i] += al * ph[i];
}

// x = (x + alpha phat) + omega shat; r = s - omega t; partials of ||r||^2 and (rhat, r).
// One pass over x per iteration, with the two additions in the order of the two updates.
static __global__ __launch_bounds__(WG) void k_bicg_xr(size_t n, const double* __restrict__ sc,
                                                const double* __restrict__ s,
                                                const double* __restrict__ t,
                                                const double* __restrict__ ph,
                                                const double* __restrict__ sh,
                                                const double* __restrict__ rh,
                                                double* __restrict__ x, double* __restrict__ r,
                                                double* __restrict__ part) {
  const double al = sc[SC_ALPHA], om = sc[SC_OMEGA];
  double rr = 0.0, rho = 0.0;
  GRID_STRIDE(i, n) {
    x[i] = (x[i] + al * ph[i]) + om * sh[i];
    const double ri = s[i] - om * t[i];
    r[i] = ri;
    rr += ri * ri;
    rho += rh[i] * ri;
  }
  wg_sum2(rr, rho);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rr;
    part[gridDim.x + blockIdx.x] = rho;
  }
}

// y = a * x (a read from sc[ia] inverted when inv) or y = x.
static __global__ __launch_bounds__(WG) void k_scale(size_t n, const double* __restrict__ sc, int ia,
                                              int sqrt_inv, const double* __restrict__ x,
                                              double* __restrict__ y) {
  const double a = sqrt_inv ? 1.0 / sqrt(sc[ia]) : sc[ia];
  GRID_STRIDE(i, n) y[i] = a * x[i];
}

static __global__ __launch_bounds__(WG) void k_scal(size_t n, double a, const double* __restrict__ x,
                                              double* __restrict__ y) {
  GRID_STRIDE(i, n) y[i] = a * x[i];
}

static __global__ __launch_bounds__(WG) void k_copy(size_t n, const double* __restrict__ x,
                                             double* __restrict__ y) {
  GRID_STRIDE(i, n) y[i] = x[i];
}

static __global__ __launch_bounds__(WG) void k_fill(size_t n, double v, double* __restrict__ y) {
  GRID_STRIDE(i, n) y[i] = v;
}

// ---- FGMRES: classical Gram-Schmidt with one reorthogonalization -------------

constexpr int MAXM = 32;

// part[q * grid + blk] = <V_q, w> for q < m <= MQ (V_q = V + q * ld).  MQ bounds the
// accumulators a thread keeps; launch through multidot(), which picks the
// smallest MQ that holds m (the summation order does not depend on MQ).
template <int MQ>
static __global__ __launch_bounds__(WG) void k_multidot(size_t n, int m, const double* __restrict__ V,
                                                 size_t ld, const double* __restrict__ w,
                                                 double* __restrict__ part) {
  double acc[MQ];
#pragma unroll
  for (int q = 0; q < MQ; ++q) acc[q] = 0.0;
  GRID_STRIDE(i, n) {
    const double wi = w[i];
#pragma unroll
    for (int q = 0; q < MQ; ++q)
      if (q < m) acc[q] += V[q * ld + i] * wi;
  }
  for (int q = 0; q < m; ++q) {
    double a = acc[q], dummy = 0.0;
    wg_sum2(a, dummy);
    if (threadIdx.x == 0) part[(size_t)q * gridDim.x + blockIdx.x] = a;
    __syncthreads();
  }
}

static inline void multidot(hipStream_t st, int g, size_t n, int m, const double* V, size_t ld,
                            const double* w, double* part) {
  if (m <= 4) k_multidot<4><<<g, WG, 0, st>>>(n, m, V, ld, w, part);
  else if (m <= 8) k_multidot<8><<<g, WG, 0, st>>>(n, m, V, ld, w, part);
  else if (m <= 16) k_multidot<16><<<g, WG, 0, st>>>(n, m, V, ld, w, part);
  else k_multidot<MAXM><<<g, WG, 0, st>>>(n, m, V, ld, w, part);
}

// h[q] = sum of the partials of dot q (count each); h2 accumulates into hsum.
static __global__ __launch_bounds__(WG) void k_multifin(const double* __restrict__ part, int count,
                                                 int m, double* __restrict__ h,
                                                 double* __restrict__ hsum, int add) {
  for (int q = 0; q < m; ++q) {
    double a = 0.0, dummy = 0.0;
    for (int k = threadIdx.x; k < count; k += WG) a += part[(size_t)q * count + k];
    wg_sum2(a, dummy);
    if (threadIdx.x == 0) {
      h[q] = a;
      hsum[q] = add ? hsum[q] + a : a;
    }
    __syncthreads();
  }
}

// w -= V h (m vectors), optionally partials of ||w||^2.
static __global__ __launch_bounds__(WG) void k_multiaxpy(size_t n, int m, const double* __restrict__ V,
                                                  size_t ld, const double* __restrict__ h,
                                                  double* __restrict__ w,
                                                  double* __restrict__ part) {
  double ss = 0.0, dummy = 0.0;
  GRID_STRIDE(i, n) {
    double wi = w[i];
    for (int q = 0; q < m; ++q) wi -= h[q] * V[q * ld + i];
    w[i] = wi;
    ss += wi * wi;
  }
  if (part) {
    wg_sum2(ss, dummy);
    if (threadIdx.x == 0) part[blockIdx.x] = ss;
  }
}

// x += sum_q y_q Z_q (y on the device).
static __global__ __launch_bounds__(WG) void k_update_x(size_t n, int m, const double* __restrict__ Z,
                                                 size_t ld, const double* __restrict__ y,
                                                 double* __restrict__ x) {
  GRID_STRIDE(i, n) {
    double xi = x[i];
    for (int q = 0; q < m; ++q) xi += y[q] * Z[q * ld + i];
    x[i] = xi;
  }
}

// ---- Schur split / merge --------------------------------------------------------

// out = (TO) in.
template <class TI, class TO>
__global__ __launch_bounds__(WG) void k_cast(size_t n, const TI* __restrict__ in,
                                             TO* __restrict__ out) {
  GRID_STRIDE(i, n) out[i] = (TO)in[i];
}

// out = a + b.
template <class T, class TO>
__global__ __launch_bounds__(WG) void k_add(size_t n, const T* __restrict__ a,
                                            const T* __restrict__ b, TO* __restrict__ out) {
  GRID_STRIDE(i, n) out[i] = (TO)(a[i] + b[i]);
}

// y = m .* x (diagonal preconditioner step).
template <class T>
__global__ __launch_bounds__(WG) void k_diag_mul(size_t n, const T* __restrict__ m,
                                                 const T* __restrict__ x, T* __restrict__ y) {
  GRID_STRIDE(i, n) y[i] = m[i] * x[i];
}

// Interleaved [u,v,w,p] FP64 -> velocity (3 per node) and pressure (1 per node).
template <class TX>
__global__ __launch_bounds__(WG) void k_split(size_t nn, const double* __restrict__ r,
                                              TX* __restrict__ ru, TX* __restrict__ rp) {
  GRID_STRIDE(g, nn) {
    ru[3 * g] = (TX)r[4 * g];
    ru[3 * g + 1] = (TX)r[4 * g + 1];
    ru[3 * g + 2] = (TX)r[4 * g + 2];
    rp[g] = (TX)r[4 * g + 3];
  }
}

template <class TX>
__global__ __launch_bounds__(WG) void k_merge(size_t nn, const TX* __restrict__ zu,
                                              const TX* __restrict__ zp, double* __restrict__ z) {
  GRID_STRIDE(g, nn) {
    z[4 * g] = (double)zu[3 * g];
    z[4 * g + 1] = (double)zu[3 * g + 1];
    z[4 * g + 2] = (double)zu[3 * g + 2];
    z[4 * g + 3] = (double)zp[g];
  }
}

// ---- gradients ---------------------------------------------------------------

// G_k = -lambda_I x_J^T for every stored b x b block k = (I, J).
template <int B>
__global__ __launch_bounds__(WG) void k_bsr_grad(int nbr, const int* __restrict__ ptr,
                                                 const int* __restrict__ col,
                                                 const double* __restrict__ lam,
                                                 const double* __restrict__ x,
                                                 double* __restrict__ g) {
  const int i = blockIdx.x * (WG / (B * B)) + threadIdx.x / (B * B);
  const int e = threadIdx.x % (B * B);
  if (i >= nbr || threadIdx.x >= (WG / (B * B)) * B * B) return;
  const int r = e / B, c = e % B;
  const double li = lam[(size_t)i * B + r];
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) g[(size_t)k * B * B + e] = -li * x[(size_t)col[k] * B + c];
}

// Per-cell viscosity gradient of the finite-difference Stokes operator.
static __global__ __launch_bounds__(WG) void k_theta_grad(int n, const double* __restrict__ lam,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ g) {
  const int nc = n - 1;
  const size_t e = (size_t)blockIdx.x * WG + threadIdx.x;
  if (e >= (size_t)nc * nc * nc) return;
  const int ci = (int)(e % nc), cj = (int)((e / nc) % nc), ck = (int)(e / ((size_t)nc * nc));
  const double inv_h2 = (double)nc * (double)nc;
  auto inner = [&](int i, int j, int k) {
    return i > 0 && j > 0 && k > 0 && i < n - 1 && j < n - 1 && k < n - 1;
  };
  double sum = 0.0;
  for (int d = 0; d < 3; ++d)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        int p[3] = {ci, cj, ck};
        p[(d + 1) % 3] += a;
        p[(d + 2) % 3] += b;
        int q[3] = {p[0], p[1], p[2]};
        q[d] += 1;
        const size_t gp = p[0] + (size_t)n * (p[1] + (size_t)n * p[2]);
        const size_t gq = q[0] + (size_t)n * (q[1] + (size_t)n * q[2]);
        double dmu = 0.0;
        if (inner(p[0], p[1], p[2]))
          for (int c = 0; c < 3; ++c) dmu += lam[4 * gp + c] * (x[4 * gp + c] - x[4 * gq + c]);
        if (inner(q[0], q[1], q[2]))
          for (int c = 0; c < 3; ++c) dmu += lam[4 * gq + c] * (x[4 * gq + c] - x[4 * gp + c]);
        sum -= inv_h2 * dmu;
      }
  g[e] = 0.25 * sum;
}

}  // namespace mgk
