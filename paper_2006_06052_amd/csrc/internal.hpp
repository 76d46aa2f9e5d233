#pragma once
// Internal declarations shared by the translation units of libmgk: device
// memory, stored operators, kernel launchers, the hierarchy, the V-cycle and
// the solver object.
//
// Solve-phase orchestration overview (implemented in solver.hip and multi.hip):
//
// Setup runs on the host in FP64 (host.hpp) and is then moved to the device
// once (Section 2.3: setup with built-in structures, then transfer to the
// backend).  The solve phase composes the kernels of kernels.hpp:
//   V(1,1) cycle per level: z = M r; t = r - A z; r_c = R t; recurse;
//     z += P z_c; z_out = z + M (r - A z); coarsest level: dense FP64 inverse;
//   BiCGStab (right preconditioned) with every scalar kept on the device and
//     convergence read back through pinned memory while the next stage is
//     already queued, so the host never drains the stream inside an
//     iteration;
//   flexible GMRES(m) with classical Gram-Schmidt plus one reorthogonalization
//     (multi-dot kernels) and host Givens rotations;
//   the Schur pressure correction: one velocity cycle, the pressure cycle on
//     r_p - B_lo z_u, and a second velocity cycle on r_u - B_up z_p (Section 4,
//     eqs. SchurP and SchurU).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/mgk.h"
#include "host.hpp"
#include "kernels.hpp"

namespace mgk {

inline thread_local std::string g_err;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCK(x)                                                                      \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess)                                                             \
      throw Error(MGK_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_));         \
  } while (0)

static inline int grid_for(size_t n) {
  size_t g = (n + WG - 1) / WG;
  return (int)std::max<size_t>(1, std::min<size_t>(g, 1024));
}

// ---------------------------------------------------------------- memory

struct Device {
  std::vector<void*> owned;
  int64_t bytes = 0;
  hipStream_t stream = nullptr;
  void* alloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 16;
    n = (n + 255) & ~(size_t)255;
    if (hipMalloc(&p, n) != hipSuccess) throw Error(MGK_E_NOMEM, "hipMalloc failed");
    owned.push_back(p);
    bytes += (int64_t)n;
    return p;
  }
  // The copy has completed when upload returns, so the host buffer (often a temporary
  // of the caller) may be released at once.
  template <class T>
  T* upload(const T* h, size_t count) {
    T* d = (T*)alloc(sizeof(T) * count);
    if (count) {
      HIPCK(hipMemcpyAsync(d, h, sizeof(T) * count, hipMemcpyHostToDevice, stream));
      HIPCK(hipStreamSynchronize(stream));
    }
    return d;
  }
  ~Device() {
    for (void* p : owned) (void)hipFree(p);
  }
};

inline uint16_t f32_to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}

struct Tile {
  int s = 1, u = 4, rpl = 1;
};

// Device block matrix in a storage precision, with optional column index
// (CSC over blocks) for products with the transpose.
struct DMat {
  int br = 1, bc = 1, nbr = 0, nbc = 0;
  int64_t nnzb = 0;
  int storage = MGK_F64;
  int *ptr = nullptr, *col = nullptr;
  void* val = nullptr;
  int *tptr = nullptr, *trow = nullptr, *tblk = nullptr;
  double avg_row = 0.0, avg_col = 0.0;
  Tile tile, ttile;          // engine tiles for products with A and with A^T
  Tile dtile;                // tile of the fused SpMV-and-dots (outer operator)
  bool cached = false;       // values and columns read with cached loads
  // Diagonal layout (dia.k > 0): a copy of the values as n_brows x dia.k blocks on the
  // block diagonals dia.o, used by every product with A (not A^T) in its place.
  void* dval = nullptr;
  DiaOffs dia{};
};

// Block diagonals of a square operator for the diagonal layout: at most DIA_MAX distinct
// block offsets j - i, and the padded layout at most max_pad times the stored blocks
// (the zero blocks it adds are read like stored ones).  Returns false otherwise.
inline bool dia_offsets(const HBsr& A, DiaOffs& of, double max_pad) {
  of = DiaOffs{};
  if (A.br != A.bc || A.nbr != A.nbc || A.nbr == 0) return false;
  int k = 0;
  for (int32_t i = 0; i < A.nbr; ++i)
    for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q) {
      const int off = A.col[q] - i;
      int p = 0;
      while (p < k && of.o[p] < off) ++p;
      if (p < k && of.o[p] == off) continue;
      if (k == DIA_MAX) return false;
      for (int t = k; t > p; --t) of.o[t] = of.o[t - 1];
      of.o[p] = off;
      ++k;
    }
  of.k = k;
  if ((double)A.nbr * k > max_pad * (double)A.nnzb()) {
    of = DiaOffs{};
    return false;
  }
  return true;
}

// Value and column loads of the block-row kernels: the preconditioner's operators
// (every level, prolongator and restriction, in any storage precision) are read with
// ordinary cached loads, the FP64 outer operator of the Krylov iteration with streaming
// (non-temporal) loads.  Measured at 96^3 over four right-hand sides: cached loads made
// the FP64 and BF16 hierarchy solves 5% faster and left FP32 unchanged, while on the
// outer operator they cost 10% (its value stream then evicts the gathered x, a 28 MB
// vector, from L2).  The environment variable MGK_CACHED_LOADS, read at setup,
// overrides the choice with a bit mask of the operators read with cached loads: 1 BF16,
// 2 FP32 and 4 FP64 preconditioner operators, 8 the FP64 outer operator (in every product
// with it, the fused SpMV-and-dots included) together with the level 0 of an FP64
// hierarchy, which shares the outer operator's arrays (default 7).  Results are bitwise
// the same either way.
inline bool operator_cached(int storage, bool outer) {
  const char* e = getenv("MGK_CACHED_LOADS");
  const int mask = e ? atoi(e) : 7;
  if (outer) return (mask & 8) != 0;
  return (mask & (storage == MGK_BF16 ? 1 : storage == MGK_F32 ? 2 : 4)) != 0;
}

// Values in storage precision (FP64, FP32, or BF16 rounded through FP32).
inline void* upload_values(Device& D, const std::vector<double>& val, int storage) {
  const size_t nv = val.size();
  if (storage == MGK_F64) return D.upload(val.data(), nv);
  if (storage == MGK_F32) {
    std::vector<float> v(nv);
    for (size_t i = 0; i < nv; ++i) v[i] = (float)val[i];
    void* d = D.upload(v.data(), nv);
    HIPCK(hipStreamSynchronize(D.stream));
    return d;
  }
  std::vector<uint16_t> v(nv);
  for (size_t i = 0; i < nv; ++i) v[i] = f32_to_bf16((float)val[i]);
  void* d = D.upload(v.data(), nv);
  HIPCK(hipStreamSynchronize(D.stream));
  return d;
}

inline DMat upload_mat(Device& D, const HBsr& A, int storage, bool transpose_index,
                       int dia_mode = 0) {
  DMat M;
  M.br = A.br;
  M.bc = A.bc;
  M.nbr = A.nbr;
  M.nbc = A.nbc;
  M.nnzb = A.nnzb();
  M.storage = storage;
  M.ptr = D.upload(A.ptr.data(), A.ptr.size());
  M.col = D.upload(A.col.data(), A.col.size());
  const size_t nv = A.val.size();
  if (storage == MGK_F64) {
    M.val = D.upload(A.val.data(), nv);
  } else if (storage == MGK_F32) {
    std::vector<float> v(nv);
    for (size_t i = 0; i < nv; ++i) v[i] = (float)A.val[i];
    M.val = D.upload(v.data(), nv);
  } else {
    std::vector<uint16_t> v(nv);
    for (size_t i = 0; i < nv; ++i) v[i] = f32_to_bf16((float)A.val[i]);
    M.val = D.upload(v.data(), nv);
  }
  M.cached = operator_cached(storage, false);
  M.avg_row = A.nbr ? (double)M.nnzb / A.nbr : 0.0;
  DiaOffs of;
  if (dia_mode && (A.br == 3 || A.br == 4) &&
      dia_offsets(A, of, dia_mode == 1 ? 1.15 : 1e300)) {
    const int bb = A.br * A.bc;
    std::vector<double> dv((size_t)A.nbr * of.k * bb, 0.0);
    std::vector<uint8_t> mask(A.nbr, 0);
    for (int32_t i = 0; i < A.nbr; ++i)
      for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q) {
        int d = 0;
        while (of.o[d] != A.col[q] - i) ++d;
        std::copy(A.blk(q), A.blk(q) + bb, dv.begin() + ((size_t)i * of.k + d) * bb);
        mask[i] |= (uint8_t)(1u << d);
      }
    M.dval = upload_values(D, dv, storage);
    if ((int64_t)A.nbr * of.k != A.nnzb()) of.mask = D.upload(mask.data(), mask.size());
    M.dia = of;
  }
  if (transpose_index) {
    std::vector<int> tp(A.nbc + 1, 0), tr(M.nnzb), tb(M.nnzb);
    for (int64_t k = 0; k < M.nnzb; ++k) tp[A.col[k] + 1]++;
    for (int j = 0; j < A.nbc; ++j) tp[j + 1] += tp[j];
    std::vector<int> fill(tp.begin(), tp.end() - 1);
    for (int i = 0; i < A.nbr; ++i)
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        const int d = fill[A.col[k]]++;
        tr[d] = i;
        tb[d] = (int)k;
      }
    M.tptr = D.upload(tp.data(), tp.size());
    M.trow = D.upload(tr.data(), tr.size());
    M.tblk = D.upload(tb.data(), tb.size());
    M.avg_col = A.nbc ? (double)M.nnzb / A.nbc : 0.0;
  }
  // the host vectors must outlive the async copies
  HIPCK(hipStreamSynchronize(D.stream));
  return M;
}

// ---------------------------------------------------------------- sparse launch

template <int BR, int S, int RPL = 1>
static int nwg_rows(int nbr) {
  return std::max(1, (nbr + RowMap<BR, S, RPL>::ROWS - 1) / RowMap<BR, S, RPL>::ROWS);
}

template <class TV>
using AccOf = typename std::conditional<std::is_same<TV, double>::value, double, float>::type;

// Tile of the block-row engine: S lanes split a block row, U blocks per step.
// Candidates below: few lanes and deep unrolling for the short fine-level rows,
// many lanes for the long rows of coarse Galerkin levels and restrictions.
#define MGK_TILES_B(CASE) \
  CASE(1, 4) CASE(1, 8) CASE(2, 2) CASE(2, 4) CASE(2, 8) CASE(4, 2) CASE(4, 4) CASE(8, 4) CASE(16, 2)
#define MGK_TILES_1(CASE) CASE(1, 8) CASE(2, 4) CASE(4, 4) CASE(8, 4) CASE(16, 2) CASE(32, 2)
// Wide-lane tiles (S, U, RPL) for 4x4 blocks: a lane owns RPL adjacent rows of a
// block, reads them with 16-byte loads and gathers the block's x entries once for
// all of them (a BF16 block row is only 8 bytes; for FP32 and FP64 the point is the
// x gather, shared by fewer lanes).
#define MGK_TILES_W(CASE) \
  CASE(2, 4, 2) CASE(4, 2, 2) CASE(4, 4, 2) CASE(8, 2, 2) CASE(16, 2, 2) CASE(4, 2, 4) \
  CASE(8, 1, 4) CASE(16, 1, 4)

// Products that may read the diagonal layout (square 3x3 and 4x4 blocks).
template <int BR, int BC>
constexpr bool dia_ok() {
  return BR == BC && (BR == 3 || BR == 4);
}

// Products that may use the wide-lane tiles (square 4x4 blocks in any storage).
template <int BR, int BC, class TV>
constexpr bool wide_ok() {
  return BR == 4 && BC == 4;
}

template <int BR, class F>
static void tile_switch(const Tile& t, F&& launch) {
#define MGK_TCASE(SS, UU)                                   \
  if (t.s == SS && t.u == UU) {                             \
    launch(std::integral_constant<int, SS>(), std::integral_constant<int, UU>()); \
    return;                                                 \
  }
  if constexpr (BR == 1) {
    MGK_TILES_1(MGK_TCASE)
  } else {
    MGK_TILES_B(MGK_TCASE)
  }
#undef MGK_TCASE
  throw Error(MGK_E_INVALID, "no kernel for tile s=" + std::to_string(t.s) + " u=" +
                                 std::to_string(t.u));
}

// Tile dispatch including the wide-lane tiles (when WIDE): launch(S, U, RPL).
template <int BR, bool WIDE, class F>
static void tile_switch_r(const Tile& t, F&& launch) {
  if (t.rpl == 1) {
    tile_switch<BR>(t, [&](auto SS, auto UU) { launch(SS, UU, std::integral_constant<int, 1>()); });
    return;
  }
  if constexpr (WIDE) {
#define MGK_WCASE(SS, UU, RR)                                                              \
  if (t.s == SS && t.u == UU && t.rpl == RR) {                                             \
    launch(std::integral_constant<int, SS>(), std::integral_constant<int, UU>(),            \
           std::integral_constant<int, RR>());                                              \
    return;                                                                                 \
  }
    MGK_TILES_W(MGK_WCASE)
#undef MGK_WCASE
  }
  throw Error(MGK_E_INVALID, "no kernel for tile s=" + std::to_string(t.s) + " u=" +
                                 std::to_string(t.u) + " rpl=" + std::to_string(t.rpl));
}

// y = alpha A x + beta y.
template <int BR, int BC, class TV, class TX, class TY>
static void spmv_s(hipStream_t st, const DMat& M, bool trans, const Tile& tile, const TX* x,
                   TY* y, double alpha, double beta) {
  using TA = AccOf<TV>;
  const int nrows = trans ? M.nbc : M.nbr;
  const int* p = trans ? M.tptr : M.ptr;
  const int* c = trans ? M.trow : M.col;
  const int* b = trans ? M.tblk : nullptr;
  const TV* v = (const TV*)M.val;
  if (trans) {
    tile_switch<BR>(tile, [&](auto SS, auto UU) {
      constexpr int S_ = decltype(SS)::value, U_ = decltype(UU)::value;
      const int g = nwg_rows<BR, S_>(nrows);
      k_spmv<BR, BC, S_, U_, true, TV, TX, TY, TA><<<g, WG, 0, st>>>(nrows, p, c, b, v, x, y,
                                                                     (TA)alpha, (TA)beta,
                                                                     DiaOffs{});
    });
    return;
  }
  tile_switch_r<BR, wide_ok<BR, BC, TV>()>(tile, [&](auto SS, auto UU, auto RR) {
    constexpr int S_ = decltype(SS)::value, U_ = decltype(UU)::value, R_ = decltype(RR)::value;
    const int g = nwg_rows<BR, S_, R_>(nrows);
    if constexpr (dia_ok<BR, BC>()) {
      if (M.dia.k) {
        const TV* dv = (const TV*)M.dval;
        if (M.cached)
          k_spmv<BR, BC, S_, U_, false, TV, TX, TY, TA, R_, true, true><<<g, WG, 0, st>>>(
              nrows, p, c, b, dv, x, y, (TA)alpha, (TA)beta, M.dia);
        else
          k_spmv<BR, BC, S_, U_, false, TV, TX, TY, TA, R_, false, true><<<g, WG, 0, st>>>(
              nrows, p, c, b, dv, x, y, (TA)alpha, (TA)beta, M.dia);
        return;
      }
    }
    if (M.cached)
      k_spmv<BR, BC, S_, U_, false, TV, TX, TY, TA, R_, true><<<g, WG, 0, st>>>(
          nrows, p, c, b, v, x, y, (TA)alpha, (TA)beta, DiaOffs{});
    else
      k_spmv<BR, BC, S_, U_, false, TV, TX, TY, TA, R_><<<g, WG, 0, st>>>(
          nrows, p, c, b, v, x, y, (TA)alpha, (TA)beta, DiaOffs{});
  });
}

// y = R x and z = Mc y (the coarse level's pre-smoothing from a zero guess) in one launch,
// with R's tile; bitwise the same as spmv_s followed by the block-diagonal kernel.
template <int B, class TV, class TX, class TM>
static void spmv_bd_s(hipStream_t st, const DMat& R, const TX* x, TX* y, const TM* Mc, TX* z) {
  using TA = AccOf<TV>;
  const int nrows = R.nbr;
  const TV* v = (const TV*)R.val;
  tile_switch_r<B, wide_ok<B, B, TV>()>(R.tile, [&](auto SS, auto UU, auto RR) {
    constexpr int S_ = decltype(SS)::value, U_ = decltype(UU)::value, R_ = decltype(RR)::value;
    const int g = nwg_rows<B, S_, R_>(nrows);
    if (R.cached)
      k_spmv_bd<B, B, S_, U_, TV, TX, TX, TA, TM, R_, true><<<g, WG, 0, st>>>(
          nrows, R.ptr, R.col, v, x, y, Mc, z);
    else
      k_spmv_bd<B, B, S_, U_, TV, TX, TX, TA, TM, R_><<<g, WG, 0, st>>>(nrows, R.ptr, R.col, v,
                                                                         x, y, Mc, z);
  });
}

// y = A x (FP64) with the fused partials of <w1, y> and, when two, <y, y>;
// returns the number of partials written per dot (one per group of dot_rows block rows).
// Launch on WG-thread workgroups; with events, the dispatch itself records the kernel's
// start and end in them (its execution time alone, as a kernel trace reports it).
template <class K, class... Args>
static void launch_ev(K kernel, int g, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                      Args... args) {
  if (e0)
    hipExtLaunchKernelGGL(kernel, dim3(g), dim3(WG), 0, st, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, dim3(g), dim3(WG), 0, st, args...);
}

template <int BR, int BC>
static int spmv_dot_s(hipStream_t st, const DMat& M, bool trans, const Tile& tile,
                      const double* x, double* y, int two, const double* w1, double* part,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  const int nrows = trans ? M.nbc : M.nbr;
  const int* p = trans ? M.tptr : M.ptr;
  const int* c = trans ? M.trow : M.col;
  const int* b = trans ? M.tblk : nullptr;
  const double* v = (const double*)M.val;
  if (trans) {
    tile_switch<BR>(tile, [&](auto SS, auto UU) {
      constexpr int S_ = decltype(SS)::value, U_ = decltype(UU)::value;
      constexpr int WR = dot_wg_rows<BR, S_, 1>();
      const int g = std::max(1, (nrows + WR - 1) / WR);
      launch_ev(k_spmv_dot<BR, BC, S_, U_, true, double, double>, g, st, e0, e1, nrows, p, c, b,
                v, x, y, two, w1, part, DiaOffs{});
    });
  } else {
    tile_switch_r<BR, wide_ok<BR, BC, double>()>(tile, [&](auto SS, auto UU, auto RR) {
      constexpr int S_ = decltype(SS)::value, U_ = decltype(UU)::value, R_ = decltype(RR)::value;
      constexpr int WR = dot_wg_rows<BR, S_, R_>();
      const int g = std::max(1, (nrows + WR - 1) / WR);
      if constexpr (dia_ok<BR, BC>()) {
        if (M.dia.k) {
          const double* dv = (const double*)M.dval;
          if (M.cached)
            launch_ev(k_spmv_dot<BR, BC, S_, U_, false, double, double, R_, true, true>, g, st,
                      e0, e1, nrows, p, c, b, dv, x, y, two, w1, part, M.dia);
          else
            launch_ev(k_spmv_dot<BR, BC, S_, U_, false, double, double, R_, false, true>, g, st,
                      e0, e1, nrows, p, c, b, dv, x, y, two, w1, part, M.dia);
          return;
        }
      }
      if (M.cached)
        launch_ev(k_spmv_dot<BR, BC, S_, U_, false, double, double, R_, true>, g, st, e0, e1,
                  nrows, p, c, b, v, x, y, two, w1, part, DiaOffs{});
      else
        launch_ev(k_spmv_dot<BR, BC, S_, U_, false, double, double, R_>, g, st, e0, e1, nrows, p,
                  c, b, v, x, y, two, w1, part, DiaOffs{});
    });
  }
  return std::max(1, (nrows + dot_rows<BR>() - 1) / dot_rows<BR>());
}

template <int BR, int BC, class TV, class TX, class TF>
static void residual_s(hipStream_t st, const DMat& M, bool trans, const Tile& tile, const TF* f,
                       const TX* z, TX* t) {
  using TA = AccOf<TV>;
  const int nrows = trans ? M.nbc : M.nbr;
  const int* p = trans ? M.tptr : M.ptr;
  const int* c = trans ? M.trow : M.col;
  const int* b = trans ? M.tblk : nullptr;
  const TV* v = (const TV*)M.val;
  if (trans) {
    tile_switch<BR>(tile, [&](auto SS, auto UU) {
      constexpr int S_ = decltype(SS)::value, U_ = decltype(UU)::value;
      const int g = nwg_rows<BR, S_>(nrows);
      k_residual<BR, BC, S_, U_, true, TV, TX, TF, TA><<<g, WG, 0, st>>>(nrows, p, c, b, v, f,
                                                                          z, t, DiaOffs{});
    });
    return;
  }
  tile_switch_r<BR, wide_ok<BR, BC, TV>()>(tile, [&](auto SS, auto UU, auto RR) {
    constexpr int S_ = decltype(SS)::value, U_ = decltype(UU)::value, R_ = decltype(RR)::value;
    const int g = nwg_rows<BR, S_, R_>(nrows);
    if constexpr (dia_ok<BR, BC>()) {
      if (M.dia.k) {
        const TV* dv = (const TV*)M.dval;
        if (M.cached)
          k_residual<BR, BC, S_, U_, false, TV, TX, TF, TA, R_, true, true><<<g, WG, 0, st>>>(
              nrows, p, c, b, dv, f, z, t, M.dia);
        else
          k_residual<BR, BC, S_, U_, false, TV, TX, TF, TA, R_, false, true><<<g, WG, 0, st>>>(
              nrows, p, c, b, dv, f, z, t, M.dia);
        return;
      }
    }
    if (M.cached)
      k_residual<BR, BC, S_, U_, false, TV, TX, TF, TA, R_, true><<<g, WG, 0, st>>>(
          nrows, p, c, b, v, f, z, t, DiaOffs{});
    else
      k_residual<BR, BC, S_, U_, false, TV, TX, TF, TA, R_><<<g, WG, 0, st>>>(
          nrows, p, c, b, v, f, z, t, DiaOffs{});
  });
}

template <int B, class TV, class TX, class TF, class TO, class TM>
static void smooth_s(hipStream_t st, const DMat& M, bool trans, const Tile& tile, const TM* Mb,
                     const TF* f, const TX* z, TO* zout) {
  using TA = AccOf<TV>;
  const int nrows = M.nbr;
  const int* p = trans ? M.tptr : M.ptr;
  const int* c = trans ? M.trow : M.col;
  const int* b = trans ? M.tblk : nullptr;
  const TV* v = (const TV*)M.val;
  if (trans) {
    tile_switch<B>(tile, [&](auto SS, auto UU) {
      constexpr int S_ = decltype(SS)::value, U_ = decltype(UU)::value;
      const int g = nwg_rows<B, S_>(nrows);
      k_smooth<B, S_, U_, true, TV, TX, TF, TO, TM, TA><<<g, WG, 0, st>>>(nrows, p, c, b, v, Mb,
                                                                           f, z, zout,
                                                                           DiaOffs{});
    });
    return;
  }
  tile_switch_r<B, wide_ok<B, B, TV>()>(tile, [&](auto SS, auto UU, auto RR) {
    constexpr int S_ = decltype(SS)::value, U_ = decltype(UU)::value, R_ = decltype(RR)::value;
    const int g = nwg_rows<B, S_, R_>(nrows);
    if constexpr (dia_ok<B, B>()) {
      if (M.dia.k) {
        const TV* dv = (const TV*)M.dval;
        if (M.cached)
          k_smooth<B, S_, U_, false, TV, TX, TF, TO, TM, TA, R_, true, true><<<g, WG, 0, st>>>(
              nrows, p, c, b, dv, Mb, f, z, zout, M.dia);
        else
          k_smooth<B, S_, U_, false, TV, TX, TF, TO, TM, TA, R_, false, true><<<g, WG, 0, st>>>(
              nrows, p, c, b, dv, Mb, f, z, zout, M.dia);
        return;
      }
    }
    if (M.cached)
      k_smooth<B, S_, U_, false, TV, TX, TF, TO, TM, TA, R_, true><<<g, WG, 0, st>>>(
          nrows, p, c, b, v, Mb, f, z, zout, DiaOffs{});
    else
      k_smooth<B, S_, U_, false, TV, TX, TF, TO, TM, TA, R_><<<g, WG, 0, st>>>(
          nrows, p, c, b, v, Mb, f, z, zout, DiaOffs{});
  });
}

// ---------------------------------------------------------------- hierarchy

struct DLevel {
  DMat A, P, R;
  void* M = nullptr;       // smoother blocks: FP64 (F64 hierarchy) or FP32
  DMat Lf, Uf;             // ILU(0) smoother factors (ilu hierarchies)
  void* Dinv = nullptr;    // ILU pivot inverses, FP64 or FP32 like M
  int nbr = 0;
  size_t n = 0;            // scalar unknowns
  void *r = nullptr, *t = nullptr, *z = nullptr, *z2 = nullptr;
};

struct DHier {
  int b = 1, storage = MGK_F64;
  bool trans_ready = false;
  bool ilu = false;        // levels smooth with block ILU(0)
  int ilu_sweeps = 2;
  void *sy = nullptr, *sy2 = nullptr, *sw = nullptr, *sz = nullptr;  // ILU scratch (level-0 size)
  std::vector<DLevel> lv;
  int nc = 0;
  double *cinv = nullptr, *cinvT = nullptr;
  HHierarchy host;         // kept only when requested
  bool keep_host = false;
  std::vector<mgk_level_desc> desc;
};

// One V(1,1) cycle on level l.  r: TIN at level 0 (else TX in lv[l].r);
// output: TOUT at level 0 (else TX).  Returns nothing; the output of a level
// l > 0 lands in lv[l].z2 (or lv[l].z on the coarsest level).
// Block ILU application with Jacobi sweeps on the factors (TX vectors, FP32 or
// FP64 accumulation): (I + L) y = r by y = r, then `sw` times y <- r - L y;
// (D + U) z = y by z = Dinv y, then `sw` times z <- Dinv (y - U z).  y, y2, w,
// zt are scratch vectors of n entries; the last product writes out (TOUT).
template <int B, class TV, class TX, class TIN, class TOUT>
static void ilu_sweeps(hipStream_t st, const DMat& Lf, const DMat& Uf, const void* Dinv, int nbr,
                       int sw, const TIN* r, TOUT* out, TX* y, TX* y2, TX* w, TX* zt) {
  using TM = typename std::conditional<std::is_same<TV, double>::value, double, float>::type;
  using TA = AccOf<TV>;
  const size_t n = (size_t)nbr * B;
  const int gd = (int)((n + WG - 1) / WG);
  const TM* D = (const TM*)Dinv;
  k_cast<TIN, TX><<<grid_for(n), WG, 0, st>>>(n, r, y);
  for (int q = 0; q < sw; ++q) {
    residual_s<B, B, TV, TX, TIN>(st, Lf, false, Lf.tile, r, y, y2);
    std::swap(y, y2);
  }
  if (sw == 0) {
    k_block_diag<B, TM, TX, TOUT, TA><<<gd, WG, 0, st>>>(nbr, 0, D, y, out);
    return;
  }
  k_block_diag<B, TM, TX, TX, TA><<<gd, WG, 0, st>>>(nbr, 0, D, y, zt);
  for (int q = 0; q < sw; ++q) {
    residual_s<B, B, TV, TX, TX>(st, Uf, false, Uf.tile, y, zt, w);
    if (q + 1 == sw)
      k_block_diag<B, TM, TX, TOUT, TA><<<gd, WG, 0, st>>>(nbr, 0, D, w, out);
    else
      k_block_diag<B, TM, TX, TX, TA><<<gd, WG, 0, st>>>(nbr, 0, D, w, zt);
  }
}

template <int B, class TV, class TX>
struct Cycle {
  using TM = typename SmootherOf<TV>::type;

  // pre: lv[l].z already holds the pre-smoothing M r (written by the restriction above).
  template <class TIN, class TOUT>
  static void run(hipStream_t st, DHier& H, int l, const TIN* r, TOUT* zout, bool trans,
                  bool pre = false) {
    DLevel& L = H.lv[l];
    const int nl = (int)H.lv.size();
    if (l == nl - 1) {
      k_coarse_gemv<TIN, TOUT><<<H.nc, WG, 0, st>>>(H.nc, trans ? H.cinvT : H.cinv, r, zout);
      return;
    }
    TX* z = (TX*)L.z;
    TX* t = (TX*)L.t;
    DLevel& C = H.lv[l + 1];
    TX *sy = (TX*)H.sy, *sy2 = (TX*)H.sy2, *sw = (TX*)H.sw, *sz = (TX*)H.sz;
    if (H.ilu)   // z = ILU^-1 r
      ilu_sweeps<B, TV, TX, TIN, TX>(st, L.Lf, L.Uf, L.Dinv, L.nbr, H.ilu_sweeps, r, z, sy, sy2,
                                     sw, sz);
    else if (!pre)
      k_block_diag<B, TM, TIN, TX, AccOf<TV>>
          <<<(unsigned)((L.n + WG - 1) / WG), WG, 0, st>>>(L.nbr, trans, (const TM*)L.M, r, z);
    residual_s<B, B, TV, TX, TIN>(st, L.A, trans, trans ? L.A.ttile : L.A.tile, r, z, t);
    // a coarse level that is not the coarsest pre-smooths from a zero guess: forward
    // block-diagonal cycles fold that product into the restriction's launch
    const bool fold = !trans && !H.ilu && l + 1 < nl - 1;
    if (fold)
      spmv_bd_s<B, TV, TX, TM>(st, L.R, t, (TX*)C.r, (const TM*)C.M, (TX*)C.z);
    else
      spmv_s<B, B, TV, TX, TX>(st, L.R, false, L.R.tile, t, (TX*)C.r, 1.0, 0.0);
    TX* zc = (l + 1 == nl - 1) ? (TX*)C.z : (TX*)C.z2;
    run<TX, TX>(st, H, l + 1, (const TX*)C.r, zc, trans, fold);
    spmv_s<B, B, TV, TX, TX>(st, L.P, false, L.P.tile, zc, z, 1.0, 1.0);
    if (H.ilu) {   // zout = z + ILU^-1 (r - A z)
      residual_s<B, B, TV, TX, TIN>(st, L.A, false, L.A.tile, r, z, t);
      ilu_sweeps<B, TV, TX, TX, TX>(st, L.Lf, L.Uf, L.Dinv, L.nbr, H.ilu_sweeps, t, (TX*)L.z2,
                                    sy, sy2, sw, sz);
      k_add<TX, TOUT><<<grid_for(L.n), WG, 0, st>>>(L.n, z, (const TX*)L.z2, zout);
    } else {
      smooth_s<B, TV, TX, TIN, TOUT, TM>(st, L.A, trans, trans ? L.A.ttile : L.A.tile,
                                         (const TM*)L.M, r, z, zout);
    }
  }
};

// Dispatch on (block size, storage) for vectors of type TIN/TOUT at the
// hierarchy boundary.
template <class TIN, class TOUT>
static void vcycle(hipStream_t st, DHier& H, const TIN* r, TOUT* z, bool trans) {
#define MGK_VC(BB)                                                                   \
  case BB:                                                                           \
    if (H.storage == MGK_F64)                                                        \
      Cycle<BB, double, double>::run<TIN, TOUT>(st, H, 0, r, z, trans);              \
    else if (H.storage == MGK_F32)                                                   \
      Cycle<BB, float, float>::run<TIN, TOUT>(st, H, 0, r, z, trans);                \
    else                                                                             \
      Cycle<BB, bf16, float>::run<TIN, TOUT>(st, H, 0, r, z, trans);                 \
    break;
  switch (H.b) {
    MGK_VC(1)
    MGK_VC(3)
    MGK_VC(4)
    default: throw Error(MGK_E_INVALID, "unsupported block size");
  }
#undef MGK_VC
}


struct MultiWork;
void multi_free(MultiWork* w);

// IDR(s) workspace (idrs.hip).
constexpr int IDR_MAX_S = 16;
struct IdrWork;
IdrWork* idr_create(mgk_solver* S);
void idr_free(IdrWork* w);
int idrs(mgk_solver* S, const double* b, double* x, double tol, bool trans, mgk_info* info);

// Solve-phase helpers shared by the Krylov methods (solver.hip).
void outer_spmv(mgk_solver* S, const double* x, double* y, bool trans, int dots = 0,
                const double* w1 = nullptr, int* nwg = nullptr);
void outer_residual(mgk_solver* S, const double* b, const double* x, double* r, bool trans);
// Sum `count` reduction partials (two arrays when two) into sc[i0] (, sc[i1]) with
// finalize op `op`; sc defaults to the solver's scalar block.
void finalize(mgk_solver* S, int count, int two, int op, int i0 = 0, int i1 = 0,
              double* sc = nullptr);
double norm2(mgk_solver* S, const double* a);
struct BatchWork;
void batch_free(BatchWork* w);

inline int fail(const Error& e) {
  g_err = e.what();
  return e.code;
}

// Run an entry point body; no exception crosses the C ABI.
template <class F>
int guard(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    return fail(e);
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return MGK_E_NOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return MGK_E_INVALID;
  }
}

void precond(mgk_solver* S, const double* r, double* z, bool trans);
void precond(mgk_solver* S, const float* r, double* z);
}  // namespace mgk

// ---------------------------------------------------------------- solver object

using namespace mgk;

struct mgk_solver {
  Device dev;
  mgk_params prm;
  int kind = MGK_AMG_SPAI0;
  int b = 4;
  int nbr = 0;
  size_t n = 0;
  HBsr A_host;               // kept for the FP64 transpose pattern and export
  DMat A;                    // FP64 outer operator
  DHier H;                   // monolithic or velocity hierarchy
  DHier Hp;                  // pressure hierarchy (Schur)
  DMat Blo, Bup;             // Schur couplings in storage precision
  void* Sm = nullptr;        // scalar SPAI(0) of the pressure operator (schur_spai0)
  DMat Lf, Uf;               // ILU factors (strict lower / upper), storage precision
  void* Dinv = nullptr;      // ILU pivot inverses (FP64, or FP32 for low-precision storage)
  void *iy = nullptr, *iy2 = nullptr, *iw = nullptr, *iz = nullptr;  // ILU sweep vectors
  IluFactors ilu_host;       // FP64 factors kept for mgk_ilu_export (keep_host / host only)
  bool ilu_kept = false;
  void *ru = nullptr, *rp = nullptr, *tu = nullptr, *tp = nullptr, *zu = nullptr, *zp = nullptr;
  // Krylov workspace (FP64)
  double *r = nullptr, *rh = nullptr, *p = nullptr, *v = nullptr, *ph = nullptr, *s = nullptr,
         *sh = nullptr, *t = nullptr;
  // FP32 copies of p and s, the BiCGStab V-cycle inputs, for a block-diagonal-smoothed AMG
  // hierarchy stored below FP64 (its kernels round their FP64 input to FP32 on reading, so
  // the copies give bitwise the same cycle while the three level-0 passes over the input
  // read half the bytes); null otherwise
  float *p32 = nullptr, *s32 = nullptr;
  double* sc = nullptr;      // device scalars
  double* part = nullptr;    // reduction partials
  double* part2 = nullptr;   // second-stage partials
  size_t part_len = 0;
  double* hsc = nullptr;     // pinned host mirror of sc
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  int time_mask = 0;             // timing of the next solves: prm.time_spmv, restricted by
                                 // mgk_set_timing
  std::vector<hipEvent_t> tev;   // timing events around outer SpMV launches
  size_t tev_used = 0;
  std::vector<hipEvent_t> pev;   // timing events around preconditioner applications
  size_t pev_used = 0;
  // FGMRES
  double *V = nullptr, *Z = nullptr, *h = nullptr, *hsum = nullptr, *yv = nullptr;
  double* hpin = nullptr;
  int m = 0;
  double setup_ms = 0.0;
  bool host_only = false;
  MultiWork* multi = nullptr;      // multi-RHS workspace, created by the first mgk_solve_multi
  IdrWork* idr = nullptr;          // IDR(s) workspace (krylov == MGK_IDRS)
  BatchWork* batch = nullptr;      // set for solvers made by mgk_batch_setup
  ~mgk_solver() {
    if (multi) mgk::multi_free(multi);
    if (idr) mgk::idr_free(idr);
    if (batch) mgk::batch_free(batch);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : tev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : pev)
      if (e) (void)hipEventDestroy(e);
    if (hsc) (void)hipHostFree(hsc);
    if (hpin) (void)hipHostFree(hpin);
  }
};

