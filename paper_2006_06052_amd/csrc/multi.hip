// K <= 32 right-hand sides solved together (mgk_solve_multi).
//
// The K BiCGStab recurrences run in lockstep: every matrix product is one block
// SpMM over [n][K] vectors (the hierarchy and the outer operator are read once
// per product for all K columns), every scalar of the recurrence is a per-column
// array kept on the device, and each column stops on its own tolerance: a
// column that converged, broke down or needs a restart is masked out of the
// vector updates.  This is K independent solves, not a block Krylov method.
#include "internal.hpp"
#include "kernels_multi.hpp"

namespace mgk {

// Flag uploads go through a ring of pinned slots, so a slot is never rewritten
// while its asynchronous copy may still be pending (the host synchronizes with
// the stream far more often than every FLAG_SLOTS uploads).
constexpr int FLAG_SLOTS = 64;

struct MLevel {
  void *r = nullptr, *t = nullptr, *z = nullptr, *z2 = nullptr;  // [n_l][K] in TX
};

struct MultiWork {
  std::vector<void*> owned;
  std::vector<MLevel> lv;
  double *r = nullptr, *rh = nullptr, *p = nullptr, *v = nullptr, *ph = nullptr, *s = nullptr,
         *sh = nullptr, *t = nullptr;
  double* scm = nullptr;     // per-column scalars [SM_COUNT][KL]
  int *active = nullptr, *mask = nullptr;
  double *part = nullptr, *part2 = nullptr;
  size_t part_rows = 0;
  double* hsc = nullptr;     // pinned mirror of scm
  int* hflags = nullptr;     // pinned ring of FLAG_SLOTS x (active[KL], mask[KL])
  int flag_slot = 0;
  int act[KL] = {0}, msk[KL] = {0};
  hipEvent_t ev = nullptr;
  int64_t bytes = 0;
  void* alloc(size_t n) {
    void* q = nullptr;
    n = (n + 255) & ~(size_t)255;
    if (hipMalloc(&q, n) != hipSuccess) throw Error(MGK_E_NOMEM, "hipMalloc failed (multi-RHS)");
    owned.push_back(q);
    bytes += (int64_t)n;
    return q;
  }
};

void multi_free(MultiWork* w) {
  if (!w) return;
  for (void* q : w->owned) (void)hipFree(q);
  if (w->hsc) (void)hipHostFree(w->hsc);
  if (w->hflags) (void)hipHostFree(w->hflags);
  if (w->ev) (void)hipEventDestroy(w->ev);
  delete w;
}

static MultiWork* ensure_multi(mgk_solver* S) {
  if (S->multi) return S->multi;
  MultiWork* W = new MultiWork();
  try {
    const size_t n = S->n;
    const size_t vb = n * KL * sizeof(double);
    double** vecs[] = {&W->r, &W->rh, &W->p, &W->v, &W->ph, &W->s, &W->sh, &W->t};
    for (double** q : vecs) *q = (double*)W->alloc(vb);
    const size_t xs = S->H.storage == MGK_F64 ? 8 : 4;
    W->lv.resize(S->H.lv.size());
    for (size_t l = 0; l < S->H.lv.size(); ++l) {
      const size_t nl = S->H.lv[l].n * KL * xs;
      W->lv[l].r = W->alloc(nl);
      W->lv[l].t = W->alloc(nl);
      W->lv[l].z = W->alloc(nl);
      W->lv[l].z2 = W->alloc(nl);
    }
    W->scm = (double*)W->alloc(sizeof(double) * SM_COUNT * KL);
    W->active = (int*)W->alloc(sizeof(int) * KL);
    W->mask = (int*)W->alloc(sizeof(int) * KL);
    // per-column partial rows: two dots per SpMM workgroup (8 block rows each)
    W->part_rows = 2 * ((size_t)S->nbr / MROWS + 2) + 2 * 1024;
    W->part = (double*)W->alloc(sizeof(double) * KL * W->part_rows);
    W->part2 = (double*)W->alloc(sizeof(double) * KL * (2 * (W->part_rows / MRED_CHUNK + 2)));
    HIPCK(hipHostMalloc((void**)&W->hsc, sizeof(double) * SM_COUNT * KL, hipHostMallocDefault));
    HIPCK(hipHostMalloc((void**)&W->hflags, sizeof(int) * 2 * KL * FLAG_SLOTS,
                        hipHostMallocDefault));
    HIPCK(hipEventCreateWithFlags(&W->ev, hipEventDisableTiming));
  } catch (...) {
    multi_free(W);
    throw;
  }
  S->multi = W;
  return W;
}

// Plane-tiled workgroup order for a diagonal-layout operator whose largest offset P (a
// grid plane) is a multiple of 8 rows and at least 1024; the linear order otherwise.
// Returns the grid size (8 tiles x planes x tile width, holes included).
static int msched_of(const DMat& A, MSched& ms) {
  ms = MSched{0, 0, 0};
  const int g = (A.nbr + MROWS - 1) / MROWS;
  if (A.dia.k == 0) return g;
  int P = 0;
  for (int d = 0; d < A.dia.k; ++d) P = std::max(P, std::abs(A.dia.o[d]));
  if (P % MROWS != 0 || P < 1024) return g;
  ms.pb = P / MROWS;
  ms.tb = (ms.pb + 7) / 8;
  ms.np = (g + ms.pb - 1) / ms.pb;
  return 8 * ms.np * ms.tb;
}

// Row slices (log2) of a BSR operator in the multi-RHS products.  A coarse level has few
// rows, each long (64^3: 3,936 rows of 71 blocks at level 2), so one 32-lane group per row
// leaves most of the GPU idle while each group walks its row step by step; its rows are
// cut into slices while the launch has fewer than 2048 workgroups and a slice keeps at
// least 6 blocks.  Rows of the fine and first coarse levels stay whole (slicing them
// measured slower: more workgroups, each with a slice combine).
static int mslices(const DMat& A) {
  const double avg = A.nbr ? (double)A.nnzb / A.nbr : 0.0;
  int qs = 0;
  while (qs < 3 && (((int64_t)A.nbr << qs) / MROWS) < 2048 && avg / (2 << qs) >= 6.0) ++qs;
  return qs;
}

// The small stage (128 blocks per pass) for an operator whose workgroups own few blocks.
static bool msmall(const DMat& A, int qs) {
  const double avg = A.nbr ? (double)A.nnzb / A.nbr : 0.0;
  return avg * (MROWS >> qs) <= 96.0;
}

static int mgrid(int nbr, int qs) {
  const int rw = MROWS >> qs;
  return (nbr + rw - 1) / rw;
}

// ---------------------------------------------------------------- multi V-cycle

// Y = A X + beta Y over [n][K] vectors (restriction, prolongation).
template <int B, class TV, class TX, class TA>
static void spmm(hipStream_t st, const DMat& A, int K, int qs, const TX* X, TX* Y, TA beta) {
  const int g = mgrid(A.nbr, qs);
  if (msmall(A, qs))
    k_spmm<B, B, TV, TX, TX, TA, true><<<g, WG, 0, st>>>(A.nbr, K, A.ptr, A.col,
                                                         (const TV*)A.val, X, Y, TA(1), beta, qs);
  else
    k_spmm<B, B, TV, TX, TX, TA, false><<<g, WG, 0, st>>>(A.nbr, K, A.ptr, A.col,
                                                          (const TV*)A.val, X, Y, TA(1), beta, qs);
}

// Y = R X and Z = Mc Y (the coarse level's pre-smoothing from a zero guess) in one launch.
template <int B, class TV, class TX, class TA, class TM>
static void spmm_bd(hipStream_t st, const DMat& R, int K, int qs, const TX* X, TX* Y,
                    const TM* Mc, TX* Z) {
  const int g = mgrid(R.nbr, qs);
  if (msmall(R, qs))
    k_spmm_bd<B, B, TV, TX, TX, TA, TM, true><<<g, WG, 0, st>>>(R.nbr, K, R.ptr, R.col,
                                                               (const TV*)R.val, X, Y, Mc, Z, qs);
  else
    k_spmm_bd<B, B, TV, TX, TX, TA, TM, false><<<g, WG, 0, st>>>(
        R.nbr, K, R.ptr, R.col, (const TV*)R.val, X, Y, Mc, Z, qs);
}

template <int B, class TV, class TX>
struct CycleM {
  using TM = typename SmootherOf<TV>::type;
  using TA = AccOf<TV>;

  // pre: W.lv[l].z already holds the pre-smoothing M r (written by the restriction above).
  template <class TIN, class TOUT>
  static void run(hipStream_t st, DHier& H, MultiWork& W, int l, int K, const TIN* r,
                  TOUT* zout, bool pre = false) {
    DLevel& L = H.lv[l];
    const int nl = (int)H.lv.size();
    if (l == nl - 1) {
      k_coarse_gemm<TIN, TOUT><<<H.nc, WG, 0, st>>>(H.nc, K, H.cinv, r, zout);
      return;
    }
    TX* z = (TX*)W.lv[l].z;
    TX* t = (TX*)W.lv[l].t;
    MLevel& C = W.lv[l + 1];
    const int g = (L.nbr + MROWS - 1) / MROWS;
    const int qa = mslices(L.A), qr = mslices(L.R), qp = mslices(L.P);
    const int ga = mgrid(L.nbr, qa);
    // a square operator stored in the diagonal layout is read in it (same sums, bitwise),
    // its row blocks taken in the plane-tiled order
    const bool dia = (B == 3 || B == 4) && L.A.dia.k > 0;
    // the small stage pays in register count for BF16 values only (FP32 residual and
    // smoother instantiations compile to as many registers either way)
    const bool small = sizeof(TV) == 2 && msmall(L.A, mslices(L.A));
    const TV* av = (const TV*)(dia ? L.A.dval : L.A.val);
    MSched ms;
    const int gd = msched_of(L.A, ms);
    if (!pre)
      k_block_diag_m<B, TM, TIN, TX, TA><<<g, WG, 0, st>>>(L.nbr, K, (const TM*)L.M, r, z);
    if (dia)
      k_residual_m<B, TV, TX, TIN, TA, true><<<gd, WG, 0, st>>>(L.nbr, K, L.A.ptr, L.A.col, av,
                                                                r, z, t, L.A.dia, ms, 0);
    else if (small)
      k_residual_m<B, TV, TX, TIN, TA, false, true><<<ga, WG, 0, st>>>(
          L.nbr, K, L.A.ptr, L.A.col, av, r, z, t, DiaOffs{}, MSched{}, qa);
    else
      k_residual_m<B, TV, TX, TIN, TA, false, false><<<ga, WG, 0, st>>>(
          L.nbr, K, L.A.ptr, L.A.col, av, r, z, t, DiaOffs{}, MSched{}, qa);
    // a coarse level that is not the coarsest pre-smooths from a zero guess: the
    // restriction's launch does that product too
    const bool fold = l + 1 < nl - 1;
    if (fold)
      spmm_bd<B, TV, TX, TA, TM>(st, L.R, K, qr, t, (TX*)C.r, (const TM*)H.lv[l + 1].M,
                                 (TX*)C.z);
    else
      spmm<B, TV, TX, TA>(st, L.R, K, qr, t, (TX*)C.r, TA(0));
    TX* zc = (l + 1 == nl - 1) ? (TX*)C.z : (TX*)C.z2;
    run<TX, TX>(st, H, W, l + 1, K, (const TX*)C.r, zc, fold);
    spmm<B, TV, TX, TA>(st, L.P, K, qp, zc, z, TA(1));
    if (dia)
      k_smooth_m<B, TV, TX, TIN, TOUT, TM, TA, true><<<gd, WG, 0, st>>>(
          L.nbr, K, L.A.ptr, L.A.col, av, (const TM*)L.M, r, z, zout, L.A.dia, ms, 0);
    else if (small)
      k_smooth_m<B, TV, TX, TIN, TOUT, TM, TA, false, true><<<ga, WG, 0, st>>>(
          L.nbr, K, L.A.ptr, L.A.col, av, (const TM*)L.M, r, z, zout, DiaOffs{}, MSched{}, qa);
    else
      k_smooth_m<B, TV, TX, TIN, TOUT, TM, TA, false, false><<<ga, WG, 0, st>>>(
          L.nbr, K, L.A.ptr, L.A.col, av, (const TM*)L.M, r, z, zout, DiaOffs{}, MSched{}, qa);
  }
};

static void vcycle_m(mgk_solver* S, int K, const double* r, double* z) {
  hipStream_t st = S->dev.stream;
  DHier& H = S->H;
  MultiWork& W = *S->multi;
#define MGK_VCM(BB)                                                                     \
  case BB:                                                                              \
    if (H.storage == MGK_F64)                                                           \
      CycleM<BB, double, double>::run<double, double>(st, H, W, 0, K, r, z);            \
    else if (H.storage == MGK_F32)                                                      \
      CycleM<BB, float, float>::run<double, double>(st, H, W, 0, K, r, z);              \
    else                                                                                \
      CycleM<BB, bf16, float>::run<double, double>(st, H, W, 0, K, r, z);               \
    break;
  switch (H.b) {
    MGK_VCM(1)
    MGK_VCM(3)
    MGK_VCM(4)
    default: throw Error(MGK_E_INVALID, "unsupported block size");
  }
#undef MGK_VCM
}

// ---------------------------------------------------------------- outer products

static void outer_residual_m(mgk_solver* S, int K, const double* B, const double* X, double* R) {
  hipStream_t st = S->dev.stream;
  const DMat& A = S->A;
  const double* v = (const double*)A.val;
  const double* dv = (const double*)A.dval;
  const bool dia = A.dia.k > 0;
  MSched ms;
  const int gd = msched_of(A, ms);
  const MSched lin{};
  const int qa = mslices(A), ga = mgrid(S->nbr, qa);
  switch (S->b) {
    case 1: k_residual_m<1, double, double, double, double, false><<<ga, WG, 0, st>>>(S->nbr, K, A.ptr, A.col, v, B, X, R, DiaOffs{}, lin, qa); break;
    case 3:
      if (dia) k_residual_m<3, double, double, double, double, true><<<gd, WG, 0, st>>>(S->nbr, K, A.ptr, A.col, dv, B, X, R, A.dia, ms, 0);
      else k_residual_m<3, double, double, double, double, false><<<ga, WG, 0, st>>>(S->nbr, K, A.ptr, A.col, v, B, X, R, DiaOffs{}, lin, qa);
      break;
    case 4:
      if (dia) k_residual_m<4, double, double, double, double, true><<<gd, WG, 0, st>>>(S->nbr, K, A.ptr, A.col, dv, B, X, R, A.dia, ms, 0);
      else k_residual_m<4, double, double, double, double, false><<<ga, WG, 0, st>>>(S->nbr, K, A.ptr, A.col, v, B, X, R, DiaOffs{}, lin, qa);
      break;
  }
}

// Y = A X with per-column partials; returns the partial count.
static int outer_spmm_dot(mgk_solver* S, int K, const double* X, double* Y, int two,
                          const double* W1) {
  hipStream_t st = S->dev.stream;
  const int g = (S->nbr + MROWS - 1) / MROWS;
  const DMat& A = S->A;
  double* part = S->multi->part;
  // with time_spmv, the kernel's dispatch records its own start and end
  const bool timed = (S->time_mask & 1) && S->tev_used + 2 <= S->tev.size();
  hipEvent_t e0 = timed ? S->tev[S->tev_used] : nullptr;
  hipEvent_t e1 = timed ? S->tev[S->tev_used + 1] : nullptr;
  const double* v = (const double*)A.val;
  const double* dv = (const double*)A.dval;
  const DiaOffs no{};
  const bool dia = A.dia.k > 0;
  MSched ms;
  const int gd = msched_of(A, ms);
  const MSched lin{};
  switch (S->b) {
    case 1: launch_ev(k_spmm_dot<1, false>, g, st, e0, e1, S->nbr, K, A.ptr, A.col, v, X, Y, two, W1, part, no, lin); break;
    case 3:
      if (dia) launch_ev(k_spmm_dot<3, true>, gd, st, e0, e1, S->nbr, K, A.ptr, A.col, dv, X, Y, two, W1, part, A.dia, ms);
      else launch_ev(k_spmm_dot<3, false>, g, st, e0, e1, S->nbr, K, A.ptr, A.col, v, X, Y, two, W1, part, no, lin);
      break;
    case 4:
      if (dia) launch_ev(k_spmm_dot<4, true>, gd, st, e0, e1, S->nbr, K, A.ptr, A.col, dv, X, Y, two, W1, part, A.dia, ms);
      else launch_ev(k_spmm_dot<4, false>, g, st, e0, e1, S->nbr, K, A.ptr, A.col, v, X, Y, two, W1, part, no, lin);
      break;
  }
  if (timed) {
    HIPCK(hipGetLastError());
    S->tev_used += 2;
  }
  return g;
}

static int vec_grid(size_t n) {
  return (int)std::max<size_t>(1, std::min<size_t>((n + MROWS - 1) / MROWS, 1024));
}

static void finalize_m(mgk_solver* S, int K, int count, int two, int op, int i0 = 0,
                       int i1 = 0) {
  MultiWork& W = *S->multi;
  hipStream_t st = S->dev.stream;
  const double* src = W.part;
  if (count > MRED_CHUNK) {
    const int nb = (count + MRED_CHUNK - 1) / MRED_CHUNK;
    k_reduce_stage_m<<<nb, WG, 0, st>>>(W.part, count, two, W.part2);
    src = W.part2;
    count = nb;
  }
  k_finalize_m<<<K, WG, 0, st>>>(src, count, two, op, i0, i1, K, W.active, W.scm);
}

static void publish_m(mgk_solver* S) {
  MultiWork& W = *S->multi;
  HIPCK(hipMemcpyAsync(W.hsc, W.scm, sizeof(double) * SM_COUNT * KL, hipMemcpyDeviceToHost,
                       S->dev.stream));
  HIPCK(hipEventRecord(W.ev, S->dev.stream));
  HIPCK(hipEventSynchronize(W.ev));
  HIPCK(hipGetLastError());
}

static void push_flags(mgk_solver* S) {
  MultiWork& W = *S->multi;
  int* slot = W.hflags + (size_t)W.flag_slot * 2 * KL;
  W.flag_slot = (W.flag_slot + 1) % FLAG_SLOTS;
  std::memcpy(slot, W.act, sizeof(int) * KL);
  std::memcpy(slot + KL, W.msk, sizeof(int) * KL);
  HIPCK(hipMemcpyAsync(W.active, slot, sizeof(int) * KL, hipMemcpyHostToDevice, S->dev.stream));
  HIPCK(hipMemcpyAsync(W.mask, slot + KL, sizeof(int) * KL, hipMemcpyHostToDevice,
                       S->dev.stream));
}

__global__ void k_set_scalars_m(int K, const int* __restrict__ mask, double* __restrict__ scm) {
  const int k = threadIdx.x;
  if (k >= K || !mask[k]) return;
  scm[SM_RHO * KL + k] = 1.0;
  scm[SM_ALPHA * KL + k] = 1.0;
  scm[SM_OMEGA * KL + k] = 1.0;
}

__global__ void k_zero_cols_m(size_t n, int K, const int* __restrict__ mask,
                              double* __restrict__ x) {
  const int k = threadIdx.x % KL;
  if (k >= K || !mask[k]) return;
  MROW_STRIDE(row, n) x[row * K + k] = 0.0;
}

// ---------------------------------------------------------------- lockstep BiCGStab

static int bicgstab_multi(mgk_solver* S, int K, const double* B, double* X, double tol,
                          mgk_info* infos) {
  MultiWork& W = *ensure_multi(S);
  hipStream_t st = S->dev.stream;
  const size_t n = S->n;
  const int gv = vec_grid(n);
  int* act = W.act;
  int* msk = W.msk;
  double* hs = W.hsc;
  auto sc = [&](int idx, int k) { return hs[idx * KL + k]; };

  // ||b_k||
  k_dot_m<<<gv, WG, 0, st>>>(n, K, B, B, nullptr, nullptr, W.part);
  for (int k = 0; k < KL; ++k) act[k] = msk[k] = 0;
  for (int k = 0; k < K; ++k) act[k] = 1;
  push_flags(S);
  finalize_m(S, K, gv, 0, FINM_STORE1, SM_NB);
  publish_m(S);
  std::vector<double> nb(K), tol2(K);
  std::vector<int> iters(K, 0), restarts(K, 0), done(K, 0);
  for (int k = 0; k < K; ++k) {
    nb[k] = std::sqrt(sc(SM_NB, k));
    tol2[k] = (tol * nb[k]) * (tol * nb[k]);
    msk[k] = nb[k] == 0.0;
  }
  for (int k = 0; k < K; ++k)
    if (nb[k] == 0.0) {
      act[k] = 0;
      done[k] = 1;
    }
  push_flags(S);
  k_zero_cols_m<<<gv, WG, 0, st>>>(n, K, W.mask, X);
  int it = 0;
  const int maxit = S->prm.maxiter;
  for (int round = 0;; ++round) {
    // (re)start every column that is still active
    for (int k = 0; k < K; ++k) msk[k] = act[k];
    push_flags(S);
    outer_residual_m(S, K, B, X, W.r);
    k_restart_m<<<gv, WG, 0, st>>>(n, K, W.mask, W.r, W.rh, W.p, W.v);
    k_set_scalars_m<<<1, KL, 0, st>>>(K, W.mask, W.scm);
    k_dot_m<<<gv, WG, 0, st>>>(n, K, W.r, W.r, W.rh, W.r, W.part);
    finalize_m(S, K, gv, 1, FINM_STORE2, SM_RR, SM_RHO1);
    publish_m(S);
    for (int k = 0; k < K; ++k)
      if (act[k] && sc(SM_RR, k) <= tol2[k]) act[k] = 0;
    push_flags(S);
    auto any_active = [&]() {
      for (int k = 0; k < K; ++k)
        if (act[k]) return true;
      return false;
    };
    while (any_active() && it < maxit) {
      bool changed = false;
      for (int k = 0; k < K; ++k)
        if (act[k] && sc(SM_RHO1, k) == 0.0) {
          act[k] = 0;   // breakdown: restarted in the next round
          changed = true;
        }
      if (changed) push_flags(S);
      if (!any_active()) break;
      ++it;
      for (int k = 0; k < K; ++k) iters[k] += act[k];
      k_bicg_p_m<<<gv, WG, 0, st>>>(n, K, W.active, W.scm, W.r, W.v, W.p);
      vcycle_m(S, K, W.p, W.ph);
      int g1 = outer_spmm_dot(S, K, W.ph, W.v, 0, W.rh);
      finalize_m(S, K, g1, 0, FINM_ALPHA);
      k_bicg_s_m<<<gv, WG, 0, st>>>(n, K, W.active, W.scm, W.r, W.v, W.s, W.part);
      finalize_m(S, K, gv, 0, FINM_STORE1, SM_SS);
      publish_m(S);
      changed = false;
      for (int k = 0; k < K; ++k) {
        msk[k] = act[k] && sc(SM_SS, k) <= tol2[k];
        if (msk[k]) {
          act[k] = 0;   // stops at s: x_k += alpha_k phat_k below
          changed = true;
        }
      }
      if (changed) {
        push_flags(S);
        k_bicg_x_m<<<gv, WG, 0, st>>>(n, K, W.mask, W.scm, W.ph, X);
      }
      if (!any_active()) break;
      vcycle_m(S, K, W.s, W.sh);
      int g2 = outer_spmm_dot(S, K, W.sh, W.t, 1, W.s);
      finalize_m(S, K, g2, 1, FINM_OMEGA);
      k_bicg_xr_m<<<gv, WG, 0, st>>>(n, K, W.active, W.scm, W.s, W.t, W.ph, W.sh, W.rh, X,
                                      W.r, W.part);
      finalize_m(S, K, gv, 1, FINM_RHO);
      publish_m(S);
      changed = false;
      for (int k = 0; k < K; ++k)
        if (act[k] && (sc(SM_RR, k) <= tol2[k] || sc(SM_TT, k) == 0.0)) {
          act[k] = 0;
          changed = true;
        }
      if (changed) push_flags(S);
    }
    // true residuals of every column
    outer_residual_m(S, K, B, X, W.r);
    k_dot_m<<<gv, WG, 0, st>>>(n, K, W.r, W.r, nullptr, nullptr, W.part);
    finalize_m(S, K, gv, 0, FINM_STORE1, SM_RR);
    publish_m(S);
    bool again = false;
    for (int k = 0; k < K; ++k) {
      if (done[k]) continue;
      const double rel = std::sqrt(sc(SM_RR, k)) / nb[k];
      infos[k].rel_resid = rel;
      if (rel <= tol) {
        done[k] = 1;
        act[k] = 0;
      } else if (it < maxit && restarts[k] < S->prm.max_restarts) {
        act[k] = 1;
        restarts[k] += 1;
        again = true;
      } else {
        act[k] = 0;
      }
    }
    if (!again) break;
  }
  int worst = MGK_OK;
  for (int k = 0; k < K; ++k) {
    infos[k].iters = iters[k];
    infos[k].restarts = restarts[k];
    infos[k].status = done[k] ? MGK_OK : MGK_NOT_CONVERGED;
    if (nb[k] == 0.0) infos[k].rel_resid = 0.0;
    if (!done[k]) worst = MGK_NOT_CONVERGED;
  }
  return worst;
}

}  // namespace mgk

extern "C" int mgk_solve_multi(mgk_solver* s, int32_t nrhs, const double* d_B, double* d_X,
                               double rtol, mgk_info* infos) {
  if (!s || !d_B || !d_X || !infos || nrhs < 1 || nrhs > mgk::KL || !(rtol > 0.0)) {
    mgk::g_err = "mgk_solve_multi: need 1 <= nrhs <= 32, non-null arguments, rtol > 0";
    return MGK_E_INVALID;
  }
  if (s->host_only || s->batch || s->kind == MGK_SCHUR || s->kind == MGK_ILU ||
      s->prm.ilu_smoother) {
    mgk::g_err = "mgk_solve_multi: needs a monolithic AMG solver with device data";
    return MGK_E_STATE;
  }
  return mgk::guard([&]() -> int {
    auto t0 = std::chrono::steady_clock::now();
    std::memset(infos, 0, sizeof(mgk_info) * nrhs);
    s->tev_used = 0;
    const int rc = mgk::bicgstab_multi(s, nrhs, d_B, d_X, rtol, infos);
    HIPCK(hipStreamSynchronize(s->dev.stream));
    HIPCK(hipGetLastError());
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    double spmm_ms = 0.0;   // the outer SpMM launches (time_spmv bit 1)
    for (size_t e = 0; e + 1 < s->tev_used; e += 2) {
      float t = 0.0f;
      HIPCK(hipEventElapsedTime(&t, s->tev[e], s->tev[e + 1]));
      spmm_ms += t;
    }
    for (int k = 0; k < nrhs; ++k) {
      infos[k].levels = (int)s->H.lv.size();
      infos[k].setup_ms = s->setup_ms;
      infos[k].solve_ms = ms;
      infos[k].device_bytes = s->dev.bytes + s->multi->bytes;
      infos[k].spmv_ms = spmm_ms;
      infos[k].spmv_calls = (int32_t)(s->tev_used / 2);
    }
    return rc;
  });
}
