// IDR(s) outer solver on the device: induced dimension reduction with residual
// updates kept biorthogonal to an s-dimensional shadow space (van Gijzen and
// Sonneveld, ACM TOMS 38, 2011), right preconditioned, FP64 vectors.  The paper's
// own outer solver is IDR(5) (Section 4, table of solver variants).
//
// Per inner step k (k = 0 .. s-1) of a cycle:
//   c   = M(k:s, k:s)^-1 f(k:s)                  lower triangular, on the device
//   v   = r - sum_{i>=k} c_i G_i
//   U_k = omega K^-1 v + sum_{i>=k} c_i U_i,      G_k = A U_k
//   G_k, U_k -= sum_{i<k} alpha_i (G_i, U_i)      alpha = M(0:k, 0:k)^-1 P(0:k)^T G_k
//   M(:, k) = P^T G_k,  beta = f_k / M_kk,  r -= beta G_k,  x += beta U_k,
//   f(k+1:s) -= beta M(k+1:s, k)
// then one dimension-reduction step: t = A K^-1 r, omega = (t, r) / (t, t)
// (enlarged when |cos(t, r)| < 0.7), r -= omega t, x += omega K^-1 r.
//
// One pass of shadow dots d = P^T G_k per inner step serves the whole step: the
// orthogonalization against the first k shadow vectors solves for all alpha_i
// at once (a forward substitution with the stored lower triangle of M, which is
// the sequential projection of the algorithm written in one pass), and the new
// column of M follows as M(i, k) = d_i - sum_j alpha_j M(i, j).
// Every scalar stays in device memory.  The convergence flag of step j is read
// through pinned memory while the preconditioner and SpMV of step j+1, which do
// not touch x or r, are already queued.
#include "internal.hpp"

namespace mgk {

namespace {

// Device scalar slots.
constexpr int I_F = 0;                          // f[s]
constexpr int I_C = I_F + IDR_MAX_S;            // c[s]
constexpr int I_A = I_C + IDR_MAX_S;            // alpha[s]
constexpr int I_D = I_A + IDR_MAX_S;            // dots[s]
constexpr int I_X = I_D + IDR_MAX_S;            // scratch[s]
constexpr int I_M = I_X + IDR_MAX_S;            // M[s][s], row-major, IDR_MAX_S stride
constexpr int I_OM = I_M + IDR_MAX_S * IDR_MAX_S;
constexpr int I_BETA = I_OM + 1;
constexpr int I_RR = I_BETA + 1;                // ||r||^2   (published)
constexpr int I_BRK = I_RR + 1;                 // breakdown flag (published)
constexpr int I_TR = I_BRK + 1;
constexpr int I_TT = I_TR + 1;
constexpr int I_COUNT = I_TT + 1;
constexpr int RING = 2;

__device__ __forceinline__ double& Mat(double* d, int i, int j) {
  return d[I_M + i * IDR_MAX_S + j];
}

// M = I, omega = 1, flags cleared.
__global__ void k_idr_reset(int s, double* __restrict__ d) {
  for (int q = threadIdx.x; q < I_COUNT; q += blockDim.x) d[q] = 0.0;
  __syncthreads();
  if (threadIdx.x < s) Mat(d, threadIdx.x, threadIdx.x) = 1.0;
  if (threadIdx.x == 0) d[I_OM] = 1.0;
}

// c(k:s) = M(k:s, k:s)^-1 f(k:s) (forward substitution).
__global__ void k_idr_coef(int s, int k, double* __restrict__ d) {
  if (threadIdx.x != 0) return;
  for (int i = k; i < s; ++i) {
    double a = d[I_F + i];
    for (int j = k; j < i; ++j) a = a - Mat(d, i, j) * d[I_C + j];
    d[I_C + i] = a / Mat(d, i, i);
  }
}

// From the shadow dots d = P^T G_k of the new direction (before it is made
// orthogonal to p_0 .. p_{k-1}):
//   alpha(0:k) = M(0:k, 0:k)^-1 d(0:k)                  (forward substitution)
//   M(i, k) = d_i - sum_{j<k} alpha_j M(i, j), i >= k    (= p_i^T of the orthogonalized G_k,
//                                                          since M(i, j) = p_i^T G_j)
//   beta = f_k / M_kk (breakdown: beta = 0, flag set); f(k+1:s) -= beta M(k+1:s, k).
__global__ void k_idr_proj(int s, int k, double* __restrict__ d) {
  if (threadIdx.x != 0) return;
  for (int i = 0; i < k; ++i) {
    double a = d[I_D + i];
    for (int j = 0; j < i; ++j) a = a - Mat(d, i, j) * d[I_A + j];
    d[I_A + i] = a / Mat(d, i, i);
  }
  for (int i = k; i < s; ++i) {
    double m = d[I_D + i];
    for (int j = 0; j < k; ++j) m = m - d[I_A + j] * Mat(d, i, j);
    Mat(d, i, k) = m;
  }
  const double mkk = Mat(d, k, k);
  if (mkk == 0.0) {
    d[I_BETA] = 0.0;
    d[I_BRK] = 1.0;
    return;
  }
  const double beta = d[I_F + k] / mkk;
  d[I_BETA] = beta;
  for (int i = k + 1; i < s; ++i) d[I_F + i] = d[I_F + i] - beta * Mat(d, i, k);
}

// omega = (t, r) / (t, t), enlarged when |cos(t, r)| < 0.7; breakdown: omega = 0.
__global__ void k_idr_omega(double* __restrict__ d) {
  if (threadIdx.x != 0) return;
  const double tr = d[I_TR], tt = d[I_TT];
  const double rho = fabs(tr) / (sqrt(tt) * sqrt(d[I_RR]));
  if (tt == 0.0 || rho == 0.0 || !(rho == rho)) {
    d[I_OM] = 0.0;
    d[I_BRK] = 1.0;
    return;
  }
  double om = tr / tt;
  if (rho < 0.7) om = om * 0.7 / rho;
  d[I_OM] = om;
}

// v = r - sum_{i=k}^{s-1} c_i G_i.
__global__ __launch_bounds__(WG) void k_idr_v(size_t n, int s, int k, const double* __restrict__ r,
                                              const double* __restrict__ G,
                                              const double* __restrict__ d,
                                              double* __restrict__ v) {
  GRID_STRIDE(q, n) {
    double a = r[q];
    for (int i = k; i < s; ++i) a = a - d[I_C + i] * G[(size_t)i * n + q];
    v[q] = a;
  }
}

// U_k = omega vh + sum_{i=k}^{s-1} c_i U_i (the old U_k enters the sum).
__global__ __launch_bounds__(WG) void k_idr_u(size_t n, int s, int k, const double* __restrict__ vh,
                                              const double* __restrict__ d,
                                              double* __restrict__ U) {
  const double om = d[I_OM];
  GRID_STRIDE(q, n) {
    double a = om * vh[q];
    for (int i = k; i < s; ++i) a = a + d[I_C + i] * U[(size_t)i * n + q];
    U[(size_t)k * n + q] = a;
  }
}

// G_k -= sum_{i<k} alpha_i G_i; U_k -= sum_{i<k} alpha_i U_i.
__global__ __launch_bounds__(WG) void k_idr_orth(size_t n, int k, const double* __restrict__ d,
                                                 double* __restrict__ G, double* __restrict__ U) {
  GRID_STRIDE(q, n) {
    double g = G[(size_t)k * n + q], u = U[(size_t)k * n + q];
    for (int i = 0; i < k; ++i) {
      const double a = d[I_A + i];
      g = g - a * G[(size_t)i * n + q];
      u = u - a * U[(size_t)i * n + q];
    }
    G[(size_t)k * n + q] = g;
    U[(size_t)k * n + q] = u;
  }
}

// r -= coef gv; x += coef uv; partial ||r||^2 per workgroup (coef = d[slot]).
__global__ __launch_bounds__(WG) void k_idr_update(size_t n, const double* __restrict__ gv,
                                                   const double* __restrict__ uv,
                                                   const double* __restrict__ d, int slot,
                                                   double* __restrict__ r, double* __restrict__ x,
                                                   double* __restrict__ part) {
  const double cf = d[slot];
  double ss = 0.0, dummy = 0.0;
  GRID_STRIDE(q, n) {
    const double ri = r[q] - cf * gv[q];
    r[q] = ri;
    x[q] = x[q] + cf * uv[q];
    ss = fma_(ri, ri, ss);
  }
  wg_sum2(ss, dummy);
  if (threadIdx.x == 0) part[blockIdx.x] = ss;
}

// ---- shadow space ----------------------------------------------------------------

// SplitMix64 (Steele, Lea and Flood, 2014), output number c from state 0, top 53
// bits mapped to [-1, 1).
double splitmix64_unit(uint64_t c) {
  uint64_t z = (c + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

// n x s shadow space (column j = entries j*n .. j*n+n-1 of the sequence), made
// orthonormal by modified Gram-Schmidt in column order; FP64 on the host.
std::vector<double> shadow_space(size_t n, int s) {
  std::vector<double> P(n * (size_t)s);
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < (int64_t)(n * s); ++q) P[q] = splitmix64_unit((uint64_t)q);
  for (int j = 0; j < s; ++j) {
    double* pj = &P[(size_t)j * n];
    for (int i = 0; i < j; ++i) {
      const double* pi = &P[(size_t)i * n];
      double dd = 0.0;
      for (size_t q = 0; q < n; ++q) dd = dd + pi[q] * pj[q];
      for (size_t q = 0; q < n; ++q) pj[q] = pj[q] - dd * pi[q];
    }
    double nn = 0.0;
    for (size_t q = 0; q < n; ++q) nn = nn + pj[q] * pj[q];
    nn = std::sqrt(nn);
    for (size_t q = 0; q < n; ++q) pj[q] = pj[q] / nn;
  }
  return P;
}

}  // namespace

struct IdrWork {
  int s = 0;
  size_t n = 0;
  double *P = nullptr, *G = nullptr, *U = nullptr;
  double* d = nullptr;      // device scalars
  double* hp = nullptr;     // pinned ring: RING x (||r||^2, breakdown)
  hipEvent_t ev[RING] = {nullptr, nullptr};
  ~IdrWork() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (hp) (void)hipHostFree(hp);
  }
};

IdrWork* idr_create(mgk_solver* S) {
  auto* w = new IdrWork();
  try {
    w->s = S->prm.idr_s;
    w->n = S->n;
    const size_t nb = sizeof(double) * w->n * w->s;
    w->P = (double*)S->dev.alloc(nb);
    w->G = (double*)S->dev.alloc(nb);
    w->U = (double*)S->dev.alloc(nb);
    w->d = (double*)S->dev.alloc(sizeof(double) * I_COUNT);
    const std::vector<double> P = shadow_space(w->n, w->s);
    HIPCK(hipMemcpyAsync(w->P, P.data(), nb, hipMemcpyHostToDevice, S->dev.stream));
    HIPCK(hipStreamSynchronize(S->dev.stream));
    HIPCK(hipHostMalloc((void**)&w->hp, sizeof(double) * 2 * RING, hipHostMallocDefault));
    for (auto& e : w->ev) HIPCK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  } catch (...) {
    delete w;
    throw;
  }
  return w;
}

void idr_free(IdrWork* w) { delete w; }

int idrs(mgk_solver* S, const double* b, double* x, double tol, bool trans, mgk_info* info) {
  IdrWork& W = *S->idr;
  hipStream_t st = S->dev.stream;
  const size_t n = S->n;
  const int s = W.s, g = grid_for(n);
  double* d = W.d;
  double *r = S->r, *v = S->v, *vh = S->ph, *t = S->t;
  const double nb = norm2(S, b);
  info->iters = 0;
  info->restarts = 0;
  if (nb == 0.0) {
    k_fill<<<g, WG, 0, st>>>(n, 0.0, x);
    info->rel_resid = 0.0;
    return MGK_OK;
  }
  const double tol2 = (tol * nb) * (tol * nb);
  const int maxiter = S->prm.maxiter;
  int slot = 0;
  auto publish = [&]() {
    HIPCK(hipMemcpyAsync(W.hp + 2 * slot, d + I_RR, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
    HIPCK(hipEventRecord(W.ev[slot], st));
    const int mine = slot;
    slot = (slot + 1) % RING;
    return mine;
  };
  auto wait = [&](int e) {
    HIPCK(hipEventSynchronize(W.ev[e]));
    HIPCK(hipGetLastError());
    return std::make_pair(W.hp[2 * e], W.hp[2 * e + 1]);
  };
  auto rnorm = [&]() {
    k_dot2<<<g, WG, 0, st>>>(n, r, r, nullptr, nullptr, S->part);
    finalize(S, g, 0, FIN_STORE1, I_RR, 0, d);
  };
  // shadow dots of w into d[slot0 .. slot0+m)
  auto pdots = [&](int m, const double* w, int slot0) {
    multidot(st, g, n, m, W.P, n, w, S->part);
    k_multifin<<<1, WG, 0, st>>>(S->part, g, m, d + slot0, d + I_X, 0);
  };

  int it = 0;
  for (int restart = 0;; ++restart) {
    outer_residual(S, b, x, r, trans);
    k_fill<<<g, WG, 0, st>>>(n * s, 0.0, W.G);
    k_fill<<<g, WG, 0, st>>>(n * s, 0.0, W.U);
    k_idr_reset<<<1, 64, 0, st>>>(s, d);
    rnorm();
    auto st0 = wait(publish());
    bool done = st0.first <= tol2, brk = false;
    int pending = -1;   // ring slot of the last unchecked residual update
    // Queue the part of an inner step that leaves x and r alone.
    auto inner_pre = [&](int k) {
      double* Gk = W.G + (size_t)k * n;
      double* Uk = W.U + (size_t)k * n;
      k_idr_coef<<<1, 64, 0, st>>>(s, k, d);
      k_idr_v<<<g, WG, 0, st>>>(n, s, k, r, W.G, d, v);
      precond(S, v, vh, trans);
      k_idr_u<<<g, WG, 0, st>>>(n, s, k, vh, d, W.U);
      outer_spmv(S, Uk, Gk, trans);
      pdots(s, Gk, I_D);
      k_idr_proj<<<1, 64, 0, st>>>(s, k, d);
      if (k > 0) k_idr_orth<<<g, WG, 0, st>>>(n, k, d, W.G, W.U);
    };
    auto reduce_pre = [&]() {
      precond(S, r, vh, trans);
      int nw = 0;
      outer_spmv(S, vh, t, trans, 2, r, &nw);   // partials (r, t), (t, t)
      finalize(S, nw, 1, FIN_STORE2, I_TR, I_TT, d);
      k_idr_omega<<<1, 64, 0, st>>>(d);
    };
    // Check the pending update (if any); true when the iteration must stop.
    auto check = [&]() {
      if (pending < 0) return false;
      auto res = wait(pending);
      pending = -1;
      if (res.second != 0.0) brk = true;
      if (res.first <= tol2) done = true;
      return done || brk;
    };
    while (!done && !brk && it < maxiter) {
      pdots(s, r, I_F);   // f = P^T r (queued after the last update)
      for (int k = 0; k < s; ++k) {
        inner_pre(k);
        if (check()) break;
        k_idr_update<<<g, WG, 0, st>>>(n, W.G + (size_t)k * n, W.U + (size_t)k * n, d, I_BETA, r,
                                      x, S->part);
        finalize(S, g, 0, FIN_STORE1, I_RR, 0, d);
        pending = publish();
        if (++it >= maxiter) break;
      }
      if (done || brk || it >= maxiter) break;
      // dimension reduction
      reduce_pre();
      if (check()) break;
      k_idr_update<<<g, WG, 0, st>>>(n, t, vh, d, I_OM, r, x, S->part);
      finalize(S, g, 0, FIN_STORE1, I_RR, 0, d);
      pending = publish();
      ++it;
    }
    check();
    // true residual
    outer_residual(S, b, x, r, trans);
    const double rn = norm2(S, r);
    info->rel_resid = rn / nb;
    info->iters = it;
    info->restarts = restart;
    if (info->rel_resid <= tol) return MGK_OK;
    if (it >= maxiter || restart >= S->prm.max_restarts) return MGK_NOT_CONVERGED;
  }
}

}  // namespace mgk
