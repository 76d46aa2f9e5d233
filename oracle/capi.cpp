// C entry points of the oracle, loaded by the tests through ctypes.
// TEST INFRASTRUCTURE ONLY (see oracle.hpp).
#include <omp.h>

#include <cstring>
#include <exception>
#include <memory>
#include <string>
#include "oracle.hpp"

using namespace orc;

namespace {
thread_local std::string g_err;

struct Identity : Precond {
  i64 n;
  explicit Identity(i64 n_) : n(n_) {}
  void apply(const double* r, double* z) const override { std::memcpy(z, r, sizeof(double) * n); }
};
struct AmgPre : Precond {
  const Hierarchy* H;
  explicit AmgPre(const Hierarchy* h) : H(h) {}
  void apply(const double* r, double* z) const override { vcycle(*H, 0, r, z); }
};
struct IluPre : Precond {
  const Ilu* F;
  explicit IluPre(const Ilu* f) : F(f) {}
  void apply(const double* r, double* z) const override { ilu_apply(*F, r, z); }
};
struct SchurPre : Precond {
  const Schur* S;
  explicit SchurPre(const Schur* s) : S(s) {}
  void apply(const double* r, double* z) const override { schur_apply(*S, r, z); }
};

Csr make_csr(i64 nr, i64 nc, const i64* ptr, const i32* col, const double* val) {
  Csr A;
  A.nr = nr;
  A.nc = nc;
  A.ptr.assign(ptr, ptr + nr + 1);
  A.col.assign(col, col + ptr[nr]);
  A.val.assign(val, val + ptr[nr]);
  return A;
}
}  // namespace

extern "C" {

struct orc_params {
  int32_t krylov;        // 0 BiCGStab, 1 FGMRES
  int32_t fgmres_m;
  int32_t maxiter;
  int32_t max_restarts;
  double eps_strong;
  int32_t coarse_enough;
  int32_t max_levels;
  int32_t smoother;      // 0 block SPAI0, 1 damped Jacobi, 2 scalar SPAI0, 3 block ILU(0)
  int32_t kind;          // 0 monolithic AMG, 1 Schur pressure correction, 2 identity
  double jacobi_omega;
  int32_t coarsening;    // 0 smoothed aggregation, 1 plain aggregation
  int32_t schur_approx;  // 1: diagonal-only Schur approximation
  int32_t schur_spai0;   // 1: SPAI(0) pressure step
  int32_t schur_lower;   // 1: lower block factorization
  int32_t idr_s;         // shadow space dimension of IDR(s)
  int32_t ilu_level;     // fill level of the block ILU(k) preconditioner (kind 3)
  int32_t ilu_sweeps;    // Jacobi sweeps per triangular factor
  int32_t schur_scalar_u;  // 1: Schur velocity AMG on scalar values
  int32_t ilu_kind;      // kind 3: 0 block ILU(k), 1 block ILUT(p, tau)
  double ilut_p;
  double ilut_tau;
};

struct orc_info {
  int32_t iters, restarts, converged, pad;
  double rel_resid;
};

struct orc_solver {
  Csr A;
  int b = 1;
  orc_params prm;
  AmgParams aprm;
  Hierarchy H, Ht;
  bool have_t = false;
  Schur S;
  Ilu F;
};

const char* orc_last_error(void) { return g_err.c_str(); }

int64_t orc_stokes_nnz(int n) { return stokes_nnz(n); }

int orc_stokes_assemble(int n, const double* theta, int64_t* ptr, int32_t* col, double* val) {
  if (n < 3) return -1;
  Csr A;
  stokes_assemble(n, theta, A);
  std::memcpy(ptr, A.ptr.data(), sizeof(int64_t) * (A.nr + 1));
  std::memcpy(col, A.col.data(), sizeof(int32_t) * A.col.size());
  std::memcpy(val, A.val.data(), sizeof(double) * A.val.size());
  return 0;
}

int orc_theta_grad(int n, const double* lambda, const double* x, double* g) {
  theta_gradient(n, lambda, x, g);
  return 0;
}

int orc_spmv(int64_t nr, int64_t nc, const int64_t* ptr, const int32_t* col, const double* val,
             const double* x, double* y) {
  Csr A = make_csr(nr, nc, ptr, col, val);
  spmv(A, x, y);
  return 0;
}

orc_solver* orc_setup(int64_t nr, const int64_t* ptr, const int32_t* col, const double* val,
                      int block, const orc_params* prm) {
  try {
    auto s = std::make_unique<orc_solver>();
    s->A = make_csr(nr, nr, ptr, col, val);
    s->b = block;
    s->prm = *prm;
    s->aprm.eps_strong = prm->eps_strong;
    s->aprm.coarse_enough = prm->coarse_enough;
    s->aprm.max_levels = prm->max_levels;
    s->aprm.smoother = prm->smoother;
    s->aprm.jacobi_omega = prm->jacobi_omega;
    s->aprm.smooth_p = prm->coarsening == 0;
    s->aprm.ilu_sweeps = prm->ilu_sweeps;
    s->aprm.ilut_p = prm->ilut_p;
    s->aprm.ilut_tau = prm->ilut_tau;
    if (prm->krylov == 2 && (prm->idr_s < 1 || prm->idr_s > 32)) {
      g_err = "oracle: IDR(s) needs 1 <= s <= 32";
      return nullptr;
    }
    const char* msg = nullptr;
    if (prm->kind == 0) {
      if (!amg_build(s->A, block, s->aprm, s->H, &msg)) {
        g_err = msg ? msg : "oracle: setup failed";
        return nullptr;
      }
    } else if (prm->kind == 3) {
      if (prm->ilu_level < 0 || prm->ilu_level > 1 || prm->ilu_sweeps < 0) {
        g_err = "oracle: ILU(k) needs k in {0, 1} and sweeps >= 0";
        return nullptr;
      }
      const bool ok = prm->ilu_kind == 1
                          ? ilut_build(s->A, block, prm->ilut_p, prm->ilut_tau, prm->ilu_sweeps,
                                       s->F, &msg)
                          : ilu_build(s->A, block, prm->ilu_level, prm->ilu_sweeps, s->F, &msg);
      if (!ok) {
        g_err = msg ? msg : "oracle: ILU setup failed";
        return nullptr;
      }
    } else if (prm->kind == 1) {
      if (block != 4) {
        g_err = "oracle: Schur needs interleaved 4-component unknowns";
        return nullptr;
      }
      SchurOptions so;
      so.diag_approx = prm->schur_approx != 0;
      so.spai0_p = prm->schur_spai0 != 0;
      so.lower = prm->schur_lower != 0;
      so.scalar_u = prm->schur_scalar_u != 0;
      if (!schur_build(s->A, s->aprm, so, s->S, &msg)) {
        g_err = msg ? msg : "oracle: Schur setup failed";
        return nullptr;
      }
    }
    return s.release();
  } catch (const std::exception& e) {
    g_err = e.what();
    return nullptr;
  }
}

void orc_free(orc_solver* s) { delete s; }

static const Hierarchy* pick(orc_solver* s, int which) {
  if (s->prm.kind == 0) return which == 0 ? &s->H : (which == 2 && s->have_t ? &s->Ht : nullptr);
  if (s->prm.kind == 1)
    return which == 0 ? &s->S.Hu : (which == 1 && !s->S.Hp.levels.empty() ? &s->S.Hp : nullptr);
  return nullptr;
}

int orc_nlevels(orc_solver* s, int which) {
  const Hierarchy* H = pick(s, which);
  return H ? (int)H->levels.size() : -1;
}

// out: [A rows, A nnz, P cols, P nnz, R nnz, n_agg, block]
int orc_level_sizes(orc_solver* s, int which, int l, int64_t* out) {
  const Hierarchy* H = pick(s, which);
  if (!H || l < 0 || l >= (int)H->levels.size()) return -1;
  const Level& L = H->levels[l];
  out[0] = L.A.nr;
  out[1] = (int64_t)L.A.col.size();
  out[2] = L.P.nc;
  out[3] = (int64_t)L.P.col.size();
  out[4] = (int64_t)L.R.col.size();
  out[5] = L.n_agg;
  out[6] = H->b;
  return 0;
}

int orc_level_get(orc_solver* s, int which, int l, int mat, int64_t* ptr, int32_t* col, double* val) {
  const Hierarchy* H = pick(s, which);
  if (!H || l < 0 || l >= (int)H->levels.size()) return -1;
  const Level& L = H->levels[l];
  const Csr& M = mat == 0 ? L.A : (mat == 1 ? L.P : L.R);
  std::memcpy(ptr, M.ptr.data(), sizeof(int64_t) * M.ptr.size());
  std::memcpy(col, M.col.data(), sizeof(int32_t) * M.col.size());
  std::memcpy(val, M.val.data(), sizeof(double) * M.val.size());
  return 0;
}

int orc_level_agg(orc_solver* s, int which, int l, int32_t* agg, double* omega) {
  const Hierarchy* H = pick(s, which);
  if (!H || l < 0 || l >= (int)H->levels.size()) return -1;
  const Level& L = H->levels[l];
  const i64 nn = L.A.nr / H->b;
  for (i64 i = 0; i < nn; ++i) agg[i] = L.agg.empty() ? -1 : L.agg[i];
  *omega = L.omega;
  return 0;
}

int orc_level_smoother(orc_solver* s, int which, int l, double* M) {
  const Hierarchy* H = pick(s, which);
  if (!H || l < 0 || l >= (int)H->levels.size()) return -1;
  std::memcpy(M, H->levels[l].M.data(), sizeof(double) * H->levels[l].M.size());
  return 0;
}

static int ensure_transposed(orc_solver* s) {
  if (s->have_t) return 0;
  if (s->prm.kind != 0) {
    g_err = "oracle: transposed solves need the monolithic AMG";
    return -1;
  }
  const char* msg = nullptr;
  if (!amg_transpose(s->H, s->Ht, &msg)) {
    g_err = msg;
    return -1;
  }
  s->have_t = true;
  return 0;
}

int orc_precond(orc_solver* s, const double* r, double* z, int transposed) {
  if (transposed && ensure_transposed(s)) return -1;
  if (s->prm.kind == 0) {
    vcycle(transposed ? s->Ht : s->H, 0, r, z);
  } else if (s->prm.kind == 1) {
    schur_apply(s->S, r, z);
  } else if (s->prm.kind == 3) {
    ilu_apply(s->F, r, z);
  } else {
    std::memcpy(z, r, sizeof(double) * s->A.nr);
  }
  return 0;
}

int orc_solve(orc_solver* s, const double* b, double* x, double tol, int transposed, orc_info* info) {
  if (transposed && ensure_transposed(s)) return -1;
  Csr At;
  const Csr* A = &s->A;
  if (transposed) {
    At = transpose(s->A);
    A = &At;
  }
  std::unique_ptr<Precond> M;
  if (s->prm.kind == 0) M.reset(new AmgPre(transposed ? &s->Ht : &s->H));
  else if (s->prm.kind == 1) M.reset(new SchurPre(&s->S));
  else if (s->prm.kind == 3) M.reset(new IluPre(&s->F));
  else M.reset(new Identity(s->A.nr));
  SolveInfo si;
  if (s->prm.krylov == 0)
    bicgstab(*A, *M, b, x, tol, s->prm.maxiter, s->prm.max_restarts, si);
  else if (s->prm.krylov == 1)
    fgmres(*A, *M, b, x, tol, s->prm.fgmres_m, s->prm.maxiter, si);
  else
    idrs(*A, *M, b, x, tol, s->prm.idr_s, s->prm.maxiter, s->prm.max_restarts, si);
  info->iters = si.iters;
  info->restarts = si.restarts;
  info->converged = si.converged;
  info->rel_resid = si.rel_resid;
  return si.converged ? 0 : 1;
}

}  // extern "C"

// Combined ILU factor as scalar CSR (block entries expanded, zeros kept):
// returns the number of entries, fills ptr/col/val when they are non-null.
extern "C" int64_t orc_ilu_factor(orc_solver* s, int64_t* ptr, int32_t* col, double* val) {
  const Ilu& F = s->F;
  const int b = F.b;
  int64_t nz = 0;
  for (i64 i = 0; i < F.nn; ++i)
    for (int r = 0; r < b; ++r) {
      if (ptr) ptr[i * b + r] = nz;
      for (size_t t = 0; t < F.cols[i].size(); ++t)
        for (int c = 0; c < b; ++c) {
          if (col) {
            col[nz] = F.cols[i][t] * b + c;
            val[nz] = F.vals[i][t * b * b + r * b + c];
          }
          ++nz;
        }
    }
  if (ptr) ptr[F.nn * b] = nz;
  return nz;
}

extern "C" void orc_ilu_dinv(orc_solver* s, double* out) {
  std::copy(s->F.Dinv.begin(), s->F.Dinv.end(), out);
}

extern "C" void orc_idr_shadow(int64_t n, int s, double* out) {
  const std::vector<double> P = idr_shadow(n, s);
  std::copy(P.begin(), P.end(), out);
}

extern "C" int orc_gather_block_row(int64_t nr, const int64_t* ptr, const int32_t* col,
                                    const double* val, int b, int64_t i, int32_t* cols,
                                    double* vals, int32_t cap) {
  Csr A = make_csr(nr, nr, ptr, col, val);
  BlockRow br = gather_block_row(A, b, i);
  const int32_t m = (int32_t)br.cols.size();
  for (int32_t t = 0; t < m && t < cap; ++t) {
    cols[t] = br.cols[t];
    for (int q = 0; q < b * b; ++q) vals[(size_t)t * b * b + q] = br.vals[(size_t)t * b * b + q];
  }
  return m;
}

// Thread count of the OpenMP loops (SpMV, sparse products) and the iteration limits of
// an existing solver, for timing bounded samples of a solve.
extern "C" void orc_set_threads(int n) { omp_set_num_threads(n); }
extern "C" int orc_max_threads() { return omp_get_max_threads(); }
extern "C" void orc_set_limits(orc_solver* s, int maxiter, int max_restarts) {
  s->prm.maxiter = maxiter;
  s->prm.max_restarts = max_restarts;
}
