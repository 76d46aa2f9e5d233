// Oracle Krylov solvers and the Schur-complement pressure correction
// preconditioner.  TEST INFRASTRUCTURE ONLY (see oracle.hpp).
//
// BiCGStab (van der Vorst, 1992) and flexible GMRES(m) (Saad, 1993), both
// right-preconditioned so the monitored residual is the residual of the
// original system.  The Schur preconditioner follows Section 4 (eqs. SchurP
// and SchurU): one velocity cycle, the pressure correction on the Schur
// complement approximation S = C - B_lo diag(A_uu)^-1 B_up (the explicitly
// assembled form the paper describes for its PETSc comparison), then a second
// velocity cycle on the corrected right-hand side.
#include <cmath>
#include <cstring>
#include <vector>
#include "oracle.hpp"

namespace orc {

namespace {
void residual(const Csr& A, const double* b, const double* x, double* r) {
  spmv(A, x, r);
  for (i64 i = 0; i < A.nr; ++i) r[i] = b[i] - r[i];
}
}  // namespace

// Right-preconditioned BiCGStab.  Exit tests use ||.||_2 relative to ||b||.
// A breakdown (rho' = 0 or (t,t) = 0) or a final true residual above tol
// restarts from r = b - A x with rhat = r.
void bicgstab(const Csr& A, const Precond& M, const double* b, double* x,
              double tol, int maxiter, int max_restarts, SolveInfo& info) {
  const i64 n = A.nr;
  info = SolveInfo();
  const double nb = nrm2(n, b);
  if (nb == 0.0) {
    for (i64 i = 0; i < n; ++i) x[i] = 0.0;
    info.converged = 1;
    return;
  }
  std::vector<double> r(n), rh(n), p(n), v(n), ph(n), s(n), sh(n), t(n);
  int it = 0;
  for (int restart = 0;; ++restart) {
    residual(A, b, x, r.data());
    std::memcpy(rh.data(), r.data(), sizeof(double) * n);
    std::fill(p.begin(), p.end(), 0.0);
    std::fill(v.begin(), v.end(), 0.0);
    double rho = 1.0, alpha = 1.0, omega = 1.0;
    bool breakdown = false;
    if (nrm2(n, r.data()) / nb <= tol) {
      info.converged = 1;
    }
    while (!info.converged && it < maxiter) {
      ++it;
      const double rho1 = dot(n, rh.data(), r.data());
      if (rho1 == 0.0) {
        breakdown = true;
        break;
      }
      const double beta = (rho1 / rho) * (alpha / omega);
      for (i64 i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
      M.apply(p.data(), ph.data());
      spmv(A, ph.data(), v.data());
      alpha = rho1 / dot(n, rh.data(), v.data());
      for (i64 i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
      if (nrm2(n, s.data()) / nb <= tol) {
        for (i64 i = 0; i < n; ++i) x[i] = x[i] + alpha * ph[i];
        break;
      }
      M.apply(s.data(), sh.data());
      spmv(A, sh.data(), t.data());
      const double tt = dot(n, t.data(), t.data());
      if (tt == 0.0) {
        for (i64 i = 0; i < n; ++i) x[i] = x[i] + alpha * ph[i];
        breakdown = true;
        break;
      }
      omega = dot(n, t.data(), s.data()) / tt;
      for (i64 i = 0; i < n; ++i) x[i] = x[i] + alpha * ph[i] + omega * sh[i];
      for (i64 i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
      rho = rho1;
      if (nrm2(n, r.data()) / nb <= tol) break;
    }
    residual(A, b, x, r.data());
    info.rel_resid = nrm2(n, r.data()) / nb;
    info.iters = it;
    info.restarts = restart;
    if (info.rel_resid <= tol) {
      info.converged = 1;
      return;
    }
    info.converged = 0;
    if (it >= maxiter || restart >= max_restarts) return;
    (void)breakdown;
  }
}

// Flexible GMRES(m) with modified Gram-Schmidt and Givens rotations.
// maxiter counts inner steps over all restart cycles.
void fgmres(const Csr& A, const Precond& M, const double* b, double* x,
            double tol, int m, int maxiter, SolveInfo& info) {
  const i64 n = A.nr;
  info = SolveInfo();
  const double nb = nrm2(n, b);
  if (nb == 0.0) {
    for (i64 i = 0; i < n; ++i) x[i] = 0.0;
    info.converged = 1;
    return;
  }
  std::vector<std::vector<double>> V(m + 1, std::vector<double>(n)), Z(m, std::vector<double>(n));
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), w(n), r(n);
  int total = 0;
  for (int cycle = 0;; ++cycle) {
    residual(A, b, x, r.data());
    const double beta = nrm2(n, r.data());
    info.rel_resid = beta / nb;
    info.iters = total;
    info.restarts = cycle;
    if (beta / nb <= tol) {
      info.converged = 1;
      return;
    }
    if (total >= maxiter) return;
    for (i64 i = 0; i < n; ++i) V[0][i] = r[i] / beta;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < m && total < maxiter; ++j) {
      M.apply(V[j].data(), Z[j].data());
      spmv(A, Z[j].data(), w.data());
      for (int i = 0; i <= j; ++i) {
        const double h = dot(n, w.data(), V[i].data());
        H[(size_t)i * m + j] = h;
        for (i64 q = 0; q < n; ++q) w[q] = w[q] - h * V[i][q];
      }
      const double hn = nrm2(n, w.data());
      H[(size_t)(j + 1) * m + j] = hn;
      if (hn != 0.0)
        for (i64 q = 0; q < n; ++q) V[j + 1][q] = w[q] / hn;
      for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
      }
      const double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
      const double den = std::hypot(a, c);
      cs[j] = a / den;
      sn[j] = c / den;
      H[(size_t)j * m + j] = den;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++total;
      k = j + 1;
      if (std::fabs(g[j + 1]) / nb <= tol || hn == 0.0) break;
    }
    std::vector<double> y(k);
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int q = i + 1; q < k; ++q) s = s - H[(size_t)i * m + q] * y[q];
      y[i] = s / H[(size_t)i * m + i];
    }
    for (int i = 0; i < k; ++i)
      for (i64 q = 0; q < n; ++q) x[q] = x[q] + y[i] * Z[i][q];
  }
}

// ---- IDR(s) -------------------------------------------------------------------
//
// Induced dimension reduction (Sonneveld and van Gijzen), in the variant whose
// residual updates are kept biorthogonal to the shadow space (van Gijzen and
// Sonneveld, ACM TOMS 38, 2011), with right preconditioning: every new search
// direction U_k is a preconditioned vector and G_k = A U_k.  The paper uses
// IDR(5) as its outer solver (Section 4, Table of solver variants).  The step
// length omega of the dimension-reduction step is the minimal-residual one,
// enlarged when the angle between t and r is small (|cos| < 0.7).

static double splitmix_unit(uint64_t c) {
  // SplitMix64 (Steele, Lea and Flood, 2014): output number c of the sequence
  // started from state 0, top 53 bits mapped to [-1, 1).
  uint64_t z = (c + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

std::vector<double> idr_shadow(i64 n, int s) {
  std::vector<double> P((size_t)n * s);
  for (int j = 0; j < s; ++j)
    for (i64 i = 0; i < n; ++i) P[(size_t)j * n + i] = splitmix_unit((uint64_t)j * n + i);
  for (int j = 0; j < s; ++j) {
    double* pj = &P[(size_t)j * n];
    for (int i = 0; i < j; ++i) {
      const double* pi = &P[(size_t)i * n];
      const double d = dot(n, pi, pj);
      for (i64 q = 0; q < n; ++q) pj[q] = pj[q] - d * pi[q];
    }
    const double nr = nrm2(n, pj);
    for (i64 q = 0; q < n; ++q) pj[q] = pj[q] / nr;
  }
  return P;
}

void idrs(const Csr& A, const Precond& K, const double* b, double* x, double tol, int s,
          int maxiter, int max_restarts, SolveInfo& info) {
  const i64 n = A.nr;
  info = SolveInfo();
  const double nb = nrm2(n, b);
  if (nb == 0.0) {
    for (i64 i = 0; i < n; ++i) x[i] = 0.0;
    info.converged = 1;
    return;
  }
  const std::vector<double> P = idr_shadow(n, s);
  auto col = [n](std::vector<double>& V, int j) { return &V[(size_t)j * n]; };
  auto pcol = [&](int j) { return &P[(size_t)j * n]; };
  std::vector<double> r(n), v(n), vh(n), t(n), G((size_t)n * s), U((size_t)n * s);
  std::vector<double> Mm((size_t)s * s), f(s), c(s);
  int it = 0;
  for (int restart = 0;; ++restart) {
    residual(A, b, x, r.data());
    std::fill(G.begin(), G.end(), 0.0);
    std::fill(U.begin(), U.end(), 0.0);
    std::fill(Mm.begin(), Mm.end(), 0.0);
    for (int i = 0; i < s; ++i) Mm[(size_t)i * s + i] = 1.0;
    double om = 1.0;
    double normr = nrm2(n, r.data());
    bool conv = normr / nb <= tol, breakdown = false;
    while (!conv && !breakdown && it < maxiter) {
      for (int i = 0; i < s; ++i) f[i] = dot(n, pcol(i), r.data());
      for (int k = 0; k < s && !conv && it < maxiter; ++k) {
        // lower triangular M(k:s, k:s) c = f(k:s)
        for (int i = k; i < s; ++i) {
          double a = f[i];
          for (int j = k; j < i; ++j) a = a - Mm[(size_t)i * s + j] * c[j];
          c[i] = a / Mm[(size_t)i * s + i];
        }
        for (i64 q = 0; q < n; ++q) v[q] = r[q];
        for (int i = k; i < s; ++i)
          for (i64 q = 0; q < n; ++q) v[q] = v[q] - c[i] * col(G, i)[q];
        K.apply(v.data(), vh.data());
        double* Uk = col(U, k);
        double* Gk = col(G, k);
        std::vector<double> un(n);
        for (i64 q = 0; q < n; ++q) un[q] = om * vh[q];
        for (int i = k; i < s; ++i)
          for (i64 q = 0; q < n; ++q) un[q] = un[q] + c[i] * col(U, i)[q];
        std::copy(un.begin(), un.end(), Uk);
        spmv(A, Uk, Gk);
        // make G_k orthogonal to the first k shadow vectors
        for (int i = 0; i < k; ++i) {
          const double alpha = dot(n, pcol(i), Gk) / Mm[(size_t)i * s + i];
          for (i64 q = 0; q < n; ++q) {
            Gk[q] = Gk[q] - alpha * col(G, i)[q];
            Uk[q] = Uk[q] - alpha * col(U, i)[q];
          }
        }
        for (int i = k; i < s; ++i) Mm[(size_t)i * s + k] = dot(n, pcol(i), Gk);
        if (Mm[(size_t)k * s + k] == 0.0) {
          breakdown = true;
          break;
        }
        const double beta = f[k] / Mm[(size_t)k * s + k];
        for (i64 q = 0; q < n; ++q) {
          r[q] = r[q] - beta * Gk[q];
          x[q] = x[q] + beta * Uk[q];
        }
        ++it;
        normr = nrm2(n, r.data());
        if (normr / nb <= tol) {
          conv = true;
          break;
        }
        for (int i = k + 1; i < s; ++i) f[i] = f[i] - beta * Mm[(size_t)i * s + k];
      }
      if (conv || breakdown || it >= maxiter) break;
      // dimension reduction step
      K.apply(r.data(), vh.data());
      spmv(A, vh.data(), t.data());
      const double tt = dot(n, t.data(), t.data()), tr = dot(n, t.data(), r.data());
      const double rho = std::fabs(tr) / (std::sqrt(tt) * normr);
      if (tt == 0.0 || rho == 0.0) {
        breakdown = true;
        break;
      }
      om = tr / tt;
      if (rho < 0.7) om = om * 0.7 / rho;
      for (i64 q = 0; q < n; ++q) {
        r[q] = r[q] - om * t[q];
        x[q] = x[q] + om * vh[q];
      }
      ++it;
      normr = nrm2(n, r.data());
      conv = normr / nb <= tol;
    }
    residual(A, b, x, r.data());
    info.rel_resid = nrm2(n, r.data()) / nb;
    info.iters = it;
    info.restarts = restart;
    if (info.rel_resid <= tol) {
      info.converged = 1;
      return;
    }
    if (restart >= max_restarts || it >= maxiter) return;
  }
}

bool schur_build(const Csr& A, const AmgParams& prm, const SchurOptions& opt, Schur& S,
                 const char** msg) {
  const i64 nn = A.nr / 4;
  S.nn = nn;
  S.opt = opt;
  auto init = [](Csr& M, i64 nr, i64 nc) {
    M = Csr();
    M.nr = nr;
    M.nc = nc;
    M.ptr.assign(nr + 1, 0);
  };
  init(S.Auu, 3 * nn, 3 * nn);
  init(S.Bup, 3 * nn, nn);
  init(S.Blo, nn, 3 * nn);
  init(S.C, nn, nn);
  for (i64 g = 0; g < nn; ++g)
    for (int c = 0; c < 4; ++c) {
      const i64 row = 4 * g + c;
      for (i64 k = A.ptr[row]; k < A.ptr[row + 1]; ++k) {
        const i32 m = A.col[k] / 4, cc = A.col[k] % 4;
        Csr& T = c < 3 ? (cc < 3 ? S.Auu : S.Bup) : (cc < 3 ? S.Blo : S.C);
        T.col.push_back(cc < 3 ? 3 * m + cc : m);
        T.val.push_back(A.val[k]);
      }
      if (c < 3) {
        S.Auu.ptr[3 * g + c + 1] = (i64)S.Auu.col.size();
        S.Bup.ptr[3 * g + c + 1] = (i64)S.Bup.col.size();
      } else {
        S.Blo.ptr[g + 1] = (i64)S.Blo.col.size();
        S.C.ptr[g + 1] = (i64)S.C.col.size();
      }
    }
  // W = B_lo diag(A_uu)^-1 (columns scaled by 1/d), then S = C - W B_up.
  std::vector<double> dinv(3 * nn, 0.0);
  for (i64 r = 0; r < 3 * nn; ++r)
    for (i64 k = S.Auu.ptr[r]; k < S.Auu.ptr[r + 1]; ++k)
      if (S.Auu.col[k] == r) dinv[r] = 1.0 / S.Auu.val[k];
  Csr W = S.Blo;
  for (i64 k = 0; k < (i64)W.val.size(); ++k) W.val[k] = W.val[k] * dinv[W.col[k]];
  Csr SP = spgemm(W, S.Bup);
  if (opt.diag_approx) {
    // eq. SchurApprox: only the diagonal of Blo diag(Auu)^-1 Bup is subtracted
    Csr D;
    init(D, nn, nn);
    for (i64 r = 0; r < nn; ++r) {
      for (i64 k = SP.ptr[r]; k < SP.ptr[r + 1]; ++k)
        if (SP.col[k] == r) {
          D.col.push_back((i32)r);
          D.val.push_back(SP.val[k]);
        }
      D.ptr[r + 1] = (i64)D.col.size();
    }
    SP = D;
  }
  init(S.S, nn, nn);
  for (i64 r = 0; r < nn; ++r) {
    i64 a = S.C.ptr[r], ae = S.C.ptr[r + 1], p = SP.ptr[r], pe = SP.ptr[r + 1];
    while (a < ae || p < pe) {
      const i32 ca = a < ae ? S.C.col[a] : INT32_MAX, cp = p < pe ? SP.col[p] : INT32_MAX;
      if (ca < cp) {
        S.S.col.push_back(ca);
        S.S.val.push_back(S.C.val[a++]);
      } else if (cp < ca) {
        S.S.col.push_back(cp);
        S.S.val.push_back(0.0 - SP.val[p++]);
      } else {
        S.S.col.push_back(ca);
        S.S.val.push_back(S.C.val[a++] - SP.val[p++]);
      }
    }
    S.S.ptr[r + 1] = (i64)S.S.col.size();
  }
  if (!amg_build(S.Auu, opt.scalar_u ? 1 : 3, prm, S.Hu, msg)) return false;
  if (opt.spai0_p) {
    // scalar SPAI(0): m_i = s_ii / sum_j s_ij^2 (the b = 1 case of the block formula)
    S.Sm.assign(nn, 0.0);
    for (i64 r = 0; r < nn; ++r) {
      double d = 0.0, q = 0.0;
      for (i64 k = S.S.ptr[r]; k < S.S.ptr[r + 1]; ++k) {
        q = q + S.S.val[k] * S.S.val[k];
        if (S.S.col[k] == r) d = S.S.val[k];
      }
      if (!(q > 0.0)) {
        *msg = "oracle: empty Schur complement row";
        return false;
      }
      S.Sm[r] = d / q;
    }
    return true;
  }
  if (!amg_build(S.S, 1, prm, S.Hp, msg)) return false;
  return true;
}

// z_u = V_u(r_u); z_p = V_S(r_p - B_lo z_u); z_u = V_u(r_u - B_up z_p) (eqs. SchurP,
// SchurU).  The lower factorization stops after z_p; with spai0_p the pressure step
// is z_p = m .* (r_p - B_lo z_u).
void schur_apply(const Schur& S, const double* r, double* z) {
  const i64 nn = S.nn;
  std::vector<double> ru(3 * nn), rp(nn), zu(3 * nn), zp(nn), tu(3 * nn), tp(nn);
  for (i64 g = 0; g < nn; ++g) {
    for (int c = 0; c < 3; ++c) ru[3 * g + c] = r[4 * g + c];
    rp[g] = r[4 * g + 3];
  }
  vcycle(S.Hu, 0, ru.data(), zu.data());
  spmv(S.Blo, zu.data(), tp.data());
  for (i64 g = 0; g < nn; ++g) tp[g] = rp[g] - tp[g];
  if (S.opt.spai0_p) {
    for (i64 g = 0; g < nn; ++g) zp[g] = S.Sm[g] * tp[g];
  } else {
    vcycle(S.Hp, 0, tp.data(), zp.data());
  }
  if (!S.opt.lower) {
    spmv(S.Bup, zp.data(), tu.data());
    for (i64 q = 0; q < 3 * nn; ++q) tu[q] = ru[q] - tu[q];
    vcycle(S.Hu, 0, tu.data(), zu.data());
  }
  for (i64 g = 0; g < nn; ++g) {
    for (int c = 0; c < 3; ++c) z[4 * g + c] = zu[3 * g + c];
    z[4 * g + 3] = zp[g];
  }
}

}  // namespace orc
