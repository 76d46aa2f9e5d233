// FP64 host setup of the smoothed-aggregation hierarchy in block CSR form.
//
// Components (the paper's AMG composition: smoothed aggregation coarsening
// with the strong-connection threshold eps_str and SPAI(0) relaxation on each
// level, Section 2.1; the constants it leaves open are fixed as follows):
//   strength   N(i,j) = squared Frobenius norm of block (i,j), row-major sum;
//              j != i is strong iff N(i,j) > (eps^2 sqrt N(i,i)) sqrt N(j,j);
//              eps halves on every coarser level; a block row without strong
//              neighbours is isolated (Dirichlet rows are).
//   aggregates three greedy passes over block rows in ascending order.
//   prolong.   P = P_tent - omega D^-1 (A_F P_tent), A_F = strong blocks plus
//              the weak blocks lumped into the diagonal block D, omega =
//              (4/3) / (max Gershgorin row sum of D^-1 A_F), P_tent identity
//              blocks (unnormalized); patterns are structural.
//   Galerkin   R = P^T, A_c = R (A P).
//   smoother   block SPAI(0) M_i = A_ii^T (sum_j A_ij A_ij^T)^-1 (row-block
//              minimizer of ||I - M A||_F), scalar-row SPAI(0) a_rr/sum a_rk^2,
//              or damped block Jacobi.
//   coarsest   rows * b <= coarse_enough, the level cap, or no reduction;
//              its FP64 inverse is formed by Gauss-Jordan with pivoting.
#include <algorithm>
#include <cmath>
#include <cstring>
#include "host.hpp"

namespace mgk {

namespace {

inline double sq_frobenius(const double* B, int n) {
  double s = 0.0;
  for (int t = 0; t < n; ++t) s = s + B[t] * B[t];
  return s;
}

// W = X Y for b x b row-major blocks; each entry is 0 + sum_q X[r][q] Y[q][c]
// with q ascending.
inline void block_product(int b, const double* X, const double* Y, double* W) {
  for (int r = 0; r < b; ++r)
    for (int c = 0; c < b; ++c) {
      double s = 0.0;
      for (int q = 0; q < b; ++q) s = s + X[r * b + q] * Y[q * b + c];
      W[r * b + c] = s;
    }
}

int64_t diag_index(const HBsr& A, int32_t i) {
  const int32_t* b = A.col.data() + A.ptr[i];
  const int32_t* e = A.col.data() + A.ptr[i + 1];
  const int32_t* it = std::lower_bound(b, e, i);
  return (it != e && *it == i) ? (int64_t)(it - A.col.data()) : -1;
}

// strong[k] = 1 if stored block k is a strong off-diagonal connection.
void strength(const HBsr& A, double eps, std::vector<char>& strong, std::vector<char>& iso) {
  const int b2 = A.br * A.bc;
  const int32_t n = A.nbr;
  std::vector<double> nd(n, 0.0);
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    const int64_t k = diag_index(A, i);
    nd[i] = k >= 0 ? sq_frobenius(A.blk(k), b2) : 0.0;
  }
  strong.assign(A.nnzb(), 0);
  iso.assign(n, 1);
  const double e2 = eps * eps;
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    const double si = e2 * std::sqrt(nd[i]);
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const int32_t j = A.col[k];
      if (j == i) continue;
      if (sq_frobenius(A.blk(k), b2) > si * std::sqrt(nd[j])) {
        strong[k] = 1;
        iso[i] = 0;
      }
    }
  }
}

// Greedy aggregation: (1) a row whose non-isolated strong neighbours are all
// unassigned seeds an aggregate with them; (2) leftovers join the phase-1
// aggregate of their first (lowest) strong neighbour that has one.  No row can be
// left after (2) (the classical third phase for leftovers never runs); -1 reports a
// broken invariant.
int32_t aggregation(const HBsr& A, const std::vector<char>& strong, const std::vector<char>& iso,
                    std::vector<int32_t>& agg) {
  const int32_t n = A.nbr;
  agg.assign(n, -1);
  int32_t count = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (iso[i] || agg[i] != -1) continue;
    bool ok = true;
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1] && ok; ++k)
      if (strong[k] && !iso[A.col[k]] && agg[A.col[k]] != -1) ok = false;
    if (!ok) continue;
    agg[i] = count;
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (strong[k] && !iso[A.col[k]]) agg[A.col[k]] = count;
    ++count;
  }
  std::vector<int32_t> seeded(agg);
  for (int32_t i = 0; i < n; ++i) {
    if (iso[i] || agg[i] != -1) continue;
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const int32_t j = A.col[k];
      if (strong[k] && !iso[j] && seeded[j] != -1) {
        agg[i] = seeded[j];
        break;
      }
    }
  }
  // Every connected row is assigned now: phase 1 passes over a connected row only when a
  // connected strong neighbour already sits in a phase-1 aggregate, and phase 2 joins it.
  for (int32_t i = 0; i < n; ++i)
    if (!iso[i] && agg[i] == -1) return -1;
  return count;
}

HBsr block_transpose(const HBsr& P) {
  HBsr R;
  R.br = P.bc;
  R.bc = P.br;
  R.nbr = P.nbc;
  R.nbc = P.nbr;
  R.ptr.assign(R.nbr + 1, 0);
  const int64_t nnz = P.nnzb();
  for (int64_t k = 0; k < nnz; ++k) R.ptr[P.col[k] + 1]++;
  for (int32_t i = 0; i < R.nbr; ++i) R.ptr[i + 1] += R.ptr[i];
  R.col.resize(nnz);
  R.val.resize(P.val.size());
  std::vector<int32_t> fill(R.ptr.begin(), R.ptr.end() - 1);
  const int br = P.br, bc = P.bc;
  for (int32_t i = 0; i < P.nbr; ++i)
    for (int64_t k = P.ptr[i]; k < P.ptr[i + 1]; ++k) {
      const int64_t d = fill[P.col[k]]++;
      R.col[d] = i;
      const double* s = P.blk(k);
      double* t = R.blk(d);
      for (int r = 0; r < br; ++r)
        for (int c = 0; c < bc; ++c) t[c * br + r] = s[r * bc + c];
    }
  return R;
}

// Block Gustavson product C = A B.  Entry (r, c) of output block (i, J)
// accumulates A(i,j)[r][q] B(j,J)[q][c] over stored j ascending, then q
// ascending.  Every reached block is stored (no value-based dropping).
HBsr block_spgemm(const HBsr& A, const HBsr& B) {
  HBsr C;
  C.br = A.br;
  C.bc = B.bc;
  C.nbr = A.nbr;
  C.nbc = B.nbc;
  C.ptr.assign(C.nbr + 1, 0);
  const int br = A.br, bk = A.bc, bc = B.bc, bs = br * bc;
  std::vector<std::vector<int32_t>> rc(C.nbr);
  std::vector<std::vector<double>> rv(C.nbr);
#pragma omp parallel
  {
    std::vector<int64_t> slot(B.nbc, -1);
    std::vector<int32_t> cols;
    std::vector<double> acc;
    std::vector<int32_t> order;
#pragma omp for schedule(dynamic, 512)
    for (int32_t i = 0; i < A.nbr; ++i) {
      cols.clear();
      acc.clear();
      for (int64_t ka = A.ptr[i]; ka < A.ptr[i + 1]; ++ka) {
        const double* X = A.blk(ka);
        const int32_t j = A.col[ka];
        for (int64_t kb = B.ptr[j]; kb < B.ptr[j + 1]; ++kb) {
          const int32_t J = B.col[kb];
          if (slot[J] < 0) {
            slot[J] = (int64_t)cols.size();
            cols.push_back(J);
            acc.resize(acc.size() + bs, 0.0);
          }
          double* W = acc.data() + slot[J] * bs;
          const double* Y = B.blk(kb);
          for (int r = 0; r < br; ++r)
            for (int c = 0; c < bc; ++c) {
              double s = W[r * bc + c];
              for (int q = 0; q < bk; ++q) s = s + X[r * bk + q] * Y[q * bc + c];
              W[r * bc + c] = s;
            }
        }
      }
      order.resize(cols.size());
      for (size_t t = 0; t < cols.size(); ++t) order[t] = (int32_t)t;
      std::sort(order.begin(), order.end(), [&](int32_t u, int32_t v) { return cols[u] < cols[v]; });
      rc[i].resize(cols.size());
      rv[i].resize(cols.size() * bs);
      for (size_t t = 0; t < cols.size(); ++t) {
        rc[i][t] = cols[order[t]];
        std::memcpy(&rv[i][t * bs], &acc[(size_t)order[t] * bs], sizeof(double) * bs);
        slot[cols[order[t]]] = -1;
      }
    }
  }
  for (int32_t i = 0; i < C.nbr; ++i) C.ptr[i + 1] = C.ptr[i] + (int32_t)rc[i].size();
  C.col.resize(C.ptr[C.nbr]);
  C.val.resize((size_t)C.ptr[C.nbr] * bs);
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < C.nbr; ++i) {
    std::copy(rc[i].begin(), rc[i].end(), C.col.begin() + C.ptr[i]);
    std::copy(rv[i].begin(), rv[i].end(), C.val.begin() + (size_t)C.ptr[i] * bs);
  }
  return C;
}

// Smoothed prolongator of one level.  Returns 0, or a negative status.
int smoothed_prolongator(const HBsr& A, const std::vector<char>& strong,
                         const std::vector<char>& iso, const std::vector<int32_t>& agg,
                         int32_t n_agg, HLevel& L, std::string& err) {
  const int b = A.br, bs = b * b;
  const int32_t n = A.nbr;
  std::vector<double> D((size_t)n * bs), Dinv((size_t)n * bs);
  int bad = 0;
  double rho = 0.0;
#pragma omp parallel for schedule(static) reduction(max : rho) reduction(| : bad)
  for (int32_t i = 0; i < n; ++i) {
    const int64_t kd = diag_index(A, i);
    if (kd < 0) {
      bad |= 1;
      continue;
    }
    double* Di = &D[(size_t)i * bs];
    std::memcpy(Di, A.blk(kd), sizeof(double) * bs);
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (A.col[k] != i && !strong[k])
        for (int t = 0; t < bs; ++t) Di[t] = Di[t] + A.blk(k)[t];
    if (!gauss_jordan_inverse(b, Di, &Dinv[(size_t)i * bs])) {
      bad |= 2;
      continue;
    }
    if (iso[i]) continue;
    double W[16], rs[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const double* X = A.col[k] == i ? Di : (strong[k] ? A.blk(k) : nullptr);
      if (!X) continue;
      block_product(b, &Dinv[(size_t)i * bs], X, W);
      for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) rs[r] = rs[r] + std::fabs(W[r * b + c]);
    }
    for (int r = 0; r < b; ++r) rho = std::max(rho, rs[r]);
  }
  if (bad & 1) {
    err = "setup: a block row has no diagonal block";
    return -1;
  }
  if (bad & 2) {
    err = "setup: singular filtered diagonal block";
    return -4;
  }
  if (!(rho > 0.0)) {
    err = "setup: zero spectral radius estimate";
    return -4;
  }
  L.omega = (4.0 / 3.0) / rho;
  const double om = L.omega;

  HBsr& P = L.P;
  P.br = P.bc = b;
  P.nbr = n;
  P.nbc = n_agg;
  P.ptr.assign(n + 1, 0);
  std::vector<std::vector<int32_t>> pc(n);
  std::vector<std::vector<double>> pv(n);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t i = 0; i < n; ++i) {
    if (agg[i] < 0) continue;
    // T(i, J) = sum of the kept blocks (i, j) with agg(j) = J, j ascending.
    std::vector<int32_t> J;
    std::vector<double> T;
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const int32_t j = A.col[k];
      const double* X = j == i ? &D[(size_t)i * bs] : (strong[k] ? A.blk(k) : nullptr);
      if (!X || agg[j] < 0) continue;
      size_t t = 0;
      while (t < J.size() && J[t] != agg[j]) ++t;
      if (t == J.size()) {
        J.push_back(agg[j]);
        T.insert(T.end(), X, X + bs);
      } else {
        for (int q = 0; q < bs; ++q) T[t * bs + q] = T[t * bs + q] + X[q];
      }
    }
    std::vector<int32_t> ord(J.size());
    for (size_t t = 0; t < J.size(); ++t) ord[t] = (int32_t)t;
    std::sort(ord.begin(), ord.end(), [&](int32_t u, int32_t v) { return J[u] < J[v]; });
    pc[i].resize(J.size());
    pv[i].resize(J.size() * bs);
    double W[16];
    for (size_t t = 0; t < J.size(); ++t) {
      const int32_t jj = J[ord[t]];
      block_product(b, &Dinv[(size_t)i * bs], &T[(size_t)ord[t] * bs], W);
      pc[i][t] = jj;
      for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) {
          const double e = (jj == agg[i] && r == c) ? 1.0 : 0.0;
          pv[i][t * bs + r * b + c] = e - om * W[r * b + c];
        }
    }
  }
  for (int32_t i = 0; i < n; ++i) P.ptr[i + 1] = P.ptr[i] + (int32_t)pc[i].size();
  P.col.resize(P.ptr[n]);
  P.val.resize((size_t)P.ptr[n] * bs);
  for (int32_t i = 0; i < n; ++i) {
    std::copy(pc[i].begin(), pc[i].end(), P.col.begin() + P.ptr[i]);
    std::copy(pv[i].begin(), pv[i].end(), P.val.begin() + (size_t)P.ptr[i] * bs);
  }
  return 0;
}

// Tentative prolongator (plain aggregation): one identity block at (i, agg(i))
// for every aggregated block row.
static void tentative_prolongator(int b, int32_t n, const std::vector<int32_t>& agg,
                                  int32_t n_agg, HLevel& L) {
  HBsr& P = L.P;
  P = HBsr();
  P.br = P.bc = b;
  P.nbr = n;
  P.nbc = n_agg;
  P.ptr.assign(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) {
    P.ptr[i + 1] = P.ptr[i];
    if (agg[i] < 0) continue;
    P.col.push_back(agg[i]);
    for (int r = 0; r < b; ++r)
      for (int c = 0; c < b; ++c) P.val.push_back(r == c ? 1.0 : 0.0);
    P.ptr[i + 1] = P.ptr[i] + 1;
  }
  L.omega = 0.0;
}

int build_smoother(const HBsr& A, const SetupParams& prm, std::vector<double>& M,
                   std::string& err) {
  const int b = A.br, bs = b * b;
  const int32_t n = A.nbr;
  M.assign((size_t)n * bs, 0.0);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int32_t i = 0; i < n; ++i) {
    const int64_t kd = diag_index(A, i);
    if (kd < 0) {
      bad |= 1;
      continue;
    }
    const double* Aii = A.blk(kd);
    double* Mi = &M[(size_t)i * bs];
    if (prm.smoother == SM_JACOBI) {
      double inv[16];
      if (!gauss_jordan_inverse(b, Aii, inv)) {
        bad |= 2;
        continue;
      }
      for (int t = 0; t < bs; ++t) Mi[t] = prm.jacobi_omega * inv[t];
    } else if (prm.smoother == SM_SPAI0_SCALAR) {
      for (int r = 0; r < b; ++r) {
        double s = 0.0;
        for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
          for (int c = 0; c < b; ++c) s = s + A.blk(k)[r * b + c] * A.blk(k)[r * b + c];
        Mi[r * b + r] = Aii[r * b + r] / s;
      }
    } else {
      double G[16] = {0.0}, Gi[16];
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        const double* X = A.blk(k);
        for (int r = 0; r < b; ++r)
          for (int c = 0; c < b; ++c)
            for (int q = 0; q < b; ++q) G[r * b + c] = G[r * b + c] + X[r * b + q] * X[c * b + q];
      }
      if (!gauss_jordan_inverse(b, G, Gi)) {
        bad |= 2;
        continue;
      }
      for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) {
          double s = 0.0;
          for (int q = 0; q < b; ++q) s = s + Aii[q * b + r] * Gi[q * b + c];
          Mi[r * b + c] = s;
        }
    }
  }
  if (bad & 1) {
    err = "setup: a block row has no diagonal block";
    return -1;
  }
  if (bad & 2) {
    err = "setup: singular smoother block";
    return -4;
  }
  return 0;
}

}  // namespace

// Gauss-Jordan elimination on [D | I]: for each pivot column take the first
// row of largest magnitude at or below the diagonal, swap it up, divide the
// pivot row by the pivot, and subtract multiples of it from every other row.
bool gauss_jordan_inverse(int n, const double* D, double* Dinv) {
  const int w = 2 * n;
  double aug[2 * 4 * 4];
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < w; ++c) aug[r * w + c] = c < n ? D[r * n + c] : (c - n == r ? 1.0 : 0.0);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double mx = std::fabs(aug[k * w + k]);
    for (int r = k + 1; r < n; ++r) {
      const double v = std::fabs(aug[r * w + k]);
      if (v > mx) {
        mx = v;
        p = r;
      }
    }
    if (!(mx > 0.0) || !std::isfinite(mx)) return false;
    if (p != k)
      for (int c = 0; c < w; ++c) std::swap(aug[k * w + c], aug[p * w + c]);
    const double pv = aug[k * w + k];
    for (int c = 0; c < w; ++c) aug[k * w + c] = aug[k * w + c] / pv;
    for (int r = 0; r < n; ++r) {
      if (r == k) continue;
      const double f = aug[r * w + k];
      for (int c = 0; c < w; ++c) aug[r * w + c] = aug[r * w + c] - f * aug[k * w + c];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) Dinv[r * n + c] = aug[r * w + n + c];
  return true;
}

// Dense inverse of the coarsest matrix (row-major, overwritten).
bool dense_inverse(int n, std::vector<double>& a, std::vector<double>& inv) {
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double mx = std::fabs(a[(size_t)k * n + k]);
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * n + k]) > mx) {
        mx = std::fabs(a[(size_t)r * n + k]);
        p = r;
      }
    if (!(mx > 0.0) || !std::isfinite(mx)) return false;
    if (p != k) {
      std::swap_ranges(a.begin() + (size_t)k * n, a.begin() + (size_t)(k + 1) * n,
                       a.begin() + (size_t)p * n);
      std::swap_ranges(inv.begin() + (size_t)k * n, inv.begin() + (size_t)(k + 1) * n,
                       inv.begin() + (size_t)p * n);
    }
    const double pv = a[(size_t)k * n + k];
    for (int c = 0; c < n; ++c) {
      a[(size_t)k * n + c] /= pv;
      inv[(size_t)k * n + c] /= pv;
    }
#pragma omp parallel for schedule(static)
    for (int r = 0; r < n; ++r) {
      if (r == k) continue;
      const double f = a[(size_t)r * n + k];
      if (f == 0.0) continue;
      double* ar = &a[(size_t)r * n];
      double* ir = &inv[(size_t)r * n];
      const double* ak = &a[(size_t)k * n];
      const double* ik = &inv[(size_t)k * n];
      for (int c = 0; c < n; ++c) {
        ar[c] -= f * ak[c];
        ir[c] -= f * ik[c];
      }
    }
  }
  return true;
}

int build_hierarchy(const HBsr& A0, const SetupParams& prm, HHierarchy& H, std::string& err) {
  H.b = A0.br;
  H.levels.clear();
  H.levels.emplace_back();
  H.levels[0].A = A0;
  double eps = prm.eps_strong;
  const int b = A0.br;
  for (int l = 0;; ++l) {
    bool coarsest = (int64_t)H.levels[l].A.nbr * b <= prm.coarse_enough || l == prm.max_levels - 1;
    HBsr Ac;
    if (!coarsest) {
      HLevel& L = H.levels[l];
      std::vector<char> strong, iso;
      strength(L.A, eps, strong, iso);
      L.n_agg = aggregation(L.A, strong, iso, L.agg);
      if (L.n_agg < 0) {
        err = "aggregation left a connected block row unassigned";
        return -1;
      }
      if (L.n_agg == 0 || L.n_agg >= L.A.nbr) {
        coarsest = true;
        L.agg.clear();
        L.n_agg = 0;
      } else {
        int rc = 0;
        if (prm.smooth_p) rc = smoothed_prolongator(L.A, strong, iso, L.agg, L.n_agg, L, err);
        else tentative_prolongator(b, L.A.nbr, L.agg, L.n_agg, L);
        if (rc) return rc;
        L.R = block_transpose(L.P);
        HBsr AP = block_spgemm(L.A, L.P);
        Ac = block_spgemm(L.R, AP);
        rc = !prm.ilu_smoother ? build_smoother(L.A, prm, L.M, err)
             : prm.ilu_kind == 1 ? ilut_factor(L.A, prm.ilut_p, prm.ilut_tau, L.ilu, err)
                                 : ilu_factor(L.A, 0, L.ilu, err);
        if (rc) return rc;
      }
    }
    if (coarsest) {
      const HBsr& C = H.levels[l].A;
      const int nc = C.nbr * b;
      std::vector<double> dense((size_t)nc * nc, 0.0);
      for (int32_t i = 0; i < C.nbr; ++i)
        for (int64_t k = C.ptr[i]; k < C.ptr[i + 1]; ++k)
          for (int r = 0; r < b; ++r)
            for (int c = 0; c < b; ++c)
              dense[(size_t)(i * b + r) * nc + C.col[k] * b + c] = C.blk(k)[r * b + c];
      H.nc = nc;
      if (!dense_inverse(nc, dense, H.coarse_inv)) {
        err = "setup: singular coarsest matrix";
        return -4;
      }
      return 0;
    }
    eps = 0.5 * eps;
    H.levels.emplace_back();
    H.levels.back().A = std::move(Ac);
  }
}

}  // namespace mgk
