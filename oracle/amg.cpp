// Oracle smoothed-aggregation AMG hierarchy and V(1,1) cycle.
// TEST INFRASTRUCTURE ONLY (see oracle.hpp).
//
// The paper composes its monolithic preconditioner from smoothed-aggregation
// coarsening with a strong-connection threshold eps_str and the SPAI(0)
// smoother on every level (Section 2.1, the AMG composition listing and its
// parameters), and uses a single V-cycle per preconditioner application
// (Section 4, one application of each nested preconditioner).  The paper does
// not fix the remaining constants; the readings taken here are:
//   strength   j != i strong iff N_ij > eps^2 sqrt(N_ii) sqrt(N_jj), with
//              N_ij the squared Frobenius norm of block (i,j) summed row-major;
//              eps halves from one level to the next;
//   aggregates greedy phases in ascending node order: seed full strong
//              neighbourhoods, then attach leftovers to the phase-1 aggregate of
//              their lowest strong neighbour (the classical third phase for
//              leftovers is unreachable after these two); a node with no strong
//              neighbour is isolated and joins no aggregate;
//   P          (I - omega D^-1 A_F) P_tent with the row-sum lumped filtered
//              matrix A_F, D = diagonal block of A_F, omega = (4/3)/rho and
//              rho the Gershgorin bound of D^-1 A_F;
//   R, A_c     R = P^T and A_c = R (A P);
//   smoother   block SPAI(0): M_i = A_ii^T (sum_j A_ij A_ij^T)^-1, the
//              block-diagonal minimizer of ||I - M A||_F (scalar rows: a_ii /
//              sum_j a_ij^2); or damped block Jacobi omega_J A_ii^-1;
//   coarsest   FP64 dense LU with partial pivoting.
#include <algorithm>
#include <cmath>
#include <cstring>
#include "oracle.hpp"

namespace orc {

namespace {

double block_norm2(int b, const double* B) {
  double s = 0.0;
  for (int t = 0; t < b * b; ++t) s = s + B[t] * B[t];
  return s;
}

const double* find_block(const BlockRow& br, int b, i32 j) {
  auto it = std::lower_bound(br.cols.begin(), br.cols.end(), j);
  if (it == br.cols.end() || *it != j) return nullptr;
  return &br.vals[(size_t)(it - br.cols.begin()) * b * b];
}

// W = X Y for b x b row-major blocks; each entry sums over q ascending.
void block_mul(int b, const double* X, const double* Y, double* W) {
  for (int r = 0; r < b; ++r)
    for (int c = 0; c < b; ++c) {
      double s = 0.0;
      for (int q = 0; q < b; ++q) s = s + X[r * b + q] * Y[q * b + c];
      W[r * b + c] = s;
    }
}

// Append node row i of a matrix whose every stored block is dense.
void push_block_row(Csr& M, int b, i64 i, const std::vector<i32>& cols,
                    const std::vector<double>& vals) {
  for (int r = 0; r < b; ++r) {
    for (size_t t = 0; t < cols.size(); ++t)
      for (int c = 0; c < b; ++c) {
        M.col.push_back(cols[t] * b + c);
        M.val.push_back(vals[t * b * b + r * b + c]);
      }
    M.ptr[i * b + r + 1] = (i64)M.col.size();
  }
}

struct Strength {
  std::vector<std::vector<i32>> S;   // strong neighbours, ascending
  std::vector<char> iso;
};

Strength strength(const Csr& A, int b, double eps) {
  const i64 nn = A.nr / b;
  std::vector<double> Nd(nn, 0.0);
  for (i64 i = 0; i < nn; ++i) {
    BlockRow br = gather_block_row(A, b, i);
    const double* D = find_block(br, b, (i32)i);
    Nd[i] = D ? block_norm2(b, D) : 0.0;
  }
  Strength st;
  st.S.resize(nn);
  st.iso.assign(nn, 0);
  const double e2 = eps * eps;
  for (i64 i = 0; i < nn; ++i) {
    BlockRow br = gather_block_row(A, b, i);
    for (size_t t = 0; t < br.cols.size(); ++t) {
      const i32 j = br.cols[t];
      if (j == i) continue;
      const double Nij = block_norm2(b, &br.vals[t * b * b]);
      if (Nij > (e2 * std::sqrt(Nd[i])) * std::sqrt(Nd[j])) st.S[i].push_back(j);
    }
    st.iso[i] = st.S[i].empty();
  }
  return st;
}

// Greedy aggregation in ascending node order; returns -1 if a node were left over.
i64 aggregate(const Strength& st, std::vector<i32>& agg) {
  const i64 nn = (i64)st.S.size();
  agg.assign(nn, -1);
  i32 next = 0;
  // Phase 1: a node whose whole (non-isolated) strong neighbourhood is free
  // becomes a new aggregate together with that neighbourhood.
  for (i64 i = 0; i < nn; ++i) {
    if (st.iso[i] || agg[i] >= 0) continue;
    bool free = true;
    for (i32 j : st.S[i])
      if (!st.iso[j] && agg[j] >= 0) free = false;
    if (!free) continue;
    agg[i] = next;
    for (i32 j : st.S[i])
      if (!st.iso[j]) agg[j] = next;
    ++next;
  }
  // Phase 2: a free node joins the phase-1 aggregate of its lowest-numbered
  // strong neighbour that has one.
  const std::vector<i32> phase1 = agg;
  for (i64 i = 0; i < nn; ++i) {
    if (st.iso[i] || agg[i] >= 0) continue;
    for (i32 j : st.S[i])
      if (!st.iso[j] && phase1[j] >= 0) {
        agg[i] = phase1[j];
        break;
      }
  }
  // No third phase is needed: phase 1 skips a non-isolated node only when one of its
  // non-isolated strong neighbours is already in a phase-1 aggregate, and phase 2
  // attaches it to the first such neighbour's aggregate, so every non-isolated node is
  // aggregated here.  A node left over would be a broken invariant.
  for (i64 i = 0; i < nn; ++i)
    if (!st.iso[i] && agg[i] < 0) return -1;
  return next;
}

bool build_smoother(const Csr& A, int b, const AmgParams& prm, std::vector<double>& M) {
  const i64 nn = A.nr / b;
  M.assign((size_t)nn * b * b, 0.0);
  for (i64 i = 0; i < nn; ++i) {
    BlockRow br = gather_block_row(A, b, i);
    const double* D = find_block(br, b, (i32)i);
    if (!D) return false;
    double* Mi = &M[(size_t)i * b * b];
    if (prm.smoother == JACOBI) {
      double Dinv[64];
      if (!gj_inverse(b, D, Dinv)) return false;
      for (int t = 0; t < b * b; ++t) Mi[t] = prm.jacobi_omega * Dinv[t];
    } else if (prm.smoother == SPAI0_SCALAR) {
      for (int r = 0; r < b; ++r) {
        double s = 0.0;
        const i64 row = i * b + r;
        for (i64 k = A.ptr[row]; k < A.ptr[row + 1]; ++k) s = s + A.val[k] * A.val[k];
        Mi[r * b + r] = D[r * b + r] / s;
      }
    } else {
      // G = sum_j A_ij A_ij^T (j ascending, then q ascending), M = A_ii^T G^-1.
      double G[64] = {0}, Ginv[64];
      for (size_t t = 0; t < br.cols.size(); ++t) {
        const double* X = &br.vals[t * b * b];
        for (int r = 0; r < b; ++r)
          for (int c = 0; c < b; ++c)
            for (int q = 0; q < b; ++q) G[r * b + c] = G[r * b + c] + X[r * b + q] * X[c * b + q];
      }
      if (!gj_inverse(b, G, Ginv)) return false;
      for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) {
          double s = 0.0;
          for (int q = 0; q < b; ++q) s = s + D[q * b + r] * Ginv[q * b + c];
          Mi[r * b + c] = s;
        }
    }
  }
  return true;
}

// One coarsening step: aggregates, P, R and the Galerkin operator.  With
// smooth_p false the prolongator is the tentative one (plain aggregation).
bool coarsen(Level& L, int b, double eps, bool smooth_p, Csr& Ac, const char** msg) {
  const Csr& A = L.A;
  const i64 nn = A.nr / b;
  Strength st = strength(A, b, eps);
  L.isolated = st.iso;
  L.n_agg = aggregate(st, L.agg);
  if (L.n_agg < 0) {
    *msg = "oracle: aggregation left a connected node unassigned";
    return false;
  }
  if (L.n_agg == 0 || L.n_agg >= nn) return false;

  // Tentative prolongator: identity block at (i, agg(i)), unnormalized.
  Csr Pt;
  Pt.nr = A.nr;
  Pt.nc = L.n_agg * b;
  Pt.ptr.assign(Pt.nr + 1, 0);
  for (i64 i = 0; i < nn; ++i)
    for (int r = 0; r < b; ++r) {
      if (L.agg[i] >= 0) {
        Pt.col.push_back(L.agg[i] * b + r);
        Pt.val.push_back(1.0);
      }
      Pt.ptr[i * b + r + 1] = (i64)Pt.col.size();
    }
  if (!smooth_p) {
    L.omega = 0.0;
    L.P = Pt;
    L.R = transpose(L.P);
    Csr AP = spgemm(A, L.P);
    Ac = spgemm(L.R, AP);
    return true;
  }

  // Filtered matrix: strong blocks kept, weak blocks added to the diagonal
  // block (starting from A_ii, weak blocks in ascending column order).
  Csr AF;
  AF.nr = A.nr;
  AF.nc = A.nc;
  AF.ptr.assign(AF.nr + 1, 0);
  std::vector<double> Dinv((size_t)nn * b * b);
  double rho = 0.0;
  for (i64 i = 0; i < nn; ++i) {
    BlockRow br = gather_block_row(A, b, i);
    const double* Aii = find_block(br, b, (i32)i);
    if (!Aii) {
      *msg = "oracle: missing diagonal block";
      return false;
    }
    std::vector<double> D(Aii, Aii + b * b);
    for (size_t t = 0; t < br.cols.size(); ++t) {
      const i32 j = br.cols[t];
      if (j == i || std::binary_search(st.S[i].begin(), st.S[i].end(), j)) continue;
      for (int q = 0; q < b * b; ++q) D[q] = D[q] + br.vals[t * b * b + q];
    }
    std::vector<i32> cols;
    std::vector<double> vals;
    for (size_t t = 0; t < br.cols.size(); ++t) {
      const i32 j = br.cols[t];
      if (j == i) {
        cols.push_back(j);
        vals.insert(vals.end(), D.begin(), D.end());
      } else if (std::binary_search(st.S[i].begin(), st.S[i].end(), j)) {
        cols.push_back(j);
        vals.insert(vals.end(), br.vals.begin() + t * b * b, br.vals.begin() + (t + 1) * b * b);
      }
    }
    push_block_row(AF, b, i, cols, vals);
    if (!gj_inverse(b, D.data(), &Dinv[(size_t)i * b * b])) {
      *msg = "oracle: singular filtered diagonal block";
      return false;
    }
    if (st.iso[i]) continue;
    // Gershgorin row sums of D^-1 A_F over S_i and i, ascending block column.
    std::vector<double> W(b * b);
    std::vector<double> rowsum(b, 0.0);
    for (size_t t = 0; t < cols.size(); ++t) {
      block_mul(b, &Dinv[(size_t)i * b * b], &vals[t * b * b], W.data());
      for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) rowsum[r] = rowsum[r] + std::fabs(W[r * b + c]);
    }
    for (int r = 0; r < b; ++r) rho = std::max(rho, rowsum[r]);
  }
  if (!(rho > 0.0)) {
    *msg = "oracle: zero spectral radius estimate";
    return false;
  }
  L.omega = (4.0 / 3.0) / rho;

  // P = P_tent - omega D^-1 (A_F P_tent).
  Csr T = spgemm(AF, Pt);
  L.P.nr = A.nr;
  L.P.nc = Pt.nc;
  L.P.ptr.assign(L.P.nr + 1, 0);
  for (i64 i = 0; i < nn; ++i) {
    std::vector<i32> cols;
    std::vector<double> vals;
    if (L.agg[i] >= 0) {
      BlockRow tr = gather_block_row(T, b, i);
      std::vector<double> W(b * b);
      for (size_t t = 0; t < tr.cols.size(); ++t) {
        block_mul(b, &Dinv[(size_t)i * b * b], &tr.vals[t * b * b], W.data());
        cols.push_back(tr.cols[t]);
        for (int r = 0; r < b; ++r)
          for (int c = 0; c < b; ++c) {
            const double id = (tr.cols[t] == L.agg[i] && r == c) ? 1.0 : 0.0;
            vals.push_back(id - L.omega * W[r * b + c]);
          }
      }
    }
    push_block_row(L.P, b, i, cols, vals);
  }
  L.R = transpose(L.P);
  Csr AP = spgemm(A, L.P);
  Ac = spgemm(L.R, AP);
  return true;
}

}  // namespace

bool amg_build(const Csr& A, int b, const AmgParams& prm, Hierarchy& H, const char** msg) {
  H.b = b;
  H.levels.clear();
  H.levels.emplace_back();
  H.levels[0].A = A;
  double eps = prm.eps_strong;
  for (int l = 0;; ++l) {
    Level& L = H.levels[l];
    bool last = L.A.nr <= prm.coarse_enough || l == prm.max_levels - 1;
    Csr Ac;
    if (!last) {
      *msg = nullptr;
      if (!coarsen(L, b, eps, prm.smooth_p, Ac, msg)) {
        if (*msg) return false;
        last = true;
        L.P = Csr();
        L.R = Csr();
        L.agg.clear();
      }
    }
    if (last) {
      if (!lu_factor(L.A, H.coarse)) {
        *msg = "oracle: singular coarsest matrix";
        return false;
      }
      return true;
    }
    if (prm.smoother == ILU0) {
      if (!ilu_build(L.A, b, 0, prm.ilu_sweeps, L.F, msg)) return false;
    } else if (prm.smoother == ILUT) {
      if (!ilut_build(L.A, b, prm.ilut_p, prm.ilut_tau, prm.ilu_sweeps, L.F, msg)) return false;
    } else if (!build_smoother(L.A, b, prm, L.M)) {
      *msg = "oracle: singular smoother block";
      return false;
    }
    eps = 0.5 * eps;
    H.levels.emplace_back();
    H.levels.back().A = std::move(Ac);
  }
}

bool amg_transpose(const Hierarchy& H, Hierarchy& Ht, const char** msg) {
  const int b = H.b;
  for (const Level& L : H.levels)
    if (!L.F.cols.empty()) {
      *msg = "oracle: no transposed cycle with the ILU smoother";
      return false;
    }
  Ht.b = b;
  Ht.transposed = true;
  Ht.levels.resize(H.levels.size());
  for (size_t l = 0; l < H.levels.size(); ++l) {
    const Level& L = H.levels[l];
    Level& T = Ht.levels[l];
    T.A = transpose(L.A);
    T.P = L.P;
    T.R = L.R;
    T.agg = L.agg;
    T.n_agg = L.n_agg;
    T.M.resize(L.M.size());
    const i64 nn = (i64)L.M.size() / (b * b);
    for (i64 i = 0; i < nn; ++i)
      for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) T.M[i * b * b + r * b + c] = L.M[i * b * b + c * b + r];
  }
  if (!lu_factor(Ht.levels.back().A, Ht.coarse)) {
    *msg = "oracle: singular transposed coarsest matrix";
    return false;
  }
  return true;
}

namespace {
void apply_M(int b, const std::vector<double>& M, const double* r, double* z, bool add) {
  const i64 nn = (i64)M.size() / (b * b);
  for (i64 i = 0; i < nn; ++i)
    for (int p = 0; p < b; ++p) {
      double s = 0.0;
      for (int q = 0; q < b; ++q) s = s + M[i * b * b + p * b + q] * r[i * b + q];
      z[i * b + p] = add ? z[i * b + p] + s : s;
    }
}
}  // namespace

// V(1,1): z = M r; t = r - A z; r_c = R t; z_c = V(l+1, r_c); z += P z_c;
// z += M (r - A z).  The coarsest level solves exactly.
void vcycle(const Hierarchy& H, int l, const double* r, double* z) {
  const Level& L = H.levels[l];
  const i64 n = L.A.nr;
  if (l + 1 == (int)H.levels.size()) {
    lu_solve(H.coarse, r, z);
    return;
  }
  const int b = H.b;
  std::vector<double> t(n), rc(L.P.nc), zc(L.P.nc), pz(n);
  const bool ilu = !L.F.cols.empty();
  if (ilu) ilu_apply(L.F, r, z);   // z = ILU^-1 r
  else apply_M(b, L.M, r, z, false);
  spmv(L.A, z, t.data());
  for (i64 i = 0; i < n; ++i) t[i] = r[i] - t[i];
  spmv(L.R, t.data(), rc.data());
  vcycle(H, l + 1, rc.data(), zc.data());
  spmv(L.P, zc.data(), pz.data());
  for (i64 i = 0; i < n; ++i) z[i] = z[i] + pz[i];
  spmv(L.A, z, t.data());
  for (i64 i = 0; i < n; ++i) t[i] = r[i] - t[i];
  if (ilu) {
    std::vector<double> w(n);
    ilu_apply(L.F, t.data(), w.data());
    for (i64 i = 0; i < n; ++i) z[i] = z[i] + w[i];
  } else {
    apply_M(b, L.M, t.data(), z, true);
  }
}

}  // namespace orc
