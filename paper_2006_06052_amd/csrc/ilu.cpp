// Host factorization of the block ILU(k) preconditioner (k = 0 or 1).
//
// The paper's monolithic variant preconditions IDR(5) with ILU(1) (Section 4,
// the ILU(1) solver listing).  The factorization is taken on the b x b blocks:
// the pattern of block row i is A's pattern (level 0) plus the blocks (i, j)
// reached through an eliminated block k < i with lev(i,k) + lev(k,j) + 1 <= K;
// the numeric phase eliminates k < i in ascending order, L(i,k) = W(i,k)
// U(k,k)^-1 and W(i,j) -= L(i,k) U(k,j) for every later j of both patterns.
// All arithmetic is FP64 without contraction, block products with the inner
// index ascending, so the factors are reproducible bit for bit.
//
// The result is split for the device: L (blocks strictly below the diagonal),
// U (strictly above) and Dinv = U(i,i)^-1, which the solve phase applies with
// Jacobi sweeps on each triangular factor.
#include "host.hpp"

#include <algorithm>
#include <cmath>
#include <map>

namespace mgk {

namespace {

void block_mul(int b, const double* X, const double* Y, double* W) {
  for (int r = 0; r < b; ++r)
    for (int c = 0; c < b; ++c) {
      double s = 0.0;
      for (int q = 0; q < b; ++q) s = s + X[r * b + q] * Y[q * b + c];
      W[r * b + c] = s;
    }
}

}  // namespace

int ilu_factor(const HBsr& A, int level, IluFactors& out, std::string& err) {
  if (A.br != A.bc) {
    err = "ILU needs square blocks";
    return -1;
  }
  if (level < 0 || level > 1) {
    err = "ILU(k) supports k = 0 and k = 1";
    return -1;
  }
  const int b = A.br, bs = b * b;
  const int32_t n = A.nbr;
  std::vector<std::vector<int32_t>> cols(n);
  std::vector<std::vector<int>> lev(n);
  std::vector<std::vector<double>> vals(n);
  std::vector<double> Dinv((size_t)n * bs);
  std::vector<double> T(bs), Pr(bs);
  for (int32_t i = 0; i < n; ++i) {
    std::map<int32_t, int> L;
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) L[A.col[k]] = 0;
    for (auto it = L.begin(); it != L.end() && it->first < i; ++it) {
      const int32_t k = it->first;
      const int lik = it->second;
      for (size_t t = 0; t < cols[k].size(); ++t) {
        const int32_t j = cols[k][t];
        if (j <= k) continue;
        const int l = lik + lev[k][t] + 1;
        if (l > level) continue;
        auto f = L.find(j);
        if (f == L.end()) L[j] = l;
        else f->second = std::min(f->second, l);
      }
    }
    std::vector<int32_t>& ci = cols[i];
    for (auto& kv : L) {
      ci.push_back(kv.first);
      lev[i].push_back(kv.second);
    }
    std::vector<double>& W = vals[i];
    W.assign(ci.size() * bs, 0.0);
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const size_t p = std::lower_bound(ci.begin(), ci.end(), A.col[k]) - ci.begin();
      std::copy(A.blk(k), A.blk(k) + bs, &W[p * bs]);
    }
    for (size_t p = 0; p < ci.size() && ci[p] < i; ++p) {
      const int32_t k = ci[p];
      block_mul(b, &W[p * bs], &Dinv[(size_t)k * bs], T.data());
      std::copy(T.begin(), T.end(), &W[p * bs]);
      for (size_t t = 0; t < cols[k].size(); ++t) {
        const int32_t j = cols[k][t];
        if (j <= k) continue;
        const auto q = std::lower_bound(ci.begin(), ci.end(), j);
        if (q == ci.end() || *q != j) continue;
        block_mul(b, &W[p * bs], &vals[k][t * bs], Pr.data());
        double* Wij = &W[(size_t)(q - ci.begin()) * bs];
        for (int e = 0; e < bs; ++e) Wij[e] = Wij[e] - Pr[e];
      }
    }
    const auto d = std::lower_bound(ci.begin(), ci.end(), i);
    if (d == ci.end() || *d != i) {
      err = "ILU: a block row has no diagonal block";
      return -1;
    }
    if (!gauss_jordan_inverse(b, &W[(size_t)(d - ci.begin()) * bs], &Dinv[(size_t)i * bs])) {
      err = "ILU: singular pivot block";
      return -4;
    }
  }
  auto init = [&](HBsr& M) {
    M = HBsr();
    M.br = M.bc = b;
    M.nbr = M.nbc = n;
    M.ptr.assign(n + 1, 0);
  };
  init(out.L);
  init(out.U);
  for (int32_t i = 0; i < n; ++i) {
    for (size_t t = 0; t < cols[i].size(); ++t) {
      const int32_t j = cols[i][t];
      if (j == i) continue;
      HBsr& M = j < i ? out.L : out.U;
      M.col.push_back(j);
      M.val.insert(M.val.end(), &vals[i][t * bs], &vals[i][t * bs] + bs);
    }
    out.L.ptr[i + 1] = (int32_t)out.L.col.size();
    out.U.ptr[i + 1] = (int32_t)out.U.col.size();
  }
  out.Dinv = std::move(Dinv);
  return 0;
}

// Block ILUT(p, tau) (Saad's threshold ILU, Iterative Methods for Sparse Linear Systems,
// Sec. 10.4), the smoother the paper names for its Schur velocity AMG (Section 4, the V2
// and V3 listings), on b x b blocks with Frobenius norms in place of magnitudes.  Block
// row i is eliminated against the already finished rows:
//   drop tolerance t_i = tau * ||A(i, :)||_F over the row's stored entries (block
//     columns ascending, entries row-major);
//   working row w = A(i, :); for k < i in ascending order, fill included: w(k) = w(k)
//     U(k,k)^-1, dropped when ||w(k)||_F < t_i, otherwise w(j) -= w(k) U(k,j) for the
//     stored blocks j > k of U's row k (absent w(j) start at zero);
//   upper blocks with ||w(j)||_F < t_i are dropped;
//   L keeps at most floor(p n_L) and U at most floor(p n_U) blocks, n_L and n_U being
//     A's stored blocks of row i below and above the diagonal: the largest norms, ties to
//     the smaller block column; the diagonal block is always kept.
// Same arithmetic rules as ILU(k), so the factors are reproducible bit for bit.
int ilut_factor(const HBsr& A, double p, double tau, IluFactors& out, std::string& err) {
  if (A.br != A.bc) {
    err = "ILUT needs square blocks";
    return -1;
  }
  if (!(p >= 0.0) || !(tau >= 0.0) || !std::isfinite(p) || !std::isfinite(tau)) {
    err = "ILUT needs finite p >= 0 and tau >= 0";
    return -1;
  }
  const int b = A.br, bs = b * b;
  const int32_t n = A.nbr;
  auto norm = [bs](const double* X) {
    double s = 0.0;
    for (int e = 0; e < bs; ++e) s = s + X[e] * X[e];
    return std::sqrt(s);
  };
  auto init = [&](HBsr& M) {
    M = HBsr();
    M.br = M.bc = b;
    M.nbr = M.nbc = n;
    M.ptr.assign(n + 1, 0);
  };
  init(out.L);
  init(out.U);
  std::vector<double> Dinv((size_t)n * bs);
  std::vector<double> T(bs), Pr(bs);
  struct Cand {
    int32_t col;
    double nrm;
  };
  std::vector<Cand> lo, up;
  for (int32_t i = 0; i < n; ++i) {
    double s2 = 0.0;
    int nL = 0, nU = 0;
    std::map<int32_t, std::vector<double>> w;
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const double* X = A.blk(k);
      for (int e = 0; e < bs; ++e) s2 = s2 + X[e] * X[e];
      nL += A.col[k] < i;
      nU += A.col[k] > i;
      w[A.col[k]].assign(X, X + bs);
    }
    const double tol = tau * std::sqrt(s2);
    for (auto it = w.begin(); it != w.end() && it->first < i;) {
      const int32_t k = it->first;
      block_mul(b, it->second.data(), &Dinv[(size_t)k * bs], T.data());
      if (norm(T.data()) < tol) {
        it = w.erase(it);
        continue;
      }
      it->second.assign(T.begin(), T.end());
      for (int32_t q = out.U.ptr[k]; q < out.U.ptr[k + 1]; ++q) {
        block_mul(b, T.data(), &out.U.val[(size_t)q * bs], Pr.data());
        std::vector<double>& wj = w[out.U.col[q]];
        if (wj.empty()) wj.assign(bs, 0.0);
        for (int e = 0; e < bs; ++e) wj[e] = wj[e] - Pr[e];
      }
      ++it;
    }
    const auto d = w.find(i);
    if (d == w.end()) {
      err = "ILUT: a block row has no diagonal block";
      return -1;
    }
    lo.clear();
    up.clear();
    for (const auto& kv : w) {
      const double nr = norm(kv.second.data());
      if (kv.first < i) lo.push_back({kv.first, nr});
      else if (kv.first > i && !(nr < tol)) up.push_back({kv.first, nr});
    }
    auto select = [](std::vector<Cand>& v, size_t cap) {
      std::stable_sort(v.begin(), v.end(), [](const Cand& a, const Cand& c) {
        return a.nrm > c.nrm;
      });
      if (v.size() > cap) v.resize(cap);
      std::sort(v.begin(), v.end(), [](const Cand& a, const Cand& c) { return a.col < c.col; });
    };
    select(lo, (size_t)std::floor(p * nL));
    select(up, (size_t)std::floor(p * nU));
    if (!gauss_jordan_inverse(b, d->second.data(), &Dinv[(size_t)i * bs])) {
      err = "ILUT: singular pivot block";
      return -4;
    }
    for (const Cand& c : lo) {
      out.L.col.push_back(c.col);
      out.L.val.insert(out.L.val.end(), w[c.col].begin(), w[c.col].end());
    }
    for (const Cand& c : up) {
      out.U.col.push_back(c.col);
      out.U.val.insert(out.U.val.end(), w[c.col].begin(), w[c.col].end());
    }
    out.L.ptr[i + 1] = (int32_t)out.L.col.size();
    out.U.ptr[i + 1] = (int32_t)out.U.col.size();
  }
  out.Dinv = std::move(Dinv);
  return 0;
}

}  // namespace mgk
