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

}  // namespace mgk
