// Block incomplete LU factorization with level of fill k, applied with Jacobi
// sweeps on the triangular factors.
//
// The paper's monolithic variant preconditions IDR(5) with ILU(1) (Section 4,
// the ILU(1) solver listing), and its Schur variants smooth the velocity AMG
// with ILUT (ilut_build below).  ILU(k) is taken on b x b node blocks:
//   symbolic: the pattern of block row i is A's pattern (level 0) plus every
//     (i, j) reached through an eliminated k < i with level
//     lev(i,k) + lev(k,j) + 1 <= K, smallest level kept;
//   numeric (row-wise elimination in ascending k): W = A(i, :) on the pattern;
//     for k < i ascending: L(i,k) = W(i,k) U(k,k)^-1, then
//     W(i,j) -= L(i,k) U(k,j) for j > k in both patterns (j ascending);
//     U(i, j>=i) = W(i, j>=i).
// The factors are applied approximately, by Jacobi iterations on the two
// triangular systems (Anzt, Chow and Dongarra, 2015):
//   (I + L) y = r:  y = r, then `sweeps` times y <- r - L y;
//   (D + U) z = y:  z = D^-1 y, then `sweeps` times z <- D^-1 (y - U z),
// with L strictly lower, U strictly upper and D the diagonal blocks of U.
// With at least as many sweeps as the depth of the triangular dependency graph
// the application is the exact LU solve.
#include "oracle.hpp"

#include <algorithm>
#include <cmath>
#include <map>

namespace orc {

namespace {
// W = X Y for b x b row-major blocks, inner index ascending.
void bmul(int b, const double* X, const double* Y, double* W) {
  for (int r = 0; r < b; ++r)
    for (int c = 0; c < b; ++c) {
      double s = 0.0;
      for (int q = 0; q < b; ++q) s = s + X[r * b + q] * Y[q * b + c];
      W[r * b + c] = s;
    }
}
}  // namespace

bool ilu_build(const Csr& A, int b, int level, int sweeps, Ilu& F, const char** msg) {
  const i64 nn = A.nr / b;
  const int bs = b * b;
  F = Ilu();
  F.b = b;
  F.nn = nn;
  F.sweeps = sweeps;
  F.cols.resize(nn);
  F.vals.resize(nn);
  std::vector<std::vector<int>> lev(nn);
  F.Dinv.assign((size_t)nn * bs, 0.0);
  for (i64 i = 0; i < nn; ++i) {
    BlockRow br = gather_block_row(A, b, i);
    // symbolic: level of every (i, j), starting from A's pattern
    std::map<i32, int> L;
    for (i32 j : br.cols) L[j] = 0;
    for (auto it = L.begin(); it != L.end() && it->first < i; ++it) {
      const i32 k = it->first;
      const int lik = it->second;
      for (size_t t = 0; t < F.cols[k].size(); ++t) {
        const i32 j = F.cols[k][t];
        if (j <= k) continue;
        const int l = lik + lev[k][t] + 1;
        if (l > level) continue;
        auto f = L.find(j);
        if (f == L.end()) L[j] = l;
        else f->second = std::min(f->second, l);
      }
    }
    std::vector<i32> cols;
    for (auto& kv : L) {
      cols.push_back(kv.first);
      lev[i].push_back(kv.second);
    }
    // numeric
    std::vector<double> W(cols.size() * bs, 0.0);
    for (size_t t = 0; t < br.cols.size(); ++t) {
      const size_t p = std::lower_bound(cols.begin(), cols.end(), br.cols[t]) - cols.begin();
      std::copy(&br.vals[t * bs], &br.vals[t * bs] + bs, &W[p * bs]);
    }
    std::vector<double> T(bs);
    for (size_t p = 0; p < cols.size() && cols[p] < i; ++p) {
      const i32 k = cols[p];
      bmul(b, &W[p * bs], &F.Dinv[(size_t)k * bs], T.data());
      std::copy(T.begin(), T.end(), &W[p * bs]);   // L(i, k)
      for (size_t t = 0; t < F.cols[k].size(); ++t) {
        const i32 j = F.cols[k][t];
        if (j <= k) continue;
        const auto q = std::lower_bound(cols.begin(), cols.end(), j);
        if (q == cols.end() || *q != j) continue;
        std::vector<double> Pr(bs);
        bmul(b, &W[p * bs], &F.vals[k][t * bs], Pr.data());
        double* Wij = &W[(size_t)(q - cols.begin()) * bs];
        for (int e = 0; e < bs; ++e) Wij[e] = Wij[e] - Pr[e];
      }
    }
    const auto d = std::lower_bound(cols.begin(), cols.end(), (i32)i);
    if (d == cols.end() || *d != i) {
      *msg = "oracle: ILU needs a diagonal block in every row";
      return false;
    }
    if (!gj_inverse(b, &W[(size_t)(d - cols.begin()) * bs], &F.Dinv[(size_t)i * bs])) {
      *msg = "oracle: singular ILU pivot block";
      return false;
    }
    F.cols[i] = std::move(cols);
    F.vals[i] = std::move(W);
  }
  return true;
}

namespace {
double fnorm(int bs, const double* X) {
  double s = 0.0;
  for (int e = 0; e < bs; ++e) s = s + X[e] * X[e];
  return std::sqrt(s);
}
}  // namespace

// Block ILUT(p, tau): incomplete LU with threshold dropping and a cap on the fill per
// row (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Sec. 10.4, ILUT),
// taken on b x b node blocks with block norms in place of entry magnitudes.  Row i:
//   tol = tau * ||A(i, :)||_F (all stored entries of the block row);
//   w = A(i, :); for k < i in ascending order among w's blocks (fill included):
//     w(k) <- w(k) U(k,k)^-1; if ||w(k)||_F < tol drop it, else w(j) -= w(k) U(k,j)
//     for every block j > k of U's row k (creating fill);
//   U part: drop blocks j > i with ||w(j)||_F < tol;
//   keep at most floor(p * nL) blocks of the L part and floor(p * nU) of the U part (nL,
//   nU: A's blocks of row i below / above the diagonal), the largest norms first, ties
//   to the smaller column; the diagonal block is always kept and inverted.
bool ilut_build(const Csr& A, int b, double p, double tau, int sweeps, Ilu& F,
                const char** msg) {
  const i64 nn = A.nr / b;
  const int bs = b * b;
  F = Ilu();
  F.b = b;
  F.nn = nn;
  F.sweeps = sweeps;
  F.cols.resize(nn);
  F.vals.resize(nn);
  F.Dinv.assign((size_t)nn * bs, 0.0);
  std::vector<double> T(bs), Pr(bs);
  for (i64 i = 0; i < nn; ++i) {
    BlockRow br = gather_block_row(A, b, i);
    double s2 = 0.0;
    for (size_t e = 0; e < br.vals.size(); ++e) s2 = s2 + br.vals[e] * br.vals[e];
    const double tol = tau * std::sqrt(s2);
    int nL = 0, nU = 0;
    std::map<i32, std::vector<double>> w;
    for (size_t t = 0; t < br.cols.size(); ++t) {
      if (br.cols[t] < i) ++nL;
      if (br.cols[t] > i) ++nU;
      w[br.cols[t]].assign(&br.vals[t * bs], &br.vals[t * bs] + bs);
    }
    for (auto it = w.begin(); it != w.end() && it->first < i;) {
      const i32 k = it->first;
      bmul(b, it->second.data(), &F.Dinv[(size_t)k * bs], T.data());
      if (fnorm(bs, T.data()) < tol) {
        it = w.erase(it);
        continue;
      }
      it->second = T;
      for (size_t t = 0; t < F.cols[k].size(); ++t) {
        const i32 j = F.cols[k][t];
        if (j <= k) continue;
        bmul(b, T.data(), &F.vals[k][t * bs], Pr.data());
        auto f = w.find(j);
        if (f == w.end()) f = w.emplace(j, std::vector<double>(bs, 0.0)).first;
        for (int e = 0; e < bs; ++e) f->second[e] = f->second[e] - Pr[e];
      }
      ++it;
    }
    auto d = w.find((i32)i);
    if (d == w.end()) {
      *msg = "oracle: ILUT needs a diagonal block in every row";
      return false;
    }
    // candidates of each triangle in ascending column order, then the largest kept
    std::vector<std::pair<i32, double>> lo, up;
    for (auto& kv : w) {
      const double nr = fnorm(bs, kv.second.data());
      if (kv.first < i) lo.push_back({kv.first, nr});
      else if (kv.first > i && !(nr < tol)) up.push_back({kv.first, nr});
    }
    auto keep = [](std::vector<std::pair<i32, double>>& v, size_t cap) {
      std::stable_sort(v.begin(), v.end(), [](const std::pair<i32, double>& a,
                                              const std::pair<i32, double>& c) {
        return a.second > c.second;
      });
      if (v.size() > cap) v.resize(cap);
      std::sort(v.begin(), v.end());
    };
    keep(lo, (size_t)std::floor(p * nL));
    keep(up, (size_t)std::floor(p * nU));
    if (!gj_inverse(b, d->second.data(), &F.Dinv[(size_t)i * bs])) {
      *msg = "oracle: singular ILUT pivot block";
      return false;
    }
    for (auto& c : lo) {
      F.cols[i].push_back(c.first);
      F.vals[i].insert(F.vals[i].end(), w[c.first].begin(), w[c.first].end());
    }
    F.cols[i].push_back((i32)i);
    F.vals[i].insert(F.vals[i].end(), d->second.begin(), d->second.end());
    for (auto& c : up) {
      F.cols[i].push_back(c.first);
      F.vals[i].insert(F.vals[i].end(), w[c.first].begin(), w[c.first].end());
    }
  }
  return true;
}

void ilu_apply(const Ilu& F, const double* r, double* z) {
  const int b = F.b, bs = b * b;
  const i64 n = F.nn * b;
  std::vector<double> y(r, r + n), y2(n), w(n), z2(n);
  for (int s = 0; s < F.sweeps; ++s) {
    for (i64 i = 0; i < F.nn; ++i)
      for (int rr = 0; rr < b; ++rr) {
        double acc = 0.0;
        for (size_t t = 0; t < F.cols[i].size() && F.cols[i][t] < i; ++t) {
          const double* X = &F.vals[i][t * bs + rr * b];
          const double* v = &y[(size_t)F.cols[i][t] * b];
          for (int c = 0; c < b; ++c) acc = acc + X[c] * v[c];
        }
        y2[i * b + rr] = r[i * b + rr] - acc;
      }
    y.swap(y2);
  }
  auto dmul = [&](const double* in, double* out) {
    for (i64 i = 0; i < F.nn; ++i)
      for (int rr = 0; rr < b; ++rr) {
        double acc = 0.0;
        for (int c = 0; c < b; ++c) acc = acc + F.Dinv[(size_t)i * bs + rr * b + c] * in[i * b + c];
        out[i * b + rr] = acc;
      }
  };
  dmul(y.data(), z);
  for (int s = 0; s < F.sweeps; ++s) {
    for (i64 i = 0; i < F.nn; ++i)
      for (int rr = 0; rr < b; ++rr) {
        double acc = 0.0;
        for (size_t t = 0; t < F.cols[i].size(); ++t) {
          if (F.cols[i][t] <= i) continue;
          const double* X = &F.vals[i][t * bs + rr * b];
          const double* v = &z[(size_t)F.cols[i][t] * b];
          for (int c = 0; c < b; ++c) acc = acc + X[c] * v[c];
        }
        w[i * b + rr] = y[i * b + rr] - acc;
      }
    dmul(w.data(), z2.data());
    std::copy(z2.begin(), z2.end(), z);
  }
}

}  // namespace orc
