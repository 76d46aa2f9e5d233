// Oracle sparse and dense primitives.  TEST INFRASTRUCTURE ONLY (see oracle.hpp).
//
// The solve-phase vocabulary the paper names for its backends: the matrix-vector
// product inside the residual, and inner products (Section 2.3, "Backends").
#include <algorithm>
#include <cmath>
#include <cstring>
#include "oracle.hpp"

namespace orc {

// y = A x.  Each row sums its entries in ascending column order.  Rows are
// independent, so threading over rows does not change any result.
void spmv(const Csr& A, const double* x, double* y) {
#pragma omp parallel for schedule(static)
  for (i64 r = 0; r < A.nr; ++r) {
    double s = 0.0;
    for (i64 k = A.ptr[r]; k < A.ptr[r + 1]; ++k) s = s + A.val[k] * x[A.col[k]];
    y[r] = s;
  }
}

double dot(i64 n, const double* a, const double* b) {
  double s = 0.0;
  for (i64 i = 0; i < n; ++i) s = s + a[i] * b[i];
  return s;
}

double nrm2(i64 n, const double* a) { return std::sqrt(dot(n, a, a)); }

Csr transpose(const Csr& A) {
  Csr T;
  T.nr = A.nc;
  T.nc = A.nr;
  T.ptr.assign(T.nr + 1, 0);
  for (i64 k = 0; k < A.ptr[A.nr]; ++k) T.ptr[A.col[k] + 1]++;
  for (i64 r = 0; r < T.nr; ++r) T.ptr[r + 1] += T.ptr[r];
  T.col.resize(A.ptr[A.nr]);
  T.val.resize(A.ptr[A.nr]);
  std::vector<i64> next(T.ptr.begin(), T.ptr.end() - 1);
  // Visiting source rows in ascending order leaves every output row sorted.
  for (i64 r = 0; r < A.nr; ++r)
    for (i64 k = A.ptr[r]; k < A.ptr[r + 1]; ++k) {
      i64 d = next[A.col[k]]++;
      T.col[d] = (i32)r;
      T.val[d] = A.val[k];
    }
  return T;
}

// Gustavson product.  Output entry (r, c) accumulates A(r,k) * B(k,c) for k in
// ascending order, starting from the first product.  Every structurally
// reached entry is stored, including exact zeros (no value-based dropping).
Csr spgemm(const Csr& A, const Csr& B) {
  Csr C;
  C.nr = A.nr;
  C.nc = B.nc;
  C.ptr.assign(C.nr + 1, 0);
  std::vector<std::vector<i32>> rcols(C.nr);
  std::vector<std::vector<double>> rvals(C.nr);
#pragma omp parallel
  {
    std::vector<i64> pos(B.nc, -1);
    std::vector<i32> cols;
    std::vector<double> acc;
#pragma omp for schedule(dynamic, 256)
    for (i64 r = 0; r < A.nr; ++r) {
      cols.clear();
      acc.clear();
      for (i64 ka = A.ptr[r]; ka < A.ptr[r + 1]; ++ka) {
        const double a = A.val[ka];
        const i64 k = A.col[ka];
        for (i64 kb = B.ptr[k]; kb < B.ptr[k + 1]; ++kb) {
          const i32 c = B.col[kb];
          const double p = a * B.val[kb];
          if (pos[c] < 0) {
            pos[c] = (i64)cols.size();
            cols.push_back(c);
            acc.push_back(p);
          } else {
            acc[pos[c]] = acc[pos[c]] + p;
          }
        }
      }
      std::vector<i32> order(cols.size());
      for (size_t t = 0; t < cols.size(); ++t) order[t] = (i32)t;
      std::sort(order.begin(), order.end(),
                [&](i32 u, i32 v) { return cols[u] < cols[v]; });
      rcols[r].resize(cols.size());
      rvals[r].resize(cols.size());
      for (size_t t = 0; t < cols.size(); ++t) {
        rcols[r][t] = cols[order[t]];
        rvals[r][t] = acc[order[t]];
        pos[cols[order[t]]] = -1;
      }
    }
  }
  for (i64 r = 0; r < C.nr; ++r) C.ptr[r + 1] = C.ptr[r] + (i64)rcols[r].size();
  C.col.resize(C.ptr[C.nr]);
  C.val.resize(C.ptr[C.nr]);
  for (i64 r = 0; r < C.nr; ++r) {
    std::copy(rcols[r].begin(), rcols[r].end(), C.col.begin() + C.ptr[r]);
    std::copy(rvals[r].begin(), rvals[r].end(), C.val.begin() + C.ptr[r]);
  }
  return C;
}

BlockRow gather_block_row(const Csr& A, int b, i64 i) {
  BlockRow br;
  for (int r = 0; r < b; ++r) {
    const i64 row = i * b + r;
    for (i64 k = A.ptr[row]; k < A.ptr[row + 1]; ++k) {
      const i32 j = A.col[k] / b;
      auto it = std::lower_bound(br.cols.begin(), br.cols.end(), j);
      size_t t = (size_t)(it - br.cols.begin());
      if (it == br.cols.end() || *it != j) {
        br.cols.insert(it, j);
        br.vals.insert(br.vals.begin() + t * b * b, (size_t)b * b, 0.0);
      }
      br.vals[t * b * b + r * b + (A.col[k] % b)] = A.val[k];
    }
  }
  return br;
}

// Gauss-Jordan on the augmented matrix [D | I].  For pivot column k: choose
// the row p >= k with the largest |D(p,k)| (first such row), swap rows k and p,
// divide row k by the pivot, then for every other row r (ascending) subtract
// D(r,k) times row k.  All 2b columns are updated in ascending order.
bool gj_inverse(int b, const double* D, double* Dinv) {
  const int w = 2 * b;
  double M[2 * 8 * 8];
  for (int r = 0; r < b; ++r)
    for (int c = 0; c < w; ++c)
      M[r * w + c] = c < b ? D[r * b + c] : (c - b == r ? 1.0 : 0.0);
  for (int k = 0; k < b; ++k) {
    int p = k;
    double best = std::fabs(M[k * w + k]);
    for (int r = k + 1; r < b; ++r)
      if (std::fabs(M[r * w + k]) > best) {
        best = std::fabs(M[r * w + k]);
        p = r;
      }
    if (!(best > 0.0) || !std::isfinite(best)) return false;
    if (p != k)
      for (int c = 0; c < w; ++c) std::swap(M[k * w + c], M[p * w + c]);
    const double piv = M[k * w + k];
    for (int c = 0; c < w; ++c) M[k * w + c] = M[k * w + c] / piv;
    for (int r = 0; r < b; ++r) {
      if (r == k) continue;
      const double f = M[r * w + k];
      for (int c = 0; c < w; ++c) M[r * w + c] = M[r * w + c] - f * M[k * w + c];
    }
  }
  for (int r = 0; r < b; ++r)
    for (int c = 0; c < b; ++c) Dinv[r * b + c] = M[r * w + b + c];
  return true;
}

bool lu_factor(const Csr& A, DenseLU& F) {
  const int n = (int)A.nr;
  F.n = n;
  F.lu.assign((size_t)n * n, 0.0);
  F.piv.resize(n);
  for (i64 r = 0; r < n; ++r)
    for (i64 k = A.ptr[r]; k < A.ptr[r + 1]; ++k) F.lu[(size_t)r * n + A.col[k]] = A.val[k];
  double* a = F.lu.data();
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(a[(size_t)k * n + k]);
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * n + k]) > best) {
        best = std::fabs(a[(size_t)r * n + k]);
        p = r;
      }
    if (!(best > 0.0)) return false;
    F.piv[k] = p;
    if (p != k)
      for (int c = 0; c < n; ++c) std::swap(a[(size_t)k * n + c], a[(size_t)p * n + c]);
    const double piv = a[(size_t)k * n + k];
#pragma omp parallel for schedule(static)
    for (int r = k + 1; r < n; ++r) {
      const double l = a[(size_t)r * n + k] / piv;
      a[(size_t)r * n + k] = l;
      for (int c = k + 1; c < n; ++c) a[(size_t)r * n + c] = a[(size_t)r * n + c] - l * a[(size_t)k * n + c];
    }
  }
  return true;
}

// z = A^-1 r from P A = L U: apply the row swaps, then L y = Pr, then U z = y.
void lu_solve(const DenseLU& F, const double* r, double* z) {
  const int n = F.n;
  std::vector<double> y(r, r + n);
  for (int k = 0; k < n; ++k) std::swap(y[k], y[F.piv[k]]);
  const double* a = F.lu.data();
  for (int i = 0; i < n; ++i) {
    double s = y[i];
    for (int k = 0; k < i; ++k) s = s - a[(size_t)i * n + k] * y[k];
    y[i] = s;
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < n; ++k) s = s - a[(size_t)i * n + k] * y[k];
    y[i] = s / a[(size_t)i * n + i];
  }
  std::memcpy(z, y.data(), sizeof(double) * n);
}

}  // namespace orc
