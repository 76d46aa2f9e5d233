// Problem ingest on the host: validation, scalar CSR to block CSR, the
// synthetic finite-difference Stokes assembler, and the velocity/pressure
// split of the Schur pressure correction.
#include <algorithm>
#include <cmath>
#include <cstring>
#include "host.hpp"

namespace mgk {

int validate_bsr(const HBsr& A, std::string& err) {
  if (A.nbr < 0 || A.nbc < 0 || (int)A.ptr.size() != A.nbr + 1 || A.ptr[0] != 0) {
    err = "invalid BSR: row pointer size or origin";
    return -1;
  }
  for (int32_t i = 0; i < A.nbr; ++i) {
    if (A.ptr[i + 1] < A.ptr[i]) {
      err = "invalid BSR: row pointer decreases at block row " + std::to_string(i);
      return -1;
    }
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      if (A.col[k] < 0 || A.col[k] >= A.nbc) {
        err = "invalid BSR: column out of range in block row " + std::to_string(i);
        return -1;
      }
      if (k > A.ptr[i] && A.col[k] <= A.col[k - 1]) {
        err = "invalid BSR: block columns not strictly ascending in block row " +
              std::to_string(i);
        return -1;
      }
    }
  }
  for (double v : A.val)
    if (!std::isfinite(v)) {
      err = "invalid BSR: non-finite value";
      return -1;
    }
  return 0;
}

// Block row i gathers scalar rows i*b .. i*b+b-1; a block is stored when any
// of its scalar entries is, and absent entries of a stored block are zero
// (the layout of the worked 6x6 example in Section 4).
int csr_to_bsr(int32_t nrows, const int32_t* ptr, const int32_t* col, const double* val, int b,
               HBsr& out, std::string& err) {
  if (b < 1 || b > 4 || nrows < 0 || nrows % b) {
    err = "csr_to_bsr: rows must be a multiple of the block size (1..4)";
    return -1;
  }
  const int32_t nb = nrows / b;
  out = HBsr();
  out.br = out.bc = b;
  out.nbr = out.nbc = nb;
  out.ptr.assign(nb + 1, 0);
  std::vector<int32_t> cols;
  for (int32_t i = 0; i < nb; ++i) {
    cols.clear();
    for (int r = 0; r < b; ++r) {
      const int32_t row = i * b + r;
      for (int32_t k = ptr[row]; k < ptr[row + 1]; ++k) {
        if (col[k] < 0 || col[k] >= nrows || (k > ptr[row] && col[k] <= col[k - 1])) {
          err = "csr_to_bsr: columns out of range or not ascending in row " + std::to_string(row);
          return -1;
        }
        cols.push_back(col[k] / b);
      }
    }
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    out.col.insert(out.col.end(), cols.begin(), cols.end());
    out.ptr[i + 1] = (int32_t)out.col.size();
  }
  out.val.assign((size_t)out.col.size() * b * b, 0.0);
  for (int32_t i = 0; i < nb; ++i)
    for (int r = 0; r < b; ++r) {
      const int32_t row = i * b + r;
      for (int32_t k = ptr[row]; k < ptr[row + 1]; ++k) {
        const int32_t J = col[k] / b;
        const int32_t* f = std::lower_bound(out.col.data() + out.ptr[i],
                                            out.col.data() + out.ptr[i + 1], J);
        const int64_t t = f - out.col.data();
        out.val[(size_t)t * b * b + r * b + (col[k] % b)] = val[k];
      }
    }
  return 0;
}

void stokes_sizes(int n, int32_t& nbr, int64_t& nnzb) {
  const int64_t nn = (int64_t)n * n * n, ni = (int64_t)(n - 2) * (n - 2) * (n - 2);
  nbr = (int32_t)nn;
  nnzb = 7 * ni + (nn - ni);
}

// 7-point stabilized FD Stokes on n^3 nodes (see mgk.h for the scheme).
// Velocity row c of an interior node g, neighbour m = g + s e_d:
//   (c,c) = -mu_E / h^2,  (c,3) = s/(2h) when d == c,
// pressure row of g:  (3,d) = -s/(2h),  (3,3) = 1;
// the self block holds sum_E mu_E / h^2 on the velocity diagonal and -6 for
// the pressure.  mu_E is the mean of theta over the four cells around edge E,
// summed in ascending cell id and scaled by 1/4.
void stokes_assemble(int n, const double* theta, int32_t* ptr, int32_t* col, double* val) {
  const double inv_h2 = (double)((n - 1) * (n - 1));
  const double inv_2h = 0.5 * (double)(n - 1);
  const int64_t n1 = n - 1;
  auto cell = [&](int64_t i, int64_t j, int64_t k) { return i + n1 * (j + n1 * k); };
  auto edge_mu = [&](int i, int j, int k, int d, int s) -> double {
    if (!theta) return 1.0;
    int lo[3] = {i, j, k};
    if (s < 0) lo[d] -= 1;
    int64_t ids[4];
    int t = 0;
    for (int a = 0; a < 2; ++a)
      for (int bb = 0; bb < 2; ++bb) {
        int q[3] = {lo[0], lo[1], lo[2]};
        const int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
        q[e1] -= a;
        q[e2] -= bb;
        ids[t++] = cell(q[0], q[1], q[2]);
      }
    std::sort(ids, ids + 4);
    double s4 = theta[ids[0]];
    for (int u = 1; u < 4; ++u) s4 = s4 + theta[ids[u]];
    return 0.25 * s4;
  };
  int64_t nz = 0;
  ptr[0] = 0;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const int64_t g = i + (int64_t)n * (j + (int64_t)n * k);
        const bool inner = i > 0 && j > 0 && k > 0 && i < n - 1 && j < n - 1 && k < n - 1;
        if (!inner) {
          col[nz] = (int32_t)g;
          double* B = val + nz * 16;
          std::memset(B, 0, sizeof(double) * 16);
          for (int c = 0; c < 4; ++c) B[c * 5] = 1.0;
          ++nz;
          ptr[g + 1] = (int32_t)nz;
          continue;
        }
        double mu[3][2];
        for (int d = 0; d < 3; ++d) {
          mu[d][0] = edge_mu(i, j, k, d, -1);
          mu[d][1] = edge_mu(i, j, k, d, +1);
        }
        double diag = 0.0;
        for (int d = 0; d < 3; ++d) {
          diag = diag + mu[d][0] * inv_h2;
          diag = diag + mu[d][1] * inv_h2;
        }
        const int64_t stride[3] = {1, n, (int64_t)n * n};
        // ascending neighbour order: -z, -y, -x, self, +x, +y, +z
        const int dirs[7] = {2, 1, 0, -1, 0, 1, 2};
        const int sgn[7] = {-1, -1, -1, 0, 1, 1, 1};
        for (int q = 0; q < 7; ++q) {
          double* B = val + nz * 16;
          std::memset(B, 0, sizeof(double) * 16);
          if (dirs[q] < 0) {
            col[nz] = (int32_t)g;
            for (int c = 0; c < 3; ++c) B[c * 4 + c] = diag;
            B[15] = -6.0;
          } else {
            const int d = dirs[q], s = sgn[q];
            col[nz] = (int32_t)(g + s * stride[d]);
            const double w = mu[d][s > 0 ? 1 : 0] * inv_h2;
            for (int c = 0; c < 3; ++c) B[c * 4 + c] = -w;
            B[d * 4 + 3] = s > 0 ? inv_2h : -inv_2h;
            B[3 * 4 + d] = s > 0 ? -inv_2h : inv_2h;
            B[15] = 1.0;
          }
          ++nz;
        }
        ptr[g + 1] = (int32_t)nz;
      }
}

// The scalar structure of the split is the set of nonzero entries: stored
// sub-blocks that are entirely zero are dropped, and zero entries inside the
// 1x3 and 3x1 coupling blocks take no part in the product that forms S.
int schur_split(const HBsr& A, bool diag_only, SchurParts& S, std::string& err) {
  if (A.br != 4 || A.bc != 4) {
    err = "Schur split needs 4x4 blocks with interleaved [u,v,w,p]";
    return -1;
  }
  const int32_t n = A.nbr;
  auto init = [&](HBsr& M, int br, int bc) {
    M = HBsr();
    M.br = br;
    M.bc = bc;
    M.nbr = M.nbc = n;
    M.ptr.assign(n + 1, 0);
  };
  init(S.Auu, 3, 3);
  init(S.Bup, 3, 1);
  init(S.Blo, 1, 3);
  init(S.C, 1, 1);
  for (int32_t i = 0; i < n; ++i) {
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const double* B = A.blk(k);
      double uu[9], up[3], lo[3], pp = B[15];
      bool nuu = false, nup = false, nlo = false;
      for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) {
          uu[r * 3 + c] = B[r * 4 + c];
          nuu |= uu[r * 3 + c] != 0.0;
        }
        up[r] = B[r * 4 + 3];
        lo[r] = B[12 + r];
        nup |= up[r] != 0.0;
        nlo |= lo[r] != 0.0;
      }
      const int32_t j = A.col[k];
      if (nuu) {
        S.Auu.col.push_back(j);
        S.Auu.val.insert(S.Auu.val.end(), uu, uu + 9);
      }
      if (nup) {
        S.Bup.col.push_back(j);
        S.Bup.val.insert(S.Bup.val.end(), up, up + 3);
      }
      if (nlo) {
        S.Blo.col.push_back(j);
        S.Blo.val.insert(S.Blo.val.end(), lo, lo + 3);
      }
      if (pp != 0.0) {
        S.C.col.push_back(j);
        S.C.val.push_back(pp);
      }
    }
    S.Auu.ptr[i + 1] = (int32_t)S.Auu.col.size();
    S.Bup.ptr[i + 1] = (int32_t)S.Bup.col.size();
    S.Blo.ptr[i + 1] = (int32_t)S.Blo.col.size();
    S.C.ptr[i + 1] = (int32_t)S.C.col.size();
  }
  // dinv = 1 / diag(A_uu) (scalar diagonal), W = B_lo dinv, S = C - W B_up.
  std::vector<double> dinv((size_t)n * 3, 0.0);
  for (int32_t i = 0; i < n; ++i) {
    const int32_t* b = S.Auu.col.data() + S.Auu.ptr[i];
    const int32_t* e = S.Auu.col.data() + S.Auu.ptr[i + 1];
    const int32_t* f = std::lower_bound(b, e, i);
    if (f == e || *f != i) {
      err = "Schur split: velocity block row without a diagonal block";
      return -1;
    }
    const double* D = S.Auu.blk(f - S.Auu.col.data());
    for (int c = 0; c < 3; ++c) {
      if (D[c * 4] == 0.0) {
        err = "Schur split: zero velocity diagonal";
        return -4;
      }
      dinv[(size_t)i * 3 + c] = 1.0 / D[c * 4];
    }
  }
  S.S = HBsr();
  S.S.br = S.S.bc = 1;
  S.S.nbr = S.S.nbc = n;
  S.S.ptr.assign(n + 1, 0);
  std::vector<int64_t> slot(n, -1);
  std::vector<int32_t> cols;
  std::vector<double> acc;
  for (int32_t i = 0; i < n; ++i) {
    cols.clear();
    acc.clear();
    // product row: sum over B_lo blocks (i,m) ascending, then component c, of
    // (B_lo(i,m)[c] * dinv(m,c)) * B_up(m,j)[c]
    for (int64_t k = S.Blo.ptr[i]; k < S.Blo.ptr[i + 1]; ++k) {
      const int32_t m = S.Blo.col[k];
      const double* lo = S.Blo.blk(k);
      for (int c = 0; c < 3; ++c) {
        if (lo[c] == 0.0) continue;   // zero entries of a stored sub-block are absent
        const double w = lo[c] * dinv[(size_t)m * 3 + c];
        for (int64_t q = S.Bup.ptr[m]; q < S.Bup.ptr[m + 1]; ++q) {
          const int32_t jj = S.Bup.col[q];
          if (S.Bup.blk(q)[c] == 0.0) continue;
          if (diag_only && jj != i) continue;   // only the diagonal of the product
          const double p = w * S.Bup.blk(q)[c];
          if (slot[jj] < 0) {
            slot[jj] = (int64_t)cols.size();
            cols.push_back(jj);
            acc.push_back(p);
          } else {
            acc[slot[jj]] = acc[slot[jj]] + p;
          }
        }
      }
    }
    // merge with C: C - product (an entry only in the product is 0 - product)
    std::vector<std::pair<int32_t, double>> row;
    for (size_t t = 0; t < cols.size(); ++t) row.emplace_back(cols[t], 0.0 - acc[t]);
    for (int64_t k = S.C.ptr[i]; k < S.C.ptr[i + 1]; ++k) {
      const int32_t jj = S.C.col[k];
      if (slot[jj] >= 0) row[slot[jj]].second = S.C.val[k] - acc[slot[jj]];
      else row.emplace_back(jj, S.C.val[k]);
    }
    for (int32_t jj : cols) slot[jj] = -1;
    std::sort(row.begin(), row.end());
    for (auto& e : row) {
      S.S.col.push_back(e.first);
      S.S.val.push_back(e.second);
    }
    S.S.ptr[i + 1] = (int32_t)S.S.col.size();
  }
  return 0;
}

int scalar_spai0(const HBsr& A, std::vector<double>& m, std::string& err) {
  if (A.br != 1 || A.bc != 1) {
    err = "scalar SPAI(0) needs 1x1 blocks";
    return -1;
  }
  m.assign(A.nbr, 0.0);
  for (int32_t i = 0; i < A.nbr; ++i) {
    double d = 0.0, q = 0.0;
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      q = q + A.val[k] * A.val[k];
      if (A.col[k] == i) d = A.val[k];
    }
    if (!(q > 0.0)) {
      err = "scalar SPAI(0): empty row";
      return -4;
    }
    m[i] = d / q;
  }
  return 0;
}

HBsr scalar_form(const HBsr& A) {
  const int b = A.br;
  HBsr S;
  S.br = S.bc = 1;
  S.nbr = A.nbr * b;
  S.nbc = A.nbc * b;
  S.ptr.assign(S.nbr + 1, 0);
  for (int32_t i = 0; i < A.nbr; ++i)
    for (int r = 0; r < b; ++r) {
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
        for (int c = 0; c < b; ++c) {
          const double v = A.blk(k)[r * b + c];
          if (v == 0.0) continue;
          S.col.push_back(A.col[k] * b + c);
          S.val.push_back(v);
        }
      S.ptr[(size_t)i * b + r + 1] = (int32_t)S.col.size();
    }
  return S;
}

}  // namespace mgk
