// Oracle assembly of the stabilized equal-order finite-difference Stokes system
// and the exact gradient of a solve with respect to the per-cell viscosity.
// TEST INFRASTRUCTURE ONLY (see oracle.hpp).
//
// PDE: steady Stokes, -mu lap(u) + grad(p) = f, div(u) = 0 (Section 3, eq.
// StokesPDE).  The paper discretizes it with weak Galerkin elements; here the
// synthetic stand-in is a 7-point finite-difference scheme on the unit cube:
//   nodes (i,j,k) h, h = 1/(n-1); node id g = i + n (j + n k); unknown 4g+c
//   with c = 0,1,2 the velocity components and c = 3 the pressure.
//   Boundary node: identity row for all four unknowns.
//   Interior velocity row c:
//     sum_{d,s} mu_{g,d,s}/h^2 (u_c(g) - u_c(g + s e_d)) + (p(g+e_c) - p(g-e_c))/(2h)
//   Interior pressure row:
//     -sum_c (u_c(g+e_c) - u_c(g-e_c))/(2h) + sum_{6 nbrs} (p(nbr) - p(g))
//   i.e. -div_h u + h^2 lap_h p = 0 (pressure-stabilized, symmetric interior
//   blocks as in the symmetric indefinite systems of Section 3).
//   Columns of boundary nodes are kept in interior rows.
//   mu on an edge is the mean of the per-cell viscosity of the four cells that
//   share the edge, summed in ascending cell id and scaled by 0.25.
#include <cmath>
#include "oracle.hpp"

namespace orc {

namespace {

struct Grid {
  int n;
  i64 node(int i, int j, int k) const { return i + (i64)n * (j + (i64)n * k); }
  i64 cell(int i, int j, int k) const { return i + (i64)(n - 1) * (j + (i64)(n - 1) * k); }
  bool interior(int i, int j, int k) const {
    return i > 0 && j > 0 && k > 0 && i < n - 1 && j < n - 1 && k < n - 1;
  }
};

// Viscosity of the edge from node (i,j,k) to its neighbour in direction d
// (0 = x, 1 = y, 2 = z) with offset s = -1 or +1.
double edge_mu(const Grid& G, const double* theta, int i, int j, int k, int d, int s) {
  if (!theta) return 1.0;
  int c[3] = {i, j, k};
  c[d] = s > 0 ? c[d] : c[d] - 1;        // cell index along the edge
  int d1 = d == 0 ? 1 : 0;               // the two other directions, d1 < d2
  int d2 = d == 2 ? 1 : 2;
  double sum = 0.0;
  bool first = true;
  for (int b2 = -1; b2 <= 0; ++b2)        // d2 is the more significant index
    for (int b1 = -1; b1 <= 0; ++b1) {
      int q[3] = {c[0], c[1], c[2]};
      q[d1] = c[d1] + b1;
      q[d2] = c[d2] + b2;
      const double t = theta[G.cell(q[0], q[1], q[2])];
      sum = first ? t : sum + t;
      first = false;
    }
  return 0.25 * sum;
}

}  // namespace

i64 stokes_nnz(int n) {
  const i64 ni = (i64)(n - 2) * (n - 2) * (n - 2);
  const i64 nn = (i64)n * n * n;
  return 40 * ni + 4 * (nn - ni);
}

void stokes_assemble(int n, const double* theta, Csr& A) {
  Grid G{n};
  const i64 nn = (i64)n * n * n;
  const double inv_h2 = (double)((n - 1) * (n - 1));
  const double inv_2h = 0.5 * (double)(n - 1);
  A.nr = A.nc = 4 * nn;
  A.ptr.assign(A.nr + 1, 0);
  A.col.clear();
  A.val.clear();
  A.col.reserve(stokes_nnz(n));
  A.val.reserve(stokes_nnz(n));
  auto push = [&](i64 c, double v) {
    A.col.push_back((i32)c);
    A.val.push_back(v);
  };
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const i64 g = G.node(i, j, k);
        if (!G.interior(i, j, k)) {
          for (int c = 0; c < 4; ++c) {
            push(4 * g + c, 1.0);
            A.ptr[4 * g + c + 1] = (i64)A.col.size();
          }
          continue;
        }
        // Neighbours in ascending node id: -z, -y, -x, self, +x, +y, +z.
        const int nd[7] = {2, 1, 0, -1, 0, 1, 2};
        const int ns[7] = {-1, -1, -1, 0, 1, 1, 1};
        double mu[3][2];
        for (int d = 0; d < 3; ++d)
          for (int t = 0; t < 2; ++t) mu[d][t] = edge_mu(G, theta, i, j, k, d, t ? 1 : -1);
        double diag = 0.0;
        for (int d = 0; d < 3; ++d)
          for (int t = 0; t < 2; ++t) diag = diag + mu[d][t] * inv_h2;
        auto nbr = [&](int q) {
          int c[3] = {i, j, k};
          if (nd[q] >= 0) c[nd[q]] += ns[q];
          return G.node(c[0], c[1], c[2]);
        };
        for (int c = 0; c < 3; ++c) {            // velocity rows
          for (int q = 0; q < 7; ++q) {
            const i64 m = nbr(q);
            if (nd[q] < 0) {
              push(4 * m + c, diag);
            } else {
              push(4 * m + c, -(mu[nd[q]][ns[q] > 0] * inv_h2));
              if (nd[q] == c) push(4 * m + 3, ns[q] > 0 ? inv_2h : -inv_2h);
            }
          }
          A.ptr[4 * g + c + 1] = (i64)A.col.size();
        }
        for (int q = 0; q < 7; ++q) {            // pressure row
          const i64 m = nbr(q);
          if (nd[q] < 0) {
            push(4 * m + 3, -6.0);
          } else {
            push(4 * m + nd[q], ns[q] > 0 ? -inv_2h : inv_2h);
            push(4 * m + 3, 1.0);
          }
        }
        A.ptr[4 * g + 4] = (i64)A.col.size();
      }
}

// dL/dtheta_e = 1/4 sum over the 12 edges E of cell e of dL/dmu_E, where
// dL/dmu_E = -(1/h^2) sum over interior endpoints g of E (other endpoint g')
//            sum_{c<3} lambda_{g,c} (x_{g,c} - x_{g',c}).
// This is -lambda^T (dA/dtheta_e) x for the assembly above, with lambda the
// adjoint solution A^T lambda = dL/dx.
void theta_gradient(int n, const double* lambda, const double* x, double* g) {
  Grid G{n};
  const double inv_h2 = (double)((n - 1) * (n - 1));
  const int nc = n - 1;
#pragma omp parallel for schedule(static)
  for (int ck = 0; ck < nc; ++ck)
    for (int cj = 0; cj < nc; ++cj)
      for (int ci = 0; ci < nc; ++ci) {
        double sum = 0.0;
        for (int d = 0; d < 3; ++d) {
          const int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
          for (int b2 = 0; b2 <= 1; ++b2)
            for (int b1 = 0; b1 <= 1; ++b1) {
              int a[3] = {ci, cj, ck};
              a[d1] += b1;
              a[d2] += b2;
              int e[3] = {a[0], a[1], a[2]};
              e[d] += 1;
              const i64 ga = G.node(a[0], a[1], a[2]);
              const i64 ge = G.node(e[0], e[1], e[2]);
              double dmu = 0.0;
              if (G.interior(a[0], a[1], a[2]))
                for (int c = 0; c < 3; ++c)
                  dmu = dmu + lambda[4 * ga + c] * (x[4 * ga + c] - x[4 * ge + c]);
              if (G.interior(e[0], e[1], e[2]))
                for (int c = 0; c < 3; ++c)
                  dmu = dmu + lambda[4 * ge + c] * (x[4 * ge + c] - x[4 * ga + c]);
              sum = sum + (-inv_h2) * dmu;
            }
        }
        g[G.cell(ci, cj, ck)] = 0.25 * sum;
      }
}

}  // namespace orc
