// Plain FP64 CPU oracle for the AMG-preconditioned Krylov Stokes solver
// (Demidov, Mu, Wang: "Accelerating linear solvers for Stokes problems with
// C++ metaprogramming").
//
// TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU path.  Only the
// test suite, the smoke check and the CPU-baseline leg of the benchmark may
// load it.  It shares no code, header, table or helper with the GPU library.
//
// Every matrix is held as scalar CSR with ascending columns per row.  Where an
// algorithm is defined on nodes (b x b blocks), the node quantities are
// gathered from the b consecutive scalar rows of that node.  Arithmetic is
// FP64, compiled with -ffp-contract=off, and every sum runs in the ascending
// order stated at its definition.
//
// Pins (tests/test_oracle_pins.py) cover every function below: the strength test
// (eps^2 threshold against the geometric mean of the two diagonal norms, hand-derived
// chains), eps halving per level and the lumping of weak connections into the filtered
// diagonal (hand-derived anisotropic lines: aggregates, omega, P and the level-1 matrix),
// the damped block Jacobi smoother (its closed form), that two aggregation phases leave
// no connected node over (random matrices), and further the
// plain-aggregation prolongator (hand-derived 1D case, block invariants,
// Galerkin product), the diagonal Schur approximation and its SPAI(0) pressure
// step (derived from the pinned full approximation; least-squares optimality),
// the lower block factorization (dense algebra), and IDR(s) (SplitMix64's
// published outputs for the shadow space, the m + m/s termination bound, dense
// LU), and block ILU(k) (exact LU of a tridiagonal matrix, (LU)_ij = A_ij on the
// factor's pattern, exactness of enough Jacobi sweeps, block Jacobi at zero
// sweeps), and block ILUT (a hand-derived 4 x 4 case with a fill block dropped by the
// tolerance and one by the cap, the exact LU at tau = 0, block Jacobi for a tolerance
// above every row norm, the per-row cap on random matrices).
#pragma once
#include <cstdint>
#include <vector>

namespace orc {

using i64 = int64_t;
using i32 = int32_t;

struct Csr {
  i64 nr = 0, nc = 0;
  std::vector<i64> ptr;     // nr + 1
  std::vector<i32> col;     // ascending within a row
  std::vector<double> val;
};

// ---- sparse and dense primitives (csr.cpp) -------------------------------
void spmv(const Csr& A, const double* x, double* y);      // y = A x
Csr transpose(const Csr& A);
Csr spgemm(const Csr& A, const Csr& B);                   // C = A B, Gustavson
double dot(i64 n, const double* a, const double* b);      // ascending order
double nrm2(i64 n, const double* a);

// All nonzero b x b blocks of node row i, ascending block column.  Blocks are
// dense row-major; entries absent from the CSR are 0.
struct BlockRow {
  std::vector<i32> cols;
  std::vector<double> vals;   // cols.size() * b * b
};
BlockRow gather_block_row(const Csr& A, int b, i64 i);

// Gauss-Jordan inverse of a b x b row-major matrix with partial pivoting (the
// first row holding the largest |pivot| wins).  Returns false when singular.
bool gj_inverse(int b, const double* D, double* Dinv);

// Dense LU with partial pivoting for the coarsest level.
struct DenseLU {
  int n = 0;
  std::vector<double> lu;   // row-major n x n
  std::vector<int> piv;
};
bool lu_factor(const Csr& A, DenseLU& F);
void lu_solve(const DenseLU& F, const double* r, double* z);

// ---- Stokes assembly (stokes.cpp) ----------------------------------------
i64 stokes_nnz(int n);
void stokes_assemble(int n, const double* theta, Csr& A);
void theta_gradient(int n, const double* lambda, const double* x, double* g);

// ---- smoothed-aggregation hierarchy (amg.cpp) ----------------------------
enum Smoother { SPAI0_BLOCK = 0, JACOBI = 1, SPAI0_SCALAR = 2, ILU0 = 3, ILUT = 4 };

struct AmgParams {
  double eps_strong = 0.08;
  int coarse_enough = 3000;   // scalar unknowns on the coarsest level
  int max_levels = 20;
  int smoother = SPAI0_BLOCK;
  double jacobi_omega = 2.0 / 3.0;
  bool smooth_p = true;       // false: plain aggregation, P = P_tent
  int ilu_sweeps = 2;         // Jacobi sweeps per factor of the ILU0 / ILUT smoother
  double ilut_p = 2.0;        // ILUT fill cap relative to A's blocks per row and triangle
  double ilut_tau = 1e-2;     // ILUT drop tolerance relative to the block row's norm
};

// Block ILU(k) (ilu.cpp): per block row, the sorted block columns of the
// combined factor (L strictly below the diagonal, U on and above it) and their
// b x b blocks; Dinv holds U(i,i)^-1.  Applied with `sweeps` Jacobi iterations
// on each triangular factor.
struct Ilu {
  int b = 1;
  i64 nn = 0;
  int sweeps = 2;
  std::vector<std::vector<i32>> cols;
  std::vector<std::vector<double>> vals;
  std::vector<double> Dinv;
};
bool ilu_build(const Csr& A, int b, int level, int sweeps, Ilu& F, const char** msg);
// Block ILUT(p, tau) (threshold dropping and a fill cap per row), same factor layout.
bool ilut_build(const Csr& A, int b, double p, double tau, int sweeps, Ilu& F,
                const char** msg);
void ilu_apply(const Ilu& F, const double* r, double* z);

struct Level {
  Csr A, P, R;                // P, R empty on the coarsest level
  std::vector<i32> agg;       // aggregate of each node, -1 if isolated
  std::vector<char> isolated;
  std::vector<double> M;      // smoother: one b x b block per node
  Ilu F;                      // block ILU(0) / ILUT factors when the smoother is one
  double omega = 0;           // prolongator damping used to build P
  i64 n_agg = 0;
};

struct Hierarchy {
  int b = 1;
  std::vector<Level> levels;
  DenseLU coarse;
  bool transposed = false;
};

// Build the hierarchy; returns false (with msg) on a singular block or pivot.
bool amg_build(const Csr& A, int b, const AmgParams& prm, Hierarchy& H,
               const char** msg);
// Hierarchy of the transposed operator: A_l^T, M_l^T, same R and P, and the
// coarse factorization of A_L^T.
bool amg_transpose(const Hierarchy& H, Hierarchy& Ht, const char** msg);
void vcycle(const Hierarchy& H, int l, const double* r, double* z);

// ---- Krylov solvers (krylov.cpp) -----------------------------------------
struct Precond {
  virtual ~Precond() {}
  virtual void apply(const double* r, double* z) const = 0;
};

struct SolveInfo {
  int iters = 0, restarts = 0, converged = 0;
  double rel_resid = 0;
};

void bicgstab(const Csr& A, const Precond& M, const double* b, double* x,
              double tol, int maxiter, int max_restarts, SolveInfo& info);
void fgmres(const Csr& A, const Precond& M, const double* b, double* x,
            double tol, int m, int maxiter, SolveInfo& info);
// IDR(s) with biorthogonal residuals, right preconditioned; iters counts products
// with A.  The shadow space is idr_shadow(n, s).
void idrs(const Csr& A, const Precond& M, const double* b, double* x, double tol, int s,
          int maxiter, int max_restarts, SolveInfo& info);
// n x s shadow space, column-major: entry (i, j) from SplitMix64 at counter j*n + i
// mapped to [-1, 1), columns orthonormalized by modified Gram-Schmidt.
std::vector<double> idr_shadow(i64 n, int s);

// Schur-complement pressure correction for interleaved [u,v,w,p] unknowns.
struct SchurOptions {
  bool diag_approx = false;   // S = C - diag(Blo diag(Auu)^-1 Bup)   (eq. SchurApprox)
  bool spai0_p = false;       // pressure step: one SPAI(0) application instead of a V-cycle
  bool lower = false;         // lower block factorization: no second velocity cycle
  bool scalar_u = false;      // velocity AMG on scalar values instead of 3x3 blocks
};
struct Schur {
  Csr Auu, Bup, Blo, C, S;    // S = C - Blo diag(Auu)^-1 Bup, or its diagonal-only form
  Hierarchy Hu, Hp;
  std::vector<double> Sm;     // scalar SPAI(0) of S (spai0_p)
  SchurOptions opt;
  i64 nn = 0;                 // nodes
};
bool schur_build(const Csr& A, const AmgParams& prm, const SchurOptions& opt, Schur& S,
                 const char** msg);
void schur_apply(const Schur& S, const double* r, double* z);



}  // namespace orc
