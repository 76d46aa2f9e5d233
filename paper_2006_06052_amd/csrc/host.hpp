// Host-side block CSR structures and the FP64 setup phase of the solver.
//
// The paper builds the multigrid hierarchy with built-in CPU structures and
// then moves the result to the compute backend (Section 2, opening paragraph,
// and Section 2.3).  This file declares that CPU phase for the MI355X
// library: every matrix is block CSR with small dense row-major blocks, all
// setup arithmetic is FP64 and compiled without FMA contraction, and every
// accumulation runs in ascending (block column, inner index) order so that the
// resulting patterns are reproducible bit for bit.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace mgk {

struct HBsr {
  int br = 1, bc = 1;             // block shape (rows x cols)
  int32_t nbr = 0, nbc = 0;       // block rows / block columns
  std::vector<int32_t> ptr, col;  // ptr has nbr + 1 entries
  std::vector<double> val;        // nnzb * br * bc, row-major blocks
  int64_t nnzb() const { return ptr.empty() ? 0 : ptr.back(); }
  const double* blk(int64_t k) const { return val.data() + k * br * bc; }
  double* blk(int64_t k) { return val.data() + k * br * bc; }
};

// Block ILU(k) factors (k = 0 or 1): L strictly below, U strictly above the
// diagonal blocks, Dinv the inverses of U's diagonal blocks (ilu.cpp).
struct IluFactors {
  HBsr L, U;
  std::vector<double> Dinv;
};

enum SmootherKind { SM_SPAI0_BLOCK = 0, SM_JACOBI = 1, SM_SPAI0_SCALAR = 2 };

struct SetupParams {
  double eps_strong = 0.08;
  int coarse_enough = 3000;
  int max_levels = 20;
  int smoother = SM_SPAI0_BLOCK;
  double jacobi_omega = 2.0 / 3.0;
  bool smooth_p = true;          // false: plain aggregation, P = P_tent
  bool ilu_smoother = false;     // block ILU smoothing instead of the block-diagonal smoother
  int ilu_kind = 0;              // ... with ILU(0) (0) or ILUT(ilut_p, ilut_tau) (1)
  double ilut_p = 2.0;
  double ilut_tau = 1e-2;
  int ilu_sweeps = 2;            // Jacobi sweeps per factor of the ILU smoother
};

struct HLevel {
  HBsr A, P, R;                  // P, R empty on the coarsest level
  std::vector<int32_t> agg;      // aggregate per block row, -1 = isolated
  std::vector<double> M;         // smoother, nbr * b * b (empty on coarsest)
  IluFactors ilu;                // block ILU(0) smoother factors (ilu_smoother)
  double omega = 0.0;
  int32_t n_agg = 0;
};

struct HHierarchy {
  int b = 1;
  std::vector<HLevel> levels;
  int nc = 0;                    // scalar size of the coarsest level
  std::vector<double> coarse_inv;// nc x nc row-major inverse of the coarsest A
};

// Returns 0 or a negative mgk_status; err receives the reason.
int build_hierarchy(const HBsr& A, const SetupParams& prm, HHierarchy& H, std::string& err);

// Gauss-Jordan inverse with partial pivoting of a row-major n x n matrix.
bool gauss_jordan_inverse(int n, const double* D, double* Dinv);
bool dense_inverse(int n, std::vector<double>& a, std::vector<double>& inv);

// Interleaved [u,v,w,p] 4x4 BSR split into A_uu (3x3), B_up (3x1), B_lo (1x3)
// and C (1x1); sub-blocks that are entirely zero are not stored.  S is the
// pressure operator C - B_lo diag(A_uu)^-1 B_up, or with diag_only the
// approximation C - diag(B_lo diag(A_uu)^-1 B_up) (eq. SchurApprox).
struct SchurParts {
  HBsr Auu, Bup, Blo, C, S;
};
int schur_split(const HBsr& A, bool diag_only, SchurParts& out, std::string& err);
// Scalar (1x1-block) form of a square-block BSR matrix, zero entries dropped.
HBsr scalar_form(const HBsr& A);
// Scalar SPAI(0) of a 1x1-block matrix: m_i = a_ii / sum_j a_ij^2 (ascending j).
int scalar_spai0(const HBsr& A, std::vector<double>& m, std::string& err);

int ilu_factor(const HBsr& A, int level, IluFactors& out, std::string& err);
// Block ILUT(p, tau): threshold dropping and at most floor(p n) blocks per row and triangle.
int ilut_factor(const HBsr& A, double p, double tau, IluFactors& out, std::string& err);

// Ingest helpers.
int csr_to_bsr(int32_t nrows, const int32_t* ptr, const int32_t* col, const double* val,
               int b, HBsr& out, std::string& err);
int validate_bsr(const HBsr& A, std::string& err);
void stokes_sizes(int n, int32_t& nbr, int64_t& nnzb);
void stokes_assemble(int n, const double* theta, int32_t* ptr, int32_t* col, double* val);

}  // namespace mgk
