/* mgk: AMG-preconditioned Krylov solver for block-structured Stokes
 * saddle-point systems on AMD MI355X (gfx950).
 *
 * Method: D. Demidov, L. Mu, B. Wang, "Accelerating linear solvers for Stokes
 * problems with C++ metaprogramming".  The interface follows the paper's
 * statement of a solver: set up once from the system matrix and parameters,
 * then solve for a right-hand side and an initial guess (Section 2.1, the
 * parameter listing and `Solver S(A, prm)`; Section 2.3, the residual and
 * inner-product primitives of the solve phase).
 *
 * Conventions for every entry point:
 *  - Matrices handed to setup are HOST arrays in block CSR (BSR): square,
 *    block columns strictly ascending inside each block row, each block b x b
 *    row-major (Section 4, the block-valued backend and its worked 6x6
 *    example).  Setup deep-copies them; the caller may free them on return.
 *  - Vectors handed to solve calls are DEVICE pointers owned by the caller,
 *    FP64, laid out as n_brows * block scalars (block row i holds scalars
 *    i*b .. i*b+b-1).  All device work runs on the HIP stream given at setup.
 *    A solve call returns after the result is final in device memory.
 *  - Return values are mgk_status codes.  Nothing throws across the ABI.
 *    Invalid arguments are rejected before any device work and the message
 *    is available from mgk_last_error() (thread-local).
 *  - MGK_NOT_CONVERGED is a positive status: info is still filled and x holds
 *    the last iterate.
 */
#ifndef MGK_H
#define MGK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgk_solver mgk_solver;  /* opaque; owns all device hierarchy memory */

typedef enum {
  MGK_OK = 0,
  MGK_NOT_CONVERGED = 1,
  MGK_E_INVALID = -1,   /* bad argument or malformed matrix */
  MGK_E_HIP = -2,       /* a HIP runtime call failed */
  MGK_E_NOMEM = -3,     /* device or host allocation failed */
  MGK_E_SINGULAR = -4,  /* singular diagonal block, smoother block or coarse matrix */
  MGK_E_STATE = -5      /* call not valid for this solver (e.g. wrong kind) */
} mgk_status;

/* Preconditioner kinds.
 *  MGK_AMG_SPAI0  monolithic smoothed-aggregation AMG, SPAI(0) smoother on
 *                 every level, one V(1,1) cycle per application (Section
 *                 2.1, the AMG composition listing).
 *  MGK_AMG_JACOBI the same hierarchy with damped block Jacobi smoothing.
 *  MGK_SCHUR      Schur-complement pressure correction (Section 4, eqs.
 *                 SchurP and SchurU) for interleaved [u,v,w,p] unknowns
 *                 (block size 4): velocity AMG on the 3x3 block A_uu, scalar
 *                 pressure AMG on S = C - B_lo diag(A_uu)^-1 B_up.
 *  MGK_ILU        block ILU(k), k = mgk_params.ilu_level in {0, 1}, of the
 *                 whole system (the paper's monolithic variant uses ILU(1) under
 *                 IDR(5), Section 4), applied with mgk_params.ilu_sweeps Jacobi
 *                 sweeps on each triangular factor. */
typedef enum { MGK_AMG_SPAI0 = 0, MGK_AMG_JACOBI = 1, MGK_SCHUR = 2, MGK_ILU = 3 } mgk_precond_kind;

/* Storage precision of the preconditioner hierarchy values (Section 4, the
 * mixed-precision variant: single-precision nested solvers under a double
 * precision outer iteration).  F32 and BF16 hierarchies accumulate in FP32;
 * the outer Krylov iteration and the coarsest dense solve stay FP64. */
typedef enum { MGK_F64 = 0, MGK_F32 = 1, MGK_BF16 = 2 } mgk_storage;

/* Outer Krylov method: BiCGStab, flexible GMRES(m), or IDR(s) with biorthogonal
 * residual updates (the paper's outer solver, IDR(5); Section 4 and the table of
 * solver variants), all right preconditioned with FP64 vectors and scalars. */
typedef enum { MGK_BICGSTAB = 0, MGK_FGMRES = 1, MGK_IDRS = 2 } mgk_krylov;

/* AMG coarsening: smoothed aggregation, P = (I - omega D^-1 A_F) P_tent (Section
 * 2.1 composition listing), or plain aggregation, P = P_tent (the coarsening of the
 * paper's Schur-complement velocity solvers, Section 4 listings V2-V4). */
typedef enum { MGK_SMOOTHED_AGGREGATION = 0, MGK_PLAIN_AGGREGATION = 1 } mgk_coarsening;

typedef struct {
  int32_t n_brows;        /* block rows (= block columns) */
  int32_t block;          /* b in {1, 3, 4} */
  const int32_t* rowptr;  /* n_brows + 1 */
  const int32_t* col;     /* rowptr[n_brows] block column indices */
  const double* val;      /* rowptr[n_brows] * b * b values */
} mgk_bsr;

typedef struct {
  int32_t krylov;          /* mgk_krylov, default MGK_BICGSTAB */
  int32_t fgmres_m;        /* restart length, default 30 */
  int32_t maxiter;         /* default 1000 (FGMRES: inner steps over all cycles) */
  int32_t max_restarts;    /* BiCGStab restarts after breakdown or a final true
                              residual above rtol, default 5 */
  int32_t hier;            /* mgk_storage of the preconditioner: the hierarchy's A_l, P_l,
                              R_l and smoother blocks (ILU pivot inverses FP32 below FP64),
                              vectors FP32 below FP64; default MGK_F64 */
  int32_t coarse_enough;   /* scalar unknowns at which coarsening stops, default 3000 */
  int32_t max_levels;      /* default 20 */
  int32_t block_spai0;     /* 1: block SPAI(0) (default), 0: scalar-row SPAI(0) */
  double eps_strong;       /* strong-connection threshold on level 0, halved per
                              level, default 0.08 */
  double jacobi_omega;     /* damping of MGK_AMG_JACOBI, default 2/3 */
  int32_t keep_host;       /* 1: keep FP64 host copies of every level for
                              mgk_level_export (default 0) */
  int32_t enable_transpose;/* 1: build the A^T indices for adjoint solves (default 0) */
  int32_t time_spmv;       /* bit mask: 1 times every outer-operator SpMV of a solve
                              (mgk_info.spmv_ms; the fused SpMV-and-dots kernels record their
                              own start and end events through their dispatch, other products
                              are bracketed by events), 2 every preconditioner application
                              (mgk_info.precond_ms, bracketed), on the solver's stream */
  int32_t force_tile;      /* 0: the autotuner picks each operator's kernel tile;
                              otherwise 10000*RPL + 100*S + U (S lanes per block row, U
                              blocks per step, RPL scalar rows per lane) for every
                              operator.  RPL 2 or 4 exists for 4x4 blocks only (and not for
                              transposed products); other products then take (S, U) if that
                              tile exists for them, else the autotuner's tile.  An unknown
                              tile is MGK_E_INVALID.  Results are bitwise the same for every
                              tile.  The autotuner times each candidate after clearing the
                              caches (512 MB of transient device memory during setup) */
  int32_t coarsening;      /* mgk_coarsening, default MGK_SMOOTHED_AGGREGATION */
  int32_t schur_approx;    /* MGK_SCHUR pressure operator: 0 (default) S = C - B_lo
                              diag(A_uu)^-1 B_up assembled; 1 S = C - diag(B_lo
                              diag(A_uu)^-1 B_up) (eq. SchurApprox) */
  int32_t schur_spai0;     /* MGK_SCHUR pressure step: 0 (default) one AMG V-cycle on S;
                              1 one application of the scalar SPAI(0) of S (the paper's
                              pressure preconditioner, Section 4) */
  int32_t schur_lower;     /* MGK_SCHUR factorization: 0 (default) full, eqs. SchurP and
                              SchurU (two velocity cycles); 1 lower block factorization
                              (one velocity cycle, the PETSc LOWER variant of Section 4) */
  int32_t idr_s;           /* shadow space dimension of MGK_IDRS, 1..16, default 5 */
  int32_t ilu_level;       /* MGK_ILU fill level k in {0, 1}, default 0 */
  int32_t ilu_sweeps;      /* Jacobi sweeps per triangular factor for MGK_ILU and the ILU
                              smoother, 0..64, default 2 */
  int32_t ilu_smoother;    /* 1: every AMG level (monolithic, or the Schur velocity and
                              pressure hierarchies) smooths with block ILU(0) instead of
                              SPAI(0) / Jacobi: pre z = ILU^-1 r, post z += ILU^-1 (r - A z)
                              (the paper smooths its velocity AMG with ILUT, Section 4).
                              Not with enable_transpose, multi-RHS or batched solves. */
  int32_t schur_scalar_u;  /* MGK_SCHUR: 1 builds the velocity AMG on the scalar values of
                              A_uu (1x1 blocks, zero entries dropped) instead of 3x3 blocks -
                              the paper's scalar (V2) versus block-valued (V3) solver */
  int32_t ilu_kind;        /* factorization of MGK_ILU and of the ILU smoother: 0 (default)
                              block ILU(k) (k = ilu_level for MGK_ILU, 0 for the smoother);
                              1 block ILUT(ilut_p, ilut_tau) - threshold ILU (Saad), the
                              smoother of the paper's velocity AMG (Section 4, listings V2
                              and V3): blocks below ilut_tau times the block row's Frobenius
                              norm are dropped during and after elimination, and each row
                              keeps at most floor(ilut_p * n) blocks per triangle (n: A's
                              blocks of that row and triangle), the largest first */
  double ilut_p;           /* ILUT fill cap factor, 0..1e6, default 2 */
  double ilut_tau;         /* ILUT drop tolerance, >= 0, default 0.01 */
  int32_t layout;          /* 0 (default): a square 3x3 / 4x4 operator whose blocks lie on at
                              most 8 block diagonals, padded by at most 15%, is also stored in
                              a diagonal layout (values only, columns implied by the diagonal
                              offsets) that the forward products read instead of the BSR
                              arrays (the outer operator and the matching hierarchy levels of
                              a structured grid); 1: BSR only; 2: the diagonal layout for
                              every such operator whatever its padding.  Results agree to
                              rounding (bit for bit when every block row holds either all the
                              operator's block diagonals or only its diagonal block; always
                              bit for bit in mgk_solve_multi).  mgk_batch_setup takes 0 and 2
                              alike (every system's eligible fine operator in the diagonal
                              layout), 1 keeps BSR. */
  int32_t reserved;
} mgk_params;

typedef struct {
  int32_t iters;           /* Krylov iterations (BiCGStab) or inner steps (FGMRES) */
  int32_t levels;          /* levels of the (velocity) hierarchy */
  int32_t restarts;
  int32_t status;          /* MGK_OK or MGK_NOT_CONVERGED */
  double rel_resid;        /* final true ||b - A x|| / ||b|| */
  double setup_ms;
  double solve_ms;
  int64_t device_bytes;    /* device memory held by the solver */
  double spmv_ms;          /* with time_spmv bit 1: summed duration of the outer SpMVs */
  int32_t spmv_calls;      /* ... and their number */
  int32_t outer_tile;      /* kernel tile of the outer operator's fused SpMV-and-dots (the
                              Krylov products of BiCGStab and IDR(s)), 10000*RPL + 100*S + U */
  double precond_ms;       /* with time_spmv bit 2: summed duration of the preconditioner
                              applications */
  int32_t precond_calls;   /* ... and their number */
  int32_t outer_dia;       /* block diagonals of the outer operator's diagonal layout
                              (0: read as BSR) */
} mgk_info;

typedef struct {
  int32_t n_brows, block;  /* rows of A_l in blocks, block size */
  int64_t nnzb;            /* stored blocks of A_l */
  int32_t n_agg;           /* block columns of P_l (0 on the coarsest level) */
  int32_t dia;             /* block diagonals of A_l's diagonal layout on the device (0: BSR
                              only, or a host-only setup) */
  int64_t p_nnzb, r_nnzb;  /* stored blocks of P_l and R_l */
  double omega;            /* prolongator damping used to build P_l */
} mgk_level_desc;

/* Fill prm with the defaults listed above. */
int mgk_params_default(mgk_params* prm);

/* ---- problem ingest (host only, no device work) ------------------------- */

/* Sizes of the synthetic stabilized finite-difference Stokes system on n^3
 * nodes (n >= 3) in 4x4 BSR: n^3 block rows; 7 blocks per interior node row,
 * 1 per boundary node row. */
int mgk_stokes_sizes(int32_t n, int32_t* n_brows, int64_t* nnzb);

/* Assemble that system into caller-allocated host BSR arrays.  PDE: steady
 * Stokes (Section 3, eq. StokesPDE) discretized by 7-point differences with
 * h = 1/(n-1), pressure stabilization h^2 lap_h p in the continuity row,
 * identity rows at boundary nodes (columns to them kept), and per-edge
 * viscosity = mean of theta over the 4 cells sharing the edge.  theta may be
 * NULL (viscosity 1) or hold (n-1)^3 per-cell values, cell (i,j,k) at
 * i + (n-1)(j + (n-1)k).  Unknown 4g+c, node g = i + n(j + n k), c = u,v,w,p. */
int mgk_stokes_assemble(int32_t n, const double* theta, int32_t* rowptr, int32_t* col,
                        double* val);

/* Convert scalar CSR (sorted columns) into BSR with block size b (Section 4,
 * worked example).  nrows must be a multiple of b.  With bcol == NULL only
 * *nnzb is computed; otherwise bptr (nrows/b + 1), bcol (*nnzb) and bval
 * (*nnzb * b * b) are written, missing entries of a stored block being 0. */
int mgk_csr_to_bsr(int32_t nrows, const int32_t* ptr, const int32_t* col, const double* val,
                   int32_t b, int32_t* bptr, int32_t* bcol, double* bval, int64_t* nnzb);

/* ---- setup and solve --------------------------------------------------- */

/* Build the preconditioner for A on the host in FP64 (smoothed aggregation:
 * Section 2.1; Schur split: Section 4), cast it to prm->hier and upload it on
 * `hip_stream` (a hipStream_t, NULL for the default stream).  block_size
 * must equal A->block.  *out receives the solver. */
int mgk_setup(const mgk_bsr* A, int32_t block_size, mgk_precond_kind kind,
              const mgk_params* prm, void* hip_stream, mgk_solver** out);

/* The same FP64 host setup without any device work: the resulting solver
 * only answers mgk_level_count / mgk_level_info / mgk_level_export (keep_host
 * is implied) and mgk_destroy.  For inspecting or planning a hierarchy on a
 * machine without a GPU. */
int mgk_setup_host(const mgk_bsr* A, int32_t block_size, mgk_precond_kind kind,
                   const mgk_params* prm, mgk_solver** out);

/* Solve A x = b to ||b - A x||_2 <= rtol ||b||_2 with the configured Krylov
 * method, right-preconditioned.  d_x holds the initial guess on entry. */
int mgk_solve(mgk_solver* s, const double* d_b, double* d_x, double rtol, mgk_info* info);

/* mgk_solve without any device allocation, for callers that cannot allocate
 * device memory while they run (tight serving loops, code that must not call
 * hipMalloc between set-up and tear-down).  It runs the same BiCGStab kernels as
 * mgk_solve with the same results bit for bit, but its Krylov workspace (eight
 * vectors, the reduction partials and the device scalars) lives in one static
 * device array of the library, 34 MiB per GPU, held from the library's first use
 * on that GPU until the process ends; the preconditioner's own buffers belong to
 * the solver as for mgk_solve.  The call itself allocates nothing (no hipMalloc,
 * no hipFree, no allocating library routine).
 *  - s: a solver from mgk_setup with prm.krylov = MGK_BICGSTAB (else
 *    MGK_E_STATE) and at most 524288 scalar unknowns (n_brows * block; larger
 *    systems return MGK_E_INVALID before any device work).  Its stream must
 *    belong to the current device (else MGK_E_INVALID).
 *  - d_b, d_x, rtol, info: as for mgk_solve.
 * Every call on a GPU shares that GPU's one array, which keeps the last call's
 * contents (every buffer is written before it is read, so nothing needs to start
 * at zero).  Calls that overlap in time on one GPU - from several threads, or
 * while another such call's work is still queued - race on the array and give
 * wrong results; calls in sequence are safe (each returns after its work is
 * done). */
int mgk_solve_noalloc(mgk_solver* s, const double* d_b, double* d_x, double rtol,
                      mgk_info* info);

/* Adjoint solve A^T lambda = g with BiCGStab preconditioned by the transpose
 * of the forward V-cycle (A_l^T, M_l^T, same R_l and P_l, transposed coarse
 * inverse).  Needs prm->enable_transpose and a monolithic AMG kind. */
int mgk_solve_transposed(mgk_solver* s, const double* d_g, double* d_lambda, double rtol,
                         mgk_info* info);

/* nrhs independent solves run in lockstep as block operations.  d_B and d_X
 * are [n_brows*b][nrhs] row-major (RHS fastest).  Each column stops on its own
 * tolerance.  infos has nrhs entries.  nrhs in 1..32. */
int mgk_solve_multi(mgk_solver* s, int32_t nrhs, const double* d_B, double* d_X, double rtol,
                    mgk_info* infos);

/* Several independent systems of uneven size behind one solver: every stage
 * of the solve is one launch over a work list of (system, row tile). */
int mgk_batch_setup(int32_t nsys, const mgk_bsr* const* A, int32_t block_size,
                    mgk_precond_kind kind, const mgk_params* prm, void* hip_stream,
                    mgk_solver** out);
int mgk_batch_solve(mgk_solver* s, const double* const* d_b, double* const* d_x, double rtol,
                    mgk_info* infos);

/* ---- kernels exposed for measurement and checks -------------------------- */

/* y = M x for one stored operator: level -1 is the FP64 outer matrix (x, y
 * FP64); level l >= 0 selects A_l (which 0), P_l (1), R_l (2) or A_l^T (3) of
 * the (velocity, hier 0) or pressure (hier 1) hierarchy in its storage
 * precision, with x, y in the hierarchy vector precision (FP64 for MGK_F64,
 * FP32 otherwise).  Level -1 with which 3 is the FP64 A^T. */
int mgk_spmv(mgk_solver* s, int32_t hier, int32_t level, int32_t which, const void* d_x,
             void* d_y);

/* Restricts the timing events of later solves (mgk_info.spmv_ms, precond_ms) to the
 * bits of mask (same meaning as mgk_params.time_spmv) that were set at setup; 0 turns
 * them off, so a solve carries no event records, and setting the setup value again turns
 * them back on.  Rejects a mask outside 0..3 (MGK_E_INVALID). */
int mgk_set_timing(mgk_solver* s, int32_t mask);

/* z = B r for one preconditioner application (FP64 in and out). */
int mgk_precond_apply(mgk_solver* s, const double* d_r, double* d_z, int32_t transposed);

/* Block ILU factor inspection (MGK_ILU solvers set up with prm->keep_host, or
 * with mgk_setup_host): sizes, then which 0 = L (blocks strictly below the
 * diagonal), 1 = U (strictly above), as BSR with n_brows + 1 row pointers and
 * row-major b x b blocks; which 2 = the n_brows pivot inverses U(i,i)^-1 in val.
 * Arrays are caller-allocated; null arrays are skipped.  MGK_E_STATE if no
 * factors were kept. */
int mgk_ilu_info(mgk_solver* s, int32_t* n_brows, int64_t* l_nnzb, int64_t* u_nnzb);
int mgk_ilu_export(mgk_solver* s, int32_t which, int32_t* rowptr, int32_t* col, double* val);

/* Hierarchy inspection (host copies need prm->keep_host).  hier 0: the
 * monolithic or velocity hierarchy, 1: the pressure hierarchy (MGK_SCHUR). */
int mgk_level_count(mgk_solver* s, int32_t hier);
int mgk_level_info(mgk_solver* s, int32_t hier, int32_t level, mgk_level_desc* out);
/* which 0: A_l, 1: P_l, 2: R_l; writes BSR arrays sized by mgk_level_info;
 * agg (may be NULL) receives the aggregate of each block row (-1 isolated).
 * which 3: the smoother blocks M_l (SPAI(0) or damped Jacobi, n_brows row-major
 * b x b blocks) into val only; MGK_E_STATE on the coarsest level or with the ILU
 * smoother. */
int mgk_level_export(mgk_solver* s, int32_t hier, int32_t level, int32_t which,
                     int32_t* rowptr, int32_t* col, double* val, int32_t* agg);

/* ---- gradients (device) ------------------------------------------------- */

/* Per-cell viscosity gradient of L(x) given the adjoint lambda (A^T lambda =
 * dL/dx) and the solution x of the Stokes system assembled by
 * mgk_stokes_assemble on n^3 nodes: g_e = -lambda^T (dA/dtheta_e) x, i.e. a
 * quarter of the sum over the 12 edges of cell e of
 * -(1/h^2) sum_{interior endpoints} sum_{c<3} lambda_c (x_c - x_c(other end)).
 * d_g has (n-1)^3 entries. */
int mgk_theta_grad(int32_t n, const double* d_lambda, const double* d_x, double* d_g,
                   void* hip_stream);

/* dL/dA on the stored block pattern of the level-0 (FP64) matrix:
 * G_k = -lambda_I x_J^T for every stored block k = (I, J).  d_gval has
 * nnzb * b * b entries in the BSR value layout. */
int mgk_bsr_grad(mgk_solver* s, const double* d_lambda, const double* d_x, double* d_gval);

void mgk_destroy(mgk_solver* s);
const char* mgk_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MGK_H */
