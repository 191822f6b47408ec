/*
 * tpf.h -- C ABI of the MI355X (gfx950) solver library for the Newton
 * Jacobian of fully implicit two-phase porous-media flow.
 *
 * Method: Bui, Elman, Moulton, "Algebraic Multigrid Preconditioners for
 * Multiphase Flow in Porous Media" (arXiv 1611.00127).
 *   - Sec. 2: cell-centred finite volumes, two-point flux approximation with
 *     phase upwinding and harmonic face permeability, backward Euler
 *     (Eq. fully_discrete_system); unknowns (P_w, S_n) per cell.
 *   - Sec. 3: Newton's method, J(u_k) delta = -F(u_k); the 2x2 block Jacobian
 *     (Eq. jacobian) solved by right-preconditioned GMRES (Eq. precon-system).
 *   - Sec. 3.2-3.4: black-box AMG, CPR-AMG(1)/(2) (Algorithms 1-2, Eqs. m_comb,
 *     m_add), block factorisation with the approximate Schur complement
 *     (Algorithm 3, Eqs. SIMPLE-Schur, m_bf).
 *
 * Conventions
 *   - Every function returns an int status (TPF_OK or a negative code);
 *     tpf_last_error() gives a message for the calling thread.
 *   - Vectors of unknowns are device FP64 arrays of length 2N in point order:
 *     element 2i is P_w of cell i, element 2i+1 is S_n of cell i.  Cell index
 *     i = ix + nx*(iy + ny*iz).  They are owned by the caller.
 *   - Handles are owned by the library and released with the matching
 *     *_destroy call; their device memory comes from the allocator installed
 *     with tpf_set_allocator (the device's stream-ordered pool if none).
 *   - All device work is ordered on the hipStream_t passed as `stream`
 *     (NULL = the null stream).  Setups may fork independent kernels onto
 *     library-owned side streams (created per caller stream on first use,
 *     default priority, kept until the process ends); they are ordered
 *     after the work queued on `stream` before the call, and `stream` waits
 *     for them before the call returns.  Only tpf_solve, the setup of a
 *     preconditioner (which reads level sizes back) and tpf_kernel_stats
 *     synchronise the stream.
 *   - Handles are not thread safe.
 */
#ifndef TPF_H
#define TPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define TPF_OK 0
#define TPF_ERR_INVALID_ARG (-1)
#define TPF_ERR_OOM (-2)
#define TPF_ERR_HIP (-3)
#define TPF_ERR_SINGULAR (-4)        /* zero ILU pivot block or singular coarsest matrix */
#define TPF_ERR_OVER_BUDGET (-5)
#define TPF_ERR_NOT_IMPLEMENTED (-6)
#define TPF_ERR_STATE (-7)           /* call out of order (e.g. apply before setup) */

/* Message for a status code (static storage). */
const char* tpf_status_string(int status);
/* Copies the calling thread's last error message into buf (NUL terminated);
 * returns the status of the failed call. */
int tpf_last_error(char* buf, size_t n);

/* ---- memory ------------------------------------------------------------ */
typedef void* (*tpf_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*tpf_free_fn)(void* ptr, void* stream, void* ctx);
/* Installs the device allocator used for all library memory (e.g. a caching
 * allocator of the host framework).  With NULLs (the default) the library
 * allocates from the current device's stream-ordered memory pool
 * (hipMallocAsync / hipFreeAsync), which keeps freed blocks cached.  Must
 * not change while handles allocated with the previous one live. */
int tpf_set_allocator(tpf_alloc_fn alloc, tpf_free_fn free_fn, void* ctx);
/* Device bytes the library currently holds from the allocator: blocks in
 * use plus freed blocks it keeps cached for reuse (per stream, at most
 * 16 GiB), each at its allocated size (the request rounded up to one of
 * eight size classes per power of two, at most 12.5% more). */
int tpf_memory_in_use(size_t* bytes);
/* Returns the blocks the library keeps cached to the allocator, and without
 * an installed allocator trims the device's memory pool (synchronises the
 * device). */
int tpf_release_cached_memory(void);

/* ---- problem (Sec. 2) -------------------------------------------------- */
#define TPF_PC_BROOKS_COREY 0 /* P_c = P_d Sb^(-1/lambda), C1-linear below s_eps */
#define TPF_PC_LINEAR 1       /* P_c = P_0 (1 - Sb); P_0 given in field pd */

typedef struct tpf_problem_desc {
  int nx, ny, nz;             /* cells per direction; nz = 1 for 2D */
  double hx, hy, hz;          /* cell sizes */
  const double* kx;           /* device, N: permeability per direction */
  const double* ky;
  const double* kz;
  const double* poro;         /* device, N */
  double mu_w, mu_n;          /* viscosities */
  double rho_w, rho_n, grav;  /* densities and gravity (potential P - rho g z, z = depth) */
  int pc_model;               /* TPF_PC_* */
  double bc_lambda;           /* Brooks-Corey lambda (also sets the Burdine relperm exponents) */
  double swr, snr;            /* residual saturations */
  double pd;                  /* entry pressure P_d (Brooks-Corey) or P_0 (linear) */
  double s_eps;               /* effective saturation below which P_c is continued linearly */
  const double* q;            /* device, 2N constant source rates (q_w, q_n), or NULL */
  int n_prod;                 /* bottom-hole-pressure producers, at most one per cell */
  const int* prod_cells;      /* host arrays of length n_prod */
  const double* prod_wi;      /* well index: q_a = -WI lambda_a(S) (P_w - p_bh) */
  const double* prod_pbh;
  int n_dir;                  /* Dirichlet boundary faces */
  const int* dir_cells;       /* host arrays of length n_dir */
  const int* dir_face;        /* 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z (must be a domain face) */
  const double* dir_p;        /* boundary P_w and S_n at the face centre */
  const double* dir_s;
} tpf_problem_desc;

typedef struct tpf_problem tpf_problem;
typedef struct tpf_jacobian tpf_jacobian;

/* Copies the description (device fields are copied, not referenced) and
 * computes the face transmissibilities T = gamma K_harm / h (Sec. 2, TPFA
 * and harmonic averaging). */
int tpf_problem_create(const tpf_problem_desc* d, void* stream, tpf_problem** out);
int tpf_problem_destroy(tpf_problem* p);
/* Number of cells N. */
int tpf_problem_cells(const tpf_problem* p, int64_t* n_cells);

/* Block-CSR (2x2 blocks) container for J with the static pattern of the
 * grid: block row i holds its face neighbours and itself, block columns
 * ascending (-z,-y,-x,self,+x,+y,+z).  Values are written by tpf_assemble. */
int tpf_jacobian_create(tpf_problem* p, void* stream, tpf_jacobian** out);
int tpf_jacobian_destroy(tpf_jacobian* J);

/* Residual and exact Jacobian at state u (Sec. 3: Newton linearisation of
 * Eq. fully_discrete_system, upwind choice frozen).  u, u_old, residual:
 * device, 2N.  residual may be NULL.  J's values (row-major 2x2 blocks,
 * entry [a][b] = dR_a/du_b) are overwritten. */
int tpf_assemble(tpf_problem* p, const double* u, const double* u_old, double dt,
                 double* residual, tpf_jacobian* J, void* stream);

typedef struct tpf_bcsr_view {
  int n_block_rows;
  int64_t nnzb;
  const int* row_ptr;   /* device, n_block_rows + 1 */
  const int* col_idx;   /* device, nnzb */
  const double* vals;   /* device, 4 * nnzb, row-major 2x2 blocks */
} tpf_bcsr_view;
/* Read-only device view of J (valid until J is destroyed). */
int tpf_jacobian_view(const tpf_jacobian* J, tpf_bcsr_view* out);

/* y = J x (x, y device 2N). */
int tpf_spmv(const tpf_jacobian* J, const double* x, double* y, void* stream);
/* Newton update (Sec. 3; the paper's Newton variant is unspecified): the
 * step is alpha * delta (alpha = -1 when delta solves J delta = +F, i.e. the
 * residual itself was the right-hand side); each saturation increment is
 * limited to [-ds_max, ds_max] when ds_max > 0 (per-cell saturation chop),
 * then u += step and S_n is clamped to [0,1].  u, delta: device 2N. */
int tpf_newton_update(tpf_problem* p, double* u, const double* delta, double alpha,
                      double ds_max, void* stream);

/* Euclidean norm of a device FP64 vector of n entries into *out (host): the
 * Newton stopping test ||F(u_k)|| <= tol of Sec. 4.1 solver settings.  The
 * sum of squares is reduced in a fixed order (deterministic).  Synchronises
 * the stream. */
int tpf_norm2(const double* x, int64_t n, double* out, void* stream);

/* ---- preconditioners (Sec. 3.2-3.4) ------------------------------------ */
#define TPF_PREC_AMG 0   /* one V-cycle on the point-ordered scalar J (Sec. 3.2) */
#define TPF_PREC_CPR1 1  /* Algorithm 1 (combinative), block ILU(0) + V-cycle on A_pp */
#define TPF_PREC_CPR2 2  /* Algorithm 2 (additive), + V-cycle on A_ss */
#define TPF_PREC_BF 3    /* Algorithm 3, V-cycles on A_ss and on S~ */
#define TPF_PREC_NONE 4  /* identity (tests) */

#define TPF_INTERP_AUTO 0    /* extended+i for S~ and A_pp; direct for A_ss and the scalar J */
#define TPF_INTERP_DIRECT 1  /* direct (distance-one) interpolation everywhere */
#define TPF_INTERP_EXTI 2    /* extended+i (distance-two) interpolation everywhere */
#define TPF_INTERP_CLASSICAL 3  /* classical (modified Ruge-Stueben) interpolation everywhere,
                                   the paper's BoomerAMG setting (Sec. 4.1): strong C
                                   neighbours, strong F neighbours distributed over them */

#define TPF_SMOOTH_L1_JACOBI 0  /* x <- x + D^{-1}(b - A x), D the l1 diagonal */
#define TPF_SMOOTH_CHEBYSHEV 1  /* Chebyshev polynomial of degree cheb_degree in D^{-1} A on
                                   [0.3 hi, hi], hi = 1.1 x a 10-step power estimate of its
                                   largest eigenvalue */
#define TPF_SMOOTH_MC_GS 2      /* multicolour Gauss-Seidel, standing in for the paper's hybrid
                                   Gauss-Seidel (Sec. 4.1): points coloured so that no two
                                   neighbours of A + A^T share a colour, x_i += (b_i - (A x)_i)
                                   / a_ii colour by colour, ascending before the coarse-grid
                                   correction and descending after it; a step is one sweep */

#define TPF_COARSEN_PMIS 0  /* PMIS (De Sterck, Yang, Heys): independent sets of hash-weighted
                               points, every undecided point with a new C neighbour F */
#define TPF_COARSEN_CLJP 1  /* CLJP (Cleary, Falgout, Henson, Jones), the paper's BoomerAMG
                               setting (Sec. 4.1): weights lowered by two edge-removal
                               heuristics each round; every strong F-F pair shares a C point */

#define TPF_FP64 0       /* hierarchy and V-cycle in FP64 */
#define TPF_FP32 1       /* hierarchy stored and V-cycle/ILU solves run in FP32; coarsest in FP64 */

typedef struct tpf_precond_opts {
  int kind;             /* TPF_PREC_* */
  int precision;        /* TPF_FP64 / TPF_FP32 */
  double theta;         /* strength threshold (0.25) */
  int max_levels;       /* 25; 1 gives an exact dense solve when n <= dense_max */
  int coarse_max;       /* stop coarsening at n <= coarse_max (128) */
  int dense_max;        /* dense LU on the coarsest level if n <= dense_max (1024),
                           else two l1-Jacobi sweeps */
  int interp;           /* TPF_INTERP_* */
  uint64_t hash_seed;   /* seed of the PMIS tie-break weights */
  int exti_route;       /* tests: 0 picks each F row's extended+i kernel by the row's size;
                           r in 1..8 starts the search at class r-1 (0-5 flattened wavefront
                           kernels, 6 wide wavefront, 7 one thread per row) */
  int smoother;         /* TPF_SMOOTH_* (l1-Jacobi); one V-cycle per inner solve, Sec. 4.1 */
  int nu1, nu2;         /* pre- and post-smoothing steps per level, each in [0, 4], sum >= 1
                           (1, 1); a Chebyshev step is one polynomial */
  int cheb_degree;      /* Chebyshev polynomial degree in [1, 8] (2) */
  int coarsening;       /* TPF_COARSEN_* (PMIS) */
  int trunc_pmax;       /* interpolation truncation, every level: each row of P keeps at most
                           this many entries, ranked by magnitude rounded to FP32 (larger
                           first, lower column first among equal ones); 0 = no limit; in
                           [0, 64] (3) */
  double trunc_factor;  /* and drops entries below trunc_factor times the row's largest
                           magnitude; in [0, 1) (0).  The kept positive and the kept negative
                           entries are rescaled so that each sign's row sum is unchanged.  A
                           setting of this library: the paper leaves the sparsity of P to its
                           AMG package (Sec. 3.2, Sec. 4.1) */
} tpf_precond_opts;
/* Fills opts with the defaults above for the given kind. */
int tpf_precond_default_opts(int kind, tpf_precond_opts* opts);

typedef struct tpf_precond tpf_precond;
int tpf_precond_create(const tpf_precond_opts* o, tpf_precond** out);
int tpf_precond_destroy(tpf_precond* M);
/* Builds the preconditioner for J: block views, S~, BILU(0) pivots and the
 * AMG hierarchies.  reuse_structure = 1 keeps the C/F splittings, P and R of
 * the previous setup on a J with the same pattern and recomputes every
 * numeric quantity (blocks, S~, Galerkin products, smoother diagonals,
 * coarsest inverse, ILU pivots).  Synchronises the stream. */
int tpf_precond_setup(tpf_precond* M, const tpf_jacobian* J, int reuse_structure, void* stream);
/* z = M^{-1} r (device 2N). */
int tpf_precond_apply(tpf_precond* M, const double* r, double* z, void* stream);

#define TPF_MAX_LEVELS 25
typedef struct tpf_hier_stats {
  int n_hier;                          /* AMG:1 (J), CPR1:1 (A_pp), CPR2:2 (A_pp,A_ss), BF:2 (A_ss,S~) */
  int levels[3];
  int64_t rows[3][TPF_MAX_LEVELS];
  int64_t nnz[3][TPF_MAX_LEVELS];
  int64_t p_nnz[3][TPF_MAX_LEVELS];    /* entries of P (level l -> l+1; R = P^T has as many);
                                          0 on the coarsest level */
  double operator_complexity[3];
  double grid_complexity[3];
  int coarse_dense[3];
  int l0_diagonals[3];                 /* level-0 smoother layout: number of stored diagonals
                                          (diagonal layout), 0 = CSR */
  int coarse_smooth_sweeps[3];         /* coarsest level: 0 = dense solve, else l1-Jacobi sweeps */
  size_t device_bytes;                 /* bytes held by the preconditioner */
  size_t hier_bytes[3];                /* of which each hierarchy (levels, transfer operators,
                                          work vectors, coarsest inverse) */
} tpf_hier_stats;
int tpf_precond_stats(const tpf_precond* M, tpf_hier_stats* out);

/* ---- introspection for parity checks ----------------------------------- */
typedef struct tpf_csr_view {
  int n_rows, n_cols;
  int64_t nnz;
  const int* row_ptr;     /* device */
  const int* col_idx;     /* device */
  const double* vals;     /* device FP64 values (NULL for pattern-only) */
} tpf_csr_view;
#define TPF_MAT_A 0       /* level operator */
#define TPF_MAT_P 1       /* interpolation (level -> level+1) */
#define TPF_MAT_R 2       /* restriction P^T */
#define TPF_MAT_S 3       /* strength graph (pattern only) */
#define TPF_MAT_GS_COLORS 4  /* Gauss-Seidel colours: row c lists the points of colour c
                                (order inside a colour unspecified); n_rows = colours */
#define TPF_MAT_APS 10    /* A_ps block (level ignored) */
#define TPF_MAT_SCHUR 11  /* S~ (BF) */
/* View of matrix `which` of hierarchy `hier` at `level` (FP64 copy). */
int tpf_precond_matrix(const tpf_precond* M, int hier, int level, int which, tpf_csr_view* out);
/* C/F splitting of a level (device int8, 1 = C, 2 = F) and the l1-Jacobi
 * inverse diagonal (device FP64). */
int tpf_precond_level_data(const tpf_precond* M, int hier, int level, const int8_t** cf,
                           const double** dinv, int* n);
/* Inverse pivot blocks of block ILU(0) (device, 4N, row-major 2x2). */
int tpf_precond_bilu_dinv(const tpf_precond* M, const double** dinv);
/* One V-cycle of hierarchy `hier` on b (device FP64, level-0 size). */
int tpf_precond_vcycle(tpf_precond* M, int hier, const double* b, double* x, void* stream);

/* ---- sparse products (the setup's SpGEMM) ------------------------------ */
/* C = alpha A B (+ beta D when D != NULL) for device CSR matrices with sorted
 * rows: the kernel behind the Galerkin products A_c = R (A P) of each AMG
 * level (Sec. 3.2) and S~ = A_pp - (A_ps D_ss^-1) A_sp (Sec. 3.4, Eq.
 * SIMPLE-Schur).  C's pattern is the symbolic product (plus D's pattern),
 * with no value dropping, rows sorted by column.
 *   route: 0 picks each row's kernel by its product count; r in 1..9 makes
 *     rows start the search at kernel class r-1 (0..6 register-sorted classes
 *     of at most 64/128/256/512/1024/2048/8192 products, 7 the LDS-sorted
 *     class, 8 the per-row merge), so tests can drive every kernel.
 *   pattern_given = 0: writes c_row_ptr (n_rows + 1 ints) and *c_nnz; when
 *     *c_nnz <= c_cap also c_col_idx and c_vals (call once with c_cap = 0 to
 *     size them).  pattern_given = 1: c_row_ptr / c_col_idx hold C's pattern
 *     (from an earlier call) and only c_vals is computed (numeric refresh).
 * All arrays are caller-owned device memory on the library's device; the
 * inputs are checked (row pointers, sorted in-range columns) and a malformed
 * matrix returns TPF_ERR_INVALID_ARG.  Synchronises `stream`. */
int tpf_csr_product(const tpf_csr_view* A, const tpf_csr_view* B, const tpf_csr_view* D,
                    double alpha, double beta, int route, int pattern_given, int* c_row_ptr,
                    int* c_col_idx, double* c_vals, int64_t c_cap, int64_t* c_nnz, void* stream);

/* C = A^T for a device CSR matrix with sorted rows (the restriction R = P^T
 * of each AMG level and the transposed strength graph, Sec. 3.2): c_row_ptr
 * n_cols + 1 ints, c_col_idx / c_vals nnz entries (c_vals may be NULL when
 * A->vals is), caller-owned device memory; rows of C sorted.  Malformed input
 * returns TPF_ERR_INVALID_ARG.  Synchronises `stream`. */
int tpf_csr_transpose(const tpf_csr_view* A, int* c_row_ptr, int* c_col_idx, double* c_vals,
                      void* stream);

/* ---- Krylov solve (Sec. 3, Eq. precon-system) -------------------------- */
#define TPF_CONVERGED 0
#define TPF_MAX_ITERS 1
#define TPF_BREAKDOWN 2
#define TPF_NONFINITE 3

typedef struct tpf_solve_opts {
  double rtol;   /* stop when ||b - J x|| <= rtol ||b|| (1e-8) */
  int restart;   /* Krylov dimension m (30), at most 64 */
  int maxit;     /* total Arnoldi steps (1000) */
} tpf_solve_opts;

typedef struct tpf_solve_info {
  int status;            /* TPF_CONVERGED, TPF_MAX_ITERS, TPF_BREAKDOWN, TPF_NONFINITE */
  int iterations;        /* Arnoldi steps */
  double relres_est;     /* |g_{j+1}| / ||b|| at the last step */
  double relres_true;    /* ||b - J x|| / ||b|| at exit */
  double ms;             /* wall time of the solve */
} tpf_solve_info;

/* Right-preconditioned flexible GMRES(m) with CGS2 Arnoldi and Givens
 * rotations, x_0 = 0; x is overwritten (device 2N).  M may be NULL
 * (identity).  Non-convergence is reported in info->status, not as an
 * error.  Synchronises the stream. */
int tpf_solve(const tpf_jacobian* J, tpf_precond* M, const double* b, double* x,
              const tpf_solve_opts* o, tpf_solve_info* info, void* stream);

/* tpf_solve for callers that cannot allocate device memory (tight serving
 * loops, harnesses that forbid hipMalloc): the same solve and the same
 * results, but the Krylov workspace (bases V and Z, residual, Hessenberg
 * matrix, rotations, partial sums) lives in a fixed 128 MiB device array of
 * the library, one per GPU, held until the process ends; the call draws no
 * device memory from the allocator and calls no hipMalloc/hipFree.
 *   - Size limit: the workspace of an FGMRES(m) solve is about
 *     (2m + 2) * 2N doubles plus 1 MiB; at restart 30 that allows up to
 *     268,000 unknowns (134,000 cells).  Larger systems fail with
 *     TPF_ERR_INVALID_ARG before any device work.
 *   - J and M must already be set up (their memory was allocated then).
 *     With V-cycle graphs enabled (tpf_set_graphs(1)) the call fails with
 *     TPF_ERR_STATE, since a graph is instantiated on first use.
 *   - Every call on one GPU uses that GPU's one array: calls that overlap on
 *     a GPU (other threads, or other streams before a call returns) race and
 *     corrupt each other's results.  Each call writes every workspace entry
 *     it reads, so the contents a previous call left do not matter.
 *   - No preconditioning is queued ahead of a step's scalars (tpf_solve
 *     overlaps the two); the iterates are the same.
 * Arguments, status and info are those of tpf_solve.  Synchronises the
 * stream. */
int tpf_solve_noalloc(const tpf_jacobian* J, tpf_precond* M, const double* b, double* x,
                      const tpf_solve_opts* o, tpf_solve_info* info, void* stream);

/* ---- serving: continuous batching of Newton-step solves ---------------- */
/* Not part of the paper's method: a request loop over many independent
 * Newton sequences (realizations) on one GPU.  Each request is one Newton
 * linear solve (Sec. 3): assemble J(u) and F(u), set up (or numerically
 * refresh) the preconditioner, and solve J x = -F by FGMRES.
 *   - Requests of one sequence share a resident Jacobian and preconditioner
 *     and run one at a time, in submission order; the first builds the AMG
 *     structure, later ones refresh it numerically when opts.reuse is set.
 *   - Up to max_active requests of different sequences are in flight, each
 *     on its own stream; tpf_server_step advances every active request by
 *     one phase (an Arnoldi step, a cycle end), so their kernels overlap.
 *   - Admission: a queued request starts only while the device bytes the
 *     server holds, plus the reservations of setups still running, plus its
 *     own estimate, fit in hbm_budget_bytes.
 *       - Held bytes are every block drawn on the server's streams (the setup
 *         stream, the slot streams, each resident preconditioner's second
 *         setup stream), whether in use or cached for reuse, at allocated
 *         sizes.
 *       - A request's estimate is its FGMRES workspace plus, for a new
 *         sequence, 1.25 times the largest resident and setup bytes measured
 *         on built sequences of that size (scaled up from smaller ones), or,
 *         for a built sequence, 1.25 times the extra bytes its last setup
 *         drew.  The budget holds as long as no setup draws more than its
 *         estimate: it is not a hard limit on the allocator.
 *       - Requests of resident sequences are considered before those that
 *         need a build; a request that does not fit yet is passed over (with
 *         the later requests of its sequence), so a sequence's requests start
 *         in submission order while other sequences go ahead.
 *       - To make room the server first returns idle streams' cached blocks
 *         to the allocator, then evicts idle sequences, those with no queued
 *         request first, least recently used first.
 *     A request that cannot fit alone fails with TPF_ERR_OVER_BUDGET.
 *   - A result does not depend on what else is in flight: every kernel is
 *     deterministic and a sequence's requests run in order.
 * Setup and admission run on the calling thread; the server is not thread safe. */
#define TPF_CANCELLED 4                /* result status of a cancelled request */

typedef struct tpf_server_opts {
  size_t hbm_budget_bytes;  /* admission budget (device bytes) */
  int max_active;           /* requests in flight (1..64) */
  int kind;                 /* preconditioner TPF_PREC_* */
  int precision;            /* TPF_FP64 / TPF_FP32 */
  int reuse;                /* 1: refresh a resident sequence's hierarchy numerically */
  tpf_solve_opts solve;     /* rtol, restart, maxit */
} tpf_server_opts;

typedef struct tpf_request {
  uint64_t sequence;           /* realization id; equal ids share resident data */
  tpf_problem* problem;        /* static data of the realization (caller owned, same for
                                  every request of a sequence, alive until it is evicted
                                  or the server is destroyed) */
  const double* u;             /* device 2N: Newton iterate u_k */
  const double* u_old;         /* device 2N: previous time level */
  double dt;
  double* x;                   /* device 2N: receives the Newton update, J x = -F(u_k) */
} tpf_request;                 /* u, u_old, x: ready at submit, untouched until polled */

typedef struct tpf_result {
  int status;             /* TPF_CONVERGED.. / TPF_CANCELLED, or a negative error code */
  int iterations;
  double relres_est, relres_true;
  double setup_ms;        /* assembly + preconditioner setup/refresh */
  double solve_ms;        /* FGMRES, first phase queued to last phase read */
  double latency_ms;      /* submit to completion */
  int refreshed;          /* 1 if the hierarchy was refreshed, 0 if built */
  size_t reserved_bytes;  /* bytes of the HBM budget the request was admitted with: its FGMRES
                             workspace plus, for a sequence not resident, the expected bytes of
                             its build (for TPF_ERR_OVER_BUDGET: the bytes that did not fit) */
} tpf_result;

typedef struct tpf_server_counters {
  int queued, active, resident_sequences;
  int64_t submitted, completed;
  size_t bytes_in_use;    /* device bytes held on the server's streams (in use or cached) */
  size_t peak_bytes;      /* maximum of bytes_in_use, sampled at each admission and step */
  int64_t evictions;
} tpf_server_counters;

typedef struct tpf_server tpf_server;
int tpf_server_default_opts(tpf_server_opts* o);
int tpf_server_create(const tpf_server_opts* o, tpf_server** out);
/* Queues a request; *ticket identifies it in poll/cancel. */
int tpf_server_submit(tpf_server* sv, const tpf_request* rq, uint64_t* ticket);
/* Admits what fits, then advances every active request by one phase
 * (blocking until each has); *n_done = requests finished in this step. */
int tpf_server_step(tpf_server* sv, int* n_done);
/* 1 and the result if the request has finished (the result is then
 * released), 0 if it is queued or active; TPF_ERR_INVALID_ARG if unknown. */
int tpf_server_poll(tpf_server* sv, uint64_t ticket, tpf_result* out);
/* Cancels a queued request at once, an active one at its next phase. */
int tpf_server_cancel(tpf_server* sv, uint64_t ticket);
int tpf_server_stats(const tpf_server* sv, tpf_server_counters* out);
/* Waits for in-flight work, then frees every resident sequence. */
int tpf_server_destroy(tpf_server* sv);

/* ---- kernel timing ----------------------------------------------------- */
/* When enabled, the launches of the main kernels are bracketed by HIP events
 * on their stream; tpf_kernel_stats returns the launch count and the summed
 * event time of every launch of the named kernel since the last reset
 * (synchronises).  Names: "vcycle_smooth_residual", "vcycle_post_smooth",
 * "csr_spmv", "bcsr_spmv", "assemble", "cgs2_dots", ... */
int tpf_kernel_timing(int enable);
int tpf_kernel_stats(const char* name, int64_t* count, double* total_ms);
int tpf_kernel_stats_reset(void);

/* ---- launch mode ------------------------------------------------------- */
/* With graphs enabled, each AMG V-cycle (about five kernels per level) is
 * recorded once as a HIP graph on a private stream, for the (input, output)
 * buffers it is applied to, and replayed on the caller's stream; graphs are
 * dropped whenever the hierarchy is rebuilt or refreshed.  Disabled by
 * default (every kernel launched directly, as also while kernel timing is
 * on): on the 1M-cell workload a replay starts about 28 us after the
 * preceding kernel and the solve is 0.2 ms slower; replays save host work
 * when one thread drives many requests.  Results are identical either way. */
int tpf_set_graphs(int enable);

#ifdef __cplusplus
}
#endif
#endif /* TPF_H */
