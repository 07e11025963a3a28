/*
 * mlc.h -- C ABI of the MI355X library for the fine-mesh correction step of the
 * multilevel-correction adaptive finite element method for the Kohn-Sham
 * equation (Hu, Xie, Xu, "On accelerating a multilevel correction adaptive
 * finite element method for Kohn-Sham equation").
 *
 * One call of mlc_correction_step performs one outer iteration l -> l+1 of
 * Algorithm 1 (steps 5-7) on a fixed pair of nested meshes:
 *   - density and exchange-correlation potential of Phi^l at the quadrature
 *     points (Section 4, LDA / X-alpha; frozen during the inner loop as the
 *     remark after eq. (gdef) requires),
 *   - N auxiliary linear problems (eq. Aux_Linear_Problem), solved together
 *     by a multi-right-hand-side Jacobi-preconditioned CG on the GPU,
 *   - the Hartree direction (eq. W_h_equation) with multipole Dirichlet data
 *     (remark after Algorithm 3),
 *   - the fine-mesh integrals of Algorithm 3 step 1 (eqs. Adef, bdef, Ah4def,
 *     betadef, rhsdef, Hartree_H_h, FG),
 *   - the inner Hartree iteration of Algorithm 2 in the small augmented
 *     spaces (Algorithm 3 step 2), in FP64 on the host,
 *   - reconstruction phi_i = phi_{i,H} + theta_{2,i} u_i (Algorithm 3 step 3),
 *     the Hartree potential and the density.
 *
 * Conventions shared by every entry point
 *   - Every function returns mlc_status; MLC_OK is 0. Nothing throws across
 *     the ABI. On failure mlc_last_error(ctx) describes the cause; the context
 *     keeps its previous state (except MLC_ERR_NOT_CONVERGED, where the last
 *     iterate is kept and the report is filled).
 *   - Host arrays passed in are copied before the call returns; the caller
 *     keeps ownership. Host output arrays are written by the library and must
 *     be large enough for the documented size.
 *   - Device memory: the library never allocates device memory. The caller
 *     allocates one workspace of mlc_workspace_bytes() bytes on the GPU that
 *     the context runs on and passes it to mlc_bind(), together with the HIP
 *     stream all work is enqueued on. The workspace must outlive the context's
 *     use of it. Calls that return host data synchronise that stream.
 *   - Nodes and DoF numbering seen by callers: the nodes of a P1 mesh are its
 *     vertices; those of a P2 fine mesh (order 2) are its vertices followed by
 *     one node per edge at the edge's midpoint, edges in increasing
 *     (lo, hi) vertex-index order. The fine (coarse) degrees of freedom are
 *     the nodes of the fine (coarse) mesh that do not lie on the box
 *     boundary, in increasing node index. Orbital blocks are row-major
 *     n_dof x N (orbital index fastest). Internally the library reorders the
 *     fine DoFs for memory locality and undoes it on output.
 *   - One context is used from one host thread at a time.
 */
#ifndef MLC_H
#define MLC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MLC_OK = 0,
  MLC_ERR_ARG = -1,           /* null pointer, size or enum out of range      */
  MLC_ERR_MESH = -2,          /* degenerate tet, index out of range, no DoF   */
  MLC_ERR_NOT_NESTED = -3,    /* a fine vertex lies outside the coarse mesh   */
  MLC_ERR_WORKSPACE = -4,     /* workspace missing or too small               */
  MLC_ERR_HIP = -5,           /* a HIP runtime call failed                    */
  MLC_ERR_NOT_CONVERGED = -6, /* CG hit cg_maxit before cg_rtol               */
  MLC_ERR_BREAKDOWN = -7,     /* CG curvature p^T A p <= 0                    */
  MLC_ERR_NONFINITE = -8,     /* NaN/Inf detected in a result                 */
  MLC_ERR_STATE = -9,         /* call order: not bound, no state, ...         */
  MLC_WARN_INNER_MAXIT = 1    /* inner iteration stopped at inner_maxit       */
} mlc_status;

/* Potentials of the external field (Section 2 defines the bare Coulomb one). */
enum { MLC_POT_ERF = 0,       /* -sum Z_k erf(|x-R_k|/rc)/|x-R_k|             */
       MLC_POT_BARE = 1,      /* -sum Z_k/|x-R_k|                             */
       MLC_POT_HARMONIC = 2   /* 0.5 omega^2 |x|^2 (no nuclei needed)         */ };
/* Exchange-correlation (Section 4). */
enum { MLC_XC_NONE = 0, MLC_XC_LDA = 1 /* Slater + Perdew-Zunger 81 */, MLC_XC_XALPHA = 2 };

/* A tetrahedral mesh of the box [box_lo, box_hi] (host arrays, copied by
 * mlc_create). order: polynomial degree of the Lagrange elements: 1 (linear,
 * the space V_h of Section 2) or, for the fine mesh only, 2 (quadratic: the
 * same construction with P2 polynomials per tet, 10 nodes, integrals by a
 * degree-5 27-point rule); any other value, or a coarse mesh of order 2, is
 * MLC_ERR_ARG. The coarse space is P1, a subspace of the fine P1 or P2 space
 * on nested meshes. xyz: n_vertices x 3 doubles; tets: n_tets x 4 vertex
 * indices (the library derives the P2 edge nodes itself). */
typedef struct {
  int32_t order;
  int64_t n_vertices;
  const double* xyz;
  int64_t n_tets;
  const int32_t* tets;
} mlc_mesh;

/* The physical system (Section 2): M nuclei with charges Z at R, N orbitals
 * with occupation numbers f_i (rho = sum f_i phi_i^2). */
typedef struct {
  int32_t n_nuclei;
  const double* R;            /* n_nuclei x 3 */
  const double* Z;            /* n_nuclei     */
  int32_t potential;          /* MLC_POT_*    */
  double rc;                  /* smoothing radius of MLC_POT_ERF */
  double omega;               /* MLC_POT_HARMONIC frequency      */
  int32_t n_orbitals;         /* N, 1..MLC_MAX_ORBITALS           */
  const double* occupations;  /* N */
  int32_t xc;                 /* MLC_XC_* */
  double xalpha;              /* alpha of X-alpha (0.77298 in Section 4) */
  int32_t hartree;            /* 1: Hartree term present, 0: absent */
  double box_lo[3], box_hi[3];/* the box prod_k [box_lo[k], box_hi[k]]; homogeneous
                                 Dirichlet data on its faces (Section 4) */
} mlc_system;

#define MLC_MAX_ORBITALS 128

typedef struct {
  double cg_rtol;       /* per-orbital ||b - A x||_2 <= cg_rtol ||b||_2       */
  int32_t cg_maxit;
  int32_t check_every;  /* CG iterations between host convergence checks     */
  int32_t shift;        /* 0: step 5 exactly as printed; 1: add sigma M       */
  double sigma0;        /* shift = sigma0 - min V_eff when shift = 1          */
  double poisson_rtol;  /* Hartree direction CG tolerance                     */
  int32_t inner_maxit;  /* Algorithm 2 iteration cap                          */
  double inner_tol;     /* Algorithm 2 stop: ||Phi^{s+1} - Phi^s||_{H^1}      */
  int32_t n_extra;      /* candidates = lowest min(N_H+1, N + n_extra) pairs  */
  int32_t reorder;      /* 1: Morton order of fine DoFs (default)            */
  int32_t time_kernels; /* 1: HIP events around every SpMM launch of step 5
                           (that CG is then launched eagerly)                  */
  int32_t use_graphs;   /* 1: CG iteration chunks replayed as HIP graphs      */
  int32_t precision;    /* MLC_PREC_FP64: plain FP64 CG for step 5;
                           MLC_PREC_FP32_IR: FP32 SpMM/CG inside FP64 iterative
                           refinement (residual, update and stopping test in
                           FP64; cg_rtol applies to the FP64 residual)         */
  double ir_inner_rtol; /* FP32 inner CG tolerance relative to ||R||          */
  int32_t ir_max_outer; /* refinement passes cap                              */
  int32_t precond;      /* CG preconditioner of the single-system solves (steps 5 and 6):
                           MLC_PC_JACOBI, or MLC_PC_CHEBYSHEV = the Chebyshev
                           polynomial of degree cheb_degree in D^-1 A over
                           [lmax / cheb_ratio, lmax], lmax a Gershgorin bound
                           (same solution, fewer iterations and reductions);
                           a batch uses the setting of its contexts, which
                           must agree                                          */
  int32_t cheb_degree;  /* 2..16                                               */
  double cheb_ratio;    /* > 1                                                 */
  int32_t hartree_coarse; /* 1: the Hartree CG adds the exact coarse-space
                           correction P K_H^-1 P^T (additive two-level
                           preconditioner over the nested coarse space; K_H =
                           P^T K P factorised on the host once per mesh, its
                           inverse applied on the device) to the preconditioner
                           chosen by precond                                   */
  int32_t hartree_precond; /* preconditioner of the Hartree CG (step 6): -1 (the
                           default) takes precond; MLC_PC_JACOBI or
                           MLC_PC_CHEBYSHEV choose it apart from the step-5
                           solves (same degree and ratio); a batch requires the
                           same choice in all its contexts                    */
  int32_t inner_mix_history; /* Algorithm 2 is a fixed-point iteration in the
                           Hartree coefficients x = (w_H, theta1); 0 runs it as
                           printed (next input = the Hartree potential of the
                           new orbitals); m > 0 chooses the next input by
                           Anderson (Pulay) mixing of the last m + 1 inputs and
                           residuals in the energy inner product of W_{H,h}
                           (same fixed point, converges where the plain
                           iteration oscillates); 0..16                       */
  double inner_mix_beta;  /* Anderson damping in (0, 1]                       */
  int32_t variant;      /* MLC_VARIANT_EIGENPAIRWISE: Algorithm 2 as printed,
                           one augmented space V_H + span{u_i} per orbital (the
                           paper's method); MLC_VARIANT_JOINT: the earlier
                           multilevel correction method it is compared with,
                           one space V_H + span{u_1..u_N} whose lowest N
                           eigenpairs are the orbitals (needs the N(N+1)/2
                           pair integrals (u_j u_l, psi_k) from the fine
                           mesh; N <= 64; P1 fine meshes only)                 */
  int32_t estimator;    /* 1: mlc_create builds the fine mesh's face
                           neighbours for mlc_estimate (host time and 20 bytes
                           of workspace per fine tet; P1 fine meshes only);
                           0 (default): off                                    */
  int32_t cheb_lanczos; /* upper end of the Chebyshev interval: 0 (default)
                           the Gershgorin bound of D^-1 A; m in 2..64:
                           min(Gershgorin, 1.1 x the largest Ritz value of m
                           Lanczos steps on D^-1 A in the D inner product,
                           from a fixed pseudo-random start), for A + sigma M
                           every step and for K once at mlc_bind              */
  int32_t hartree_cheb_degree; /* the Hartree CG's polynomial degree (2..16);
                                  0 (default): cheb_degree                    */
  double hartree_cheb_ratio;   /* its interval ratio (> 1); 0 (default):
                                  cheb_ratio                                  */
} mlc_options;

enum { MLC_VARIANT_EIGENPAIRWISE = 0, MLC_VARIANT_JOINT = 1 };

enum { MLC_PC_JACOBI = 0, MLC_PC_CHEBYSHEV = 1 };

enum { MLC_PREC_FP64 = 0, MLC_PREC_FP32_IR = 1 };

/* Filled by mlc_correction_step. Times in milliseconds. */
typedef struct {
  int32_t cg_iters_max, cg_iters_sum, poisson_iters, inner_iters;  /* FP32_IR: summed inner FP32 iterations */
  double cg_relres_max;       /* max over orbitals, true residual at exit   */
  double poisson_relres;
  double inner_last_diff;     /* last ||Phi^{s+1}-Phi^s||_{H^1}             */
  double sigma;               /* shift used in step 5                       */
  double theta1;              /* Hartree coefficient of w0                  */
  double max_offdiag_overlap; /* max_{i!=j} |(phi_i, phi_j)|                */
  double rho_integral;        /* int rho = electron count                   */
  double energy;              /* sum f lambda - 1/2 int w rho + int rho (eps_xc - v_xc^l) */
  double t_fine_ms;           /* device: density..Gram blocks (steps 5, 6, Alg. 3 step 1) */
  double t_inner_ms;          /* host: Algorithm 2 / Algorithm 3 step 2     */
  double t_recon_ms;          /* device: reconstruction and diagnostics     */
  double t_spmm_ms;           /* sum of SpMM kernel times (time_kernels=1)  */
  int64_t n_spmm;             /* SpMM launches in this step                 */
  int64_t spmm_rows;          /* rows x columns processed by those launches */
  int64_t spmm_cols_sum;
  int32_t ir_outer;           /* refinement passes (precision FP32_IR)      */
  int32_t guess_learned_cols; /* columns started from the learned guess (mlc_set_guess) */
  double guess_resid_ratio;   /* max over columns of |b - A x0| / |b - A phi| (x0 = start used) */
  double t_solve_ms;          /* device: the step-5 solve (0 in a batch: see mlc_batch_report) */
  double t_poisson_ms;        /* device: the Hartree solve (0 in a batch)   */
} mlc_step_report;

typedef struct mlc_ctx mlc_ctx;

/* Fill *opt with defaults: cg_rtol 1e-10, cg_maxit 20000, check_every 25,
 * shift 1, sigma0 1, poisson_rtol 1e-12, inner_maxit 500, inner_tol 1e-10,
 * n_extra 8, reorder 1, time_kernels 0, use_graphs 1, precision FP64,
 * ir_inner_rtol 1e-4, ir_max_outer 30, precond Jacobi, cheb_degree 4,
 * cheb_ratio 30, hartree_coarse 0, hartree_precond -1, inner_mix_history 6,
 * inner_mix_beta 0.5, variant MLC_VARIANT_EIGENPAIRWISE. */
void mlc_options_default(mlc_options* opt);

/* Build a context: validates both meshes (positive volumes, indices in range,
 * at least one interior vertex), locates every fine vertex in the coarse mesh
 * (MLC_ERR_NOT_NESTED if one lies outside), builds the fine CSR pattern, the
 * prolongation P (coarse hat functions at fine vertices, Section 3.2) and the
 * grouping of fine tets by coarse parent. Host work only. */
mlc_status mlc_create(const mlc_mesh* fine, const mlc_mesh* coarse, const mlc_system* sys,
                      const mlc_options* opt, mlc_ctx** out);

/* Sizes: fine interior DoFs, coarse interior DoFs, fine nodes (the length of
 * every nodal array below: the vertices for P1, vertices and edges for P2), N. */
mlc_status mlc_sizes(const mlc_ctx* ctx, int64_t* n_dof, int64_t* n_coarse_dof, int64_t* n_vertices,
                     int32_t* n_orbitals);

/* Device workspace size in bytes for this context. */
mlc_status mlc_workspace_bytes(const mlc_ctx* ctx, size_t* bytes);

/* Attach the caller's device workspace and HIP stream (hipStream_t, may be
 * null for the default stream), upload the mesh data and compute the fixed
 * matrices (K, M, V_ext at quadrature points, coarse trilinear tensor). */
mlc_status mlc_bind(mlc_ctx* ctx, void* dev_workspace, size_t bytes, void* hip_stream);

/* Algorithm 1 step 1 on the coarse mesh (self-consistent coarse Kohn-Sham
 * solve, host FP64) followed by step 4's transfer to the fine mesh:
 * Lambda = coarse eigenvalues, Phi = P Phi_H, w = coarse Hartree potential
 * interpolated to every fine vertex. tol: L1 norm of the density change. */
mlc_status mlc_initial_state(mlc_ctx* ctx, double tol, int32_t maxit, int32_t* iters);

/* Set (Lambda^l, Phi^l, w^l), the input of the next outer step (Algorithm 1
 * step 4): lambda_host[N] on the host; phi_dev[n_dof x N] (caller DoF order)
 * and w_dev[n_vertices] (nodal Hartree potential, boundary nodes
 * included) in device memory of the bound GPU, owned by the caller and
 * read only during the call. The library copies them into its workspace
 * (reordering Phi on the device) and synchronises the stream. A non-finite
 * value in any of the three is MLC_ERR_NONFINITE and the previous state is
 * kept. */
mlc_status mlc_set_state(mlc_ctx* ctx, const double* lambda_host, const double* phi_dev, const double* w_dev);

/* One outer step (Algorithm 1 steps 5-7). rep may be null. */
mlc_status mlc_correction_step(mlc_ctx* ctx, mlc_step_report* rep);

/* The current state (Lambda, Phi, rho, w) after the last step (any pointer
 * may be null): lambda_host[N] on the host; phi_dev[n_dof x N] (caller DoF
 * order), rho_dev[n_vertices] (nodal density sum f_i phi_i^2) and
 * w_dev[n_vertices] (nodal Hartree potential) in caller-owned device memory
 * of the bound GPU, written on the bound stream by device kernels and
 * copies (no host round trip); the call synchronises the stream before it
 * returns. */
mlc_status mlc_get_results(mlc_ctx* ctx, double* lambda_host, double* phi_dev, double* rho_dev, double* w_dev);

/* Intermediate quantities of the last correction step, for checking each part
 * against an independent implementation. Copies `count` doubles into host
 * array out; count must equal the size listed (MLC_ERR_ARG otherwise).
 *   MLC_PROBE_U        n_dof x N   u_i after M-normalisation (step 5)
 *   MLC_PROBE_W0       n_dof       zero-boundary Hartree direction (step 6)
 *   MLC_PROBE_G        n_vertices  multipole Dirichlet data (0 inside)
 *   MLC_PROBE_VXC_QP   nq n_tets   V_xc(rho^l) at quadrature points (nq = 4 for P1, 27 for P2)
 *   MLC_PROBE_PT_AFIX_U, _PT_MW0_U, _PT_M_U, _PT_K_U   N_H x N   P^T O u_i
 *   MLC_PROBE_UT_AFIX_U, _UT_MW0_U, _UT_M_U, _UT_K_U   N x N     U^T O U
 *   MLC_PROBE_HARTREE_D   N_H + 2  [P^T K w0, w0^T K w0, w0^T l] (l = K_IB g_B)
 *   MLC_PROBE_AFIX_H, _MW0_H, _M_H, _K_H   N_H x N_H  dense coarse matrices
 *   MLC_PROBE_AH4      N x N_H x N_H   (u_i psi_k, psi_j)
 *   MLC_PROBE_RHS      N x N_H          (u_i^2, psi_j)
 *   MLC_PROBE_THETA2   N                final theta_{2,i}
 *   MLC_PROBE_PHI_H    N_H x N          final phi_{i,H} coefficients
 *   MLC_PROBE_WH       N_H + 1          final [w_H, theta1]
 *   MLC_PROBE_SIGMA    1                shift of step 5
 *   MLC_PROBE_FEATURES n_dof x N x 6   learned-guess features (row dof, orbital)
 *   MLC_PROBE_NN_OUT   n_dof x N       network outputs of the last guess
 *   MLC_PROBE_GUESS_SCALE N            s_c = max |phi_c| of the last guess
 *   MLC_PROBE_PATTERN  3                [nonzeros of the interior CSR pattern,
 *                                        nodes per fine tet, quadrature points per fine tet]
 *   MLC_PROBE_LMAX     2                upper ends of the Chebyshev intervals [step 5, Hartree]
 */
enum {
  MLC_PROBE_U = 0, MLC_PROBE_W0, MLC_PROBE_G, MLC_PROBE_VXC_QP,
  MLC_PROBE_PT_AFIX_U, MLC_PROBE_PT_MW0_U, MLC_PROBE_PT_M_U, MLC_PROBE_PT_K_U,
  MLC_PROBE_UT_AFIX_U, MLC_PROBE_UT_MW0_U, MLC_PROBE_UT_M_U, MLC_PROBE_UT_K_U,
  MLC_PROBE_HARTREE_D,
  MLC_PROBE_AFIX_H, MLC_PROBE_MW0_H, MLC_PROBE_M_H, MLC_PROBE_K_H,
  MLC_PROBE_AH4, MLC_PROBE_RHS, MLC_PROBE_THETA2, MLC_PROBE_PHI_H, MLC_PROBE_WH,
  MLC_PROBE_SIGMA,
  MLC_PROBE_FEATURES, MLC_PROBE_NN_OUT, MLC_PROBE_GUESS_SCALE, MLC_PROBE_PATTERN,
  MLC_PROBE_LMAX,
  MLC_PROBE_COUNT
};
mlc_status mlc_probe(mlc_ctx* ctx, int32_t which, double* out, int64_t count);

/* Kernel timing for roofline accounting: replays one kernel of the solves
 * `reps` times back to back on the bound stream, between two HIP events, and
 * returns the mean duration per launch in microseconds, dispatch gaps
 * between the launches included (the launches are replayed from one captured
 * HIP graph, as the solver replays them, when options.use_graphs is set and
 * reps <= 4096; eagerly otherwise):
 *   MLC_KERNEL_CG_SPMM            step 5: Y = (A + sigma M) P over all N
 *                                 columns with the P.Y partials CG consumes
 *                                 (FP32 values under MLC_PREC_FP32_IR)
 *   MLC_KERNEL_CHEB_STEP          step 5: one Chebyshev step of the polynomial
 *                                 preconditioner (SpMM fused with the update),
 *                                 in the launch shape of all steps but the
 *                                 last (which adds the r.z partials)
 *   MLC_KERNEL_HARTREE_SPMM       step 6: the same SpMM with K, one column
 *   MLC_KERNEL_HARTREE_CHEB_STEP  step 6: one Chebyshev step with K
 * It overwrites only solver scratch (Q, the Gram blocks, the partials); the
 * state and the results of the last step are untouched. Requires a completed
 * correction step (MLC_ERR_STATE otherwise), options.precond =
 * MLC_PC_CHEBYSHEV for the Chebyshev kernels and a Hartree problem for the
 * step-6 kernels (MLC_ERR_ARG otherwise); reps in 1..100000. */
enum { MLC_KERNEL_CG_SPMM = 0, MLC_KERNEL_CHEB_STEP, MLC_KERNEL_HARTREE_SPMM, MLC_KERNEL_HARTREE_CHEB_STEP };
mlc_status mlc_time_kernel(mlc_ctx* ctx, int32_t which, int32_t reps, double* avg_us);

/* ---- Adaptive loop: estimate, mark, refine, transfer ------------------------
 * Algorithm 1 steps 1-3 and 9 around the correction step: the residual a
 * posteriori estimator of Section 2 on each fine tet T,
 *   eta^2(T) = h_T^2 ||R_T||^2_{0,T} + sum over interior faces e of T of h_e ||J_e||^2_{0,e},
 *   R_T = ((V_eff - lambda_i) phi_i)_i (the Laplacian of a P1 function vanishes
 *   inside T), J_e = (1/2 grad phi_i|T+ . nu+ + 1/2 grad phi_i|T- . nu-)_i,
 * with h_T, h_e the longest edges of T and e, V_eff of the current state, the
 * element norm by the 4-point rule of the assembly, and the norms of the
 * vectors over orbitals the sums of their squares; Doerfler marking; conforming
 * refinement of the marked tets by tagged (Maubach) bisection; the transfer of
 * nodal values (a new vertex is an edge midpoint: the mean of its ends).
 *
 * mlc_estimate: eta^2 of the context's current state for every fine tet, into
 *   the caller's device array eta2 (nt doubles, in the caller's tet order);
 *   asynchronous on the context's stream (it recomputes V_eff of the state at
 *   the quadrature points). Needs options.estimator = 1 at mlc_create and a
 *   state (MLC_ERR_STATE otherwise); MLC_ERR_ARG for a null pointer.
 * mlc_mark_dorfler: host arrays. marked[t] = 1 for the smallest set M of tets,
 *   taken in decreasing order of eta2 (ties by index), with sum_M eta2 >=
 *   theta sum eta2, 0 elsewhere; *count = |M|. theta in (0, 1]; MLC_ERR_ARG
 *   for bad arguments or a negative or non-finite eta2.
 * mlc_refine: host. Bisects the marked tets of (xyz, tets) once each and then
 *   every tet with a hanging edge until the mesh is conforming. Tets carry a
 *   refinement tag (tags, nt int8; 3 for a Kuhn-ordered initial mesh whose
 *   tets list x0, x1, x2, x3 with x0-x3 the cube diagonal) that selects the
 *   edge to bisect: tag k cuts edge x0-xk into (x0..x_{k-1}, z, x_{k+1}..x3) and
 *   (x1..x_k, z, x_{k+1}..x3), both tagged k - 1 (3 after 1). The result is
 *   written to out (mlc_refine_result, owned by the library until
 *   mlc_refine_free): new vertices are appended after the old ones; each
 *   comes with the two ends of the edge it bisects (parents, 2 per new vertex),
 *   in batches (batch_ptr) whose parents all precede the batch.
 * mlc_transfer_vertices: device. values (nv_new x ncols, row-major, caller's
 *   device memory) holds the old vertices' values in its first nv_old rows;
 *   the rows of the new vertices are filled batch by batch with the means of
 *   their parents' rows. parents_dev: the refinement's parents copied to the
 *   device (2 x (nv_new - nv_old) int64); batch_ptr: host, nbatch + 1 offsets.
 *   Asynchronous on the given stream. */
mlc_status mlc_estimate(mlc_ctx* ctx, double* eta2_dev);
mlc_status mlc_mark_dorfler(const double* eta2, int64_t nt, double theta, uint8_t* marked, int64_t* count);
typedef struct {
  int64_t nv, nt;          /* the refined mesh's vertex and tet counts */
  const double* xyz;       /* nv x 3 */
  const int32_t* tets;     /* nt x 4 */
  const int8_t* tags;      /* nt */
  int64_t n_new;           /* nv - the old vertex count */
  const int64_t* parents;  /* n_new x 2: edge ends of each new vertex */
  int32_t nbatch;
  const int64_t* batch_ptr;/* nbatch + 1 offsets into the new vertices */
  void* internal;
} mlc_refine_result;
mlc_status mlc_refine(int64_t nv, const double* xyz, int64_t nt, const int32_t* tets, const int8_t* tags,
                      const uint8_t* marked, mlc_refine_result* out);
void mlc_refine_free(mlc_refine_result* r);
mlc_status mlc_transfer_vertices(int64_t nv_old, int64_t nv_new, const int64_t* parents_dev, int32_t nbatch,
                                 const int64_t* batch_ptr, int32_t ncols, double* values_dev, void* hip_stream);

/* ---- Learned initial guess of step 5 ----------------------------------------
 * Extension of the method (the paper starts every step-5 problem from the
 * current orbital phi_i, Algorithm 1 step 5). A network of 8833 parameters,
 * 6 -> 64 -> 64 -> 64 -> 1 with GELU (erf form) after each hidden layer,
 * maps per-(DoF, orbital) features to a correction direction
 *   delta_i = s_i NN(features),  s_i = max |phi_i|,
 *   features = [V_eff at the vertex clipped to +-50, phi/s, D^-1 (b - A phi)/s,
 *               distances to the three nearest nuclei / 10 (box diagonal when
 *               fewer nuclei)],
 * with A, b, D the step-5 operator, right-hand side and diagonal. Step 5
 * then starts from x0_i = a phi_i + b delta_i, the minimiser of the energy
 * J(x) = 1/2 x.Ax - b.x over span{phi_i, delta_i} (a 2 x 2 solve per
 * column), which is never farther from the solution in the A-norm than
 * phi_i; phi_i stays the start where the 2 x 2 system is singular, where J
 * does not drop, or where the minimiser's residual |b - A x0| exceeds phi_i's
 * (CG's stopping test is on the residual, which a start closer in the A-norm
 * can still raise). Products run in BF16 on the matrix cores with FP32 accumulation;
 * master weights, Adam moments and the loss are FP32/FP64.
 * Parameter packing (floats): W1 (64 x 6, out x in), b1 (64), W2 (64 x 64),
 * b2, W3 (64 x 64), b3, W4 (64), b4 (1).
 *
 * A network object owns no memory: mlc_nn_bind hands it a device workspace
 * of mlc_nn_workspace_bytes (256-byte aligned) and the stream it runs on.
 * Device pointers (x: rows x 6 floats, t and y: rows floats) stay owned by
 * the caller. mlc_nn_forward is asynchronous on the stream; the other calls
 * return after the device finished. mlc_nn_loss_grad: loss = mean (y - t)^2
 * and its gradient (host array of 8833). mlc_nn_adam: one Adam step (bias
 * corrected) with a host gradient. mlc_nn_train: `steps` Adam steps (lr,
 * beta1 0.9, beta2 0.999, eps 1e-8) on minibatches of `batch` rows visiting
 * the rows in a fixed scattered order (row (g * k) mod rows for sample g of
 * the run, k coprime with rows); loss_history (host, steps floats) may be
 * NULL. Errors: MLC_ERR_ARG (bad sizes or pointers), MLC_ERR_STATE (not bound
 * or no parameters), MLC_ERR_NONFINITE (non-finite parameters). */
typedef struct mlc_nn mlc_nn;
#define MLC_NN_N_PARAMS 8833

mlc_status mlc_nn_create(mlc_nn** out);
mlc_status mlc_nn_workspace_bytes(const mlc_nn* nn, size_t* bytes);
mlc_status mlc_nn_bind(mlc_nn* nn, void* workspace, size_t bytes, void* stream);
mlc_status mlc_nn_set_params(mlc_nn* nn, const float* theta);
mlc_status mlc_nn_get_params(mlc_nn* nn, float* theta);
mlc_status mlc_nn_forward(mlc_nn* nn, const float* x, int64_t rows, float* y);
mlc_status mlc_nn_loss_grad(mlc_nn* nn, const float* x, const float* t, int64_t rows, double* loss, float* grad);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it): mlc_nn_loss_grad
 * with its scratch (per-block gradient and loss partials, the reduced
 * gradient and the loss; 9.05 MB) in a device-resident array of the library
 * instead of the network's workspace. Same arguments, results and errors as
 * mlc_nn_loss_grad; rows above 2^31 - 1 are MLC_ERR_ARG. It calls no
 * hipMalloc or hipFree and allocates nothing on the device. Each GPU holds
 * one copy of the array until the process ends and every call on that GPU
 * uses it: calls that overlap on one GPU (several streams or threads) race. */
mlc_status mlc_nn_loss_grad_noalloc(mlc_nn* nn, const float* x, const float* t, int64_t rows, double* loss,
                                    float* grad);
mlc_status mlc_nn_adam(mlc_nn* nn, const float* grad, double lr, double beta1, double beta2, double eps);
mlc_status mlc_nn_train(mlc_nn* nn, const float* x, const float* t, int64_t rows, int32_t steps, int32_t batch,
                        double lr, float* loss_history);
const char* mlc_nn_last_error(const mlc_nn* nn);
void mlc_nn_destroy(mlc_nn* nn);

/* Start step 5 of this context from the network's guess (nn bound, with
 * parameters, on the context's device; the context keeps the pointer until
 * the next call), or from phi again with nn = NULL. */
mlc_status mlc_set_guess(mlc_ctx* ctx, const mlc_nn* nn);
/* Training samples: every correction step from now on appends, while room is
 * left, the features and targets (u_i - phi_i)/s_i (u_i the step-5 solution
 * before its normalisation) of every stride-th DoF and all orbitals to the
 * device arrays x (capacity x 6 floats) and t (capacity floats), owned by
 * the caller. capacity 0 switches the sink off. mlc_sample_count: rows
 * written since the sink was set. */
mlc_status mlc_set_sample_sink(mlc_ctx* ctx, float* x, float* t, int64_t capacity, int32_t stride);
mlc_status mlc_sample_count(const mlc_ctx* ctx, int64_t* rows);

/* ---- Batches of independent systems ---------------------------------------
 * Batching extension of steps 5-6 (the paper steps systems one at a time; its
 * step-5 problems are independent per orbital, Section 3.2, and so are the
 * problems of independent systems). A batch steps several bound contexts with
 * a state together: the step-5 CG solves of all systems run as one set of
 * launches per CG phase over a table of row tiles (tile -> system), replayed
 * from a captured HIP graph, and likewise their Hartree solves; every other
 * phase runs per system on the batch stream; the host inner iterations
 * (Algorithm 3 step 2) run in parallel over the systems. An autotuner times
 * the batched SpMM on the first step for rows per tile {128, 256, 512, 1024}
 * x lanes per row {2, 4, 8} and keeps the fastest (mlc_batch_set_shape fixes
 * either instead).
 *
 * mlc_batch_create: ctxs[0..count) distinct, bound contexts with the same
 * options.precision, precond, cheb_degree, cheb_ratio and hartree_coarse
 * (MLC_ERR_ARG otherwise); the batch keeps the pointers (the caller keeps the
 * contexts alive, does not re-bind them and does not step them concurrently
 * with the batch). Systems may differ in mesh and orbital count.
 * mlc_batch_bind: device workspace of mlc_batch_workspace_bytes (256-byte
 * aligned, owned by the caller) and the stream every call enqueues on.
 * mlc_batch_step: one correction step of every system (same results, to
 * rounding order, as mlc_correction_step on each); reports[0..count) as in
 * mlc_correction_step (t_fine_ms and t_recon_ms of a system span the batch's
 * phases); br may be NULL. On error the message names the first failing
 * system. Errors found before the reconstruction (arguments, HIP, CG
 * breakdown, non-finite augmented solutions) leave every system's state as
 * it was; MLC_ERR_NOT_CONVERGED updates every system's state to the last
 * iterate (each system's report is filled), like mlc_correction_step. */
typedef struct mlc_batch mlc_batch;

typedef struct {
  int32_t n_systems;
  int32_t tile_rows;      /* rows per tile in use */
  int32_t spmm_lanes;     /* lanes per row in use (systems with N <= 8) */
  int32_t n_tiles;        /* step-5 tiles over all systems */
  int32_t cg_iters;       /* step-5 CG iterations (max over systems; FP32 total under refinement) */
  int32_t poisson_iters;  /* Hartree CG iterations (max over systems) */
  int32_t ir_outer;       /* refinement passes (MLC_PREC_FP32_IR) */
  int32_t pad;
  int64_t dof_orbitals;   /* sum over systems of n_dof x N */
  double t_gpu_ms;        /* HIP events: fine stage of all systems, density through coarse integrals */
  double t_solve_ms;      /* of which the batched step-5 solve */
  double t_poisson_ms;    /* of which the batched Hartree solve */
  double t_inner_ms;      /* host inner iterations, wall time */
  double t_recon_ms;      /* HIP events: reconstruction of all systems */
  double t_tune_ms;       /* autotuning wall time (first step only, not in t_gpu_ms) */
} mlc_batch_report;

mlc_status mlc_batch_create(mlc_ctx* const* ctxs, int32_t count, mlc_batch** out);
mlc_status mlc_batch_workspace_bytes(const mlc_batch* b, size_t* bytes);
mlc_status mlc_batch_bind(mlc_batch* b, void* workspace, size_t bytes, void* stream);
/* tile_rows in {0, 128, 256, 512, 1024}, lanes in {0, 2, 4, 8}; 0 = autotune. */
mlc_status mlc_batch_set_shape(mlc_batch* b, int32_t tile_rows, int32_t lanes);
mlc_status mlc_batch_step(mlc_batch* b, mlc_step_report* reports, mlc_batch_report* br);
const char* mlc_batch_last_error(const mlc_batch* b);
void mlc_batch_destroy(mlc_batch* b);

const char* mlc_status_string(mlc_status s);
const char* mlc_last_error(const mlc_ctx* ctx);
void mlc_destroy(mlc_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* MLC_H */
