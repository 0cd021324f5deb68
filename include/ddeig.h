/*
 * ddeig.h -- C ABI of the MI355X library for the smallest eigenpair of the
 * Q1 finite-element Schroedinger operator -Laplace + V on anisotropically
 * long boxes, by sigma-shifted inverse iteration whose inner solves are CG
 * preconditioned by two-level additive Schwarz with the PerFact coarse space
 * (Theisen & Stamm, arXiv 2311.08757).
 *
 * Problem (§1, eq:schroedingerEquation, eq:geometry-description):
 *   -Laplace(phi) + V phi = lambda phi on Omega_L = (0,L)^p x (0,ell)^q,
 *   phi = 0 on the boundary, V of period 1 in every expanding direction x_i
 *   (assumption A1) and bounded (A2).
 * Discretisation (§2, eq:discrete-weak-form): Q1 elements on the uniform
 * Cartesian grid of spacing h = 1/n_e made of translated copies of the unit
 * cell mesh; the potential term uses the tensor 2-point Gauss-Legendre rule
 * per element with V evaluated at cell-local x coordinates.  The algebraic
 * problem is A x = lambda M x with A = K + M_V (stiffness + potential mass)
 * and M the mass matrix (the paper's B); A_sigma = A - sigma M.
 *
 * Vector layout at this boundary: every vector is FP64, device resident, of
 * length n_dof, holding the interior nodes (Dirichlet nodes eliminated) in
 * lexicographic order with x1 fastest, then x2 (p = 2), then y1, then y2.
 * A node with 1-based grid index i_a (1 <= i_a <= L n_e - 1 in expanding,
 * 1 <= i_a <= ell n_e - 1 in fixed directions) sits at coordinate i_a h.
 * Cell vectors (psi) hold the unit-cell nodes with x indices 0..n_e-1
 * (periodic) and fixed-direction indices 1..ell n_e - 1, same ordering.
 *
 * Ownership: the handle owns every internal buffer; the caller owns every
 * vector passed in (e.g. torch tensors, by data pointer).  Inputs and outputs
 * must not alias.  All device work runs on the stream given to
 * ddeig_assemble.  apply_op and apply_precond are asynchronous on that
 * stream; cell_shift, pcg_solve and inverse_iteration synchronise it and
 * return host scalars.
 *
 * Errors: every call returns a ddeig_status; no exception crosses the ABI.
 * ddeig_last_error() returns a message for the last failing call of the
 * calling thread.  One handle must not be used from two threads at once.
 */
#ifndef DDEIG_H
#define DDEIG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DDEIG_OK = 0,
  DDEIG_EINVAL = -1,     /* invalid argument (geometry, h, overlap, NULL, NaN) */
  DDEIG_ENOMEM = -2,     /* device allocation failed */
  DDEIG_EHIP = -3,       /* a HIP runtime call failed */
  DDEIG_ENOTSPD = -4,    /* CG breakdown: p.A_sigma p <= 0 or r.z <= 0, or a
                            non-positive pivot while factorising */
  DDEIG_ENOCONV = -5,    /* iteration limit reached; outputs hold the last iterate */
  DDEIG_ESTATE = -6,     /* call order violated (e.g. pcg_solve before cell_shift) */
  DDEIG_EINTERNAL = -7
} ddeig_status;

/* Omega_L = (0,L)^p x (0,ell)^q (eq:geometry-description).  L >= 1 integer,
 * p >= 1, q >= 1, p + q in {2, 3}; ell * n_e must be an integer. */
typedef struct {
  int p, q;
  int L;
  double ell;
} ddeig_geometry;

/* Periodic potentials V (period 1 in x, assumption A1).
 *   CONST        V = c0
 *   SEP_FOURIER  V = sum_t a_t cos(2 pi k_t x1 + phi_t) (1 + cy prod_j sin(pi y_j / ell))
 *   FOURIER2     V = sum_t a_t cos(2 pi (k_t x1 + m_t x2) + phi_t)       (p = 2)
 *   SIN4         V = c0 prod_i sin^4(pi x_i) prod_j sin^4(pi y_j / ell)    (§4.1)
 *   SEP_SUM      V = c0 + sum_t a_t sin(2 pi k_t z_{m_t}) + sum_j g_j y_j  (§4.3;
 *                m_t is the 0-based coordinate index of term t)
 *   QUAD_TABLE   any V (periodic in x by construction), given by its values at
 *                the quadrature points of one period cell: the cell's elements
 *                (n_e per expanding, ell n_e per fixed direction) in lexicographic
 *                order, axis 0 fastest, each with its 2^(p+q) tensor Gauss points,
 *                point index sum_a b_a 2^a where b_a = 0 selects the coordinate
 *                (e_a + (1 - 1/sqrt 3) / 2) h and b_a = 1 (e_a + (1 + 1/sqrt 3) / 2) h;
 *                table_len = n_e^p (ell n_e)^q 2^(p+q) values, copied by the call.
 * Arrays have nterms entries (g has q); at most DDEIG_MAX_TERMS terms. */
typedef enum {
  DDEIG_V_CONST = 0,
  DDEIG_V_SEP_FOURIER = 1,
  DDEIG_V_FOURIER2 = 2,
  DDEIG_V_SIN4 = 3,
  DDEIG_V_SEP_SUM = 4,
  DDEIG_V_QUAD_TABLE = 5
} ddeig_vkind;

#define DDEIG_MAX_TERMS 64

typedef struct {
  ddeig_vkind kind;
  int nterms;
  const double* a;    /* host arrays */
  const double* phi;
  const int* k;
  const int* m;
  double cy;
  double c0;
  const double* g;
  const double* table;  /* QUAD_TABLE: host array of table_len values */
  long table_len;
} ddeig_potential;

typedef struct {
  int pu;          /* partition of unity: 0 equal weights 1/#covering subdomains (§2.2),
                      1 distance-based chi_i = d_i / sum_j d_j (§4.1.2) */
  int coarse;      /* 0 one-level AS (eq:dd-preconditioners), 1 two-level AS with the
                      PerFact coarse space (eq:two-level-preconditioners,
                      def:algebraic-perfact-coarse-space) */
  int local_prec;  /* local subdomain solves: 0 FP64 block-chain factors, 1 FP32 factors with
                      FP32 arithmetic, 2 dense inverses as bf16 hi/lo pairs applied on MFMA
                      (bf16x3, FP32 accumulation), 3 dense inverse and residual in single
                      bf16 (one MFMA product, FP32 accumulation); the outer CG is FP64 in
                      every case */
  int batch_iters; /* PCG iterations queued between host convergence checks (0: default 8) */
  int graphs;      /* 1: each block of batch_iters PCG iterations is captured once into a HIP
                      graph (per first iteration, maxit and iterate pointer) on a stream of the
                      problem and replayed from then on; 0: kernels are launched one by one */
  int sweep;       /* A_sigma sweep: 0 by size, 1 tiles, 2 march.  2-D grids with n_e dividing
                      64: the row march (512 columns per workgroup) once the grid has >= 1024
                      such column blocks; 3-D grids with n_e dividing 32 and 8 n < 2^31: the
                      plane march (256 x 8 lines per workgroup) once there are >= 1024 such
                      blocks.  Tiles and march give identical A_sigma x */
} ddeig_options;

typedef struct ddeig_problem ddeig_problem;

typedef struct {
  int iters;          /* PCG iterations performed */
  double relres;      /* ||r_k||_2 / ||r_0||_2 of the recursively updated residual */
  int breakdown;      /* 1 if p.A_sigma p <= 0, 2 if r.z <= 0 */
  double* hist;       /* optional host array: hist[k] = ||r_k|| / ||r_0||, k = 0..iters */
  int hist_cap;       /* capacity of hist */
  double true_relres; /* ||b - A_sigma x||_2 / ||r_0||_2 recomputed from the returned x */
  int fallback;       /* pcg_solve: 1 if r.z <= 0 under dense reduced-precision local solves
                         switched the problem to FP32 chain local solves and the solve was
                         repeated (2-D problems) */
} ddeig_pcg_info;

typedef struct {
  double lambda;      /* sigma + x^T A_sigma x for the M-normalised x */
  double dx_M;        /* ||x_k - x_{k-1}||_M of the last step */
  int outer_its;
  long inner_sum;
  int inner_max;
  double t_solve_ms;
  double spec_res;    /* ||A x - lambda M x||_2 of the returned (M-normalised) x */
  double t_setup_ms;  /* wall time of ddeig_assemble and the shift calls of the problem */
  int inner_unconverged; /* inner solves that stopped at maxit_inner (the call then
                            returns DDEIG_ENOCONV even if the outer test was met) */
  int fallback;          /* 1 if an inner solve switched the local solves to FP32 (as for
                            ddeig_pcg_info.fallback) and was repeated */
} ddeig_eig_info;

/* Builds the period-cell operator tables (K, M, M_V at one period cell: §2,
 * assumption A1), the decomposition of Omega_L into the L^p unit cells
 * extended by `overlap` element layers (§3, §4.1) and the device buffers.
 * h must be 1/n_e with n_e >= 3 an integer (checked to 1e-12 relative);
 * 1 <= overlap and 2 overlap <= n_e.  `hip_stream` is a hipStream_t (NULL:
 * the null stream).  Returns a new handle in *out. */
ddeig_status ddeig_assemble(const ddeig_geometry* geom, double h, const ddeig_potential* V,
                            int overlap, const ddeig_options* opts, void* hip_stream,
                            ddeig_problem** out);

/* Solves the periodic cell problem (eq:cell-problem, eq:weak-form-cell-problem)
 * on the device: sigma = smallest eigenvalue of (K# + M_V#) psi = sigma M# psi,
 * psi > 0, psi^T M# psi = 1.  Then finishes every sigma-dependent set-up: the
 * shifted operator, the local subdomain factorisations of A_sigma,i
 * (eq:twoLevelASMPreconditioner), the coarse basis and coarse matrix.
 * psi_cell_host (nullable) receives n_cell values. */
ddeig_status ddeig_cell_shift(ddeig_problem* P, double* sigma_out, double* psi_cell_host);

/* Test/debug override of the CG breakdown test: the next `count` PCG solves
 * of the problem that run with dense reduced-precision local solves report
 * r.z <= 0 at their first iteration (the test compares r.z with +inf instead
 * of 0), which exercises the FP32 fallback of ddeig_pcg_solve and
 * ddeig_inverse_iteration without a genuinely indefinite preconditioner. */
ddeig_status ddeig_debug_force_breakdown(ddeig_problem* P, int count);

/* Test/debug override of the shift: uses the given sigma and cell vector
 * (n_cell host values, nullable for one-level preconditioning only) instead of
 * solving the cell problem, then does the same set-up as ddeig_cell_shift. */
ddeig_status ddeig_set_shift(ddeig_problem* P, double sigma, const double* psi_cell_host);

/* y = Op x on the device, Op = 0: A_sigma, 1: A = K + M_V, 2: M, 3: K.
 * which = 0 needs a shift (cell_shift or set_shift); the others only assemble. */
ddeig_status ddeig_apply_op(ddeig_problem* P, int which, const double* x, double* y);

/* z = M_AS,2^{-1} r (or M_AS,1^{-1} r with options.coarse = 0):
 * sum_i R_i^T A_sigma,i^{-1} R_i r + R_0^T A_sigma,0^{-1} R_0 r  (§3). */
ddeig_status ddeig_apply_precond(ddeig_problem* P, const double* r, double* z);

/* Schwarz preconditioners of §3 (eq:dd-preconditioners,
 * eq:two-level-preconditioners), selected by `kind`:
 *   AS1     z = sum_i R_i^T A_sigma,i^{-1} R_i r
 *   AS2     AS1 + R_0^T A_sigma,0^{-1} R_0 r        (the PerFact coarse space)
 *   RAS1    z = sum_i R_i^T D_i A_sigma,i^{-1} R_i r (D_i: the partition of unity
 *           of options.pu; restricted additive Schwarz, not symmetric)
 *   RAS2    RAS1 + R_0^T A_sigma,0^{-1} R_0 r
 *   COARSE  R_0^T A_sigma,0^{-1} R_0 r alone (the coarse correction of
 *           eq:two-level-stationary-ras-mult-cc)
 * The local solves are those of options.local_prec.  Kinds with the coarse
 * space need options.coarse = 1 (DDEIG_ESTATE otherwise). */
#define DDEIG_PREC_AS1 0
#define DDEIG_PREC_AS2 1
#define DDEIG_PREC_RAS1 2
#define DDEIG_PREC_RAS2 3
#define DDEIG_PREC_COARSE 4

/* z = M^{-1} r for the preconditioner `kind` (asynchronous on the library
 * stream; needs the shift).  r and z: n_dof device values, not aliased. */
ddeig_status ddeig_apply_schwarz(ddeig_problem* P, int kind, const double* r, double* z);

/* Stationary RAS for A_sigma x = b: levels = 1 iterates
 * x_{k+1} = x_k + M_RAS,1^{-1} (b - A_sigma x_k) (eq:stationary-ras); levels = 2
 * follows every such half step by the coarse correction of the new residual,
 * x += R_0^T A_sigma,0^{-1} R_0 (b - A_sigma x) (multiplicative,
 * eq:two-level-stationary-ras-mult-cc; needs options.coarse = 1).  The
 * residual b - A_sigma x is recomputed after every correction.  x holds x0
 * on entry; stops when ||r_k||_2 <= rtol ||r_0||_2 or after maxit steps (a
 * half step and its coarse correction are one step).  info as for pcg_solve
 * (breakdown = 1 when the residual overflowed).  Synchronises the library
 * stream.  Returns DDEIG_ENOCONV at maxit or on divergence. */
ddeig_status ddeig_stationary_ras(ddeig_problem* P, int levels, const double* b, double* x,
                                  double rtol, int maxit, ddeig_pcg_info* info);

/* GMRES for A_sigma x = b with right preconditioning by `kind` (§3: GMRES
 * with the unsymmetric M_RAS,2 is the Krylov method for RAS; §4.2).  Arnoldi
 * by delayed classical Gram-Schmidt with reorthogonalisation (DCGS2: the
 * second projection of v_j shares its sweep over the basis with the first
 * projection of the next vector); the preconditioned vectors
 * z_j = M^{-1} v_j are kept and x = x0 + Z y (y from the Givens-rotated
 * least-squares problem), which equals x0 + M^{-1} V y for a linear M and
 * keeps the Arnoldi relation when the local solves round their input (bf16).
 * Restarts every `restart` steps from the true residual (restart <= 0: every
 * min(maxit, 300) steps; at most 1024).  x holds x0 on entry; stops when the
 * residual norm of the least-squares problem is <= rtol ||r_0||_2 or after
 * maxit steps.  info as for pcg_solve (relres and hist: the least-squares
 * residual norms; breakdown = 1 for a zero Hessenberg column).  Work space:
 * (2 restart + 1) n_dof doubles, kept by the handle.  Synchronises the library
 * stream.  Returns DDEIG_ENOCONV at maxit or on breakdown. */
ddeig_status ddeig_gmres_solve(ddeig_problem* P, int kind, const double* b, double* x, double rtol,
                               int maxit, int restart, ddeig_pcg_info* info);

/* Preconditioned CG for A_sigma x = b (§2.1, §3): x holds x0 on entry and the
 * iterate on exit; stops when ||r_k||_2 <= rtol ||r_0||_2 (§4.1).  Returns
 * DDEIG_ENOCONV after maxit iterations, DDEIG_ENOTSPD on breakdown.  With
 * dense reduced-precision local solves (local_prec 2, 3) on a 2-D problem, a
 * breakdown with r.z <= 0 (the rounded inverse made the preconditioner
 * indefinite) switches the problem to FP32 block-chain local solves for the
 * rest of its life and repeats the solve from x0 (info->fallback = 1); the
 * same holds for the inner solves of ddeig_inverse_iteration. */
ddeig_status ddeig_pcg_solve(ddeig_problem* P, const double* b, double* x, double rtol,
                             int maxit, ddeig_pcg_info* info);

/* sigma-shifted inverse iteration (§2): x_{k+1} = A_sigma^{-1} M x_k solved by
 * PCG from a zero guess to rtol_inner, M-normalised, sign fixed so that
 * 1^T M x > 0; stops when ||x_{k+1} - x_k||_M <= tol_x or after maxit_outer
 * steps.  x: on entry the start vector (all zeros selects 1/||1||_M); on exit
 * the M-normalised eigenvector (the last iterate on any error).  Returns
 * DDEIG_ENOTSPD on a CG breakdown of an inner solve, DDEIG_ENOCONV at
 * maxit_outer or when any inner solve stopped at maxit_inner (counted in
 * info->inner_unconverged: the outer test may then have settled on the fixed
 * point of the inexact solve). */
ddeig_status ddeig_inverse_iteration(ddeig_problem* P, double* x, double tol_x, int maxit_outer,
                                     double rtol_inner, int maxit_inner, ddeig_eig_info* info);

typedef struct {
  double lambda;      /* x^T A x of the final, M-normalised x */
  double res_norm;    /* ||A x - lambda M x||_2 */
  int outer_its;
  long inner_sum;     /* inner iterations (modes 0, 1) or preconditioner applications (mode 2) */
  int inner_max;
  double t_solve_ms;
} ddeig_lopcg_info;

/* Inexact shift-and-invert preconditioned LOPCG (alg:si-lopcg, §2.1; inner
 * variants of §4.3).  From the M-normalised x_k and the spectral residual
 * r_k = A x_k - R(x_k) M x_k, each outer step solves A_sigma w_k = r_k
 * inexactly and takes the minimiser of the Rayleigh quotient over
 * span{w_k, x_k, x_{k-1}} (Rayleigh-Ritz on the directions B-orthogonalised
 * against x_k, with p = x_k - x_{k-1} for x_{k-1}; directions whose scaled
 * Gram eigenvalue is below 1e-10 of the largest are dropped), M-normalised
 * with 1^T M x > 0; it stops when ||r_k||_2 <= tol_o (M-normalised x) or
 * after maxit_outer steps.  mode 0: the inner solver `inner` from zero to the
 * relative tolerance rtol_inner; 1: to min(0.1, ||r_k||_2); 2: one
 * application of the two-level preconditioner, w_k = M^{-1} r_k (no inner
 * solve; inner selects M_AS,2 (CG_AS2) or M_RAS,2 (GMRES_RAS2), the latter
 * being the fused variant of §4.3).  Inner solvers (§4.2, Table 2): CG with
 * the problem's additive Schwarz preconditioner, GMRES with M_RAS,2 (restart
 * min(maxit_inner, 300)), stationary RAS2 (multiplicative coarse
 * correction), stationary RAS1; an inner solve that reaches maxit_inner
 * leaves its last iterate and the outer iteration continues.  x: in the
 * start vector x_1 (all zeros selects the constant vector), out the
 * eigenvector; x_prev (nullable): x_0, default the first unit vector.  Needs
 * the shift (and options.coarse = 1 for the RAS2 solvers); synchronises the
 * library stream.  Returns DDEIG_ENOCONV at maxit_outer or when an inner
 * GMRES breaks down or a stationary solve diverges, DDEIG_ENOTSPD on a CG
 * breakdown of an inner solve. */
#define DDEIG_INNER_CG_AS2 0
#define DDEIG_INNER_GMRES_RAS2 1
#define DDEIG_INNER_RAS2 2
#define DDEIG_INNER_RAS1 3

ddeig_status ddeig_lopcg(ddeig_problem* P, double* x, const double* x_prev, double tol_o,
                         int maxit_outer, int mode, int inner, double rtol_inner, int maxit_inner,
                         ddeig_lopcg_info* info);

/* Measurement support: launches one kernel (or step) of the hot path `reps`
 * times on the library's stream between two HIP events and returns the mean
 * duration of one launch in *avg_us (synchronises).  which = 0: the A_sigma
 * stencil on x (y receives A_sigma x); 1: the level-1 local solves on the
 * batch left by the last apply_precond (dense: the MFMA GEMM over all
 * subdomains, m = unknowns of the unclipped box, with the coarse
 * right-hand-side workgroups it carries inside the preconditioner when the
 * problem has the coarse space and clipped subdomains; otherwise the
 * block-chain solves), so call apply_precond first; 2: the whole preconditioner on x
 * (y receives z); 3: the restriction of x into the batch; 4: the extension
 * (y receives z from the current local and coarse solutions; x plays r);
 * 5: the clipped-class correction of the dense local solves (no-op
 * otherwise).  *work receives the algorithmic work of one launch: bytes for
 * which = 0 (16 per unknown), flops for which = 1 (2 m^2 per subdomain: dense
 * inverse applied once; 4 nch b^2 per subdomain for block-chain solves), 0
 * otherwise. */
ddeig_status ddeig_profile_kernel(ddeig_problem* P, int which, int reps, const double* x, double* y,
                                  double* avg_us, double* work);

/* Measurement support: runs reps + 1 iterations of a PCG on A_sigma x = b from
 * x = 0 that cannot stop (rtol 0) on the library stream, with HIP events
 * between the parts of each iteration, and returns in us[0..4] the mean
 * duration (us) of each part over the last reps iterations: 0 the stencil with
 * the direction update (p = z + beta p, q = A_sigma p, p.q), 1 the restriction
 * with the update of x and r (||r||^2), 2 the local solves (the MFMA GEMM over
 * all subdomains, carrying R_0 r when the coarse space rides in the dense
 * launches; or the block-chain solves), 3 the clipped-class correction with
 * the coarse solve (dense local solves; 0 otherwise), 4 the extension with the
 * stopping test and r.z (with the wait for the coarse correction when that
 * runs on the second stream).  Uses the problem's internal vectors (any
 * earlier solve state is overwritten); b: n_dof device values.  Needs the
 * shift; synchronises.  1 <= reps <= 200. */
ddeig_status ddeig_profile_iteration(ddeig_problem* P, const double* b, int reps, double* us);

/* Potential-weighted bilinear form out = x^T M_W y, where M_W is the mass
 * matrix weighted by the potential W, assembled with the same quadrature as
 * M_V (§2, eq:discrete-weak-form: A = K + M_V is linear in V, so the
 * derivative of A with respect to a parameter theta of V is M_{dV/dtheta}).
 * space = 0: the global grid, x and y are n_dof device values in the
 * canonical layout; space = 1: the periodic cell, n_cell values in cell
 * order.  With W = dV/dtheta and x = y the M-normalised eigenvector of
 * inverse_iteration this is dlambda/dtheta (Hellmann-Feynman); with the
 * M#-normalised cell vector psi it is dsigma/dtheta; with an adjoint solution
 * w and u = A_sigma^{-1} b it gives w^T (dA/dtheta) u for the gradient of the
 * linear solve.  W uses the layout of ddeig_potential; it is copied during the
 * call.  Needs only ddeig_assemble; synchronises the library stream. */
ddeig_status ddeig_potential_form(ddeig_problem* P, int space, const ddeig_potential* W,
                                  const double* x, const double* y, double* out);

/* Derivatives with respect to the Fourier parameters theta = (a_1..a_T,
 * phi_1..phi_T) of the problem's own SEP_FOURIER or FOURIER2 potential (beyond
 * the paper).  A = K + M_V (§2, eq:discrete-weak-form) is linear in V, so
 * dA/dtheta_j = M_{dV/dtheta_j} with the quadrature of M_V, where
 * dV/da_t = cos(arg_t) env and dV/dphi_t = -a_t sin(arg_t) env (the t-th term
 * of the potential without, and with its amplitude, and its argument advanced
 * by pi / 2).  All 2T forms and x^T M y come from one element-walking kernel.
 * grad: host array of ngrad = 2T values (a_1..a_T, then phi_1..phi_T); other
 * kinds of potential or another ngrad return DDEIG_EINVAL.  Synchronise.
 *
 * ddeig_eig_grad: dlambda/dtheta = x^T M_{dV} x / x^T M x (Hellmann-Feynman)
 *   for the ground state x (any scaling, n_dof device values) of A x = lambda M x.
 * ddeig_shift_grad: dsigma/dtheta = psi^T M#_{dV} psi / psi^T M# psi for the
 *   cell eigenvector of the last cell_shift (eq:cell-problem; DDEIG_ESTATE
 *   without a shift or after set_shift without psi).
 * ddeig_solve_grad: for u = A_sigma^{-1} b (b independent of theta) and a
 *   scalar l(u) with w = A_sigma^{-1} dl/du (the adjoint solve: A_sigma is
 *   symmetric, so w comes from ddeig_pcg_solve with the same preconditioner),
 *   dl/dtheta = -(w^T M_{dV} u - dsigma/dtheta w^T M u), the shift moving with
 *   theta.  u, w: n_dof device values. */
ddeig_status ddeig_eig_grad(ddeig_problem* P, const double* x, double* grad, int ngrad);
ddeig_status ddeig_shift_grad(ddeig_problem* P, double* grad, int ngrad);
ddeig_status ddeig_solve_grad(ddeig_problem* P, const double* u, const double* w, double* grad,
                              int ngrad);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same form
 * out = x^T M_W y as ddeig_potential_form (same arguments, layouts and
 * errors), computed without any allocation.  Its only device memory besides x
 * and y is a static 1 MiB array per GPU held by the library until the process
 * ends (partial sums, W's description, and a QUAD_TABLE weight of at most
 * 129024 values; a larger table returns DDEIG_EINVAL).  Calls that overlap on
 * one GPU (other threads or streams) race on that array.  Synchronises the
 * library stream. */
ddeig_status ddeig_potential_form_noalloc(ddeig_problem* P, int space, const ddeig_potential* W,
                                          const double* x, const double* y, double* out);

/* Batches of independent problems (e.g. many domain lengths L or potentials
 * at once).  The instances keep their own shift, local inverse, coarse
 * space and CG state; every kernel of a PCG iteration (§3,
 * eq:cg-energy-norm-error-reduction, with the preconditioner of
 * eq:twoLevelASMPreconditioner) runs as one grouped launch over all
 * instances, and each instance stops on its own test.  Requirements, checked
 * by ddeig_batch_create (DDEIG_EINVAL otherwise): every instance is 2-D
 * (p = q = 1) with L > 4, dense local solves (local_prec 2 or 3, the same for
 * all) and the coarse space, n_e dividing 64 and at most 1024 stencil tiles
 * ((n_dof x-extent / 256 rounded up) x (ell n_e - 1) / 8 rounded up); all share
 * n_e, overlap, ell, the partition of unity and the stream.  The batch
 * borrows the problems: they must outlive it and must not be used on their
 * own while a batch call runs.  Creation runs a small autotuner that times
 * the grouped MFMA GEMM for each admissible K split and tile order on the
 * device and keeps the fastest (synchronises). */
typedef struct ddeig_batch ddeig_batch;

/* flags: DDEIG_BATCH_GRAPHS replays the grouped iterations (8 per host check)
 * from HIP graphs captured on first use (one per block start and maxit),
 * instead of launching the kernels one by one.  DDEIG_BATCH_REPRODUCIBLE
 * skips the timing: the GEMM keeps the K split of the instances' own
 * single-problem path (the smallest over the instances) in XCD-interleaved
 * order, so the batch's results are fixed by the inputs alone (and equal
 * the single-problem path's bit for bit when all instances share that
 * split).  Without it the autotuner's choice is remembered per shape
 * (local_prec, ld, the instances' subdomain counts) for the life of the
 * process: a later batch of the same shapes reuses it without timing and
 * repeats the first batch's bits. */
#define DDEIG_BATCH_GRAPHS 1
#define DDEIG_BATCH_REPRODUCIBLE 2
/* With DDEIG_BATCH_REPRODUCIBLE only: 64-row GEMM tiles instead of 128 (the
 * tile rows do not change the arithmetic: the results are the same bits). */
#define DDEIG_BATCH_TILE64 4

ddeig_status ddeig_batch_create(ddeig_problem* const* probs, int n, int flags, ddeig_batch** out);

/* Autotuner result: K split, tile order (0 instance-major, 1 XCD-interleaved),
 * number of GEMM tiles, and the six measured times in us of the 128-row tiles
 * (split 1..3 x order 0..1; 0 where a split was not admissible, and all 0
 * when nothing was timed: DDEIG_BATCH_REPRODUCIBLE or a remembered choice). */
ddeig_status ddeig_batch_query(const ddeig_batch* B, int* ksplit, int* order, int* ntiles,
                               double* tune_us);

/* The tile shape of the autotuner's choice and all twelve timings: tile_rows
 * (128, or 64 when the instances' padding rows make smaller row tiles pay),
 * tune_us[12] in us, index (tile rows 128: 0, 64: 1) x 6 + (split - 1) x 2 +
 * order (0 where a candidate was not timed). */
ddeig_status ddeig_batch_tuning(const ddeig_batch* B, int* tile_rows, double* tune_us);

/* PCG for every instance j: A_sigma,j x[j] = b[j] (host arrays of n device
 * pointers; x[j] holds x0 on entry).  info (nullable, n entries; hist is
 * ignored) receives each instance's iterations, relative residual and
 * breakdown flag.  Returns DDEIG_OK when every instance converged, else the
 * status of the failing instance (ENOTSPD before ENOCONV).  Batches have no
 * FP32 fallback: a breakdown is reported in that instance's info. */
ddeig_status ddeig_batch_pcg_solve(ddeig_batch* B, const double* const* b, double* const* x,
                                   double rtol, int maxit, ddeig_pcg_info* info);

/* sigma-shifted inverse iteration (as ddeig_inverse_iteration) for every
 * instance; converged instances drop out of the grouped launches.  x: n
 * device pointers (all-zero start vectors select 1/||1||_M).  info (nullable,
 * n entries) receives each instance's result; t_solve_ms is the batch's
 * wall time.  Returns DDEIG_OK when every instance converged. */
ddeig_status ddeig_batch_inverse_iteration(ddeig_batch* B, double* const* x, double tol_x,
                                           int maxit_outer, double rtol_inner, int maxit_inner,
                                           ddeig_eig_info* info);

/* The derivatives above for every instance of a batch in one grouped launch
 * (all instances must have T terms; ngrad = 2T).  x, u, w: host arrays of n
 * device pointers; grad: host array of n x 2T values, instance-major.
 * ddeig_batch_eig_grad: dlambda_j/dtheta_j from the eigenvectors x[j] (e.g.
 * those of ddeig_batch_inverse_iteration).  ddeig_batch_solve_grad: the
 * linear-solve gradients for u[j] = A_sigma,j^{-1} b[j] and the adjoint
 * solutions w[j] (e.g. from ddeig_batch_pcg_solve on dl/du[j]). */
ddeig_status ddeig_batch_eig_grad(ddeig_batch* B, const double* const* x, double* grad,
                                  int ngrad);
ddeig_status ddeig_batch_solve_grad(ddeig_batch* B, const double* const* u, const double* const* w,
                                    double* grad, int ngrad);

void ddeig_batch_destroy(ddeig_batch* B);

/* Sizes: interior unknowns, cell unknowns, number of subdomains (= coarse dimension). */
ddeig_status ddeig_query(const ddeig_problem* P, long* n_dof, long* n_cell, int* n_sub);

void ddeig_destroy(ddeig_problem* P);
const char* ddeig_status_string(ddeig_status s);
const char* ddeig_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DDEIG_H */
