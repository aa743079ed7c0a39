/*
 * nls.h -- C ABI of the MI355X two-level nonlinear Schwarz library (libnls).
 *
 * Method: nonlinear restricted additive Schwarz with exact tangent (RASPEN)
 * and an optional GDSW coarse level, driven by an outer Newton iteration on
 * the nonlinearly preconditioned system (Heinlein, Ho, Klawonn, Lanser,
 * "Nonlinear Two-Level Schwarz Methods: A Parallel Implementation in
 * FROSch", Section 2, eqs. (3)-(13)).
 *
 * Conventions
 *  - Every call returns an int: 0 success, negative error, positive
 *    "completed but not converged".  No C++ exception crosses the ABI.
 *  - Host arrays passed to setters are copied before the call returns; the
 *    library never keeps or frees caller memory.
 *  - Device pointers (argument names ending in _dev) must point to memory of
 *    the handle's device; the library reads and writes them in stream order
 *    on the handle's stream and synchronises that stream before returning.
 *  - Global node indices are 0-based; vectors hold d values per mesh node
 *    (d = 1 for diffusion, 2 for elasticity), node-major and interleaved:
 *    dof d*g + c is component c of node g.  Dirichlet lists name dofs.
 *  - A handle is used by one host thread at a time.
 *  - All floating point at the ABI is IEEE binary64.
 */
#ifndef NLS_H
#define NLS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define NLS_OK            0
#define NLS_ENOCONV       1   /* outer Newton hit its iteration limit; last iterate written */
#define NLS_EINVAL       -1   /* bad argument (null pointer, out-of-range index, size) */
#define NLS_EHIP         -2   /* a HIP runtime call failed */
#define NLS_ENOMEM       -3   /* device allocation failed */
#define NLS_EPARTITION   -4   /* empty subdomain, or owned nodes not inside V_i (overlap < 1) */
#define NLS_ESINGULAR    -5   /* zero pivot in a local, interior or coarse LU */
#define NLS_ELOCAL       -6   /* an inner (local or coarse) Newton iteration failed */
#define NLS_ENAN         -7   /* non-finite value in a residual */
#define NLS_ESTATE       -8   /* call out of order (e.g. solve before set_partition) */
#define NLS_ELIMIT       -9   /* a subdomain exceeds a kernel limit (band too wide for LDS) */
#define NLS_EDETF       -10   /* elasticity: a deformation with det F <= 0 at a quadrature
                                 point of a local or coarse residual (eq. (2) is defined
                                 for det F > 0 only) */

/* ---- enumerations ---------------------------------------------------- */
#define NLS_ELEM_P1_TRI   3   /* 3-node triangles, counter-clockwise */
#define NLS_ELEM_Q1_QUAD  4   /* 4-node bilinear quadrilaterals, counter-clockwise */

#define NLS_PROBLEM_DIFFUSION 1  /* -div(kappa (1 + beta u^2) grad u) = f, eq. (1);
                                    P1 triangles, d = 1 */
#define NLS_PROBLEM_NEOHOOKE  2  /* -div P(F) = 0, eq. (2), compressible Neo-Hooke
                                    P = mu (F - F^-T) + lambda ln(det F) F^-T;
                                    Q1 quadrilaterals, 2 x 2 Gauss points, d = 2 */

#define NLS_PREC_FP64     0   /* every step in binary64 */
#define NLS_PREC_FP32_IR  1   /* local LU in binary32, binary64 residuals and
                                 iterative refinement of every local solve */
#define NLS_PREC_BF16_IR  2   /* trial: as NLS_PREC_FP32_IR, with the trailing
                                 updates A22 -= L21 U12 of the blocked LU on
                                 bfloat16 operands (FP32 accumulation, matrix
                                 cores); refinement up to 30 steps per solve.
                                 Local solves whose refinement does not reach
                                 its tolerance give inexact Newton steps */

#define NLS_ONE_LEVEL     0   /* F_1(u) = sum_i P~_i T_i(u), eq. (5) with (8) */
#define NLS_ADDITIVE      1   /* F_a(u) = F_1(u) + P_0 T_0(u), eq. (10) */
#define NLS_HYBRID        2   /* F_h(u) = F_1(u - P_0 T_0(u)) + P_0 T_0(u), eq. (11):
                                 coarse correction first, local corrections at
                                 the coarse-corrected point; tangent eq. (12) */

#define NLS_COARSE_NONE   0
#define NLS_COARSE_GDSW   1   /* vertex + edge components, harmonic extension */
#define NLS_COARSE_RGDSW  2   /* reduced: one set of functions per crosspoint,
                                 option 2.2 (inverse-distance weights on edges;
                                 Dirichlet edge ends weighted the same way) */

/* ---- options --------------------------------------------------------- */
typedef struct nls_options {
    int    device;        /* HIP device ordinal */
    void*  stream;        /* hipStream_t to run on; NULL = the null stream */
    int    precision;     /* NLS_PREC_* */
    int    coupling;      /* NLS_ONE_LEVEL, NLS_ADDITIVE or NLS_HYBRID */
    double outer_rtol;    /* stop when ||F_x(u_k)||_2 <= outer_rtol ||F_x(u_0)||_2 */
    int    outer_maxit;
    double inner_rtol;    /* local/coarse Newton: ||r||_2 <= max(inner_rtol rho_0,  */
    double inner_eta;     /*   inner_eta ||b||_inf sqrt(n)), b the load vector      */
    double stagnation;    /*   or last step <= stagnation ||x||_inf                  */
    int    inner_maxit;
    double gmres_rtol;    /* GMRES on eq. (13): ||r||_2 <= gmres_rtol ||F_x(u_k)||_2 */
    int    gmres_maxit;
    int    gmres_restart;
    int    flags;         /* NLS_FLAG_* bits */
    int    lu_variant;    /* local band LU: 0 widest blocked panel the band
                             allows (NB = 16 if kl <= 48, 8 if kl <= 56),
                             1 blocked NB = 16, 2 blocked NB = 8, 3 unblocked
                             (a variant that cannot hold a band falls back
                             to the unblocked form); NLS_FLAG_AUTOTUNE
                             overrides it per size bucket */
} nls_options;

/* options.flags: time the local-solve and local-tangent kernels with HIP
   events on the handle's stream (adds one event pair per launch). */
#define NLS_FLAG_PROFILE  1
/* options.flags: run GMRES with the Hessenberg rotations on the device and
   every block of 4 Arnoldi steps replayed as one HIP graph (captured on
   first use on a stream of the library's own), one host synchronisation
   per block instead of per step.  Used when the tangent has its explicit
   local blocks and, for two-level coupling, an explicit coarse inverse;
   otherwise GMRES runs step by step. */
#define NLS_FLAG_GRAPH    2
/* options.flags: the coarse iteration for T_0 (eq. (9)) takes chord steps
   with the last factorisation of A0 (from the previous evaluation or its
   own first step), refactoring when the residual fails to halve.  This is
   a different iteration from Newton's: both stop once ||G|| meets the
   coarse stopping rule, so their T_0 agree to that tolerance, not to the
   rounding level (on the 512 x 512 workload the outer solutions differ by
   about 2e-10 relative).  A0 and its LU at the converged coarse state are
   formed in every mode (exact tangent, eq. (12)). */
#define NLS_FLAG_COARSE_CHORD 4
/* options.flags: apply A0^{-1} in the tangent by band LU solves instead of
   an explicit inverse formed once per evaluation. */
#define NLS_FLAG_COARSE_LU_APPLY 8
/* options.flags: at the first solve after the partition (or coarse space)
   is set, time the candidates on the device and keep the fastest: for each
   size bucket of local solves the band LU variant (blocked NB = 16, NB = 8,
   unblocked; each with its own LDS size and hence occupancy), timed as the
   bucket's fused local Newton launch at the initial iterate; for the coarse
   term of the tangent the explicit inverse against a band LU solve per
   GMRES step, priced at 20 steps per evaluation.  On an NLS_PREC_FP32_IR
   handle the local solves are timed in both precisions (binary32 LU with
   refinement, and binary64 LU) and the faster total is kept for all of
   them.  nls_get_tuning reports the decisions. */
#define NLS_FLAG_AUTOTUNE 16
/* options.flags: on a second stream of the handle, concurrently with the
   local work: with the additive coupling, the coarse Newton solve T_0(u)
   (eq. 9) beside the local solves T_i(u) (eq. 4), both depending on u
   only; with any two-level coupling, the tangent's coarse Galerkin matrix,
   LU and inverse at c* beside the local factorisations; with the additive
   coupling, the coarse term of each tangent product (eqs. 7, 12) beside its
   local term.  Results are those of the serial order; the reported inner
   and coarse phase times overlap. */
#define NLS_FLAG_OVERLAP  32
/* options.flags: build the exact tangent's local blocks W_i = J_ii^{-1} B_i
   (eqs. 6, 7) by per-lane band sweeps, one right-hand side per lane, instead
   of the blocked solve on the matrix cores (the default where kl <= 48 and
   kl + ku <= 112 in every subdomain), and the explicit A0^{-1} by a band
   solve step by step instead of the same blocked solve.  Both forms apply
   the same factors; they differ in rounding only. */
#define NLS_FLAG_TANGENT_SWEEP 64

/* ---- statistics of the last solve ------------------------------------ */
#define NLS_MAX_OUTER 64
typedef struct nls_stats {
    int       converged;            /* 1 if the outer stopping rule was met */
    int       outer_its;            /* outer Newton iterations taken */
    int       gmres_its[NLS_MAX_OUTER];
    int       gmres_its_total;
    int64_t   inner_its_total;      /* sum over evaluations and subdomains */
    int       inner_its_max;        /* largest local iteration count seen */
    int64_t   local_solves;         /* number of local nonlinear solves T_i */
    int       coarse_its_total;
    int       failed_subdomain;     /* -1, or the subdomain whose Newton failed */
    double    res0;                 /* ||F_x(u_0)||_2 */
    double    res_final;            /* ||F_x(u_final)||_2 */
    double    ms_inner;             /* phase times (device-synchronised wall),  */
    double    ms_coarse;            /*   the paper's schema: inner + coarse +    */
    double    ms_gmres;             /*   gmres + other = total; coarse work run  */
    double    ms_other;             /*   beside the local solves (NLS_FLAG_      */
    double    ms_total;             /*   OVERLAP) is in ms_overlap, not coarse   */
    /* with NLS_FLAG_PROFILE: event-timed launches of the fused local Newton
       kernel and of the local tangent kernel */
    int       n_local_launches;
    double    ms_local_kernel;
    int       n_tangent_launches;
    double    ms_tangent_kernel;
    /* learned initial guess (when enabled): local solves that started from
       the prediction, and those whose prediction was rejected by the judge
       or whose Newton iteration from it failed (then started from R_i u) */
    int64_t   guess_used;
    int64_t   guess_fallback;
    /* coarse Newton time that ran beside the local solves (inside ms_inner) */
    double    ms_overlap;
} nls_stats;

typedef struct nls_handle nls_handle;

/* Fill *opt with defaults: FP64, one-level, outer_rtol 1e-8, outer_maxit 50,
   inner_rtol 1e-12, inner_eta 1e-10, stagnation 1e-14, inner_maxit 30,
   gmres_rtol 1e-6, gmres_maxit 1000, gmres_restart 50. */
int nls_default_options(nls_options* opt);

/* Create a handle on opt->device.  *out receives the handle; the library
   owns it and every device buffer it allocates until nls_destroy.
   Errors: NLS_EINVAL (null pointers, bad enum), NLS_EHIP. */
int nls_create(const nls_options* opt, nls_handle** out);

/* Free every resource of h (NULL is accepted). */
int nls_destroy(nls_handle* h);

/* The mesh of the abstract discrete problem F(u) = 0 (eq. (3)).
   xy: n_nodes x 2 coordinates (row-major); conn: n_elems x 3 node indices
   per element, counter-clockwise.  Copied.  Errors: NLS_EINVAL on an index
   out of range or a non-positive element area. */
int nls_set_mesh(nls_handle* h, int elem_kind, int64_t n_nodes,
                 const double* xy, int64_t n_elems, const int32_t* conn);

/* The same as nls_set_mesh for the structured mesh of [0,lx] x [0,ly] with
   nx x ny cells: node (i,j) has index j*(nx+1) + i and coordinates
   (i*(lx/nx), j*(ly/ny)).  NLS_ELEM_P1_TRI: cell (i,j) is split along its
   diagonal (i,j)-(i+1,j+1) into elements 2(j nx + i) = [(i,j), (i+1,j),
   (i+1,j+1)] and 2(j nx + i) + 1 = [(i,j), (i+1,j+1), (i,j+1)] (the
   "regular square mesh" of Section 3 read as P1 triangles);
   NLS_ELEM_Q1_QUAD: element j nx + i = [(i,j), (i+1,j), (i+1,j+1), (i,j+1)].
   Errors: NLS_EINVAL (nx, ny < 1, lx, ly not positive and finite, or more
   than 2^27 nodes or elements). */
int nls_set_mesh_structured(nls_handle* h, int elem_kind, int32_t nx, int32_t ny,
                            double lx, double ly);

/* The nonlinear problem on that mesh.
   NLS_PROBLEM_DIFFUSION (eq. (1) generalised), P1 mesh:
     -div( kappa_e (1 + beta u^2) grad u ) = f.
   params[0] = beta.  elem_coef: kappa per element, or NULL for 1.
   elem_load: f sampled at the midpoints of each element's edges
   (v0,v1), (v1,v2), (v2,v0) (n_elems x 3), or NULL for f = 1; the load is
   integrated with the edge-midpoint rule.
   NLS_PROBLEM_NEOHOOKE (eq. (2)), Q1 mesh: params[0] = mu, params[1] =
   lambda (Lame parameters, mu > 0); elem_coef and elem_load must be NULL;
   external forces are nodal, see nls_set_nodal_load (zero until set); a
   quadrature point with det F <= 0 makes the residual non-finite
   (NLS_ENAN).  Copied.  Dirichlet data must be set after the problem. */
int nls_set_problem(nls_handle* h, int kind, const double* params,
                    const double* elem_coef, const double* elem_load);

/* Dirichlet nodes and values; F_g(u) = u_g - value on those rows.  Copied. */
int nls_set_dirichlet(nls_handle* h, int64_t n, const int64_t* nodes,
                      const double* values);

/* Element-based partition into n_sub subdomains (Section 2, last paragraph:
   the overlap is built on elements so each subdomain can assemble locally).
   elem_part[e] in [0, n_sub).  Each subdomain is grown by `overlap` layers
   of elements sharing a node with it.  V_i is the set of patch nodes whose
   every element is in the patch; node g is owned by the largest subdomain
   id among its elements (restricted prolongation, eq. (8)).
   Errors: NLS_EPARTITION (empty subdomain, overlap < 1), NLS_ELIMIT. */
int nls_set_partition(nls_handle* h, int32_t n_sub, const int32_t* elem_part,
                      int32_t overlap);

/* Build the coarse space P_0 = Phi (Section 2; GDSW family).  kind
   NLS_COARSE_GDSW: for every connected interface component (vertices:
   nodes of >= 3 subdomains, edges: 2) the null-space modes restricted to
   it (scalar: 1; elasticity: two translations, and the rotation about the
   component's centroid when it has >= 2 nodes).  NLS_COARSE_RGDSW
   (Section 2: the paper's choice, option 2.2 with its modification): one
   set of modes per crosspoint; an edge node takes inverse Euclidean
   distance weights of the crosspoints whose subdomain sets contain the
   edge's, a Dirichlet node ending the edge counting as one more ancestor
   of value 0; an edge without such crosspoints keeps its own modes.
   Interface values are extended harmonically with DF(u_lin) into every
   subdomain interior: u_lin is a host array of n_nodes * d values, or NULL
   for u_lin = 0 (the default linearisation point; diffusion: the
   kappa-weighted Laplacian, elasticity: linear elasticity).  The extension
   is fixed once built (all outer iterations and load steps use it).
   Errors: NLS_ESTATE (no partition), NLS_ESINGULAR, NLS_EINVAL (u_lin not
   finite). */
int nls_build_coarse(nls_handle* h, int kind, const double* u_lin);

/* Nodal external forces f (n_nodes * d values, dof order) of a problem
   whose load is nodal (NLS_PROBLEM_NEOHOOKE): F(u) = f_int(u) - f on free
   dofs.  Entries on Dirichlet dofs are ignored.  Like nls_set_load it keeps
   the partition and the coarse space (load stepping calls it once per
   step).  Errors: NLS_ESTATE, NLS_EINVAL. */
int nls_set_nodal_load(nls_handle* h, const double* f);

/* Replace the load samples only (same layout and meaning as elem_load of
   nls_set_problem; NULL for f = 1), keeping mesh, coefficients, Dirichlet
   data, partition and coarse space: neither the overlapping subdomains nor
   the GDSW basis (extended with DF(0), which does not involve f) depend on
   f.  The load vector b, ||b||_inf and ||Phi^T b||_inf of the stopping
   rules are recomputed.  Errors: NLS_ESTATE (no partition), NLS_EINVAL. */
int nls_set_load(nls_handle* h, const double* elem_load);

/* Outer Newton iteration on F_x(u) = 0 (eq. (13)): solve
   D F_x(u_k) du = F_x(u_k) by GMRES and set u_{k+1} = u_k - du.
   u: n_nodes values, read as the initial iterate and overwritten with the
   last iterate; a device pointer if u_on_device != 0, else host memory.
   load_factor: the external load of the problem (load samples of the
   diffusion problem, nodal forces of elasticity) scaled by this factor for
   this solve (1.0: as set; the set load is in place again on return).
   st may be NULL.  Returns NLS_OK, NLS_ENOCONV, or an error (NLS_ELOCAL
   with st->failed_subdomain, NLS_ENAN, NLS_EDETF, NLS_ESINGULAR, ...). */
int nls_solve(nls_handle* h, double* u, int u_on_device, double load_factor,
              nls_stats* st);

/* A batch of independent problems, one handle each (hs[k], n distinct
   handles, each set up completely): every handle runs nls_solve (outer
   Newton, eq. (13), with its own stopping rule, GMRES and local and coarse
   solves) on its own iterate us[k] (device pointer if u_on_device[k],
   u_on_device may be NULL for host arrays), at the same time as the others:
   one host thread per handle (at most 32 at once, taking the handles in
   order), so the kernels of handles on different streams run on the device
   together; handles sharing a stream run in that stream's order.  Results
   are those of solving each problem alone.  codes[k] receives each
   instance's return code and sts[k] (or NULL) its statistics.  Returns
   NLS_OK if every instance converged, the first negative code in index
   order if any failed, else NLS_ENOCONV.  NLS_EINVAL on null or repeated
   handles. */
int nls_solve_batch(nls_handle* const* hs, int n, double* const* us,
                    const int* u_on_device, nls_stats* sts, int* codes);

/* Load stepping (continuation, Section 3 of the paper: the beam load is
   increased in steps): the external load is set to s / n_steps of its
   full value (nodal forces, or the load samples of the diffusion problem)
   for s = 1..n_steps, and each step runs nls_solve from the previous
   step's solution.  u: initial iterate in, last solution out (device
   pointer if u_on_device).  st: n_steps records or NULL.  Stops at the
   first step that does not return NLS_OK and returns its code; the full
   load is in place again on return. */
int nls_solve_load_steps(nls_handle* h, double* u, int u_on_device, int n_steps,
                         nls_stats* st);

/* Newton-Krylov-Schwarz comparator (Section 3 of the paper, the beam test):
   Newton's method on F(u) = 0 itself; each step solves DF(u_k) du = F(u_k)
   by GMRES right-preconditioned with linear restricted additive Schwarz
   built at u_k: M^{-1} = sum_i P~_i (R_i DF(u_k) P_i)^{-1} R_i, plus
   Phi (Phi^T DF(u_k) Phi)^{-1} Phi^T on a two-level handle (the coarse
   basis of nls_build_coarse); u_{k+1} = u_k - du.  Same subdomains, band
   LU (FP64), GMRES and stopping rules as nls_solve, with ||F(u_k)||_2 in
   place of ||F_x(u_k)||_2.  u and st as for nls_solve (inner_its_total and
   local_solves stay 0; ms_inner / ms_coarse time the factorisations).
   Overwrites the state kept for nls_apply_tangent.  Returns NLS_OK,
   NLS_ENOCONV, NLS_ESINGULAR (zero pivot), NLS_ENAN, or an error. */
int nls_solve_nks(nls_handle* h, double* u, int u_on_device, nls_stats* st);

/* ---- hooks at the internal boundaries (device pointers) --------------- */

/* F(u) (eq. (3)), n_nodes values. */
int nls_eval_residual(nls_handle* h, const double* u_dev, double* F_dev);

/* F_x(u) for the handle's coupling (eqs. (5), (10)); also keeps the local
   and coarse states at u for nls_apply_tangent. */
int nls_eval_precond_residual(nls_handle* h, const double* u_dev,
                              double* Fx_dev);

/* y = D F_x(u) v at the u of the last nls_eval_precond_residual
   (eqs. (6), (7), (12)).  Errors: NLS_ESTATE if no state is kept. */
int nls_apply_tangent(nls_handle* h, const double* v_dev, double* y_dev);

/* Standalone local assembly (eqs. (3)-(4) at the first local iterate
   x = R_i u): for every subdomain the local residual R_i F(u) (at x = R_i u
   it equals the rows of F(u) at V_i, assembled from the patch elements
   only) into r_dev, sum_i |V_i| values in packed order, and, if jval_dev is
   not NULL, the values of the local Jacobian rows [J_ii | B_i] = R_i DF(u)
   restricted to the patch, in the CSR pattern of nls_get_local_pattern.
   Device pointers.  The same element kernels as the local Newton solves,
   without the factorisation: the assembly step on its own. */
int nls_eval_local(nls_handle* h, const double* u_dev, double* r_dev, double* jval_dev);

/* Row layout of the local problems and the CSR pattern of [J_ii | B_i]
   (host arrays).  Call with off_v == NULL to get counts[0] = sum_i |V_i|
   (packed rows), counts[1] = nonzeros, counts[2] = sum_i |Gamma_i|; then
   off_v (n_sub + 1): the rows of subdomain i are [off_v[i], off_v[i+1]);
   row_dof (counts[0]): global dof of each packed row; off_g (n_sub + 1) and
   gamma_dof (counts[2]): the Gamma_i dofs; rowptr (counts[0] + 1) and col
   (counts[1]): patch-local columns, c < n_i the c-th row of the subdomain,
   c >= n_i its (c - n_i)-th Gamma_i dof.  Any output may be NULL. */
int nls_get_local_pattern(nls_handle* h, int64_t* counts, int32_t* off_v, int32_t* row_dof,
                          int32_t* off_g, int32_t* gamma_dof, int64_t* rowptr, int32_t* col);

/* Local Newton iteration counts of the last evaluation, n_sub ints (host). */
int nls_get_inner_iterations(nls_handle* h, int32_t* its_host);

/* Number of subdomains and coarse functions; sizes of V_i (host, n_sub). */
int nls_get_sizes(nls_handle* h, int32_t* n_sub, int32_t* n_coarse,
                  int32_t* nv_host);

/* Coarse basis Phi (n_nodes x n_coarse) as CSR in host memory.  Call with
   rowptr == NULL to query *nnz; then rowptr (n_nodes+1), col and val (nnz)
   must be caller-allocated.  Columns are ordered by the smallest node index
   of their interface component. */
int nls_get_coarse_basis(nls_handle* h, int64_t* nnz, int64_t* rowptr,
                         int32_t* col, double* val);

/* Decisions of NLS_FLAG_AUTOTUNE (or the defaults before tuning), host
   arrays with room for one entry per size bucket (at most n_sub):
   *n_buckets; per bucket the LU variant (1 NB = 16, 2 NB = 8, 3 unblocked,
   0 by band width), its LDS bytes and its subdomain count; *coarse_inverse
   (1 explicit inverse, 0 LU solves) and coarse_ms[3] = measured ms of the
   inverse, one inverse apply and one LU solve (0 if not tuned);
   *local_precision = the NLS_PREC_* the local solves run in.  Any output
   may be NULL. */
int nls_get_tuning(nls_handle* h, int32_t* n_buckets, int32_t* lu_variant,
                   int32_t* lds_bytes, int32_t* n_sub, int32_t* coarse_inverse,
                   double* coarse_ms, int32_t* local_precision);

/* ---- learned initial guess of the local solves ------------------------
   Not part of the paper's method, which starts every inner Newton
   iteration for T_i(u) (eq. (4)) from R_i u.  A network proposes another
   start for each subdomain; the local solve takes it only when
   ||R_i F(v(x_pred))||_2 < ||R_i F(u)||_2, keeps its stopping rule relative
   to ||R_i F(u)||_2, and restarts from R_i u if Newton from the prediction
   fails, so T_i(u) is the same up to the stopping tolerance.

   Within nls_solve, an evaluation whose predictions the judge took for
   fewer than 1 in 20 subdomains makes the next two evaluations start from
   R_i u without consulting the network (guess_used + guess_fallback then
   count only the evaluations that consulted it).

   Features of subdomain i (320), diffusion: u at 64 points of the perimeter of the
   patch box (16 per side at t = j/16, counter-clockwise from the lower-left
   corner), then the nodal load (mean of the edge-midpoint samples of f
   around each node) at the 16 x 16 reference nodes (x0 + p W/15,
   y0 + q H/15), index q*16 + p; each sample is the linear interpolant of
   the nodal field in the mesh element containing the point.  Output (256):
   coefficients at the reference nodes; x_pred = transfinite (Coons)
   interpolant of the perimeter samples + bilinear interpolant of the
   coefficients, Dirichlet nodes exact.  Training target: v(x*) - Coons at
   the reference nodes, v(x*) = x* on V_i and u elsewhere (eq. (4)).

   Network: affine layers 320 -> 256 -> 256 -> 256 -> 256, GELU (exact erf)
   after the first three; parameters flat float32 W1 b1 W2 b2 W3 b3 W4 b4
   (W_l row-major [out][in]), 279552 values.

   Elasticity (Q1, two components; the same sizes, per component x then y):
   inputs u_x, u_y at 32 perimeter points (8 per side), then the external
   nodal forces f_x, f_y (zero on Dirichlet dofs) at 128 points
   (x1, y0 + j H/127) on the right side of the box (the loaded edge of the
   cantilever); outputs and targets on the 16 x 8 reference nodes
   (x0 + p W/15, y0 + q H/7), index q*16 + p, per component; samples are
   bilinear (Q1) interpolants in the quadrilateral containing the point;
   x_pred per component = Coons of its 32 trace samples + bilinear
   interpolant of its 128 coefficients, Dirichlet dofs exact.  Products in bfloat16 on the
   matrix cores with FP32 accumulation; FP32 master weights.  norm: 1152
   floats [x_mean(320) x_dev(320) y_mean(256) y_dev(256)]; the network maps
   (x - x_mean)/x_dev to (y - y_mean)/y_dev.  Arrays named _dev below are
   device pointers. */
#define NLS_GUESS_PARAMS 279552
#define NLS_GUESS_NORM   1152
#define NLS_GUESS_IN     320
#define NLS_GUESS_OUT    256

/* Set the network (copied; host arrays).  norm NULL: identity.  Resets the
   Adam state.  Errors: NLS_EINVAL (size, non-finite values). */
int nls_guess_set_model(nls_handle* h, const float* params, int64_t n_params,
                        const float* norm);
/* Copy the network out (host arrays; either may be NULL). */
int nls_guess_get_model(nls_handle* h, float* params, float* norm);
/* Use the network in every following evaluation (0 turns it off).
   Errors: NLS_ESTATE without a network. */
int nls_guess_enable(nls_handle* h, int enable);
/* Start capturing (features, target) pairs of converged local solves, up
   to `capacity` rows (subdomain order, evaluation after evaluation); the
   library allocates the store.  0 stops and frees it. */
int nls_guess_capture(nls_handle* h, int64_t capacity);
/* Copy min(rows captured, max_rows) rows to X_dev (rows x 320) and T_dev
   (rows x 256) and report the count in *n_rows; with both NULL only the
   count is reported. */
int nls_guess_captured(nls_handle* h, float* X_dev, float* T_dev,
                       int64_t max_rows, int64_t* n_rows);
/* Features of every subdomain at u_dev (n_sub x 320, raw). */
int nls_guess_features(nls_handle* h, const double* u_dev, float* X_dev);
/* x_pred (packed V rows, subdomain order, as the lengths of
   nls_get_sizes) from caller coefficients coef_dev (n_sub x 256). */
int nls_guess_lift(nls_handle* h, const double* u_dev, const float* coef_dev,
                   double* xpred_dev);
/* Network output in target units for n raw feature rows. */
int nls_guess_predict(nls_handle* h, const float* X_dev, int64_t n, float* Y_dev);
/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   network output as nls_guess_predict, for n <= NLS_GUESS_NOALLOC_ROWS raw
   feature rows, computed in a fixed working area of the library (a
   device array of 6.8 MB per GPU, held until the process ends) instead of
   buffers it allocates.  The call allocates and frees nothing and does not
   synchronise: it enqueues its kernels on the handle's stream and returns;
   Y_dev is complete in stream order.  Calls on one GPU share the working
   area, so calls that overlap in time on one GPU (other streams, other
   threads) race; serialise them.  Errors: NLS_ELIMIT (n too large),
   NLS_ESTATE (no network), NLS_EINVAL, NLS_EHIP. */
#define NLS_GUESS_NOALLOC_ROWS 4096
int nls_guess_predict_noalloc(nls_handle* h, const float* X_dev, int64_t n, float* Y_dev);
/* Mean squared error over all outputs of the standardised batch (X_dev,
   T_dev raw, n rows <= 65536) and its gradient (NLS_GUESS_PARAMS floats,
   device; may be NULL), without changing the network. */
int nls_guess_loss_grad(nls_handle* h, const float* X_dev, const float* T_dev,
                        int64_t n, float* grad_dev, double* loss);

#define NLS_TRAIN_FIT_NORM 1   /* first set norm from the training data */
#define NLS_TRAIN_COSINE   2   /* cosine decay of the learning rate to 0 */
#define NLS_MAX_EPOCHS     256
typedef struct nls_train_opts {
    int    epochs;
    int    batch;        /* rows per Adam step (<= 65536) */
    double lr;
    double beta1, beta2, eps;
    int    flags;        /* NLS_TRAIN_* bits */
} nls_train_opts;
typedef struct nls_train_stats {
    int64_t steps;
    double  final_loss;                  /* mean step loss of the last epoch */
    double  epoch_loss[NLS_MAX_EPOCHS];  /* mean step loss per epoch */
    double  ms;
} nls_train_stats;
/* Train the network by Adam (Kingma and Ba) on n rows X_dev (n x 320),
   T_dev (n x 256) in the library's own kernels.  order_dev: epochs x n
   row indices (one permutation per epoch), or NULL for the stored order.
   The last batch of an epoch may be short. */
int nls_guess_train(nls_handle* h, const nls_train_opts* opts, const float* X_dev,
                    const float* T_dev, int64_t n, const int32_t* order_dev,
                    nls_train_stats* st);

/* ---- host-only inspection (no device is touched) ----------------------- */

/* Build the overlapping subdomains of nls_set_partition on the host and
   report them.  Call once with the output arrays NULL to get
   counts[0] = sum_i |V_i| and counts[1] = sum_i |Gamma_i|; then pass
   off_v, off_g (n_sub+1), v_nodes (counts[0]), g_nodes (counts[1]),
   own_pos (n_nodes: position in v_nodes of the owner's copy of node g) and
   kl, ku (n_sub: band widths of J_ii under the ascending-node local
   order).  Any output pointer may be NULL.  Errors as nls_set_partition. */
int nls_inspect_partition(int64_t n_nodes, int64_t n_elems, const int32_t* conn,
                          int32_t n_sub, const int32_t* elem_part, int32_t overlap,
                          int64_t* counts, int32_t* off_v, int32_t* v_nodes,
                          int32_t* off_g, int32_t* g_nodes, int32_t* own_pos,
                          int32_t* kl, int32_t* ku);

/* Interface components of the GDSW coarse space (host only).  dirichlet:
   n_dir node indices excluded from the interface.  First call with
   comp_off == NULL gives counts[0] = n_coarse, counts[1] = total component
   nodes; then comp_off (n_coarse+1) and comp_nodes receive the components,
   ordered by smallest node, nodes ascending. */
int nls_inspect_coarse(int64_t n_nodes, int64_t n_elems, const int32_t* conn,
                       int32_t n_sub, const int32_t* elem_part, int64_t n_dir,
                       const int64_t* dirichlet, int64_t* counts,
                       int32_t* comp_off, int32_t* comp_nodes);

/* Message for a status code; message of the last error on h.  Strings are
   owned by the library. */
const char* nls_strerror(int code);
const char* nls_last_error(nls_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* NLS_H */
