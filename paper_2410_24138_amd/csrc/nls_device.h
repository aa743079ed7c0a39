// Device-side views (plain device pointers) shared by the solver driver and
// the HIP kernels of libnls.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

// Global mesh and problem data, all resident in HBM.
struct DevMesh {
    int N, E;
    int kind;                   // NLS_PROBLEM_*
    int nv, d, ndof;            // nodes per element, dofs per node, N*d
    const int* conn;            // nv*E
    const double* xy;           // 2N
    const int* nptr;            // N+1: node -> incident elements
    const int* nel;             // (element << 2) | vertex position
    const double* G6;           // 6E: |T| grad(phi_a).grad(phi_b): G00 G11 G22 G01 G12 G20
    const double* kappa;        // E
    const double* eload;        // 3E: element load vectors
    const double* bload;        // ndof: assembled load (diffusion) or nodal
                                //   forces (elasticity), 0 on Dirichlet rows
    const unsigned char* dflag; // ndof
    const double* dval;         // ndof
    double beta;                // diffusion
    double mu, lam;             // elasticity
};

// Overlapping-subdomain tables (see HostMaps).
struct DevMaps {
    int nsub;
    const int *off_n, *off_g, *off_e, *l2g, *g2g, *pe_conn, *pe_gid;
    const int *rinc_ptr, *rinc, *jptr, *jcol, *kl, *ku, *order, *own_pidx;
    const int64_t *off_u, *off_l;
};

// Per-evaluation state of the local level.
struct DevLocal {
    double* jval;               // CSR values of [J_ii | B_i] at the current point
    double* Uf;                 // FP64 factors (column-band U, column L)
    double* Lf;
    float* Uf32;                // FP32 factors (mixed precision)
    float* Lf32;
    int* piv;                   // packed, one per V row
    double* xstar;              // packed converged local states
    double* ghost;              // packed Gamma_i values of the last evaluation
    double* T;                  // packed T_i(u) = R_i u - x*
    double* z;                  // packed scratch of the tangent
    int* its;                   // per subdomain
    int* status;                // per subdomain: 0 ok, 1 no convergence, 2 NaN, 3 zero pivot,
                                //   4 det F <= 0 (elasticity)
    int* start;                 // per subdomain: 0 from R_i u, 1 from the predicted start,
                                //   2 prediction rejected or failed, then from R_i u
};

// Exact-tangent tables and storage: W_i = (J_ii^{-1} B_i) on owned rows.
#define NLS_MAX_BCOL 8
struct DevTangent {
    const int *bptr, *brow, *bslot;   // B_i by columns (packed over Gamma columns)
    const int *off_own, *ownrow, *rowown;
    const int64_t *off_W, *off_F;
    double* W;                        // sum |owned_i| |Gamma_i|
    double* fwd;                      // sum ceil16(n_i) ceil16(|Gamma_i|) (forward-sweep scratch)
    // blocked solve on the matrix cores: blocks of 16 rows, off_blk[i] the
    // first block of subdomain i, blk_sub the subdomain of each block
    const int *off_blk, *blk_sub;
    int* tsig;                        // 64 per block: sigma_b
    double *tG, *tUi;                 // per block: G_b, U11^{-1} in operand order
};

struct NewtonParams {
    double rtol;                // relative to ||R_i F(u)||
    double abs_tol;             // eta * ||b||_inf (times sqrt(n_i) in the kernel)
    double stagnation;
    int maxit;
    int mixed;                  // 1: FP32 LU + FP64 iterative refinement; 2: the same
                                //   with bfloat16 operands in the LU's trailing updates
    int ir_maxit;
    double ir_rtol;
    const double* xpred;        // packed predicted starts, or null
    int lu_variant;             // 0 by band width, 1 blocked NB=16, 2 NB=8, 3 unblocked
    int keep_factor;            // 1: J and its FP64 LU at x* formed by the local kernel;
                                // 0: left to launch_local_factor at (xstar, ghost)
};

// Most coarse functions nonzero at one interface dof (see HostCoarse).
#ifndef NLS_CFUN
#define NLS_CFUN 4
#endif

// GDSW coarse space tables (see HostCoarse) and state.
struct DevCoarse {
    int n0, nsub;
    const int *off_c, *cnode, *ctype, *off_k, *klist, *cfun, *off_ne, *ne_conn, *ne_gid;
    const double* cval;         // interface values of the functions named in cfun
                                //   (NLS_CFUN pairs per closure dof)
    const int *cinc_ptr, *cinc, *iidx, *off_ni, *inode, *iptr, *icol, *ikl, *iku;
    const int64_t *off_phi, *off_iu, *off_il, *off_kk;
    const int *perm, *a0ptr, *a0col, *a0src_ptr, *a0src, *gsrc_ptr, *gsrc, *cpos, *cown;
    int a0kl, a0ku;
    int nnz0;                   // entries of A0's CSR pattern
    int nblk;                   // diagonal blocks of A0 (connected components)
    const int *boff, *bkl, *bku, *rblk;
    const int64_t *offU, *offL, *offI;
    double* phi;                // dense |C_i| x |K_i| blocks
    double* zbuf;               // same shape: DF Phi rows (scratch)
    double* ybuf;               // DF^T Phi at the converged coarse point, per subdomain
                                //   column-major (|closure| rows contiguous per function)
    double* ival;               // interior CSR values (setup scratch)
    double* iU;                 // interior factors (setup scratch)
    double* iL;
    int* ipiv;
    double* gblk;               // per-subdomain Phi_i^T q (packed by off_k)
    double* ablk;               // per-subdomain Galerkin blocks (packed by off_kk)
    double* a0val;              // CSR values of A0 (band order)
    double* a0U;                // A0 factors
    double* a0L;
    int* a0piv;
    double* rhs;                // n0, band order
    double* a0inv;              // n0 x n0 inverse of A0 (band order, row-major)
    // A0^{-1} by the blocked solve on the matrix cores (inv_nblk > 0): the
    // 16-row blocks of the diagonal blocks (inv_off[b]: the first of block
    // b), their pieces, and the forward scratch (inv_offY[b] into inv_Y)
    const int* inv_off;
    const int64_t* inv_offY;
    int inv_nblk, inv_nkk;
    int* inv_sig;
    double *inv_G, *inv_Ui, *inv_Y;
    double* c;                  // n0, coarse iterate (coarse id order)
    double* w;                  // N: u - Phi c
    double* scal;               // device scalars: [0] ||G||, [1] max|dc|, [2] max|c|
    int* flag;                  // [0] zero pivot in the coarse/interior LU
};

// ---- launchers (kernels.hip) ------------------------------------------------
hipError_t launch_p1_setup(const DevMesh& M, const double* xy, const double* elem_coef,
                           const double* elem_load, double* G6, double* kappa,
                           double* eload, int* bad, hipStream_t s);
hipError_t launch_assemble_load(const DevMesh& M, double* bload, hipStream_t s);
hipError_t launch_global_residual(const DevMesh& M, const double* u, double* F,
                                  hipStream_t s);
hipError_t launch_local_newton(const DevMesh& M, const DevMaps& P, const DevLocal& L,
                               const NewtonParams& np, const double* u, int nblk, int lds_bytes,
                               int nb_per_lane, hipStream_t s);
// Standalone local assembly at x = R_i u: packed residuals r and CSR values
// jval (may be null) of every subdomain; max_rows = largest |V_i| rows,
// lds_bytes = 8 (|V_i| + |Gamma_i|) of the largest patch.
hipError_t launch_local_assemble(const DevMesh& M, const DevMaps& P, const double* u, double* r,
                                 double* jval, int max_rows, int lds_bytes, hipStream_t s);
hipError_t launch_prolong(const DevMesh& M, const DevMaps& P, const double* T,
                          const DevCoarse* C, const double* cvec, double* out,
                          const double* addv, hipStream_t s);
// z_i = J_ii^{-1} B_i v_Gamma_i (restrict_rhs = 0, the exact tangent) or
// z_i = J_ii^{-1} R_i v (restrict_rhs = 1, the linear Schwarz preconditioner)
hipError_t launch_tangent_local(const DevMesh& M, const DevMaps& P, const DevLocal& L,
                                const NewtonParams& np, const double* v, int lds_bytes,
                                int nb_per_lane, hipStream_t s, int restrict_rhs = 0);
// Newton-Krylov-Schwarz pieces: DF(u) v, Phi^T r into the coarse blocks,
// J_ii(u) and its LU
hipError_t launch_global_jv(const DevMesh& M, const double* u, const double* v, double* out,
                            hipStream_t s);
hipError_t launch_coarse_phit(const DevCoarse& C, const double* r, hipStream_t s);
// J_ii and its FP64 LU at R_i u with Gamma values from u, or, with xloc and
// gloc (packed like xstar and ghost), at that local state
hipError_t launch_local_factor(const DevMesh& M, const DevMaps& P, const DevLocal& L,
                               const NewtonParams& np, const double* u, int nblk, int lds_bytes,
                               hipStream_t s, const double* xloc = nullptr,
                               const double* gloc = nullptr);
// out = v - Phi c over all dofs (hybrid tangent)
hipError_t launch_sub_coarse(const DevMesh& M, const DevCoarse& C, const double* cvec,
                             const double* v, double* out, hipStream_t s);
// ulin: linearisation point of DF (global vector), or null for u = 0
hipError_t launch_gdsw_extend(const DevMesh& M, const DevCoarse& C, const double* ulin,
                              int lds_bytes, int nb_per_lane, hipStream_t s);
hipError_t launch_coarse_w(const DevMesh& M, const DevCoarse& C, const double* u,
                           double* w, hipStream_t s);
hipError_t launch_coarse_q(const DevMesh& M, const DevCoarse& C, const double* w,
                           const double* v, int mode, int lds_bytes, hipStream_t s);
hipError_t launch_coarse_galerkin(const DevMesh& M, const DevCoarse& C, const double* w,
                                  int with_y, hipStream_t s);
// lds_bytes: 8 bytes per closure node of the largest subdomain
hipError_t launch_coarse_ty(const DevCoarse& C, const double* v, int lds_bytes, hipStream_t s);
// sets the kernel's LDS limit (outside any stream capture)
hipError_t prepare_coarse_ty(int lds_bytes);
hipError_t launch_coarse_assemble(const DevCoarse& C, int with_matrix, hipStream_t s);
// the right-hand side part of launch_coarse_assemble, spread over the grid
hipError_t launch_coarse_gather(const DevCoarse& C, hipStream_t s);
// w -= V h (m columns) and out = ||w||^2 (deterministic, nb block partials)
hipError_t launch_maxpy_norm(const double* V, int64_t ld, int m, const double* h, double* w, int n,
                             double* partial, double* out, int nb, hipStream_t s);
hipError_t launch_coarse_lu(const DevCoarse& C, int factor, int lds_bytes, int nb_per_lane,
                            hipStream_t s);
hipError_t launch_coarse_update(const DevCoarse& C, hipStream_t s);
hipError_t launch_coarse_scatter(const DevCoarse& C, const double* src, double* cout, hipStream_t s);

int mrhs_bucket_kl(int kl, int ku);
int mrhs_lds_bytes(int kl_bucket);
hipError_t launch_tangent_prep(const DevMaps& P, const DevLocal& L, const DevTangent& Tg,
                               int kl_bucket, int max_ng, hipStream_t s);
// the same W_i by the blocked solve on the matrix cores (kl <= 48,
// kl + ku <= 112): nblk blocks in all, nkk = ceil(max (kl + ku) / 4)
hipError_t launch_tangent_blocked(const DevMaps& P, const DevLocal& L, const DevTangent& Tg,
                                  int nblk, int nkk, int max_ng, hipStream_t s);
// stream_w: nontemporal loads of W (for a W larger than the last-level cache)
hipError_t launch_tangent_gemv(const DevMaps& P, const DevTangent& Tg, const double* v, double* z,
                               int max_ng, bool stream_w, hipStream_t s);
// A0^{-1} per diagonal block from its band LU (any band up to 511 wide)
int coarse_inverse_lds_bytes(int max_block, int max_ldu);
hipError_t launch_coarse_inverse(const DevCoarse& C, int max_block, int max_ldu, hipStream_t s);
hipError_t launch_coarse_apply_inverse(const DevCoarse& C, const double* x, double* y, hipStream_t s);

// vector kernels for GMRES (deterministic reductions)
hipError_t launch_mdot(const double* V, int64_t ld, int m, const double* w, int n,
                       double* partial, double* out, int nblocks, hipStream_t s);
hipError_t launch_maxpy(const double* V, int64_t ld, int m, const double* h,
                        double* w, int n, double sign, hipStream_t s);
hipError_t launch_scale_by(const double* x, const double* denom_sq, double* y, int n,
                           hipStream_t s);
hipError_t launch_axpy(double a, const double* x, double* y, int n, hipStream_t s);
hipError_t launch_max_abs(const double* x, int n, double* partial, double* out,
                          int nblocks, hipStream_t s);
hipError_t launch_any_status(const int* status, int n, int* out, hipStream_t s);

// Device-resident state of one GMRES restart cycle (Hessenberg matrix H,
// (m+1) x m row-major, Givens rotations, residual vector g).  st[0]: 0 while
// |g_j| > tol, j when column j first met it, -j if it became non-finite;
// st[1]: columns processed.
struct GmresDev {
    double *H, *cs, *sn, *g;
    const double *h1, *h2, *tol;
    double* hn2;
    int* st;
    int m;
};
hipError_t prepare_coarse_lu(int lds_bytes, int npl);
// Both classical Gram-Schmidt passes of Arnoldi column j (h1 = V^T w,
// w -= V h1, h2 = V^T w, w -= V h2), ||w||^2 into G.hn2, rotation j and
// vnext = w / ||w||, in four launches: each kernel that consumes a
// reduction adds up its nb partial sums itself (same fixed order in every
// block), so no final-sum launches are needed, and the first update of w
// computes the second pass's partial sums for its own chunk.  pnorm: nb
// doubles, partial and partial2: nb x m each, all disjoint.
hipError_t launch_arnoldi_gs(const double* V, int64_t ld, int m, double* w, int n, double* partial,
                             double* pnorm, double* h1, double* h2, const GmresDev& G, int j,
                             double* vnext, int nb, hipStream_t s, double* partial2);
