// HIP kernels of libnls for gfx950 (CDNA4, 64-wide wavefronts).
//
// Hot path of two-level nonlinear restricted additive Schwarz (paper,
// Section 2): batched local nonlinear solves T_i (eq. 4) with P1 residual
// and Jacobian assembly, band LU with partial pivoting and band triangular
// solves, restricted prolongation (eqs. 5, 8), the GDSW coarse correction
// (eq. 9), and the exact tangent (eqs. 6, 7, 12) used by GMRES on eq. (13).
//
// Design notes
//  * One workgroup owns one subdomain for its whole inner Newton loop; the
//    patch values, residual and the LU working window stay in LDS, the
//    Jacobian values and the factors stream through HBM.
//  * Assembly is node-centric: every row sums its own incident elements in
//    a fixed order, so there are no atomics and results are bitwise
//    reproducible.
//  * The local Jacobian is banded under the lexicographic local ordering;
//    the LU keeps only the active (kl+1) x (kl+ku+1) window in an LDS ring
//    buffer and writes finished U rows / L columns to HBM (the extra ku
//    superdiagonals hold the fill of partial pivoting).
//  * Reductions are fixed-order trees (wavefront butterflies, then waves in
//    order), so norms and dot products do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cfloat>
#include <cmath>

#include "nls.h"
#include "nls_device.h"

#define NLS_BLOCK 256

namespace {

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Deterministic workgroup reductions; red must hold >= 24 doubles of LDS.
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < nw; ++i) s += red[i];
        red[16] = s;
    }
    __syncthreads();
    return red[16];
}

__device__ __forceinline__ double block_max(double v, double* red) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = red[0];
        for (int i = 1; i < nw; ++i) s = fmax(s, red[i]);
        red[17] = s;
    }
    __syncthreads();
    return red[17];
}

// Row `pos` of the element matrix G (stored G00 G11 G22 G01 G12 G20).
__device__ __forceinline__ void g_row(const double* __restrict__ G6, int pos, double& g0,
                                      double& g1, double& g2) {
    if (pos == 0) { g0 = G6[0]; g1 = G6[3]; g2 = G6[5]; }
    else if (pos == 1) { g0 = G6[3]; g1 = G6[1]; g2 = G6[4]; }
    else { g0 = G6[5]; g1 = G6[4]; g2 = G6[2]; }
}

// ----------------------------------------------------------------------------
// P1 element quantities (exact integration of the weak form of eq. 1):
//   U = u0+u1+u2, m = (U^2 + sum u_a^2)/12, s_a = sum_b G_ab u_b,
//   r_a = kappa (1 + beta m) s_a - l_a,
//   K_ac = kappa [ (1 + beta m) G_ac + beta s_a (U + u_c)/6 ].
// ----------------------------------------------------------------------------

// Residual of the rows of V_i held by this thread; vp = patch values in LDS.
// ----------------------------------------------------------------------------
// Q1 compressible Neo-Hooke (eq. 2): P = mu (F - F^-T) + lambda ln J F^-T,
// A_iJkL = mu d_ik d_JL + lambda Finv_Ji Finv_Lk - (lambda ln J - mu) Finv_Jk Finv_Li.
// Bilinear quadrilaterals, nodes counter-clockwise from the reference corner
// (-1,-1), 2 x 2 Gauss points with unit weights.
// ----------------------------------------------------------------------------
struct NHPoint {
    double wdet;        // quadrature weight x det(dX/dxi)
    double gr[4][2];    // material gradients of the shape functions
    double P[2][2];     // first Piola-Kirchhoff stress
    double Fi[2][2];    // F^{-1}
    double lnJ;
    bool ok;            // det F > 0
};

__device__ __forceinline__ void nh_point(const double X[4][2], const double ue[4][2], int q,
                                         double mu, double lam, NHPoint& o) {
    constexpr double g = 0.57735026918962576451;  // 1/sqrt(3)
    const double xa[4] = {-1.0, 1.0, 1.0, -1.0}, ya[4] = {-1.0, -1.0, 1.0, 1.0};
    const double xi = xa[q] * g, eta = ya[q] * g;
    double dN[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        dN[a][0] = 0.25 * xa[a] * (1.0 + ya[a] * eta);
        dN[a][1] = 0.25 * ya[a] * (1.0 + xa[a] * xi);
    }
    double J00 = 0, J01 = 0, J10 = 0, J11 = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        J00 += X[a][0] * dN[a][0];
        J01 += X[a][0] * dN[a][1];
        J10 += X[a][1] * dN[a][0];
        J11 += X[a][1] * dN[a][1];
    }
    const double det = J00 * J11 - J01 * J10;
    const double id = 1.0 / det;
    const double I00 = J11 * id, I01 = -J01 * id, I10 = -J10 * id, I11 = J00 * id;
    double F00 = 1.0, F01 = 0.0, F10 = 0.0, F11 = 1.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const double g0 = dN[a][0] * I00 + dN[a][1] * I10;
        const double g1 = dN[a][0] * I01 + dN[a][1] * I11;
        o.gr[a][0] = g0;
        o.gr[a][1] = g1;
        F00 += ue[a][0] * g0;
        F01 += ue[a][0] * g1;
        F10 += ue[a][1] * g0;
        F11 += ue[a][1] * g1;
    }
    const double JF = F00 * F11 - F01 * F10;
    o.ok = JF > 0.0;
    const double iJ = 1.0 / JF;
    o.Fi[0][0] = F11 * iJ;
    o.Fi[0][1] = -F01 * iJ;
    o.Fi[1][0] = -F10 * iJ;
    o.Fi[1][1] = F00 * iJ;
    o.lnJ = log(JF);
    // P_iJ = mu (F_iJ - Finv_Ji) + lambda ln J Finv_Ji
    const double a1 = lam * o.lnJ - mu;
    o.P[0][0] = mu * F00 + a1 * o.Fi[0][0];
    o.P[0][1] = mu * F01 + a1 * o.Fi[1][0];
    o.P[1][0] = mu * F10 + a1 * o.Fi[0][1];
    o.P[1][1] = mu * F11 + a1 * o.Fi[1][1];
    o.wdet = det;
}

// Element geometry and displacements: global element ge, local dof values
// from vp through the patch-local node ids, or the global vector u.
__device__ __forceinline__ void nh_coords(const DevMesh& M, int ge, double X[4][2]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int g = M.conn[4 * ge + v];
        X[v][0] = M.xy[2 * g];
        X[v][1] = M.xy[2 * g + 1];
    }
}

// Entries selected by a runtime index through unrolled compares (keeps the
// small arrays in registers).
__device__ __forceinline__ void nh_pick(const NHPoint& p, int pos, int c, double& g0, double& g1,
                                        double& P0, double& P1) {
    g0 = g1 = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
        if (a == pos) {
            g0 = p.gr[a][0];
            g1 = p.gr[a][1];
        }
    P0 = c == 0 ? p.P[0][0] : p.P[1][0];
    P1 = c == 0 ? p.P[0][1] : p.P[1][1];
}

// Internal force of dof (pos, c) of one element.
__device__ __forceinline__ double nh_force(const DevMesh& M, const double X[4][2],
                                           const double ue[4][2], int pos, int c, bool& ok) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        NHPoint p;
        nh_point(X, ue, q, M.mu, M.lam, p);
        ok = ok && p.ok;
        double g0, g1, P0, P1;
        nh_pick(p, pos, c, g0, g1, P0, P1);
        acc += p.wdet * (P0 * g0 + P1 * g1);
    }
    return acc;
}

// Stiffness row (pos, c) of one element: K[(pos,c),(b,k)] into kr[b][k].
__device__ __forceinline__ void nh_stiff_row(const DevMesh& M, const double X[4][2],
                                             const double ue[4][2], int pos, int c,
                                             double kr[4][2]) {
#pragma unroll
    for (int b = 0; b < 4; ++b) kr[b][0] = kr[b][1] = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        NHPoint p;
        nh_point(X, ue, q, M.mu, M.lam, p);
        // alpha_k = sum_J gr_pos,J Finv_Jk ; beta_k(b) = sum_L Finv_Lk gr_b,L
        double gp0, gp1, P0, P1;
        nh_pick(p, pos, c, gp0, gp1, P0, P1);
        const double al0 = gp0 * p.Fi[0][0] + gp1 * p.Fi[1][0];
        const double al1 = gp0 * p.Fi[0][1] + gp1 * p.Fi[1][1];
        const double alc = c == 0 ? al0 : al1;
        const double t = M.lam * p.lnJ - M.mu;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const double be0 = p.Fi[0][0] * p.gr[b][0] + p.Fi[1][0] * p.gr[b][1];
            const double be1 = p.Fi[0][1] * p.gr[b][0] + p.Fi[1][1] * p.gr[b][1];
            const double bec = c == 0 ? be0 : be1;
            const double gg = gp0 * p.gr[b][0] + gp1 * p.gr[b][1];
            // k = 0, 1: mu d_ck gg + lambda alpha_c beta_k - t alpha_k beta_c
            kr[b][0] += p.wdet * ((c == 0 ? M.mu * gg : 0.0) + M.lam * alc * be0 - t * al0 * bec);
            kr[b][1] += p.wdet * ((c == 1 ? M.mu * gg : 0.0) + M.lam * alc * be1 - t * al1 * bec);
        }
    }
}

__device__ __forceinline__ void nh_local_values(const DevMaps& P, int e, const double* vp,
                                                int nd[4], double ue[4][2]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        nd[v] = P.pe_conn[4 * e + v];
        ue[v][0] = vp[2 * nd[v]];
        ue[v][1] = vp[2 * nd[v] + 1];
    }
}

// detf (LDS word, or null): set to 1 when an elasticity row meets det F <= 0.
template <bool ELAST>
__device__ __forceinline__ void local_residual(const DevMesh& M, const DevMaps& P, int n, int rowbase,
                               int ebase, const double* vp, double* rb, int* detf = nullptr) {
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        const int row = rowbase + a;
        const int g = P.l2g[row];
        if (M.dflag[g]) {
            rb[a] = vp[a] - M.dval[g];
            continue;
        }
        if (ELAST) {
            // row a = dof (a & 1) of a V node; a non-admissible deformation
            // (det F <= 0) makes the residual NaN
            const int c = a & 1;
            double acc = 0.0;
            bool ok = true;
            for (int k = P.rinc_ptr[row]; k < P.rinc_ptr[row + 1]; ++k) {
                const int code = P.rinc[k];
                const int e = ebase + (code >> 2), pos = code & 3;
                double X[4][2], ue[4][2];
                int nd[4];
                nh_coords(M, P.pe_gid[e], X);
                nh_local_values(P, e, vp, nd, ue);
                acc += nh_force(M, X, ue, pos, c, ok);
            }
            rb[a] = ok ? acc - M.bload[g] : __builtin_nan("");
            if (!ok && detf) *detf = 1;
            continue;
        }
        double acc = 0.0;
        for (int k = P.rinc_ptr[row]; k < P.rinc_ptr[row + 1]; ++k) {
            const int code = P.rinc[k];
            const int e = ebase + (code >> 2), pos = code & 3;
            const double u0 = vp[P.pe_conn[3 * e]], u1 = vp[P.pe_conn[3 * e + 1]],
                         u2 = vp[P.pe_conn[3 * e + 2]];
            const int ge = P.pe_gid[e];
            const double U = u0 + u1 + u2;
            const double m = (U * U + u0 * u0 + u1 * u1 + u2 * u2) * (1.0 / 12.0);
            double g0, g1, g2;
            g_row(M.G6 + 6 * (size_t)ge, pos, g0, g1, g2);
            const double s = g0 * u0 + g1 * u1 + g2 * u2;
            acc += M.kappa[ge] * (1.0 + M.beta * m) * s;
        }
        rb[a] = acc - M.bload[g];
    }
}

// ----------------------------------------------------------------------------
// Residual and Jacobian rows of one local problem in one pass (the
// standalone assembly of eqs. (3)-(4) at the patch values vp): rows
// [a0, a1) of subdomain i, one row per thread, the row's CSR slots
// accumulated in registers and written once.  r[a] = R_i F(v)[a] (r may be
// null: no residual); jval (may be null) the values of [J_ii | B_i] in the
// fixed CSR slots.  Rows with more slots than MS (unstructured meshes of
// high valence) add into jval in place.
// ----------------------------------------------------------------------------
template <bool ELAST>
__device__ __forceinline__ void assemble_rows(const DevMesh& M, const DevMaps& P, int n, int rowbase,
                                              int ebase, const double* vp, int a0, int a1,
                                              double* __restrict__ r, double* __restrict__ jval) {
    constexpr int MS = ELAST ? 18 : 10;
    for (int a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
        const int row = rowbase + a;
        const int g = P.l2g[row];
        const int js = P.jptr[row], je = P.jptr[row + 1];
        const bool inreg = jval && je - js <= MS;
        int cl[MS];
        double acc[MS];
        // slot columns: loads from in-row addresses (a row has at least its
        // diagonal slot), selected afterwards, so that they are all in flight
#pragma unroll
        for (int t = 0; t < MS; ++t) {
            const bool in = inreg && js + t < je;
            const int c = P.jcol[in ? js + t : js];
            cl[t] = in ? c : -1;
            acc[t] = 0.0;
        }
        if (jval && !inreg)
            for (int s = js; s < je; ++s) jval[s] = 0.0;
        auto add = [&](int col, double K) {
            if (!jval) return;
            if (inreg) {
#pragma unroll
                for (int t = 0; t < MS; ++t) acc[t] += (cl[t] == col) ? K : 0.0;
            } else {
                for (int t = js; t < je; ++t)
                    if (P.jcol[t] == col) { jval[t] += K; break; }
            }
        };
        double res;
        if (M.dflag[g]) {
            res = vp[a] - M.dval[g];
            if (jval) add(a, 1.0);
        } else if (ELAST) {
            const int c = a & 1;
            double f = 0.0;
            bool ok = true;
            for (int k = P.rinc_ptr[row]; k < P.rinc_ptr[row + 1]; ++k) {
                const int code = P.rinc[k];
                const int e = ebase + (code >> 2), pos = code & 3;
                double X[4][2], ue[4][2];
                int nd[4];
                nh_coords(M, P.pe_gid[e], X);
                nh_local_values(P, e, vp, nd, ue);
                if (r) f += nh_force(M, X, ue, pos, c, ok);
                if (jval) {
                    double kr[4][2];
                    nh_stiff_row(M, X, ue, pos, c, kr);
#pragma unroll
                    for (int b = 0; b < 4; ++b)
#pragma unroll
                        for (int kk = 0; kk < 2; ++kk) add(2 * nd[b] + kk, kr[b][kk]);
                }
            }
            res = ok ? f - M.bload[g] : __builtin_nan("");
        } else {
            double f = 0.0;
            for (int k = P.rinc_ptr[row]; k < P.rinc_ptr[row + 1]; ++k) {
                const int code = P.rinc[k];
                const int e = ebase + (code >> 2), pos = code & 3;
                const int nd[3] = {P.pe_conn[3 * e], P.pe_conn[3 * e + 1], P.pe_conn[3 * e + 2]};
                const double uu[3] = {vp[nd[0]], vp[nd[1]], vp[nd[2]]};
                const int ge = P.pe_gid[e];
                const double U = uu[0] + uu[1] + uu[2];
                const double m = (U * U + uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]) * (1.0 / 12.0);
                double gr[3];
                g_row(M.G6 + 6 * (size_t)ge, pos, gr[0], gr[1], gr[2]);
                const double sg = gr[0] * uu[0] + gr[1] * uu[1] + gr[2] * uu[2];
                const double kap = M.kappa[ge];
                const double coef = kap * (1.0 + M.beta * m);
                f += coef * sg;
                if (jval) {
                    const double rk = M.beta * kap * sg * (1.0 / 6.0);
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) add(nd[cc], coef * gr[cc] + rk * (U + uu[cc]));
                }
            }
            res = f - M.bload[g];
        }
        if (r) r[a] = res;
        if (jval && inreg) {
#pragma unroll
            for (int t = 0; t < MS; ++t)
                if (js + t < je) jval[js + t] = acc[t];
        }
    }
}

// Jacobian rows [J_ii | B_i] of the whole local problem into the CSR values
// jval (slots fixed at setup), accumulated in registers row by row.
template <bool ELAST>
__device__ __forceinline__ void local_jacobian(const DevMesh& M, const DevMaps& P, int n, int rowbase,
                                               int ebase, const double* vp, double* __restrict__ jval) {
    assemble_rows<ELAST>(M, P, n, rowbase, ebase, vp, 0, n, nullptr, jval);
}

// ----------------------------------------------------------------------------
// Band LU with partial pivoting of an n x n matrix with kl sub- and ku
// superdiagonals, rows given in CSR (columns >= n are ignored).  The whole
// workgroup cooperates.  Results:
//   Uf[c*ldu + (c-r)] = U[r][c], r in [c-kl-ku, c], ldu = kl+ku+1
//   Lf[k*ldl + j]     = multiplier of row k+1+j at step k, ldl = max(kl,1)
//   piv[k]            = row swapped with row k at step k
// The interchanges are applied to the trailing columns only (interleaved
// form), so the forward solve applies swap k and then column k of L.
// Returns nonzero if a zero pivot occurred.
// ----------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ int band_lu(int n, int kl, int ku, const int* __restrict__ rptr,
                       const int* __restrict__ cols, const double* __restrict__ vals,
                       T* W, T* mult, int* sflag, T* __restrict__ Uf, T* __restrict__ Lf,
                       int* __restrict__ piv, int cbase = 0, double* rhs = nullptr) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
    // ring buffer of R rows x C columns; row r sits in slot r mod R, column c
    // in slot c mod C.  Slots of step k are tracked incrementally (kr, kc).
    const int R = kl + 1, C = kl + ku + 1;
    const int ldu = C, ldl = kl > 1 ? kl : 1;
    for (int i = tid; i < R * C; i += nt) W[i] = T(0);
    if (tid == 0) sflag[1] = 0;
    __syncthreads();
    for (int r = tid; r <= min(kl, n - 1); r += nt)
        for (int s = rptr[r]; s < rptr[r + 1]; ++s) {
            const int c = cols[s] - cbase;
            if (c < n) W[r * C + c] = T(vals[s]);
        }
    __syncthreads();
    int kr = 0, kc = 0;
    for (int k = 0; k < n; ++k) {
        const int rmax = min(k + kl, n - 1);
        if (wv == 0) {
            int d = lane;
            double a = -1.0;
            if (k + d <= rmax) {
                const int sr = kr + d < R ? kr + d : kr + d - R;
                a = fabs((double)W[sr * C + kc]);
            }
            if (lane + 64 <= rmax - k) {  // kl >= 64: second candidate per lane
                const int d2 = lane + 64;
                const int sr = kr + d2 < R ? kr + d2 : kr + d2 - R;
                const double a2 = fabs((double)W[sr * C + kc]);
                if (a2 > a) { a = a2; d = d2; }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double ao = __shfl_xor(a, o, 64);
                const int dO = __shfl_xor(d, o, 64);
                if (ao > a || (ao == a && dO < d)) { a = ao; d = dO; }
            }
            if (lane == 0) {
                sflag[0] = d;
                piv[k] = k + d;
                if (a == 0.0) sflag[1] = 1;
            }
        }
        __syncthreads();
        const int pd = sflag[0];
        T* rowk = W + kr * C;
        if (pd != 0) {
            const int sp = kr + pd < R ? kr + pd : kr + pd - R;
            T* rowp = W + sp * C;
            for (int c = tid; c < C; c += nt) {
                const T t = rowk[c];
                rowk[c] = rowp[c];
                rowp[c] = t;
            }
            if (rhs && tid == 0) {
                const double t = rhs[k];
                rhs[k] = rhs[k + pd];
                rhs[k + pd] = t;
            }
            __syncthreads();
        }
        const T pv = rowk[kc];
        const int nr = rmax - k;
        const int nc = min(k + kl + ku, n - 1) - k;
        for (int j = tid; j < nr; j += nt) {
            const int sr = kr + 1 + j < R ? kr + 1 + j : kr + 1 + j - R;
            const T l = (pv != T(0)) ? W[sr * C + kc] / pv : T(0);
            mult[j] = l;
            Lf[(size_t)k * ldl + j] = l;
            if (rhs) rhs[k + 1 + j] -= (double)l * rhs[k];
        }
        for (int c = tid; c <= nc; c += nt) {
            const int sc = kc + c < C ? kc + c : kc + c - C;
            Uf[(size_t)(k + c) * ldu + c] = rowk[sc];
        }
        __syncthreads();
        for (int j = wv; j < nr; j += nw) {
            const int sr = kr + 1 + j < R ? kr + 1 + j : kr + 1 + j - R;
            T* rowr = W + sr * C;
            const T l = mult[j];
            for (int c = lane; c < nc; c += 64) {
                const int sc = kc + 1 + c < C ? kc + 1 + c : kc + 1 + c - C;
                rowr[sc] -= l * rowk[sc];
            }
        }
        __syncthreads();
        // column k and row k leave the window; row k+R takes row k's slot and
        // column k+C takes column k's slot
        for (int r = tid; r < R; r += nt) W[r * C + kc] = T(0);
        for (int c = tid; c < C; c += nt) rowk[c] = T(0);
        __syncthreads();
        const int rn = k + R;
        if (rn < n) {
            for (int s = rptr[rn] + tid; s < rptr[rn + 1]; s += nt) {
                const int c = cols[s] - cbase;
                if (c < n) {
                    const int d = c - k;  // in [1, C]
                    const int sc = kc + d < C ? kc + d : kc + d - C;
                    rowk[sc] = T(vals[s]);
                }
            }
        }
        __syncthreads();
        kr = kr + 1 < R ? kr + 1 : 0;
        kc = kc + 1 < C ? kc + 1 : 0;
    }
    return sflag[1];
}

// Broadcast lane l's value (l uniform) through v_readlane.
__device__ __forceinline__ double rdlane(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float rdlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ unsigned dpp_umax(unsigned v) {
    return max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, ROWMASK, 0xf, false));
}

// Index (0..63) of an entry of largest |a| over the wavefront (a < 0 marks
// lanes that do not take part), compared on the high word of |a| with its 6
// low bits replaced by 63 - idx: entries within a relative 2^-14 of each
// other count as equal and the lowest index wins among them, so every
// multiplier stays below 1 + 2^-14 in magnitude.
__device__ __forceinline__ int wave_argmax_hi(double a, int idx) {
    unsigned key = 0u;
    if (a >= 0.0) key = ((unsigned)__double2hiint(a) & ~63u) | (unsigned)(63 - idx);
    key = dpp_umax<0xB1, 0xf>(key);   // quad_perm [1,0,3,2]
    key = dpp_umax<0x4E, 0xf>(key);   // quad_perm [2,3,0,1]
    key = dpp_umax<0x141, 0xf>(key);  // row_half_mirror
    key = dpp_umax<0x140, 0xf>(key);  // row_mirror
    key = dpp_umax<0x142, 0xa>(key);  // row_bcast:15 into rows 1, 3
    key = dpp_umax<0x143, 0xc>(key);  // row_bcast:31 into rows 2, 3
    key = (unsigned)__builtin_amdgcn_readlane((int)key, 63);
    return 63 - (int)(key & 63u);
}

// One 16x16x4 matrix-core step D = A B + C: A is 16 x 4 with lane l holding
// A[l % 16][l / 16], B is 4 x 16 with lane l holding B[l / 16][l % 16], and
// C, D are 16 x 16 with lane l holding four entries of column l % 16: rows
// row(l / 16, q), q = 0..3 (FP64: l / 16 + 4 q; FP32: 4 (l / 16) + q).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int q) { return g + 4 * q; }
};
template <> struct Mfma<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int q) { return 4 * g + q; }
};

// bfloat16 operands of the trial trailing update: round to nearest even.
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ short bf16_rne(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// 1/x from the hardware reciprocal and two Newton steps (a few ulp).
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float recip(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// ----------------------------------------------------------------------------
// Blocked band LU with partial pivoting (same results layout as band_lu).
// Panels of NB columns: one wavefront factors the panel in registers (lane r
// holds window row r, NB <= 64 - kl), then the workgroup applies the panel's
// row interchanges and L11^{-1} to the trailing columns (one thread per
// column) and the rank-NB update A22 -= L21 U12 with 4x4 register tiles.
// The window is an LDS ring buffer of H = NB + kl rows by Wd = NB + kl + ku
// columns; it slides by NB rows and columns per panel.
// ----------------------------------------------------------------------------
__device__ __forceinline__ int wrap(int x, int m) { return x < m ? x : x - m; }

// Workgroup barrier that orders LDS only: waits for this wave's LDS traffic
// (lgkmcnt = 0) but leaves global stores in flight.  Used inside the
// factorization, whose HBM outputs are read back only after a full
// __syncthreads().
__device__ __forceinline__ void lds_barrier() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// BF16 (T = float only): the trailing update A22 -= L21 U12 takes bfloat16
// operands on the 16x16x16 matrix-core product with FP32 accumulation.  It
// is a separate instantiation, not a run-time branch inside the update: with
// both product shapes behind one branch, the wait before the accumulators
// were read back after the FP32 product came out shorter than that product
// needs, and the binary32 factors were wrong from run to run.
template <typename T, int NB, bool BF16 = false>
__device__ __forceinline__ int band_lu_blocked(int n, int kl, int ku, const int* __restrict__ rptr,
                               const int* __restrict__ cols, const double* __restrict__ vals,
                               T* W, int* sh, T* __restrict__ Uf, T* __restrict__ Lf,
                               int* __restrict__ piv, int cbase = 0, double* rhs = nullptr) {
    static_assert(!BF16 || sizeof(T) == 4, "bfloat16 updates need binary32 factors");
    T* lt = W + (NB + kl) * (NB + kl + ku);  // L11 of the current panel by columns, NB x NB
    int* mv = (int*)(lt + NB * NB);           // moved rows of the panel (<= 64)
    // multipliers of the panel's steps, staged by wavefront 0 at the row's
    // position after the step (NB + position - step - 1), copied out by the
    // whole workgroup with the U rows
    constexpr int LSW = 64 + NB;
    T* ls = (T*)(mv + 64);
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int H = NB + kl, Wd = NB + kl + ku;
    const int ldu = kl + ku + 1, ldl = kl > 1 ? kl : 1;
    for (int i = tid; i < H * Wd; i += nt) W[i] = T(0);
    if (tid == 0) sh[NB] = 0;
    __syncthreads();
    for (int r = tid; r < min(H, n); r += nt)
        for (int s = rptr[r]; s < rptr[r + 1]; ++s) {
            const int c = cols[s] - cbase;
            if (c < n) W[r * Wd + c] = T(vals[s]);
        }
    __syncthreads();
    int rpn[NB + 1];     // row pointers of the rows entering after the next panel
#pragma unroll
    for (int q = 0; q <= NB; ++q) rpn[q] = wv > 0 ? rptr[min(H + q, min(H + NB, n))] : 0;
    int rb = 0, cb = 0;  // ring slots of global row / column k0
    for (int k0 = 0; k0 < n; k0 += NB) {
        const int nbp = min(NB, n - k0);
        const int rvalid = min(H, n - k0);
        const int k1 = k0 + NB, cb1 = wrap(cb + NB, Wd);
        // waves 1.. fetch the CSR entries of the rows that enter the window
        // after this panel while wave 0 factors it; the row pointers were
        // fetched one panel ahead, and the entries are only placed at the end
        // of the panel, so neither load is waited for before then
        constexpr int PF = 2;
        const int rn0 = k0 + H, rn1 = min(k0 + H + NB, n);
        int rp[NB + 1];
#pragma unroll
        for (int q = 0; q <= NB; ++q) rp[q] = rpn[q];
        if (wv > 0) {
            const int m1 = min(rn0 + 2 * NB, n);
#pragma unroll
            for (int q = 0; q <= NB; ++q) rpn[q] = rptr[min(rn0 + NB + q, m1)];
        }
        int pf_s[PF], pf_c[PF];
        double pf_v[PF];
#pragma unroll
        for (int e = 0; e < PF; ++e) {
            pf_s[e] = -1;
            pf_c[e] = 0;
            pf_v[e] = 0.0;
        }
        const int s_end = rp[NB], s_done = rp[0] + (nt - 64) * PF;
        if (rn0 < n && wv > 0) {
#pragma unroll
            for (int e = 0; e < PF; ++e) {
                const int sidx = rp[0] + (tid - 64) + (nt - 64) * e;
                if (sidx < s_end) {
                    pf_s[e] = sidx;
                    pf_c[e] = cols[sidx];
                    pf_v[e] = vals[sidx];
                }
            }
        }
        // ---- panel: columns k0..k0+nbp-1, rows k0..k0+rvalid-1 (wave 0).
        // Lane r keeps window row r in registers for the whole panel; the
        // interchanges are tracked as positions (pos = where row r sits in
        // the interchanged order) instead of moving data between lanes, and
        // the rows are written back to their final positions at the end.
        if (wv == 0) {
            T p[NB];
            const bool have = lane < rvalid;
            const int sr = wrap(rb + (lane < H ? lane : 0), H);
            // loads from in-window addresses, then selects: no branch and
            // no wait between the loads
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const T w = W[sr * Wd + wrap(cb + c, Wd)];
                p[c] = have ? w : T(0);
            }
            int pos = lane, sing = 0;
            bool used = false;
            // right-hand side (forward substitution fused with the
            // factorisation): each row carries its entry through the steps
            double pb = 0.0;
            if (rhs) {
                const double w = rhs[have ? k0 + lane : k0];
                pb = have ? w : 0.0;
            }
            // The steps hold no stores (the multipliers and interchanges are
            // stored after the loop) and no branch but the one around the
            // pivot search.
            int dsel = lane;        // lane j: the pivot position of step j
            int posj[NB];           // position of this row after step j
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                // a step past the last column (j >= nbp, last panel only)
                // has no candidates, so it changes nothing
                const bool act = j < nbp;
                // candidates: the rows at positions j..min(j+kl, rvalid-1),
                // i.e. the rows r <= j+kl not yet chosen as pivots.  The row
                // at position j keeps the pivot when no candidate is larger
                // in magnitude (no reduction needed); otherwise a wavefront
                // argmax, where a NaN or infinite entry is a candidate of the
                // largest key, so the chosen position belongs to a candidate.
                const bool cand = act && have && !used && lane <= j + kl;
                const double av = fabs((double)p[j]);
                const int lj = __ffsll((unsigned long long)__ballot(act && have && pos == j)) - 1;
                const double aj = fabs((double)rdlane(p[j], lj < 0 ? 0 : lj));
                int d = j, pl = lj;
                if (__ballot(cand && av > aj) != 0) {
                    d = __builtin_amdgcn_readfirstlane(
                        wave_argmax_hi(cand ? (av <= DBL_MAX ? av : DBL_MAX) : -1.0, pos));
                    pl = __ffsll((unsigned long long)__ballot(cand && pos == d)) - 1;
                }
                const int plr = pl < 0 ? 0 : pl;  // lane read when nothing is active
                dsel = (lane == j) ? d : dsel;
                pos = (pos == j) ? d : (lane == pl ? j : pos);
                posj[j] = pos;
                used = used || lane == pl;
                const T pivv = rdlane(p[j], plr);
                sing |= (act && pivv == T(0)) ? 1 : 0;
                const T inv = pivv != T(0) ? recip(pivv) : T(0);
                const bool below = cand && lane != pl;
                // l = 0 leaves the rows that are not below the pivot as they are
                const T l = below ? p[j] * inv : T(0);
                p[j] = below ? l : p[j];
#pragma unroll
                for (int c = j + 1; c < NB; ++c) p[c] -= l * rdlane(p[c], plr);
                if (rhs) pb -= (double)l * rdlane(pb, plr);
            }
            if (lane < nbp) piv[k0 + lane] = k0 + dsel;
            // every lane writes its slot (positions are distinct); the rows
            // not below a step's pivot fall outside the copied range
#pragma unroll
            for (int j = 0; j < NB; ++j) ls[j * LSW + NB + posj[j] - j - 1] = p[j];
            if (rhs && have) rhs[k0 + pos] = pb;
            if (have) {
                const int sp = wrap(rb + pos, H);
#pragma unroll
                for (int c = 0; c < NB; ++c) W[sp * Wd + wrap(cb + c, Wd)] = p[c];
                if (pos < NB) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) lt[c * NB + pos] = p[c];
                }
            }
            // rows that changed position: (new position << 8) | old position
            const bool moved = have && pos != lane;
            const unsigned long long mm = (unsigned long long)__ballot(moved);
            if (moved) {
                const int idx = __builtin_amdgcn_mbcnt_hi((unsigned)(mm >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((unsigned)mm, 0u));
                mv[idx] = (pos << 8) | lane;
            }
            if (lane == 0) {
                sh[NB + 1] = __popcll(mm);
                if (sing) sh[NB] = 1;
            }
        }
        lds_barrier();
        // ---- trailing columns: the panel's row permutation, then
        //      U12 = L11^{-1} A12 (one thread per column)
        const int ntr = min(Wd - NB, n - k0 - nbp);
        const int nmv = sh[NB + 1];
        if (nmv > 0) {
            // moved rows of the trailing columns, whole columns per round:
            // every source of a column is read before any destination of
            // that column is written
            constexpr int E = 8;
            const int cpr = (E * nt) / nmv;  // columns per round (nmv <= 2 NB)
            for (int c0 = 0; c0 < ntr; c0 += cpr) {
                const int tot = min(cpr, ntr - c0) * nmv;
                T v[E];
                int dst[E];
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int idx = tid + e * nt;
                    dst[e] = -1;
                    v[e] = T(0);
                    if (idx < tot) {
                        const int c = c0 + idx / nmv, q = idx - (idx / nmv) * nmv;
                        const int sc = wrap(cb + NB + c, Wd), m = mv[q];
                        v[e] = W[wrap(rb + (m & 255), H) * Wd + sc];
                        dst[e] = wrap(rb + (m >> 8), H) * Wd + sc;
                    }
                }
                lds_barrier();
#pragma unroll
                for (int e = 0; e < E; ++e)
                    if (dst[e] >= 0) W[dst[e]] = v[e];
                lds_barrier();
            }
        }
        for (int t = tid; t < ntr; t += nt) {
            const int sc = wrap(cb + NB + t, Wd);
            T x[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const T w = W[wrap(rb + j, H) * Wd + sc];
                x[j] = (j < nbp) ? w : T(0);
            }
            // column j of L11 is contiguous: its loads do not depend on x
            // and are issued ahead of the updates that use them
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const T xj = x[j];
#pragma unroll
                for (int r = j + 1; r < NB; ++r) x[r] -= lt[j * NB + r] * xj;
            }
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (j < nbp) W[wrap(rb + j, H) * Wd + sc] = x[j];
        }
        lds_barrier();
        // ---- A22 -= L21 U12 (rows NB..rvalid-1) on the matrix cores, one
        //      16 x 16 tile per wavefront at a time, k in steps of 4; U rows out
        {
            const int nr2 = rvalid - NB;
            if (nr2 > 0 && ntr > 0) {
                const int tr = (nr2 + 15) >> 4, tc = (ntr + 15) >> 4;
                const int li = lane & 15, lk = lane >> 4;
                // tile t = rt tc + ct, t = wv, wv + 4, ..: (rt, ct) advanced
                // without divisions.  Loads are unconditional, from clamped
                // in-window addresses: rows >= rvalid and columns >= ntr give
                // outputs that are not stored (selecting after the load lets
                // the compiler move each load under a branch of its own), and
                // with trailing columns the panel is full (nbp = NB)
                const int nw = nt >> 6;
                int rt = wv / tc, ct = wv - (wv / tc) * tc;
                for (int t = wv; t < tr * tc; t += nw) {
                    const int r0 = NB + 16 * rt, c0 = NB + 16 * ct;
                    ct += nw;
                    while (ct >= tc) {
                        ct -= tc;
                        ++rt;
                    }
                    // C: lane holds rows r0 + row(lk, q), column c0 + li
                    const int cc = c0 + li;
                    const bool cok = cc < NB + ntr;
                    const int scc = wrap(cb + (cok ? cc : 0), Wd);
                    typename Mfma<T>::acc_t acc;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int rr = r0 + Mfma<T>::row(lk, q);
                        acc[q] = W[wrap(rb + (rr < rvalid ? rr : 0), H) * Wd + scc];
                    }
                    // A = -L21 (rows r0 + li, k = 4 s + lk), B = U12 (rows k, column cc)
                    const int ra = r0 + li;
                    const int sra = wrap(rb + (ra < rvalid ? ra : 0), H);
                    if constexpr (BF16) {
                        // one 16x16x16 product: lane holds k = 4 lk .. 4 lk + 3
                        // (k >= NB, i.e. k >= 8 of an 8-column panel, are zero)
                        bf16x4_t a4, b4;
#pragma unroll
                        for (int t4 = 0; t4 < 4; ++t4) {
                            const int k = 4 * lk + t4;
                            const bool kin = k < NB;
                            const int kk = kin ? k : 0;
                            const float wa = W[sra * Wd + wrap(cb + kk, Wd)];
                            const float wb = W[wrap(rb + kk, H) * Wd + scc];
                            a4[t4] = bf16_rne(kin ? -wa : 0.f);
                            b4[t4] = bf16_rne(kin ? wb : 0.f);
                        }
                        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a4, b4, acc, 0, 0, 0);
                    } else {
                        T av[NB / 4], bv[NB / 4];
#pragma unroll
                        for (int s4 = 0; s4 < NB / 4; ++s4) {
                            const int k = 4 * s4 + lk;
                            av[s4] = -W[sra * Wd + wrap(cb + k, Wd)];
                            bv[s4] = W[wrap(rb + k, H) * Wd + scc];
                        }
#pragma unroll
                        for (int s4 = 0; s4 < NB / 4; ++s4) acc = Mfma<T>::step(av[s4], bv[s4], acc);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int rr = r0 + Mfma<T>::row(lk, q);
                        if (cok && rr < rvalid) W[wrap(rb + rr, H) * Wd + scc] = acc[q];
                    }
                }
            }
            // U rows of the panel out, column by column: the (up to NB) entries
            // of a factor column are contiguous, Uf[c * ldu + (c - r)]
            for (int idx = tid; idx < (nbp + ldu - 1) * NB; idx += nt) {
                const int c = idx / NB, r = idx - c * NB, o = c - r;
                if (r < nbp && o >= 0 && o < ldu && k0 + c < n)
                    Uf[(size_t)(k0 + c) * ldu + o] = W[wrap(rb + r, H) * Wd + wrap(cb + c, Wd)];
            }
            // multipliers of step j: Lf[(k0 + j) ldl + i], i < min(kl, n - 1 - k0 - j),
            // the steps spread over the wavefronts
            for (int j = wv; j < nbp; j += nt >> 6) {
                const int lim = min(kl, n - 1 - (k0 + j));
                for (int i = lane; i < lim; i += 64) Lf[(size_t)(k0 + j) * ldl + i] = ls[j * LSW + NB + i];
            }
        }
        lds_barrier();
        // ---- slide by NB: rows k0.. and columns k0.. leave the window
        {
            // (row q, column c) of thread tid + m nt, advanced without divisions
            const int dq = nt / Wd, dc = nt - dq * Wd;
            int q = tid / Wd, c = tid - q * Wd;
            while (q < NB) {
                W[wrap(rb + q, H) * Wd + c] = T(0);
                c += dc;
                q += dq;
                if (c >= Wd) {
                    c -= Wd;
                    ++q;
                }
            }
        }
        for (int i = tid; i < H * NB; i += nt) {
            const int r = i / NB, q = i - r * NB;
            W[r * Wd + wrap(cb + q, Wd)] = T(0);
        }
        lds_barrier();
        if (rn0 < n && wv > 0) {
#pragma unroll
            for (int e = 0; e < PF; ++e) {
                const int c = pf_c[e] - cbase;
                if (pf_s[e] >= 0 && c < n) {
                    int q = 0;
#pragma unroll
                    for (int t = 1; t < NB; ++t) q += (rp[t] <= pf_s[e]) ? 1 : 0;
                    W[wrap(rb + q, H) * Wd + wrap(cb1 + (c - k1), Wd)] = T(pf_v[e]);
                }
            }
            // rows with more entries than the prefetch covers
            for (int sidx = s_done + (tid - 64); sidx < s_end; sidx += nt - 64) {
                int q = 0;
                while (q + 1 < NB && rptr[rn0 + q + 1] <= sidx) ++q;
                const int c = cols[sidx] - cbase;
                if (c < n) W[wrap(rb + q, H) * Wd + wrap(cb1 + (c - k1), Wd)] = T(vals[sidx]);
            }
        }
        lds_barrier();
        rb = wrap(rb + NB, H);
        cb = cb1;
    }
    __syncthreads();  // factors in HBM are complete for the workgroup
    return sh[NB];
}

// Choose the blocked factorization when its panel fits a wavefront.
// With rhs (length n, LDS), the row operations are applied to it as well,
// so that it leaves holding the forward-substituted L^{-1} P rhs.
template <typename T>
__device__ __forceinline__ int band_lu_auto(int n, int kl, int ku, const int* __restrict__ rptr,
                            const int* __restrict__ cols, const double* __restrict__ vals,
                            T* W, T* mult, int* sflag, T* __restrict__ Uf, T* __restrict__ Lf,
                            int* __restrict__ piv, int cbase = 0, int variant = 0,
                            double* rhs = nullptr, bool bf16 = false) {
    // variant: 0 widest panel the band allows, 1 NB=16, 2 NB=8, 3 unblocked
    // (bf16 trailing updates exist in the blocked forms only)
    if constexpr (sizeof(T) == 4) {
        if (bf16) {
            if ((variant == 0 || variant == 1) && kl + 16 <= 64)
                return band_lu_blocked<T, 16, true>(n, kl, ku, rptr, cols, vals, W, sflag, Uf, Lf,
                                                    piv, cbase, rhs);
            if ((variant == 0 || variant == 2) && kl + 8 <= 64)
                return band_lu_blocked<T, 8, true>(n, kl, ku, rptr, cols, vals, W, sflag, Uf, Lf,
                                                   piv, cbase, rhs);
        }
    }
    if ((variant == 0 || variant == 1) && kl + 16 <= 64)
        return band_lu_blocked<T, 16>(n, kl, ku, rptr, cols, vals, W, sflag, Uf, Lf, piv, cbase, rhs);
    if ((variant == 0 || variant == 2) && kl + 8 <= 64)
        return band_lu_blocked<T, 8>(n, kl, ku, rptr, cols, vals, W, sflag, Uf, Lf, piv, cbase, rhs);
    return band_lu<T>(n, kl, ku, rptr, cols, vals, W, mult, sflag, Uf, Lf, piv, cbase, rhs);
}

// ----------------------------------------------------------------------------
// Band triangular solves with the factors of band_lu, executed by ONE
// wavefront (threads 0..63), right-hand side b in LDS (FP64).  NPL values per
// lane cover bands up to 64*NPL.  The factor columns are read in chunks of S
// steps, and the next chunk's loads are issued before the current chunk's
// steps run, so their HBM latency overlaps those steps.
// ----------------------------------------------------------------------------
template <typename T, int NPL>
__device__ __forceinline__ void band_solve_wave(int n, int kl, int ku, const T* __restrict__ Uf,
                                const T* __restrict__ Lf, const int* __restrict__ piv,
                                double* b, bool backward_only = false) {
    constexpr int S = 8;
    const int lane = threadIdx.x & 63;
    const int ldu = kl + ku + 1, ldl = kl > 1 ? kl : 1;
    if (!backward_only && n > 0) {
        T ln[S][NPL];  // columns of L and pivots of the next chunk, as loaded
        int pn[S];
        auto fetch_l = [&](int k0) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int k = k0 + s;
                const int lim = (k < n) ? min(kl, n - 1 - k) : 0;
                pn[s] = (k < n) ? piv[k] : k;
#pragma unroll
                for (int q = 0; q < NPL; ++q) {
                    const int j = lane + 64 * q;
                    ln[s][q] = (j < lim) ? Lf[(size_t)k * ldl + j] : T(0);
                }
            }
        };
        fetch_l(0);
        for (int k0 = 0; k0 < n; k0 += S) {
            double lv[S][NPL];
            int pv[S];
#pragma unroll
            for (int s = 0; s < S; ++s) {
                pv[s] = pn[s];
#pragma unroll
                for (int q = 0; q < NPL; ++q) lv[s][q] = (double)ln[s][q];
            }
            if (k0 + S < n) fetch_l(k0 + S);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int k = k0 + s;
                if (k < n) {
                    if (pv[s] != k) {
                        if (lane == 0) {
                            const double t = b[k];
                            b[k] = b[pv[s]];
                            b[pv[s]] = t;
                        }
                        wave_sync();
                    }
                    const double bk = b[k];
                    const int lim = min(kl, n - 1 - k);
#pragma unroll
                    for (int q = 0; q < NPL; ++q) {
                        const int j = lane + 64 * q;
                        if (j < lim) b[k + 1 + j] -= lv[s][q] * bk;
                    }
                    wave_sync();
                }
            }
        }
    }
    if (n > 0) {
        T un[S][NPL];  // columns of U (above the diagonal) of the next chunk
        T dn[S];       // and their diagonal entries, as loaded
        auto fetch_u = [&](int k0) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int k = k0 - s;
                const int lim = (k >= 0) ? min(kl + ku, k) : 0;
                dn[s] = (k >= 0) ? Uf[(size_t)k * ldu] : T(1);
#pragma unroll
                for (int q = 0; q < NPL; ++q) {
                    const int j = lane + 64 * q;
                    un[s][q] = (j < lim) ? Uf[(size_t)k * ldu + 1 + j] : T(0);
                }
            }
        };
        fetch_u(n - 1);
        for (int k0 = n - 1; k0 >= 0; k0 -= S) {
            double uv[S][NPL];
            double rdg[S];  // reciprocals of the diagonal, off the step chain
#pragma unroll
            for (int s = 0; s < S; ++s) {
                rdg[s] = 1.0 / (double)dn[s];
#pragma unroll
                for (int q = 0; q < NPL; ++q) uv[s][q] = (double)un[s][q];
            }
            if (k0 - S >= 0) fetch_u(k0 - S);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int k = k0 - s;
                if (k >= 0) {
                    // every lane forms x_k itself; lane 0 stores it, and no
                    // lane writes b[k] in this step otherwise
                    const double bk = b[k] * rdg[s];
                    if (lane == 0) b[k] = bk;
                    const int lim = min(kl + ku, k);
#pragma unroll
                    for (int q = 0; q < NPL; ++q) {
                        const int j = lane + 64 * q;
                        if (j < lim) b[k - 1 - j] -= uv[s][q] * bk;
                    }
                    wave_sync();
                }
            }
        }
    }
}

// ----------------------------------------------------------------------------
// Band triangular solves with the factors of band_lu for one right-hand side
// b (LDS, FP64), carried out by the whole workgroup.  Wavefront 0 runs the
// substitution steps with the rows of b that a step can touch in registers:
// R = NPL + 1 slots of 64 rows (the kl + ku <= 64 NPL rows next to step k lie
// in blocks k / 64 -+ 0..R-1), slot 0 holding the block of row k.  A step
// broadcasts the finished entry with v_readlane, keeps it in slot 0 and
// updates every slot with one FMA; when the step leaves a block, the block
// goes to b and the slots move by one, the last one taking the next block
// from b.  The other wavefronts stage the next G steps' factor entries into
// one half of an LDS double buffer while wavefront 0 reads the other half,
// already in slot order (entry (q, l) of a column is the factor entry of the
// row that lane l of slot q holds, zero outside the band) with the pivots or
// the reciprocals of the diagonal beside them, so that a step reads one entry
// per slot and applies no masks.  The workgroup synchronises every G steps.
// Same arithmetic, in the same order, as the one-wavefront solve above.  All
// threads of the workgroup call it.
// ----------------------------------------------------------------------------
template <typename T, int NPL>
__host__ __device__ __forceinline__ int band_stage_col_bytes() {
    return (NPL + 1) * 64 * (int)sizeof(T) + 8;  // slot entries + pivot or 1/d
}
template <typename T, int NPL>
__device__ __forceinline__ int band_stage_cols(int stage_bytes) {
    const int g = stage_bytes / (2 * band_stage_col_bytes<T, NPL>());
    return g >= 64 ? 64 : (g & ~7);
}

// The rows of b next to a substitution step: R blocks of 64 rows, block q in
// slot q.  Named members, not an array: every access is by a compile-time
// slot, or by a chain of selects on a uniform one, so the slots stay in
// registers.
template <int R>
struct BandRing {
    static_assert(R >= 2 && R <= 5, "1 to 4 values per lane");
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
    // row (q, lane l), q and l uniform: every slot is read at lane l and
    // the scalars are selected, so that no slot is indexed at run time
    __device__ __forceinline__ double lane_value(int q, int l) const {
        double v = rdlane(s0, l);
        const double v1 = rdlane(s1, l);
        v = q == 1 ? v1 : v;
        if constexpr (R > 2) { const double v2 = rdlane(s2, l); v = q == 2 ? v2 : v; }
        if constexpr (R > 3) { const double v3 = rdlane(s3, l); v = q == 3 ? v3 : v; }
        if constexpr (R > 4) { const double v4 = rdlane(s4, l); v = q == 4 ? v4 : v; }
        return v;
    }
    // row (q, lane of mine) := v
    __device__ __forceinline__ void put(int q, bool mine, double v) {
        s0 = (q == 0 && mine) ? v : s0;
        s1 = (q == 1 && mine) ? v : s1;
        if constexpr (R > 2) s2 = (q == 2 && mine) ? v : s2;
        if constexpr (R > 3) s3 = (q == 3 && mine) ? v : s3;
        if constexpr (R > 4) s4 = (q == 4 && mine) ? v : s4;
    }
    // slot q -= c[q] x
    template <typename C>
    __device__ __forceinline__ void axpy(const C& c, double x) {
        s0 -= c[0] * x;
        s1 -= c[1] * x;
        if constexpr (R > 2) s2 -= c[2] * x;
        if constexpr (R > 3) s3 -= c[3] * x;
        if constexpr (R > 4) s4 -= c[4] * x;
    }
    // slots move down by one; the last one takes v
    __device__ __forceinline__ void shift(double v) {
        s0 = s1;
        if constexpr (R > 2) { s1 = s2; } else { s1 = v; }
        if constexpr (R > 3) { s2 = s3; } else if constexpr (R > 2) { s2 = v; }
        if constexpr (R > 4) { s3 = s4; s4 = v; } else if constexpr (R > 3) { s3 = v; }
    }
    __device__ __forceinline__ void set(int q, double v) {
        if (q == 0) s0 = v;
        if (q == 1) s1 = v;
        if constexpr (R > 2) { if (q == 2) s2 = v; }
        if constexpr (R > 3) { if (q == 3) s3 = v; }
        if constexpr (R > 4) { if (q == 4) s4 = v; }
    }
};

template <typename T, int NPL>
__device__ __forceinline__ void band_solve_staged(int n, int kl, int ku, const T* __restrict__ Uf,
                                                  const T* __restrict__ Lf,
                                                  const int* __restrict__ piv, double* b,
                                                  void* stage, int G, bool backward_only) {
    constexpr int R = NPL + 1, S = 4, CB = 8, PER = R * 64;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
    const int ldu = kl + ku + 1, ldl = kl > 1 ? kl : 1, bw = kl + ku;
    const int t0 = nt > 64 ? 64 : 0;  // first thread of the staging waves
    // buffer h: G columns of PER entries, then G pivots or reciprocals
    T* sE[2] = {(T*)stage, (T*)stage + G * PER};
    double* sD[2] = {(double*)((T*)stage + 2 * G * PER), (double*)((T*)stage + 2 * G * PER) + G};
    BandRing<R> ring;
    // rows of block B (zeros outside 0..n-1)
    auto block = [&](int B) {
        const int r = 64 * B + lane;
        const bool in = B >= 0 && r < n;
        const double v = b[in ? r : 0];
        return in ? v : 0.0;
    };
    auto flush = [&](int B) {  // slot 0 holds the finished rows of block B
        const int r = 64 * B + lane;
        if (B >= 0 && r < n) b[r] = ring.s0;
    };
    // entry e of buffer h for the columns [c0, c0 + cnt): column c0 + e / PER,
    // slot (e % PER) / 64, lane e % 64; the value is val(k, slot, lane) or 0
    auto stage_entries = [&](T* E, int c0, int cnt, int first, auto val) {
        if (tid < first) return;
        const int step = nt - first, tot = cnt * PER;
        for (int e0 = tid - first; e0 < tot; e0 += CB * step) {
            T v[CB];
            bool ok[CB];
#pragma unroll
            for (int u = 0; u < CB; ++u) {
                const int e = min(e0 + u * step, tot - 1);
                const int c = e / PER, rem = e - c * PER;
                v[u] = val(c0 + c, rem >> 6, rem & 63, ok[u]);
            }
#pragma unroll
            for (int u = 0; u < CB; ++u) {
                const int e = e0 + u * step;
                if (e < tot) E[e] = ok[u] ? v[u] : T(0);
            }
        }
    };
    if (n <= 0) return;
    if (!backward_only) {
        // forward: slot q holds block k / 64 + q; entry (q, l) of column k is
        // the multiplier of row 64 (k / 64 + q) + l at step k
        auto stage_l = [&](int h, int c0, int first) {
            const int cnt = min(c0 + G, n) - c0;
            stage_entries(sE[h], c0, cnt, first, [&](int k, int q, int l, bool& ok) {
                const int j = 64 * ((k >> 6) + q) + l - k - 1;
                ok = j >= 0 && j < min(kl, n - 1 - k);
                return Lf[(size_t)k * ldl + (ok ? j : 0)];
            });
            if (tid >= first)
                for (int c = tid - first; c < cnt; c += nt - first)
                    ((int*)sD[h])[c] = piv[c0 + c];
        };
        stage_l(0, 0, 0);
        __syncthreads();
        if (tid < 64) {
#pragma unroll
            for (int q = 0; q < R; ++q) ring.set(q, block(q));
        }
        for (int c0 = 0, h = 0; c0 < n; c0 += G, h ^= 1) {
            const int c1 = min(c0 + G, n);
            if (c1 < n) stage_l(h ^ 1, c1, t0);
            if (tid < 64) {
                const T* E = sE[h];
                const int* pvs = (const int*)sD[h];
                T ln[S][R];
                int pn[S];
                auto fetch = [&](int k) {
#pragma unroll
                    for (int t = 0; t < S; ++t) {
                        const int ck = min(k + t, c1 - 1) - c0;
                        pn[t] = pvs[ck];
#pragma unroll
                        for (int q = 0; q < R; ++q) ln[t][q] = E[ck * PER + q * 64 + lane];
                    }
                };
                fetch(c0);
                for (int k0 = c0; k0 < c1; k0 += S) {
                    double lv[S][R];
                    int pv[S];
#pragma unroll
                    for (int t = 0; t < S; ++t) {
                        pv[t] = pn[t];
#pragma unroll
                        for (int q = 0; q < R; ++q) lv[t][q] = (double)ln[t][q];
                    }
                    if (k0 + S < c1) fetch(k0 + S);
#pragma unroll
                    for (int t = 0; t < S; ++t) {
                        const int k = k0 + t;
                        if (k < c1) {
                            const int lk = k & 63;
                            // entering block k / 64: the finished block leaves
                            if (lk == 0 && k > 0) {
                                flush((k >> 6) - 1);
                                ring.shift(block((k >> 6) + R - 1));
                            }
                            const int p = __builtin_amdgcn_readfirstlane(pv[t]);
                            const double bk = rdlane(ring.s0, lk);
                            double x = bk;
                            if (p != k) {
                                // interchange rows k and p: row p takes b_k
                                const int qp = (p >> 6) - (k >> 6), lp = p & 63;
                                x = ring.lane_value(qp, lp);
                                ring.put(qp, lane == lp, bk);
                            }
                            ring.axpy(lv[t], x);  // zero at row k itself
                            ring.s0 = lane == lk ? x : ring.s0;
                        }
                    }
                }
                if (c1 == n) flush((n - 1) >> 6);
            }
            __syncthreads();
        }
    }
    // backward: U x = b from the last column down; slot q holds block
    // k / 64 - q; entry (q, l) of column k is U(row, k) for the row
    // 64 (k / 64 - q) + l above the diagonal, and the reciprocal of U(k, k)
    // sits beside the column
    auto stage_u = [&](int h, int c1, int first) {
        const int c0 = max(c1 - G, 0), cnt = c1 - c0;
        stage_entries(sE[h], c0, cnt, first, [&](int k, int q, int l, bool& ok) {
            const int off = k - 64 * ((k >> 6) - q) - l;
            ok = off >= 1 && off <= min(bw, k);
            return Uf[(size_t)k * ldu + (ok ? off : 0)];
        });
        if (tid >= first)
            for (int c = tid - first; c < cnt; c += nt - first)
                sD[h][c] = 1.0 / (double)Uf[(size_t)(c0 + c) * ldu];
    };
    stage_u(0, n, 0);
    __syncthreads();
    if (tid < 64) {
        const int Btop = (n - 1) >> 6;
#pragma unroll
        for (int q = 0; q < R; ++q) ring.set(q, block(Btop - q));
    }
    for (int c1 = n, h = 0; c1 > 0; c1 -= G, h ^= 1) {
        const int c0 = max(c1 - G, 0);
        if (c0 > 0) stage_u(h ^ 1, c0, t0);
        if (tid < 64) {
            const T* E = sE[h];
            const double* D = sD[h];
            T un[S][R];
            double dn[S];
            auto fetch = [&](int k) {
#pragma unroll
                for (int t = 0; t < S; ++t) {
                    const int ck = max(k - t, c0) - c0;
                    dn[t] = D[ck];
#pragma unroll
                    for (int q = 0; q < R; ++q) un[t][q] = E[ck * PER + q * 64 + lane];
                }
            };
            fetch(c1 - 1);
            for (int k0 = c1 - 1; k0 >= c0; k0 -= S) {
                double uv[S][R], rdg[S];
#pragma unroll
                for (int t = 0; t < S; ++t) {
                    rdg[t] = dn[t];
#pragma unroll
                    for (int q = 0; q < R; ++q) uv[t][q] = (double)un[t][q];
                }
                if (k0 - S >= c0) fetch(k0 - S);
#pragma unroll
                for (int t = 0; t < S; ++t) {
                    const int k = k0 - t;
                    if (k >= c0) {
                        const int lk = k & 63;
                        const double xk = rdlane(ring.s0, lk) * rdg[t];
                        ring.axpy(uv[t], xk);  // zero at row k itself
                        ring.s0 = lane == lk ? xk : ring.s0;
                        // block k / 64 is finished: to b, and the slots move
                        if (lk == 0) {
                            flush(k >> 6);
                            if (k > 0) ring.shift(block((k >> 6) - R));
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
}

// The workgroup's band solve: staged when the stage holds 8 or more steps,
// otherwise the one-wavefront solve.  All threads call it; b is complete for
// every thread on return.
template <typename T, int NPL>
__device__ __forceinline__ void band_solve_group(int n, int kl, int ku, const T* __restrict__ Uf,
                                                 const T* __restrict__ Lf, const int* __restrict__ piv,
                                                 double* b, void* stage, int stage_bytes,
                                                 bool backward_only) {
    const int G = stage ? band_stage_cols<T, NPL>(stage_bytes) : 0;
    if (G >= 8) {
        band_solve_staged<T, NPL>(n, kl, ku, Uf, Lf, piv, b, stage, G, backward_only);
    } else {
        if (threadIdx.x < 64) band_solve_wave<T, NPL>(n, kl, ku, Uf, Lf, piv, b, backward_only);
        __syncthreads();
    }
}

// Solve J d = rb in place (rb in LDS).  FP64 factors: one band solve.  FP32
// factors: iterative refinement with FP64 residuals r0 - J d computed from
// the FP64 CSR values (columns < n), until ||res|| <= ir_rtol ||r0||.
// stage (LDS, stage_bytes; may be null): staging space of the band solves.
template <int NPL>
__device__ __forceinline__ void local_linear_solve(const DevMaps& P, const DevLocal& L, const NewtonParams& np,
                                   int i, int n, int rowbase, double* rb, double* r0,
                                   double* dl, double* red, bool forward_done = false,
                                   void* stage = nullptr, int stage_bytes = 0) {
    const int kl = P.kl[i], ku = P.ku[i];
    const double* Ud = L.Uf + P.off_u[i];
    const double* Ld = L.Lf + P.off_l[i];
    const float* Us = np.mixed ? L.Uf32 + P.off_u[i] : nullptr;
    const float* Ls = np.mixed ? L.Lf32 + P.off_l[i] : nullptr;
    const int* piv = L.piv + rowbase;
    if (!np.mixed) {
        band_solve_group<double, NPL>(n, kl, ku, Ud, Ld, piv, rb, stage, stage_bytes, forward_done);
        return;
    }
    double nr0 = 0.0;
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        r0[a] = rb[a];
        dl[a] = 0.0;
        nr0 += rb[a] * rb[a];
    }
    nr0 = sqrt(block_sum(nr0, red));
    for (int it = 0;; ++it) {
        band_solve_group<float, NPL>(n, kl, ku, Us, Ls, piv, rb, stage, stage_bytes, false);
        double rr = 0.0;
        for (int a = threadIdx.x; a < n; a += blockDim.x) dl[a] += rb[a];
        __syncthreads();
        for (int a = threadIdx.x; a < n; a += blockDim.x) {
            const int row = rowbase + a;
            double acc = r0[a];
            for (int s = P.jptr[row]; s < P.jptr[row + 1]; ++s) {
                const int c = P.jcol[s];
                if (c < n) acc -= L.jval[s] * dl[c];
            }
            rb[a] = acc;
            rr += acc * acc;
        }
        rr = sqrt(block_sum(rr, red));
        if (it + 1 >= np.ir_maxit || rr <= np.ir_rtol * nr0 || !(rr == rr)) break;
    }
    for (int a = threadIdx.x; a < n; a += blockDim.x) rb[a] = dl[a];
    __syncthreads();
}

// Factor J at the current point into FP64 or FP32 storage.
// rhs (FP64 only): forward substitution fused with the factorisation.
__device__ __forceinline__ int local_factor(const DevMaps& P, const DevLocal& L, const NewtonParams& np, int i,
                            int n, int rowbase, void* W, void* mult, int* sflag, bool fp64 = false,
                            double* rhs = nullptr) {
    const int kl = P.kl[i], ku = P.ku[i];
    const int* rptr = P.jptr + rowbase;
    if (np.mixed && !fp64)
        return band_lu_auto<float>(n, kl, ku, rptr, P.jcol, L.jval, (float*)W, (float*)mult, sflag,
                              L.Uf32 + P.off_u[i], L.Lf32 + P.off_l[i], L.piv + rowbase, 0,
                              np.lu_variant, nullptr, np.mixed == 2);
    return band_lu_auto<double>(n, kl, ku, rptr, P.jcol, L.jval, (double*)W, (double*)mult, sflag,
                           L.Uf + P.off_u[i], L.Lf + P.off_l[i], L.piv + rowbase, 0,
                           np.lu_variant, rhs);
}

// ----------------------------------------------------------------------------
// Fused local nonlinear solve: one workgroup per subdomain runs the whole
// inner Newton iteration for T_i(u) (eq. 4):
//   x = R_i u; loop { r = R_i F(v(x)); stop?; J = R_i DF(v(x)) P_i;
//                     LU(J); x -= J^{-1} r }
//   then J, LU at x* are kept for the exact tangent (eq. 6) and
//   T_i(u) = R_i u - x*.
// Stopping: ||r||_2 <= max(rtol rho_plain, abs_tol sqrt(n_i)) or
// max|step| <= stagnation max|x|, at most maxit steps.
// ----------------------------------------------------------------------------
template <int NPL, bool ELAST>
__global__ void __launch_bounds__(NLS_BLOCK)
k_local_newton(DevMesh M, DevMaps P, DevLocal L, NewtonParams np, const double* __restrict__ u,
               int lds_bytes) {
    extern __shared__ double smem[];
    __shared__ int sflag[20];
    __shared__ int sdetf;  // a residual met det F <= 0 (elasticity)
    const int i = P.order[blockIdx.x];
    const int rowbase = P.off_n[i], n = P.off_n[i + 1] - rowbase;
    const int gbase = P.off_g[i], ng = P.off_g[i + 1] - gbase;
    const int ebase = P.off_e[i];
    const int kl = P.kl[i];
    double* vp = smem;
    double* rb = vp + n + ng;
    double* r0 = rb + n;
    double* dl = r0 + (np.mixed ? n : 0);
    double* red = dl + (np.mixed ? n : 0);
    double* mult = red + 24;
    double* W = mult + ((kl > 1 ? kl : 1) + 1);
    for (int a = threadIdx.x; a < n; a += blockDim.x) vp[a] = u[P.l2g[rowbase + a]];
    for (int j = threadIdx.x; j < ng; j += blockDim.x) vp[n + j] = u[P.g2g[gbase + j]];
    if (threadIdx.x == 0) sdetf = 0;
    __syncthreads();
    local_residual<ELAST>(M, P, n, rowbase, ebase, vp, rb, &sdetf);
    double ss = 0.0;
    for (int a = threadIdx.x; a < n; a += blockDim.x) ss += rb[a] * rb[a];
    const double rho_plain = sqrt(block_sum(ss, red));
    const double tol = fmax(np.rtol * rho_plain, np.abs_tol * sqrt((double)n));
    double rn = rho_plain;
    // Predicted start: taken only if its residual is finite and below
    // rho_plain; the stopping rule stays relative to rho_plain.
    int start = 0;
    if (np.xpred) {
        for (int a = threadIdx.x; a < n; a += blockDim.x) vp[a] = np.xpred[rowbase + a];
        __syncthreads();
        local_residual<ELAST>(M, P, n, rowbase, ebase, vp, rb, &sdetf);
        ss = 0.0;
        for (int a = threadIdx.x; a < n; a += blockDim.x) ss += rb[a] * rb[a];
        const double rg = sqrt(block_sum(ss, red));
        if (rg == rg && !isinf(rg) && rg < rho_plain) {
            start = 1;
            rn = rg;
        } else {
            start = 2;
            // a rejected prediction's det F does not count (the reset is
            // ordered before the next residual by the barrier that follows
            // the reload of R_i u)
            if (threadIdx.x == 0) sdetf = 0;
        }
    }
    int its = 0, status = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        if (attempt == 1 || start == 2) {
            // from R_i u (plain start, or after the predicted start failed)
            for (int a = threadIdx.x; a < n; a += blockDim.x) vp[a] = u[P.l2g[rowbase + a]];
            __syncthreads();
            if (np.xpred) {
                local_residual<ELAST>(M, P, n, rowbase, ebase, vp, rb, &sdetf);
                rn = rho_plain;
            }
        }
        its = 0;
        status = 0;
        double dprev = -1.0;
        for (;;) {
            if (!(rn == rn) || isinf(rn)) {
                // the norm's reduction synchronised the block, so every
                // thread sees the flag of that residual
                status = sdetf ? 4 : 2;
                break;
            }
            if (rn <= tol) break;
            if (dprev >= 0.0) {
                double xm = 0.0;
                for (int a = threadIdx.x; a < n; a += blockDim.x) xm = fmax(xm, fabs(vp[a]));
                xm = block_max(xm, red);
                if (dprev <= np.stagnation * xm) break;
            }
            if (its == np.maxit) { status = 1; break; }
            local_jacobian<ELAST>(M, P, n, rowbase, ebase, vp, L.jval);
            __syncthreads();
            // FP64: the factorisation also carries out the forward
            // substitution on the residual, the solve only the backward one
            if (local_factor(P, L, np, i, n, rowbase, W, mult, sflag, false, np.mixed ? nullptr : rb)) {
                status = 3;
                break;
            }
            // the factorisation window is free during the solve: it holds
            // the staged factor columns
            local_linear_solve<NPL>(P, L, np, i, n, rowbase, rb, r0, dl, red, !np.mixed, W,
                                    lds_bytes - (int)((char*)W - (char*)smem));
            double dm = 0.0;
            for (int a = threadIdx.x; a < n; a += blockDim.x) {
                vp[a] -= rb[a];
                dm = fmax(dm, fabs(rb[a]));
            }
            dprev = block_max(dm, red);
            ++its;
            local_residual<ELAST>(M, P, n, rowbase, ebase, vp, rb, &sdetf);
            ss = 0.0;
            for (int a = threadIdx.x; a < n; a += blockDim.x) ss += rb[a] * rb[a];
            rn = sqrt(block_sum(ss, red));
        }
        if (status == 0 || start != 1) break;
        start = 2;
    }
    if (status == 0 && np.keep_factor) {
        // J and its LU at x*, in FP64, are kept for the exact tangent
        local_jacobian<ELAST>(M, P, n, rowbase, ebase, vp, L.jval);
        __syncthreads();
        if (local_factor(P, L, np, i, n, rowbase, W, mult, sflag, true)) status = 3;
    }
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        const int row = rowbase + a;
        L.xstar[row] = vp[a];
        L.T[row] = u[P.l2g[row]] - vp[a];
    }
    for (int j = threadIdx.x; j < ng; j += blockDim.x) L.ghost[gbase + j] = vp[n + j];
    if (threadIdx.x == 0) {
        L.its[i] = its;
        L.status[i] = status;
        L.start[i] = start;
    }
}

// ----------------------------------------------------------------------------
// ----------------------------------------------------------------------------
// Standalone local assembly (A1-A3) at x = R_i u for every subdomain: Q
// blocks per subdomain, block q stages the patch values of subdomain i in
// LDS and assembles rows [256 q, 256 (q + 1)).  r: packed local residuals;
// jval (or null): packed CSR values of [J_ii | B_i].  XCD-aware order:
// workgroups go to the eight XCDs in turn (block b to XCD b mod 8), so the
// Q blocks of subdomain i are placed at b = 8 j + (i mod 8) with consecutive
// j: they run together in the L2 of one XCD, which then serves the element
// data the neighbouring rows share.
// ----------------------------------------------------------------------------
template <bool ELAST>
__global__ void __launch_bounds__(256)
k_local_assemble(DevMesh M, DevMaps P, const double* __restrict__ u, double* __restrict__ r,
                 double* __restrict__ jval, int Q) {
    extern __shared__ double smem[];
    const int x = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int i = x + 8 * (j / Q);
    if (i >= P.nsub) return;
    const int rowbase = P.off_n[i], n = P.off_n[i + 1] - rowbase;
    const int a0 = (j % Q) * blockDim.x;
    if (a0 >= n) return;
    const int gbase = P.off_g[i], ng = P.off_g[i + 1] - gbase;
    double* vp = smem;
    for (int a = threadIdx.x; a < n; a += blockDim.x) vp[a] = u[P.l2g[rowbase + a]];
    for (int j = threadIdx.x; j < ng; j += blockDim.x) vp[n + j] = u[P.g2g[gbase + j]];
    __syncthreads();
    assemble_rows<ELAST>(M, P, n, rowbase, P.off_e[i], vp, a0, min(n, a0 + (int)blockDim.x),
                         r + rowbase, jval);
}

// Multi right-hand-side band solve X = J^{-1} R with the FP64 factors of
// band_lu: one right-hand side per lane (column c = blockIdx.y*256 + tid).
// Each lane keeps its forward window (KL+1 rows) and its backward window of
// partial sums (KW+1 rows) in registers, so the sweeps need no cross-lane
// traffic; the coefficients of MR_CH steps (pivots, L columns, U columns with
// the reciprocal of the diagonal) are staged through LDS by the whole
// workgroup, double-buffered, and read as broadcasts.  The forward results
// go to the per-column scratch fwd (row-major, ld = ldf).
// KL >= kl and KW >= kl + ku are compile-time window sizes.
// ----------------------------------------------------------------------------
constexpr int MR_CH = 8;
constexpr int MR_THREADS = 256;

// RHS columns given as sorted (row, value) lists, kept in registers.
template <int MAXE>
struct MrhsSparseSrc {
    int re[MAXE];
    double ve[MAXE];
    __device__ __forceinline__ void init(const int* __restrict__ ptr, const int* __restrict__ row,
                                         const int* __restrict__ slot,
                                         const double* __restrict__ val, int c, bool valid) {
        const int b = valid ? ptr[c] : 0, e = valid ? ptr[c + 1] : 0;
#pragma unroll
        for (int q = 0; q < MAXE; ++q) {
            re[q] = (b + q < e) ? row[b + q] : INT_MAX;
            ve[q] = (b + q < e) ? val[slot[b + q]] : 0.0;
        }
    }
    __device__ __forceinline__ double take(int r) {
        if (re[0] != r) return 0.0;
        const double v = ve[0];
#pragma unroll
        for (int q = 0; q + 1 < MAXE; ++q) {
            re[q] = re[q + 1];
            ve[q] = ve[q + 1];
        }
        re[MAXE - 1] = INT_MAX;
        return v;
    }
};


// r[j] = r[j + 1] - c[j] a for j < K (a register window shifted by one),
// with the coefficients c read from LDS in batches of 8, three batches (two
// for windows of 96 and more) in flight ahead of the multiply-adds that use
// them.  Scheduling barriers and
// empty uses of the results keep the compiler from hoisting all the reads
// (which would need K more registers) or from issuing them only just
// before their use (which leaves the LDS latency exposed on every batch).
template <int K>
__device__ __forceinline__ void shift_update(double* r, const double* c, double a) {
    static_assert(K % 8 == 0, "window sizes are multiples of 8");
    constexpr int B = 8, D = K >= 96 ? 2 : 3, NB = K / B;  // wide windows leave room for two
    double buf[D][B];
#pragma unroll
    for (int d = 0; d < D; ++d)
        if (d < NB) {
#pragma unroll
            for (int t = 0; t < B; ++t) buf[d][t] = c[d * B + t];
        }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int sl = q % D;
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < B; ++t) r[q * B + t] = r[q * B + t + 1] - buf[sl][t] * a;
#pragma unroll
        for (int t = 0; t < B; ++t) asm volatile("" ::"v"(r[q * B + t]));
        __builtin_amdgcn_sched_barrier(0);
        if (q + D < NB) {
#pragma unroll
            for (int t = 0; t < B; ++t) buf[sl][t] = c[(q + D) * B + t];
        }
    }
    __builtin_amdgcn_sched_barrier(0);
}

template <int KL, int KW, class Src, class Put>
__device__ __forceinline__ void band_solve_mrhs(int n, int kl, int ku,
                                                const double* __restrict__ Uf,
                                                const double* __restrict__ Lf,
                                                const int* __restrict__ piv, Src& src,
                                                bool valid, int col, double* __restrict__ fwd,
                                                int ldf, const int* __restrict__ tag,
                                                double* stage, int* sint, Put put) {
    constexpr int CH = MR_CH, NT = MR_THREADS;
    constexpr int FROW = KL, BROW = KW + 1;
    constexpr int PF = (CH * BROW + NT - 1) / NT;  // staged doubles per thread
    const int tid = threadIdx.x;
    const int ldu = kl + ku + 1, ldl = kl > 1 ? kl : 1;
    const int nch = (n + CH - 1) / CH;
    double pre[PF];
    int prei = 0;
    // ---------------------------------------------------------- forward sweep
    auto fload = [&](int ch) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int idx = tid + q * NT;
            double v = 0.0;
            if (idx < CH * FROW) {
                const int st = idx / FROW, j = idx - st * FROW;
                const int k = ch * CH + st;
                if (k < n && j < kl && k + 1 + j < n) v = Lf[(size_t)k * ldl + j];
            }
            pre[q] = v;
        }
        prei = 0;
        if (tid < CH) {
            const int k = ch * CH + tid;
            prei = k < n ? piv[k] : k;
        }
    };
    auto fstore = [&](int slot) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int idx = tid + q * NT;
            if (idx < CH * FROW) stage[slot * CH * BROW + idx] = pre[q];
        }
        if (tid < CH) sint[slot * CH + tid] = prei;
    };
    double x[KL + 1];
#pragma unroll
    for (int j = 0; j <= KL; ++j) x[j] = (j < n) ? src.take(j) : 0.0;
    fload(0);
    fstore(0);
    if (nch > 1) fload(1);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int slot = ch & 1;
        const double* L0 = stage + slot * CH * BROW;
#pragma unroll
        for (int st = 0; st < CH; ++st) {
            const int k = ch * CH + st;
            if (k < n) {
                const int d = sint[slot * CH + st] - k;
                if (d != 0) {
#pragma unroll
                    for (int q = 1; q <= KL; ++q)
                        if (q == d) {
                            const double t = x[0];
                            x[0] = x[q];
                            x[q] = t;
                        }
                }
                const double x0 = x[0];
                if (valid) fwd[(size_t)k * ldf + col] = x0;
                const double* Lk = L0 + st * FROW;
                shift_update<KL>(x, Lk, x0);
                x[KL] = (k + KL + 1 < n) ? src.take(k + KL + 1) : 0.0;
            }
        }
        if (ch + 1 < nch) {
            fstore((ch + 1) & 1);
            if (ch + 2 < nch) fload(ch + 2);
        }
        lds_barrier();
    }
    __syncthreads();  // forward results visible in HBM to this workgroup
    // --------------------------------------------------------- backward sweep
    // chunk ch covers steps k = n-1-ch*CH-st, st = 0..CH-1
    // the row tags tag[k] of a chunk are staged with its U columns, so that
    // a step does not wait for a load of its own
    auto bload = [&](int ch) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int idx = tid + q * NT;
            double v = 0.0;
            if (idx < CH * BROW) {
                const int st = idx / BROW, j = idx - st * BROW;
                const int k = n - 1 - ch * CH - st;
                if (k >= 0) {
                    if (j == 0) v = 1.0 / Uf[(size_t)k * ldu];
                    else if (j - 1 < min(kl + ku, k)) v = Uf[(size_t)k * ldu + j];
                }
            }
            pre[q] = v;
        }
        prei = -1;
        if (tid < CH) {
            const int k = n - 1 - ch * CH - tid;
            if (k >= 0) prei = tag[k];
        }
    };
    auto bstore = [&](int slot) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int idx = tid + q * NT;
            if (idx < CH * BROW) stage[slot * CH * BROW + idx] = pre[q];
        }
        if (tid < CH) sint[slot * CH + tid] = prei;
    };
    double p[KW + 1];
#pragma unroll
    for (int j = 0; j <= KW; ++j) {
        const int r = n - 1 - j;
        p[j] = (valid && r >= 0) ? fwd[(size_t)r * ldf + col] : 0.0;
    }
    double ent[CH], entn[CH];
    auto eload = [&](int ch, double* e) {
#pragma unroll
        for (int st = 0; st < CH; ++st) {
            const int r = n - 1 - ch * CH - st - 1 - KW;
            e[st] = (valid && r >= 0) ? fwd[(size_t)r * ldf + col] : 0.0;
        }
    };
    bload(0);
    bstore(0);
    if (nch > 1) bload(1);
    eload(0, ent);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int slot = ch & 1;
        const double* U0 = stage + slot * CH * BROW;
        if (ch + 1 < nch) eload(ch + 1, entn);
#pragma unroll
        for (int st = 0; st < CH; ++st) {
            const int k = n - 1 - ch * CH - st;
            if (k >= 0) {
                const double* Uk = U0 + st * BROW;
                const double y = p[0] * Uk[0];
                put(k, sint[slot * CH + st], y);
                shift_update<KW>(p, Uk + 1, y);
                p[KW] = ent[st];
            }
        }
#pragma unroll
        for (int st = 0; st < CH; ++st) ent[st] = entn[st];
        if (ch + 1 < nch) {
            bstore((ch + 1) & 1);
            if (ch + 2 < nch) bload(ch + 2);
        }
        lds_barrier();
    }
}

// W_i = (J_ii^{-1} B_i) on the owned rows of subdomain i (row-major, ld =
// |Gamma_i|), with J, B at the converged local state: the exact tangent's
// local term P~_i J_ii^{-1} B_i v_Gamma_i (eqs. 6, 7) becomes a GEMV.
template <int KL, int KW>
__global__ void __launch_bounds__(MR_THREADS)
k_tangent_prep(DevMaps P, DevLocal L, DevTangent Tg) {
    extern __shared__ double smem[];
    __shared__ int sint[2 * MR_CH];
    const int i = P.order[blockIdx.x];
    const int rowbase = P.off_n[i], n = P.off_n[i + 1] - rowbase;
    const int gbase = P.off_g[i], ng = P.off_g[i + 1] - gbase;
    const int kl = P.kl[i], ku = P.ku[i];
    const int col = blockIdx.y * MR_THREADS + threadIdx.x;
    const bool valid = col < ng;
    if ((int)blockIdx.y * MR_THREADS >= ng) return;  // uniform over the block
    MrhsSparseSrc<NLS_MAX_BCOL> src;
    src.init(Tg.bptr + gbase, Tg.brow, Tg.bslot, L.jval, col, valid);
    double* W = Tg.W + Tg.off_W[i];
    const int* rowown = Tg.rowown + rowbase;
    const int nown = Tg.off_own[i + 1] - Tg.off_own[i];
    auto put = [&](int k, int o, double y) {
        (void)k;
        if (valid && o >= 0) W[(size_t)col * nown + o] = y;
    };
    band_solve_mrhs<KL, KW>(n, kl, ku, L.Uf + P.off_u[i], L.Lf + P.off_l[i], L.piv + rowbase, src,
                            valid, col, Tg.fwd + Tg.off_F[i], ng, rowown, smem, sint, put);
}

// ----------------------------------------------------------------------------
// W_i = J_ii^{-1} B_i on the matrix cores.  The band LU's forward elimination
// (an interchange, then multipliers below the pivot, at every step) is taken
// 16 steps at a time: the steps of block b (rows from k0 = 16 b) act on the
// window of R = 16 + kl rows from k0 only, and their product is
// L_b^{-1} P_b, with P_b a permutation of the window and L_b unit lower
// triangular, the identity right of its first 16 columns.  With X' = P_b X
// on the window, X <- [0; X'_2] + G_b X'_1 with G_b = [L11^{-1}; -L21 L11^{-1}]
// ((16 + kl) x 16), a product on 16x16x4 FP64 matrix-core steps.  The
// backward substitution goes up in the same blocks: X_1 <- U11^{-1}
// (Y_1 - U12 X_2), U12 the 16 x (kl + ku) band strip right of the diagonal
// block.  k_tangent_blocks forms, one wavefront per block of every
// subdomain, sigma_b (P_b as a gather: position p of X' holds window row
// sigma_b(p)), G_b and U11^{-1}, stored in the operand order of the
// matrix-core steps; k_tangent_mfma runs both sweeps, one wavefront per 16
// columns of B_i, with its window of X in LDS.  Same operator as the
// per-lane sweeps above, with the rounding of a blocked elimination.
// ----------------------------------------------------------------------------
constexpr int TB_RT = 4;              // row tiles of G_b (16 + kl <= 64)
constexpr int TB_G = TB_RT * 4 * 64;  // doubles of G_b per block
constexpr int TB_U = 4 * 64;          // doubles of U11^{-1} per block
constexpr int TB_RING = 128;          // window rows in LDS (>= 16 + kl + ku)

// sigma_b, G_b and U11^{-1} of the 16-row block at row k0 of one band
// problem (n rows, band factors Lf, Uf and pivots piv of band_lu, local
// indices), by one wavefront; stored at sg (64 ints), G (TB_G doubles) and
// Ui (TB_U doubles) in the operand order of the matrix-core steps.
__device__ __forceinline__ void tb_block_pieces(int n, int kl, int ku, const double* __restrict__ Lf,
                                                const double* __restrict__ Uf,
                                                const int* __restrict__ piv, int k0,
                                                int* __restrict__ sg, double* __restrict__ G,
                                                double* __restrict__ Ui) {
    __shared__ double Lb[64 * 17];
    __shared__ double Ub[16 * 17];
    const int kw = kl + ku;
    const int ldu = kw + 1, ldl = kl > 1 ? kl : 1;
    const int lane = threadIdx.x;
    const int ns = min(16, n - k0);  // steps of this block; past n the identity
    // every load first: lane s < ns holds the pivot offset of step s, lane q
    // the multipliers of each step s for window position q
    const int pv = lane < ns ? piv[k0 + lane] - k0 : lane;
    double lv[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int j = lane - s - 1;
        const bool ok = s < ns && j >= 0 && j < kl && k0 + s + 1 + j < n;
        const double v = Lf[ok ? (size_t)(k0 + s) * ldl + j : 0];
        lv[s] = ok ? v : 0.0;
    }
    double uv[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int r = (lane + 64 * e) >> 4, c = (lane + 64 * e) & 15;
        const bool ok = c < ns && r <= c && c - r <= kw;
        const double v = Uf[ok ? (size_t)(k0 + c) * ldu + (c - r) : 0];
        uv[e] = ok ? v : (r == c ? 1.0 : 0.0);  // rows and columns past n: identity
    }
    for (int e = lane; e < 64 * 17; e += 64) Lb[e] = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) Ub[((lane + 64 * e) >> 4) * 17 + ((lane + 64 * e) & 15)] = uv[e];
    // sigma_b: the interchanges of the block applied to the window positions
    int ident = lane;
#pragma unroll
    for (int s = 0; s < 16; ++s)
        if (s < ns) {
            const int d = __builtin_amdgcn_readlane(pv, s);
            const int va = __builtin_amdgcn_readlane(ident, s);
            const int vc = __builtin_amdgcn_readlane(ident, d);
            if (lane == s) ident = vc;
            if (lane == d) ident = va;
        }
    sg[lane] = ident;
    // L_b: step s's multiplier for the row at position q after that step's
    // interchange belongs to the row's position after the whole block, m_s(q);
    // m runs backward from the identity (after the last step).  Lanes without
    // a multiplier store the zero of L_b at their position.
    __syncthreads();
    int m = lane;
#pragma unroll
    for (int s = 15; s >= 0; --s)
        if (s < ns) {
            Lb[m * 17 + s] = lv[s];
            const int d = __builtin_amdgcn_readlane(pv, s);
            const int va = __builtin_amdgcn_readlane(m, s);
            const int vc = __builtin_amdgcn_readlane(m, d);
            if (lane == s) m = vc;
            if (lane == d) m = va;
        }
    __syncthreads();
    // G_b = L_b^{-1}[:, 0:16]: lane (c, g) substitutes e_c through L11 (unit
    // diagonal; entries on and above it are not read), then forms rows
    // 16 + g + 4 t of -L21 L11^{-1}.  G_b[p][c] is lane (p & 15) + 16 (c & 3)
    // of k-step c >> 2 of row tile p >> 4.
    const int c = lane & 15, g = lane >> 4, kk = c >> 2, lc = 16 * (c & 3);
    double x[16];
#pragma unroll
    for (int p = 0; p < 16; ++p) x[p] = (p == c) ? 1.0 : 0.0;
#pragma unroll
    for (int s = 0; s < 15; ++s)
#pragma unroll
        for (int p = s + 1; p < 16; ++p) x[p] = fma(-Lb[p * 17 + s], x[s], x[p]);
#pragma unroll
    for (int p = 0; p < 16; ++p)
        if ((p & 3) == g) G[kk * 64 + p + lc] = x[p];
#pragma unroll
    for (int t = 0; t < 12; ++t) {
        const int p = 16 + g + 4 * t;
        double a = 0.0;
#pragma unroll
        for (int s = 0; s < 16; ++s) a = fma(Lb[p * 17 + s], x[s], a);
        G[((p >> 4) * 4 + kk) * 64 + (p & 15) + lc] = -a;
    }
    // U11^{-1} by columns (back substitution with e_c); entry [r][c] is lane
    // r + 16 (c & 3) of k-step c >> 2
    double y[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) y[r] = (r == c) ? 1.0 : 0.0;
#pragma unroll
    for (int jj = 15; jj >= 0; --jj) {
        y[jj] = y[jj] / Ub[jj * 17 + jj];
#pragma unroll
        for (int r = 0; r < jj; ++r) y[r] = fma(-Ub[r * 17 + jj], y[jj], y[r]);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r)
        if ((r & 3) == g) Ui[kk * 64 + r + lc] = y[r];
}

__global__ void __launch_bounds__(64) k_tangent_blocks(DevMaps P, DevLocal L, DevTangent Tg) {
    const int gb = blockIdx.x;
    const int i = Tg.blk_sub[gb];
    const int rowbase = P.off_n[i], n = P.off_n[i + 1] - rowbase;
    tb_block_pieces(n, P.kl[i], P.ku[i], L.Lf + P.off_l[i], L.Uf + P.off_u[i], L.piv + rowbase,
                    (gb - Tg.off_blk[i]) * 16, Tg.tsig + (size_t)gb * 64,
                    Tg.tG + (size_t)gb * TB_G, Tg.tUi + (size_t)gb * TB_U);
}

// Both sweeps of the blocked solve for the 16 columns of one wavefront, on
// one band problem (n rows, band widths kl, ku, U by columns in Uf; sig, Gs,
// Us its blocks' pieces; Y a scratch of ceil(n / 16) 16 x 16 tiles).
// bval(r): entry r of this lane's right-hand-side column (zero past n).
// oidx(r): the output index of row r (read one block ahead; r < n), ook(r):
// whether row r is written, put(o, v): the write.  Forward: the window rows
// [k0, k0 + R) sit in an LDS ring; rows entering it are filled by bval; each
// block gathers X' = P_b X from the ring by sigma_b, forms [0; X'_2] +
// G_b X'_1 (up to four row tiles of 16), writes rows k0 .. k0 + 15 (final)
// to Y and keeps the rest in the ring.  Backward: the solved rows above the
// block's strip sit in the ring; each block forms Y_1 - U12 X_2 (U12 read
// from the band factor, NKK k-steps of 4 columns at most), then U11^{-1}
// times it (the FP64 result layout, rows g + 4 q in lane (c, g), is already
// the operand layout of the next product), and hands the rows to put.  The
// operands of the next block are loaded once the current block's products
// have been issued.
template <int NKK, class BVal, class OIdx, class OOk, class Put>
__device__ __forceinline__ void tb_sweeps(int n, int kl, int ku, const double* __restrict__ Uf,
                                          const int* __restrict__ sig,
                                          const double* __restrict__ Gs,
                                          const double* __restrict__ Us, double* __restrict__ Y,
                                          double* ring, BVal bval, OIdx oidx, OOk ook, Put put) {
    typedef Mfma<double>::acc_t acc_t;
    constexpr int RM = TB_RING - 1;
    const int kw = kl + ku, ldu = kw + 1, R = 16 + kl;
    const int rtn = (R + 15) >> 4, nkk = (kw + 3) >> 2;
    const int lane = threadIdx.x & 63, c = lane & 15, h = lane >> 4;
    const int nb = (n + 15) >> 4;
    auto fill16 = [&](int lo) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = lo + h + 4 * q;
            ring[(r & RM) * 16 + c] = bval(r);
        }
    };
    for (int lo = 0; lo < R; lo += 16) fill16(lo);
    int sg = sig[lane];
    double ga[TB_RT * 4];
#pragma unroll
    for (int e = 0; e < TB_RT * 4; ++e) ga[e] = Gs[e * 64 + lane];
    for (int b = 0; b < nb; ++b) {
        const int k0 = b * 16;
        if (b > 0) fill16(k0 + kl);
        double bo[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int sp = __shfl(sg, 4 * kk + h);
            bo[kk] = ring[((k0 + sp) & RM) * 16 + c];
        }
        acc_t acc[TB_RT];
        acc[0] = acc_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int rt = 1; rt < TB_RT; ++rt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int p = 16 * rt + h + 4 * q;
                const int sp = __shfl(sg, p);
                const double v = ring[((k0 + sp) & RM) * 16 + c];
                acc[rt][q] = p < R ? v : 0.0;
            }
#pragma unroll
        for (int rt = 0; rt < TB_RT; ++rt)
            if (rt < rtn) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    acc[rt] = Mfma<double>::step(ga[rt * 4 + kk], bo[kk], acc[rt]);
            }
        if (b + 1 < nb) {
            sg = sig[(b + 1) * 64 + lane];
#pragma unroll
            for (int e = 0; e < TB_RT * 4; ++e) ga[e] = Gs[(size_t)(b + 1) * TB_G + e * 64 + lane];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Y[(size_t)(k0 + h + 4 * q) * 16 + c] = acc[0][q];
#pragma unroll
        for (int rt = 1; rt < TB_RT; ++rt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int p = 16 * rt + h + 4 * q;
                if (p < R) ring[((k0 + p) & RM) * 16 + c] = acc[rt][q];
            }
    }
    __syncthreads();
    for (int e = lane; e < TB_RING * 16; e += 64) ring[e] = 0.0;
    __syncthreads();
    // A[r][j] = -U[k0 + r][k0 + 16 + j] (r = c, j = 4 kk + h): column
    // k0 + 16 + j of the band factor, t = 16 + j - r above its diagonal
    // (NKK >= nkk k-steps; those past nkk have A = 0).  With them: Y_1,
    // U11^{-1} and the output index of each result row.  The loads take
    // clamped in-range addresses and are masked where they are used; those
    // of block b - 1 are issued once block b's strip products have been.
    double ua[NKK], yn[4], un[4];
    int on[4];
    auto load_blk = [&](int b) {
        const int k0 = b * 16;
#pragma unroll
        for (int kk = 0; kk < NKK; ++kk) {
            const int j = 4 * kk + h, cu = min(k0 + 16 + j, n - 1), t = min(16 + j - c, kw);
            ua[kk] = Uf[(size_t)cu * ldu + t];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = k0 + h + 4 * q;
            yn[q] = Y[(size_t)r * 16 + c];
            on[q] = oidx(min(r, n - 1));
        }
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) un[kk] = Us[(size_t)b * TB_U + kk * 64 + lane];
    };
    load_blk(nb - 1);
    for (int b = nb - 1; b >= 0; --b) {
        const int k0 = b * 16;
        double uc[4];
        int oc[4];
        acc_t acc0, acc1 = acc_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = k0 + h + 4 * q;
            acc0[q] = yn[q];
            uc[q] = un[q];
            oc[q] = (r < n && ook(r)) ? on[q] : -1;
        }
#pragma unroll
        for (int kk = 0; kk < NKK; kk += 2) {
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                if (kk + d >= NKK) break;
                const int j = 4 * (kk + d) + h;
                const bool ok = kk + d < nkk && k0 + 16 + j < n && 16 + j - c <= kw;
                const double a = ok ? -ua[kk + d] : 0.0;
                const double xb = ring[((k0 + 16 + j) & RM) * 16 + c];
                if (d == 0)
                    acc0 = Mfma<double>::step(a, xb, acc0);
                else
                    acc1 = Mfma<double>::step(a, xb, acc1);
            }
        }
        if (b > 0) load_blk(b - 1);
        acc_t xo = acc_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) xo = Mfma<double>::step(uc[kk], acc0[kk] + acc1[kk], xo);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ring[((k0 + h + 4 * q) & RM) * 16 + c] = xo[q];
            if (oc[q] >= 0) put(oc[q], xo[q]);
        }
    }
}

// W_i: one wavefront per (subdomain, 16 columns of B_i), the columns given
// by their (row, value) lists; the owned rows of the result go to W.
template <int NKK>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(NKK <= 18 ? 3 : 2)))
k_tangent_mfma(DevMaps P, DevLocal L, DevTangent Tg) {
    __shared__ double ring[TB_RING * 16];
    const int i = P.order[blockIdx.x];
    const int rowbase = P.off_n[i], n = P.off_n[i + 1] - rowbase;
    const int gbase = P.off_g[i], ng = P.off_g[i + 1] - gbase;
    const int tile = blockIdx.y;
    if (tile * 16 >= ng) return;  // uniform over the wavefront
    const int c = threadIdx.x & 15;
    const int col = tile * 16 + c;
    const bool cv = col < ng;
    const int nb = (n + 15) >> 4, b0 = Tg.off_blk[i];
    int re[NLS_MAX_BCOL];
    double ve[NLS_MAX_BCOL];
    {
        const int pb = cv ? Tg.bptr[gbase + col] : 0, pe = cv ? Tg.bptr[gbase + col + 1] : 0;
#pragma unroll
        for (int q = 0; q < NLS_MAX_BCOL; ++q) {
            re[q] = (pb + q < pe) ? Tg.brow[pb + q] : -1;
            ve[q] = (pb + q < pe) ? L.jval[Tg.bslot[pb + q]] : 0.0;
        }
    }
    auto bval = [&](int r) {
        double v = 0.0;
#pragma unroll
        for (int e = 0; e < NLS_MAX_BCOL; ++e) v = (re[e] == r) ? ve[e] : v;
        return v;
    };
    const int* __restrict__ rowown = Tg.rowown + rowbase;
    double* __restrict__ W = Tg.W + Tg.off_W[i];
    const int nown = Tg.off_own[i + 1] - Tg.off_own[i];
    tb_sweeps<NKK>(n, P.kl[i], P.ku[i], L.Uf + P.off_u[i], Tg.tsig + (size_t)b0 * 64,
                   Tg.tG + (size_t)b0 * TB_G, Tg.tUi + (size_t)b0 * TB_U,
                   Tg.fwd + Tg.off_F[i] + (size_t)tile * nb * 256, ring, bval,
                   [&](int r) { return rowown[r]; }, [&](int) { return cv; },
                   [&](int o, double v) { W[(size_t)col * nown + o] = v; });
}


// A0^{-1} by the same blocked solve: the pieces of every 16-row block of
// the diagonal blocks of A0, then one wavefront per 16 identity columns,
// the rows of the result into the row-major inverse.
__global__ void __launch_bounds__(64) k_coarse_inv_blocks(DevCoarse C) {
    const int gb = blockIdx.x;
    int b = 0;
    while (b + 1 < C.nblk && C.inv_off[b + 1] <= gb) ++b;
    const int off = C.boff[b], n = C.boff[b + 1] - off;
    tb_block_pieces(n, C.bkl[b], C.bku[b], C.a0L + C.offL[b], C.a0U + C.offU[b], C.a0piv + off,
                    (gb - C.inv_off[b]) * 16, C.inv_sig + (size_t)gb * 64,
                    C.inv_G + (size_t)gb * TB_G, C.inv_Ui + (size_t)gb * TB_U);
}

template <int NKK>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(NKK <= 18 ? 3 : 2)))
k_coarse_inv_mfma(DevCoarse C) {
    __shared__ double ring[TB_RING * 16];
    const int b = blockIdx.x, tile = blockIdx.y;
    const int off = C.boff[b], n = C.boff[b + 1] - off;
    if (tile * 16 >= n) return;  // uniform over the wavefront
    const int col = tile * 16 + (threadIdx.x & 15);
    const bool cv = col < n;
    const int nb = (n + 15) >> 4, b0 = C.inv_off[b];
    double* __restrict__ Ainv = C.a0inv + C.offI[b];
    tb_sweeps<NKK>(n, C.bkl[b], C.bku[b], C.a0U + C.offU[b], C.inv_sig + (size_t)b0 * 64,
                   C.inv_G + (size_t)b0 * TB_G, C.inv_Ui + (size_t)b0 * TB_U,
                   C.inv_Y + C.inv_offY[b] + (size_t)tile * nb * 256, ring,
                   [&](int r) { return (cv && r == col) ? 1.0 : 0.0; }, [&](int r) { return r; },
                   [&](int) { return cv; },
                   [&](int o, double v) { Ainv[(size_t)o * n + col] = v; });
}

// z[owned rows of i] = W_i v_Gamma_i: streams W (column-major, one owned
// row per thread) once; HBM-bound.  Grid (nsub, QS) splits each
// subdomain's rows over QS blocks.  STREAM: W is read with nontemporal
// loads (for a W larger than the last-level cache, which it would only
// thrash; a smaller W is left to stay cached between products).
template <bool STREAM>
__global__ void __launch_bounds__(256)
k_tangent_gemv(DevMaps P, DevTangent Tg, const double* __restrict__ v, double* __restrict__ z) {
    extern __shared__ double vg[];
    const int i = blockIdx.x;
    const int gbase = P.off_g[i], ng = P.off_g[i + 1] - gbase;
    const int ob = Tg.off_own[i], no = Tg.off_own[i + 1] - ob;
    for (int j = threadIdx.x; j < ng; j += blockDim.x) vg[j] = v[P.g2g[gbase + j]];
    __syncthreads();
    const double* W = Tg.W + Tg.off_W[i];
    const int rowbase = P.off_n[i];
    for (int r = blockIdx.y * blockDim.x + threadIdx.x; r < no; r += gridDim.y * blockDim.x) {
        // eight independent loads in flight per thread
        double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int j = 0;
        for (; j + 7 < ng; j += 8) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double* wq = W + (size_t)(j + q) * no + r;
                a[q] += (STREAM ? __builtin_nontemporal_load(wq) : *wq) * vg[j + q];
            }
        }
        for (; j < ng; ++j) a[0] += W[(size_t)j * no + r] * vg[j];
        z[rowbase + Tg.ownrow[ob + r]] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
}

// Inverse of every diagonal block of A0 (band order, row-major per block)
// from its band LU: INV_CB identity columns per workgroup, held in LDS, so
// any band width fits; the factor columns (and pivots) of INV_S steps are
// fetched into registers one chunk ahead and staged into LDS at the chunk
// boundary, so the sweeps wait for HBM only once per pipeline fill.
// Forward: interchange k, then column k of L; backward: x_k = X_k / U_kk
// (written out as row k of the inverse) and the rows above updated with
// column k of U.  One barrier per step.
constexpr int INV_CB = 8, INV_S = 8, INV_THREADS = 256, INV_MAXW = 512;
constexpr int INV_PF = (INV_S * INV_MAXW + INV_THREADS - 1) / INV_THREADS;

__global__ void __launch_bounds__(INV_THREADS) k_coarse_inverse(DevCoarse C, int max_ldu) {
    extern __shared__ double smem[];
    const int b = blockIdx.y;
    const int off = C.boff[b], n = C.boff[b + 1] - off;
    const int c0 = blockIdx.x * INV_CB;
    if (c0 >= n) return;  // uniform over the block
    const int kl = C.bkl[b], ku = C.bku[b];
    const int ldu = kl + ku + 1, ldl = kl > 1 ? kl : 1;
    const double* __restrict__ U = C.a0U + C.offU[b];
    const double* __restrict__ L = C.a0L + C.offL[b];
    const int* __restrict__ piv = C.a0piv + off;
    double* __restrict__ Ainv = C.a0inv + C.offI[b];
    double* X = smem;                                  // n x INV_CB
    double* st = X + (size_t)n * INV_CB;               // 2 x INV_S x max_ldu
    int* spiv = (int*)(st + 2 * INV_S * max_ldu);      // 2 x INV_S
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < n * INV_CB; i += nt) {
        const int r = i / INV_CB, c = i - r * INV_CB;
        X[i] = (r == c0 + c) ? 1.0 : 0.0;
    }
    const int nq = (n + INV_S - 1) / INV_S;
    double pre[INV_PF];
    int ppre = 0;
    // ---------------------------------------------------------- forward
    auto issueL = [&](int q) {
#pragma unroll
        for (int e = 0; e < INV_PF; ++e) {
            const int i = tid + e * nt;
            double v = 0.0;
            if (i < INV_S * ldl) {
                const int s = i / ldl, j = i - s * ldl, k = q * INV_S + s;
                if (k < n && j < kl && k + 1 + j < n) v = L[(size_t)k * ldl + j];
            }
            pre[e] = v;
        }
        if (tid < INV_S) {
            const int k = q * INV_S + tid;
            ppre = k < n ? piv[k] : k;
        }
    };
    auto commitL = [&](int q) {
        double* dst = st + (size_t)(q & 1) * INV_S * max_ldu;
#pragma unroll
        for (int e = 0; e < INV_PF; ++e) {
            const int i = tid + e * nt;
            if (i < INV_S * ldl) dst[(i / ldl) * max_ldu + (i % ldl)] = pre[e];
        }
        if (tid < INV_S) spiv[(q & 1) * INV_S + tid] = ppre;
    };
    issueL(0);
    commitL(0);
    __syncthreads();
    for (int q = 0; q < nq; ++q) {
        if (q + 1 < nq) issueL(q + 1);
        const double* lc = st + (size_t)(q & 1) * INV_S * max_ldu;
        const int* pc = spiv + (q & 1) * INV_S;
        for (int s = 0; s < INV_S; ++s) {
            const int k = q * INV_S + s;
            if (k >= n) break;
            const int p = pc[s];
            if (p != k) {
                if (tid < INV_CB) {
                    const double t = X[k * INV_CB + tid];
                    X[k * INV_CB + tid] = X[p * INV_CB + tid];
                    X[p * INV_CB + tid] = t;
                }
                __syncthreads();
            }
            const int lim = min(kl, n - 1 - k);
            for (int i = tid; i < lim * INV_CB; i += nt) {
                const int j = i / INV_CB, c = i - j * INV_CB;
                X[(k + 1 + j) * INV_CB + c] -= lc[s * max_ldu + j] * X[k * INV_CB + c];
            }
            __syncthreads();
        }
        if (q + 1 < nq) commitL(q + 1);
        __syncthreads();
    }
    // ---------------------------------------------------------- backward
    // chunk q covers steps k = n - 1 - (q * INV_S + s)
    auto issueU = [&](int q) {
#pragma unroll
        for (int e = 0; e < INV_PF; ++e) {
            const int i = tid + e * nt;
            double v = 0.0;
            if (i < INV_S * ldu) {
                const int s = i / ldu, o = i - s * ldu, k = n - 1 - (q * INV_S + s);
                if (k >= 0 && o <= k) v = U[(size_t)k * ldu + o];
            }
            pre[e] = v;
        }
    };
    auto commitU = [&](int q) {
        double* dst = st + (size_t)(q & 1) * INV_S * max_ldu;
#pragma unroll
        for (int e = 0; e < INV_PF; ++e) {
            const int i = tid + e * nt;
            if (i < INV_S * ldu) dst[(i / ldu) * max_ldu + (i % ldu)] = pre[e];
        }
    };
    issueU(0);
    commitU(0);
    __syncthreads();
    for (int q = 0; q < nq; ++q) {
        if (q + 1 < nq) issueU(q + 1);
        const double* uc = st + (size_t)(q & 1) * INV_S * max_ldu;
        for (int s = 0; s < INV_S; ++s) {
            const int k = n - 1 - (q * INV_S + s);
            if (k < 0) break;
            const double inv = 1.0 / uc[s * max_ldu];
            const int lim = min(ldu - 1, k);
            for (int i = tid; i < (lim + 1) * INV_CB; i += nt) {
                const int j = i / INV_CB, c = i - j * INV_CB;
                const double xk = X[k * INV_CB + c] * inv;
                if (j == 0) {
                    if (c0 + c < n) Ainv[(size_t)k * n + c0 + c] = xk;
                } else {
                    X[(k - j) * INV_CB + c] -= uc[s * max_ldu + j] * xk;
                }
            }
            __syncthreads();
        }
        if (q + 1 < nq) commitU(q + 1);
        __syncthreads();
    }
}

// y = A0^{-1} x, block by block: one wavefront per row.
__global__ void __launch_bounds__(256)
k_coarse_apply_inverse(DevCoarse C, const double* __restrict__ x, double* __restrict__ y) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= C.n0) return;
    const int b = C.rblk[row];
    const int off = C.boff[b], n = C.boff[b + 1] - off;
    const double* a = C.a0inv + C.offI[b] + (size_t)(row - off) * n;
    double acc = 0.0;
    for (int j = lane; j < n; j += 64) acc += a[j] * x[off + j];
    acc = wave_sum(acc);
    if (lane == 0) y[row] = acc;
}


// Local part of the exact tangent: z_i = J_ii^{-1} (B_i v_Gamma_i), with J,
// B at the converged local state (eq. 6 with R_i DF(u_i) v = J R_i v + B v_G).
template <int NPL>
__global__ void __launch_bounds__(NLS_BLOCK)
k_tangent_local(DevMesh M, DevMaps P, DevLocal L, NewtonParams np, const double* __restrict__ v,
                int restrict_rhs, int lds_bytes) {
    extern __shared__ double smem[];
    const int i = P.order[blockIdx.x];
    const int rowbase = P.off_n[i], n = P.off_n[i + 1] - rowbase;
    const int gbase = P.off_g[i];
    double* rb = smem;
    double* r0 = rb + n;
    double* dl = r0 + (np.mixed ? n : 0);
    double* red = dl + (np.mixed ? n : 0);
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        const int row = rowbase + a;
        double acc = 0.0;
        if (restrict_rhs) {
            acc = v[P.l2g[row]];  // R_i v (local Schwarz solve)
        } else {
            for (int s = P.jptr[row]; s < P.jptr[row + 1]; ++s) {
                const int c = P.jcol[s];
                if (c >= n) acc += L.jval[s] * v[P.g2g[gbase + c - n]];
            }
        }
        rb[a] = acc;
    }
    __syncthreads();
    double* stage = red + 24;
    local_linear_solve<NPL>(P, L, np, i, n, rowbase, rb, r0, dl, red, false, stage,
                            lds_bytes - (int)((char*)stage - (char*)smem));
    for (int a = threadIdx.x; a < n; a += blockDim.x) L.z[rowbase + a] = rb[a];
}

// out[g] = T[own(g)] (+ addv[g]) (+ sum_l Phi_o(g)[g][l] c[K_o(g)[l]]):
// restricted prolongation (eq. 8) and the coarse term P_0 c (eq. 10).
__global__ void k_prolong(int N, const int* __restrict__ own_pidx, const double* __restrict__ T,
                          const double* __restrict__ addv, DevCoarse C, int with_coarse,
                          const double* __restrict__ cvec, double* __restrict__ out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    double y = T[own_pidx[g]];
    if (addv) y += addv[g];
    if (with_coarse) {
        const int o = C.cown[g];
        const int k0 = C.off_k[o], nk = C.off_k[o + 1] - k0;
        const double* ph = C.phi + C.off_phi[o] + (int64_t)(C.cpos[g] - C.off_c[o]) * nk;
        double acc = 0.0;
        for (int l = 0; l < nk; ++l) acc += ph[l] * cvec[C.klist[k0 + l]];
        y += acc;
    }
    out[g] = y;
}

// out = DF(u) v, one thread per node (P1): the rows of the element
// Jacobians K_T = kappa [(1 + beta m) G + beta s (U 1 + u)^T / 6] (the same
// entries as the local Jacobian) over the incident elements; Dirichlet rows
// are identity rows.
__global__ void k_global_jv(DevMesh M, const double* __restrict__ u, const double* __restrict__ v,
                            double* __restrict__ out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= M.N) return;
    if (M.dflag[g]) {
        out[g] = v[g];
        return;
    }
    double acc = 0.0;
    for (int k = M.nptr[g]; k < M.nptr[g + 1]; ++k) {
        const int code = M.nel[k];
        const int e = code >> 2, pos = code & 3;
        const int nd[3] = {M.conn[3 * e], M.conn[3 * e + 1], M.conn[3 * e + 2]};
        const double uu[3] = {u[nd[0]], u[nd[1]], u[nd[2]]};
        const double U = uu[0] + uu[1] + uu[2];
        const double m = (U * U + uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]) * (1.0 / 12.0);
        double gr[3];
        g_row(M.G6 + 6 * (size_t)e, pos, gr[0], gr[1], gr[2]);
        const double sa = gr[0] * uu[0] + gr[1] * uu[1] + gr[2] * uu[2];
        const double coef = M.kappa[e] * (1.0 + M.beta * m);
        const double rk = M.beta * M.kappa[e] * sa * (1.0 / 6.0);
#pragma unroll
        for (int c = 0; c < 3; ++c) acc += (coef * gr[c] + rk * (U + uu[c])) * v[nd[c]];
    }
    out[g] = acc;
}

// out = DF(u) v for the elasticity problem, one thread per dof.
__global__ void k_global_jv_nh(DevMesh M, const double* __restrict__ u, const double* __restrict__ v,
                               double* __restrict__ out) {
    const int gd = blockIdx.x * blockDim.x + threadIdx.x;
    if (gd >= M.ndof) return;
    if (M.dflag[gd]) {
        out[gd] = v[gd];
        return;
    }
    const int g = gd >> 1, c = gd & 1;
    double acc = 0.0;
    for (int k = M.nptr[g]; k < M.nptr[g + 1]; ++k) {
        const int code = M.nel[k];
        const int e = code >> 2, pos = code & 3;
        double X[4][2], ue[4][2], kr[4][2];
        nh_coords(M, e, X);
        int gn[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            gn[a] = M.conn[4 * e + a];
            ue[a][0] = u[2 * gn[a]];
            ue[a][1] = u[2 * gn[a] + 1];
        }
        nh_stiff_row(M, X, ue, pos, c, kr);
#pragma unroll
        for (int b = 0; b < 4; ++b) acc += kr[b][0] * v[2 * gn[b]] + kr[b][1] * v[2 * gn[b] + 1];
    }
    out[gd] = acc;
}

// Per subdomain: gblk_i = Phi_i^T r over the closure dofs the subdomain owns,
// so that sum_i gblk_i = Phi^T r (each dof counted once).
__global__ void __launch_bounds__(NLS_BLOCK) k_coarse_phit(DevCoarse C, const double* __restrict__ r) {
    const int i = blockIdx.x;
    const int cb = C.off_c[i], nc = C.off_c[i + 1] - cb;
    const int k0 = C.off_k[i], nk = C.off_k[i + 1] - k0;
    const double* ph = C.phi + C.off_phi[i];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int k = wv; k < nk; k += nw) {
        double acc = 0.0;
        for (int a = lane; a < nc; a += 64) {
            const int gd = C.cnode[cb + a];
            if (C.cown[gd] == i) acc += ph[(int64_t)a * nk + k] * r[gd];
        }
        acc = wave_sum(acc);
        if (lane == 0) C.gblk[k0 + k] = acc;
    }
}

// J_ii = R_i DF(v) P_i and its FP64 band LU, at v = u (the local factors of
// the linear Schwarz preconditioner) or at a given local state (x*, Gamma
// values) for the exact tangent; status 3 on a zero pivot.  LDS as the fused
// local Newton kernel.
template <bool ELAST>
__global__ void __launch_bounds__(NLS_BLOCK)
k_local_factor(DevMesh M, DevMaps P, DevLocal L, NewtonParams np, const double* __restrict__ u,
               const double* __restrict__ xloc, const double* __restrict__ gloc) {
    extern __shared__ double smem[];
    __shared__ int sflag[20];
    const int i = P.order[blockIdx.x];
    const int rowbase = P.off_n[i], n = P.off_n[i + 1] - rowbase;
    const int gbase = P.off_g[i], ng = P.off_g[i + 1] - gbase;
    const int ebase = P.off_e[i];
    const int kl = P.kl[i];
    double* vp = smem;
    double* rb = vp + n + ng;
    double* r0 = rb + n;
    double* dl = r0 + (np.mixed ? n : 0);
    double* red = dl + (np.mixed ? n : 0);
    double* mult = red + 24;
    double* W = mult + ((kl > 1 ? kl : 1) + 1);
    for (int a = threadIdx.x; a < n; a += blockDim.x)
        vp[a] = xloc ? xloc[rowbase + a] : u[P.l2g[rowbase + a]];
    for (int j = threadIdx.x; j < ng; j += blockDim.x)
        vp[n + j] = gloc ? gloc[gbase + j] : u[P.g2g[gbase + j]];
    __syncthreads();
    local_jacobian<ELAST>(M, P, n, rowbase, ebase, vp, L.jval);
    __syncthreads();
    const int status = local_factor(P, L, np, i, n, rowbase, W, mult, sflag, true) ? 3 : 0;
    if (threadIdx.x == 0) {
        L.its[i] = 0;
        L.status[i] = status;
    }
}

// out = v - Phi c: the coarse prolongation subtracted from v, one thread per
// dof (the rows of Phi held by the dof's owner, as in k_prolong).
__global__ void k_sub_coarse(int N, DevCoarse C, const double* __restrict__ cvec,
                             const double* __restrict__ v, double* __restrict__ out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    const int o = C.cown[g];
    const int k0 = C.off_k[o], nk = C.off_k[o + 1] - k0;
    const double* ph = C.phi + C.off_phi[o] + (int64_t)(C.cpos[g] - C.off_c[o]) * nk;
    double acc = 0.0;
    for (int l = 0; l < nk; ++l) acc += ph[l] * cvec[C.klist[k0 + l]];
    out[g] = v[g] - acc;
}

// Global residual F(u) (eq. 3): node-centric over incident elements.
__global__ void k_global_residual(DevMesh M, const double* __restrict__ u, double* __restrict__ F) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= M.N) return;
    if (M.dflag[g]) {
        F[g] = u[g] - M.dval[g];
        return;
    }
    double acc = 0.0;
    for (int k = M.nptr[g]; k < M.nptr[g + 1]; ++k) {
        const int code = M.nel[k];
        const int e = code >> 2, pos = code & 3;
        const double u0 = u[M.conn[3 * e]], u1 = u[M.conn[3 * e + 1]], u2 = u[M.conn[3 * e + 2]];
        const double U = u0 + u1 + u2;
        const double m = (U * U + u0 * u0 + u1 * u1 + u2 * u2) * (1.0 / 12.0);
        double g0, g1, g2;
        g_row(M.G6 + 6 * (size_t)e, pos, g0, g1, g2);
        acc += M.kappa[e] * (1.0 + M.beta * m) * (g0 * u0 + g1 * u1 + g2 * u2);
    }
    F[g] = acc - M.bload[g];
}

// Global residual of the elasticity problem: one thread per dof.
__global__ void k_global_residual_nh(DevMesh M, const double* __restrict__ u, double* __restrict__ F) {
    const int gd = blockIdx.x * blockDim.x + threadIdx.x;
    if (gd >= M.ndof) return;
    if (M.dflag[gd]) {
        F[gd] = u[gd] - M.dval[gd];
        return;
    }
    const int g = gd >> 1, c = gd & 1;
    double acc = 0.0;
    bool ok = true;
    for (int k = M.nptr[g]; k < M.nptr[g + 1]; ++k) {
        const int code = M.nel[k];
        const int e = code >> 2, pos = code & 3;
        double X[4][2], ue[4][2];
        nh_coords(M, e, X);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int gn = M.conn[4 * e + v];
            ue[v][0] = u[2 * gn];
            ue[v][1] = u[2 * gn + 1];
        }
        acc += nh_force(M, X, ue, pos, c, ok);
    }
    F[gd] = ok ? acc - M.bload[gd] : __builtin_nan("");
}

// Element geometry G = |T| grad(phi).grad(phi), coefficient and load vectors.
// With b_a = y_{a+1}-y_{a+2}, c_a = x_{a+2}-x_{a+1}: G_ab = (b_a b_b + c_a c_b)/(4|T|).
// Load by the edge-midpoint rule: l_a = |T|/6 (f(m_{a,a+1}) + f(m_{a-1,a})).
__global__ void k_p1_setup(int E, const int* __restrict__ conn, const double* __restrict__ xy,
                           const double* __restrict__ coef, const double* __restrict__ fmid,
                           double* __restrict__ G6, double* __restrict__ kappa,
                           double* __restrict__ eload, int* bad) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double x[3], y[3];
    for (int a = 0; a < 3; ++a) {
        x[a] = xy[2 * conn[3 * e + a]];
        y[a] = xy[2 * conn[3 * e + a] + 1];
    }
    double b[3], c[3];
    for (int a = 0; a < 3; ++a) {
        b[a] = y[(a + 1) % 3] - y[(a + 2) % 3];
        c[a] = x[(a + 2) % 3] - x[(a + 1) % 3];
    }
    const double area2 = b[0] * c[1] - b[1] * c[0];
    if (!(area2 > 0.0)) atomicOr(bad, 1);
    const double d = 2.0 * area2;
    double* o = G6 + 6 * (size_t)e;
    o[0] = (b[0] * b[0] + c[0] * c[0]) / d;
    o[1] = (b[1] * b[1] + c[1] * c[1]) / d;
    o[2] = (b[2] * b[2] + c[2] * c[2]) / d;
    o[3] = (b[0] * b[1] + c[0] * c[1]) / d;
    o[4] = (b[1] * b[2] + c[1] * c[2]) / d;
    o[5] = (b[2] * b[0] + c[2] * c[0]) / d;
    kappa[e] = coef ? coef[e] : 1.0;
    const double area = 0.5 * area2;
    if (fmid) {
        const double w = area / 6.0;
        const double f01 = fmid[3 * e], f12 = fmid[3 * e + 1], f20 = fmid[3 * e + 2];
        eload[3 * e] = w * (f01 + f20);
        eload[3 * e + 1] = w * (f01 + f12);
        eload[3 * e + 2] = w * (f12 + f20);
    } else {
        for (int a = 0; a < 3; ++a) eload[3 * e + a] = area / 3.0;
    }
}

__global__ void k_assemble_load(DevMesh M, double* __restrict__ b) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= M.N) return;
    double acc = 0.0;
    for (int k = M.nptr[g]; k < M.nptr[g + 1]; ++k) {
        const int code = M.nel[k];
        acc += M.eload[3 * (code >> 2) + (code & 3)];
    }
    b[g] = M.dflag[g] ? 0.0 : acc;
}

// ----------------------------------------------------------------------------
// GDSW coarse level.  Phi_i: dense |C_i| x |K_i| block of the basis on the
// closure C_i of subdomain i (K_i: the coarse functions touching it).
// ----------------------------------------------------------------------------

// Interface value of function k (local index in K_i) at closure dof ca.
__device__ __forceinline__ double iface_value(const DevCoarse& C, int ca, int k) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < NLS_CFUN; ++q)
        if (C.cfun[NLS_CFUN * ca + q] == k) v += C.cval[NLS_CFUN * ca + q];
    return v;
}

// Element stiffness row of closure dof (pos, c) of part-i element e at the
// nodal values w (global vector), columns as closure dofs: K row entries
// kr[b][k] for closure dof ELDOF(b, k).  Diffusion: K_T = kappa[(1+beta m) G
// + beta s (U + u)/6]; elasticity: the Q1 Neo-Hooke stiffness.
template <bool ELAST>
__device__ __forceinline__ void coarse_elem_row(const DevMesh& M, const DevCoarse& C, int cb, int e,
                                                int pos, int c, const double* __restrict__ w,
                                                double kr[4][2], int cn[4]) {
    const int ge = C.ne_gid[e];
    if (ELAST) {
        double X[4][2], ue[4][2];
        nh_coords(M, ge, X);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            cn[v] = C.ne_conn[4 * e + v];
            ue[v][0] = w ? w[C.cnode[cb + 2 * cn[v]]] : 0.0;
            ue[v][1] = w ? w[C.cnode[cb + 2 * cn[v] + 1]] : 0.0;
        }
        nh_stiff_row(M, X, ue, pos, c, kr);
    } else {
        double uu[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            cn[v] = C.ne_conn[3 * e + v];
            uu[v] = w ? w[C.cnode[cb + cn[v]]] : 0.0;
        }
        cn[3] = -1;
        const double U = uu[0] + uu[1] + uu[2];
        const double m = (U * U + uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]) * (1.0 / 12.0);
        double gr[3];
        g_row(M.G6 + 6 * (size_t)ge, pos, gr[0], gr[1], gr[2]);
        const double s = gr[0] * uu[0] + gr[1] * uu[1] + gr[2] * uu[2];
        const double kap = M.kappa[ge];
        const double coef = kap * (1.0 + M.beta * m);
        const double rk = M.beta * kap * s * (1.0 / 6.0);
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            kr[v][0] = coef * gr[v] + rk * (U + uu[v]);
            kr[v][1] = 0.0;
        }
        kr[3][0] = kr[3][1] = 0.0;
    }
}

// Harmonic extension Phi_I = -A_II^{-1} A_IG Phi_G with A = DF(u_lin), u_lin
// = 0 by default (one workgroup per subdomain; setup only).
template <int NPL, bool ELAST>
__global__ void __launch_bounds__(NLS_BLOCK)
k_gdsw_extend(DevMesh M, DevCoarse C, const double* __restrict__ ulin) {
    constexpr int D = ELAST ? 2 : 1, NV = ELAST ? 4 : 3;
    extern __shared__ double smem[];
    __shared__ int sflag[20];
    const int i = blockIdx.x;
    const int cb = C.off_c[i], nc = C.off_c[i + 1] - cb;
    const int k0 = C.off_k[i], nk = C.off_k[i + 1] - k0;
    const int ib = C.off_ni[i], ni = C.off_ni[i + 1] - ib;
    const int eb = C.off_ne[i];
    const int kl = C.ikl[i], ku = C.iku[i];
    double* ph = C.phi + C.off_phi[i];
    // interface and Dirichlet rows of Phi_i
    for (int t = threadIdx.x; t < nc * nk; t += blockDim.x) {
        const int a = t / nk, k = t - a * nk;
        ph[t] = C.ctype[cb + a] == 1 ? iface_value(C, cb + a, k) : 0.0;
    }
    if (ni == 0 || nk == 0) return;
    double* rhs = smem;
    double* red = rhs + ni;
    double* mult = red + 24;
    double* W = mult + ((kl > 1 ? kl : 1) + 1);
    // A_II values (DF at u_lin; at u = 0 when ulin is null)
    for (int r = threadIdx.x; r < ni; r += blockDim.x) {
        const int ca = C.inode[ib + r];
        const int js = C.iptr[ib + r], je = C.iptr[ib + r + 1];
        for (int s = js; s < je; ++s) C.ival[s] = 0.0;
        for (int q = C.cinc_ptr[cb + ca]; q < C.cinc_ptr[cb + ca + 1]; ++q) {
            const int code = C.cinc[q];
            const int e = eb + (code >> 2), pos = code & 3;
            double kr[4][2];
            int cn[4];
            coarse_elem_row<ELAST>(M, C, cb, e, pos, ca % D, ulin, kr, cn);
#pragma unroll
            for (int b = 0; b < NV; ++b)
#pragma unroll
                for (int kk = 0; kk < D; ++kk) {
                    const int cc = C.iidx[cb + D * cn[b] + kk];
                    if (cc < 0) continue;
                    for (int s = js; s < je; ++s)
                        if (C.icol[s] == cc) { C.ival[s] += kr[b][kk]; break; }
                }
        }
    }
    __syncthreads();
    if (band_lu_auto<double>(ni, kl, ku, C.iptr + ib, C.icol, C.ival, W, mult, sflag,
                        C.iU + C.off_iu[i], C.iL + C.off_il[i], C.ipiv + ib)) {
        if (threadIdx.x == 0) atomicOr(C.flag, 1);
        return;
    }
    for (int k = 0; k < nk; ++k) {
        for (int r = threadIdx.x; r < ni; r += blockDim.x) {
            const int ca = C.inode[ib + r];
            double acc = 0.0;
            for (int q = C.cinc_ptr[cb + ca]; q < C.cinc_ptr[cb + ca + 1]; ++q) {
                const int code = C.cinc[q];
                const int e = eb + (code >> 2), pos = code & 3;
                double kr[4][2];
                int cn[4];
                coarse_elem_row<ELAST>(M, C, cb, e, pos, ca % D, ulin, kr, cn);
#pragma unroll
                for (int b = 0; b < NV; ++b)
#pragma unroll
                    for (int kk = 0; kk < D; ++kk) {
                        const int cd = cb + D * cn[b] + kk;
                        if (C.ctype[cd] == 1) acc -= kr[b][kk] * iface_value(C, cd, k);
                    }
            }
            rhs[r] = acc;
        }
        __syncthreads();
        if (threadIdx.x < 64)
            band_solve_wave<double, NPL>(ni, kl, ku, C.iU + C.off_iu[i], C.iL + C.off_il[i],
                                         C.ipiv + ib, rhs);
        __syncthreads();
        for (int r = threadIdx.x; r < ni; r += blockDim.x)
            ph[(int64_t)C.inode[ib + r] * nk + k] = rhs[r];
        __syncthreads();
    }
}

// w = u - Phi c at every dof (owner's block).
__global__ void k_coarse_w(int N, DevCoarse C, const double* __restrict__ u, double* __restrict__ w) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    const int o = C.cown[g];
    const int k0 = C.off_k[o], nk = C.off_k[o + 1] - k0;
    const double* ph = C.phi + C.off_phi[o] + (int64_t)(C.cpos[g] - C.off_c[o]) * nk;
    double acc = 0.0;
    for (int l = 0; l < nk; ++l) acc += ph[l] * C.c[C.klist[k0 + l]];
    w[g] = u[g] - acc;
}

// Per subdomain: gblk_i = Phi_i^T q_i where, on closure dofs,
//   mode 0: q = sum over part-i elements of the element residual at w
//           (so that sum_i gblk_i = Phi^T F(w)); nodal loads are counted
//           by the owner subdomain of their dof;
//   mode 1: q = sum over part-i elements of K_T(w) v_T
//           (so that sum_i gblk_i = Phi^T DF(w) v).
template <bool ELAST>
__global__ void __launch_bounds__(NLS_BLOCK)
k_coarse_q(DevMesh M, DevCoarse C, const double* __restrict__ w, const double* __restrict__ v, int mode) {
    constexpr int D = ELAST ? 2 : 1, NV = ELAST ? 4 : 3;
    extern __shared__ double smem[];
    const int i = blockIdx.x;
    const int cb = C.off_c[i], nc = C.off_c[i + 1] - cb;
    const int k0 = C.off_k[i], nk = C.off_k[i + 1] - k0;
    const int eb = C.off_ne[i];
    double* q = smem;
    for (int a = threadIdx.x; a < nc; a += blockDim.x) {
        double acc = 0.0;
        if (C.ctype[cb + a] != 2) {
            const int c = a % D;
            bool ok = true;
            for (int t = C.cinc_ptr[cb + a]; t < C.cinc_ptr[cb + a + 1]; ++t) {
                const int code = C.cinc[t];
                const int e = eb + (code >> 2), pos = code & 3;
                const int ge = C.ne_gid[e];
                if (ELAST) {
                    if (mode == 0) {
                        double X[4][2], ue[4][2];
                        nh_coords(M, ge, X);
#pragma unroll
                        for (int vv = 0; vv < 4; ++vv) {
                            const int cn = C.ne_conn[4 * e + vv];
                            ue[vv][0] = w[C.cnode[cb + 2 * cn]];
                            ue[vv][1] = w[C.cnode[cb + 2 * cn + 1]];
                        }
                        acc += nh_force(M, X, ue, pos, c, ok);
                    } else {
                        double kr[4][2];
                        int cn[4];
                        coarse_elem_row<true>(M, C, cb, e, pos, c, w, kr, cn);
#pragma unroll
                        for (int b = 0; b < 4; ++b)
#pragma unroll
                            for (int kk = 0; kk < 2; ++kk)
                                acc += kr[b][kk] * v[C.cnode[cb + 2 * cn[b] + kk]];
                    }
                } else {
                    double uu[3], vv[3];
                    for (int cc = 0; cc < 3; ++cc) {
                        const int gn = C.cnode[cb + C.ne_conn[3 * e + cc]];
                        uu[cc] = w[gn];
                        vv[cc] = mode ? v[gn] : 0.0;
                    }
                    const double U = uu[0] + uu[1] + uu[2];
                    const double m = (U * U + uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]) * (1.0 / 12.0);
                    double gr[3];
                    g_row(M.G6 + 6 * (size_t)ge, pos, gr[0], gr[1], gr[2]);
                    const double s = gr[0] * uu[0] + gr[1] * uu[1] + gr[2] * uu[2];
                    const double kap = M.kappa[ge];
                    const double coef = kap * (1.0 + M.beta * m);
                    if (mode == 0) {
                        acc += coef * s - M.eload[3 * ge + pos];
                    } else {
                        const double rk = M.beta * kap * s * (1.0 / 6.0);
                        for (int cc = 0; cc < 3; ++cc) acc += (coef * gr[cc] + rk * (U + uu[cc])) * vv[cc];
                    }
                }
            }
            if (ELAST && mode == 0) {
                const int gd = C.cnode[cb + a];
                if (C.cown[gd] == i) acc -= M.bload[gd];
                if (!ok) {
                    acc = __builtin_nan("");
                    atomicOr(C.flag, 2);  // det F <= 0
                }
            }
        }
        q[a] = acc;
    }
    (void)NV;
    __syncthreads();
    const double* ph = C.phi + C.off_phi[i];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int k = wv; k < nk; k += nw) {
        double acc = 0.0;
        for (int a = lane; a < nc; a += 64) acc += ph[(int64_t)a * nk + k] * q[a];
        acc = wave_sum(acc);
        if (lane == 0) C.gblk[k0 + k] = acc;
    }
}

// Per subdomain Galerkin block A_i = Phi_i^T K_i(w) Phi_i (K_i: part-i
// elements), first part: the rows Z_i = K_i(w) Phi_i.  With with_y, also
// Y_i = K_i(w)^T Phi_i, so that the coarse term of the tangent,
// Phi^T DF(u_0) v = sum_i Y_i^T v_i, is a GEMV.  Grid (nsub, Q): block y
// takes the closure rows [y nc / Q, (y + 1) nc / Q).
template <bool ELAST>
__global__ void __launch_bounds__(NLS_BLOCK)
k_coarse_galerkin(DevMesh M, DevCoarse C, const double* __restrict__ w, int with_y) {
    const int i = blockIdx.x;
    const int cb = C.off_c[i], nc = C.off_c[i + 1] - cb;
    const int a0 = (int)((int64_t)nc * blockIdx.y / gridDim.y);
    const int a1 = (int)((int64_t)nc * (blockIdx.y + 1) / gridDim.y);
    const int k0 = C.off_k[i], nk = C.off_k[i + 1] - k0;
    const int eb = C.off_ne[i];
    const double* ph = C.phi + C.off_phi[i];
    double* z = C.zbuf + C.off_phi[i];
    if (ELAST) {
        // the element stiffness is symmetric, so Y_i = K_i^T Phi_i = Z_i,
        // with rows on every closure dof (Dirichlet ones included: Phi is
        // zero there, so they do not change A_i, but Y needs them)
        double* y = C.ybuf + C.off_phi[i];
        for (int a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
            double* zr = z + (int64_t)a * nk;
            for (int l = 0; l < nk; ++l) zr[l] = 0.0;
            {
                for (int t = C.cinc_ptr[cb + a]; t < C.cinc_ptr[cb + a + 1]; ++t) {
                    const int code = C.cinc[t];
                    const int e = eb + (code >> 2), pos = code & 3;
                    double kr[4][2];
                    int cn[4];
                    coarse_elem_row<true>(M, C, cb, e, pos, a & 1, w, kr, cn);
#pragma unroll
                    for (int b = 0; b < 4; ++b)
#pragma unroll
                        for (int kk = 0; kk < 2; ++kk) {
                            const double* pr = ph + (int64_t)(2 * cn[b] + kk) * nk;
                            for (int l = 0; l < nk; ++l) zr[l] += kr[b][kk] * pr[l];
                        }
                }
            }
            if (with_y)
                for (int l = 0; l < nk; ++l) y[(int64_t)l * nc + a] = zr[l];
        }
        return;
    }
    // rows accumulated in registers where the subdomain meets at most
    // GAL_K coarse functions (the general loop below otherwise)
    constexpr int GAL_K = 40;
    if (nk <= GAL_K) {
        for (int a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
            double acc[GAL_K];
#pragma unroll
            for (int l = 0; l < GAL_K; ++l) acc[l] = 0.0;
            const int t0 = C.ctype[cb + a] == 2 ? 0 : C.cinc_ptr[cb + a];
            const int t1 = C.ctype[cb + a] == 2 ? 0 : C.cinc_ptr[cb + a + 1];
            for (int t = t0; t < t1; ++t) {
                const int code = C.cinc[t];
                const int e = eb + (code >> 2), pos = code & 3;
                const int ge = C.ne_gid[e];
                double uu[3];
                int cn[3];
                for (int c = 0; c < 3; ++c) {
                    cn[c] = C.ne_conn[3 * e + c];
                    uu[c] = w[C.cnode[cb + cn[c]]];
                }
                const double U = uu[0] + uu[1] + uu[2];
                const double m = (U * U + uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]) * (1.0 / 12.0);
                double gr[3];
                g_row(M.G6 + 6 * (size_t)ge, pos, gr[0], gr[1], gr[2]);
                const double s = gr[0] * uu[0] + gr[1] * uu[1] + gr[2] * uu[2];
                const double kap = M.kappa[ge];
                const double coef = kap * (1.0 + M.beta * m);
                const double rk = M.beta * kap * s * (1.0 / 6.0);
                for (int c = 0; c < 3; ++c) {
                    const double K = coef * gr[c] + rk * (U + uu[c]);
                    const double* pr = ph + (int64_t)cn[c] * nk;
#pragma unroll
                    for (int l = 0; l < GAL_K; ++l)
                        if (l < nk) acc[l] += K * pr[l];
                }
            }
            double* zr = z + (int64_t)a * nk;
#pragma unroll
            for (int l = 0; l < GAL_K; ++l)
                if (l < nk) zr[l] = acc[l];
        }
        if (with_y) {
            double* y = C.ybuf + C.off_phi[i];
            for (int c = a0 + threadIdx.x; c < a1; c += blockDim.x) {
                double acc[GAL_K];
#pragma unroll
                for (int l = 0; l < GAL_K; ++l) acc[l] = 0.0;
                for (int t = C.cinc_ptr[cb + c]; t < C.cinc_ptr[cb + c + 1]; ++t) {
                    const int code = C.cinc[t];
                    const int e = eb + (code >> 2), pc = code & 3;
                    const int ge = C.ne_gid[e];
                    double uu[3];
                    int cn[3];
                    for (int a = 0; a < 3; ++a) {
                        cn[a] = C.ne_conn[3 * e + a];
                        uu[a] = w[C.cnode[cb + cn[a]]];
                    }
                    const double U = uu[0] + uu[1] + uu[2];
                    const double m = (U * U + uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]) * (1.0 / 12.0);
                    const double kap = M.kappa[ge];
                    const double coef = kap * (1.0 + M.beta * m);
                    for (int a = 0; a < 3; ++a) {
                        double gr[3];
                        g_row(M.G6 + 6 * (size_t)ge, a, gr[0], gr[1], gr[2]);
                        const double sa = gr[0] * uu[0] + gr[1] * uu[1] + gr[2] * uu[2];
                        // K_T[a][pc]
                        const double K = coef * gr[pc] + M.beta * kap * sa * (U + uu[pc]) * (1.0 / 6.0);
                        const double* pr = ph + (int64_t)cn[a] * nk;
#pragma unroll
                        for (int l = 0; l < GAL_K; ++l)
                            if (l < nk) acc[l] += K * pr[l];
                    }
                }
#pragma unroll
                for (int l = 0; l < GAL_K; ++l)
                    if (l < nk) y[(int64_t)l * nc + c] = acc[l];
            }
        }
        return;
    }
    for (int a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
        double* zr = z + (int64_t)a * nk;
        for (int l = 0; l < nk; ++l) zr[l] = 0.0;
        if (C.ctype[cb + a] == 2) continue;
        for (int t = C.cinc_ptr[cb + a]; t < C.cinc_ptr[cb + a + 1]; ++t) {
            const int code = C.cinc[t];
            const int e = eb + (code >> 2), pos = code & 3;
            const int ge = C.ne_gid[e];
            double uu[3];
            int cn[3];
            for (int c = 0; c < 3; ++c) {
                cn[c] = C.ne_conn[3 * e + c];
                uu[c] = w[C.cnode[cb + cn[c]]];
            }
            const double U = uu[0] + uu[1] + uu[2];
            const double m = (U * U + uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]) * (1.0 / 12.0);
            double gr[3];
            g_row(M.G6 + 6 * (size_t)ge, pos, gr[0], gr[1], gr[2]);
            const double s = gr[0] * uu[0] + gr[1] * uu[1] + gr[2] * uu[2];
            const double kap = M.kappa[ge];
            const double coef = kap * (1.0 + M.beta * m);
            const double rk = M.beta * kap * s * (1.0 / 6.0);
            for (int c = 0; c < 3; ++c) {
                const double K = coef * gr[c] + rk * (U + uu[c]);
                const double* pr = ph + (int64_t)cn[c] * nk;
                for (int l = 0; l < nk; ++l) zr[l] += K * pr[l];
            }
        }
    }
    if (with_y) {
        double* y = C.ybuf + C.off_phi[i];
        for (int c = a0 + threadIdx.x; c < a1; c += blockDim.x) {
            for (int l = 0; l < nk; ++l) y[(int64_t)l * nc + c] = 0.0;
            for (int t = C.cinc_ptr[cb + c]; t < C.cinc_ptr[cb + c + 1]; ++t) {
                const int code = C.cinc[t];
                const int e = eb + (code >> 2), pc = code & 3;
                const int ge = C.ne_gid[e];
                double uu[3];
                int cn[3];
                for (int a = 0; a < 3; ++a) {
                    cn[a] = C.ne_conn[3 * e + a];
                    uu[a] = w[C.cnode[cb + cn[a]]];
                }
                const double U = uu[0] + uu[1] + uu[2];
                const double m = (U * U + uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]) * (1.0 / 12.0);
                const double kap = M.kappa[ge];
                const double coef = kap * (1.0 + M.beta * m);
                for (int a = 0; a < 3; ++a) {
                    double gr[3];
                    g_row(M.G6 + 6 * (size_t)ge, a, gr[0], gr[1], gr[2]);
                    const double sa = gr[0] * uu[0] + gr[1] * uu[1] + gr[2] * uu[2];
                    // K_T[a][pc]
                    const double K = coef * gr[pc] + M.beta * kap * sa * (U + uu[pc]) * (1.0 / 6.0);
                    const double* pr = ph + (int64_t)cn[a] * nk;
                    for (int l = 0; l < nk; ++l) y[(int64_t)l * nc + c] += K * pr[l];
                }
            }
        }
    }
}

// Second part: A_i[k][l] = sum_a Phi_i[a][k] Z_i[a][l], one wavefront per
// entry; grid (nsub, Q), block y takes every Q-th group of entries.
__global__ void __launch_bounds__(NLS_BLOCK)
k_coarse_galerkin_sum(DevCoarse C) {
    const int i = blockIdx.x;
    const int nc = C.off_c[i + 1] - C.off_c[i];
    const int nk = C.off_k[i + 1] - C.off_k[i];
    const double* ph = C.phi + C.off_phi[i];
    const double* z = C.zbuf + C.off_phi[i];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int kk = wv + nw * blockIdx.y; kk < nk * nk; kk += nw * gridDim.y) {
        const int k = kk / nk, l = kk - k * nk;
        double acc = 0.0;
        for (int a = lane; a < nc; a += 64) acc += ph[(int64_t)a * nk + k] * z[(int64_t)a * nk + l];
        acc = wave_sum(acc);
        if (lane == 0) C.ablk[C.off_kk[i] + kk] = acc;
    }
}

// gblk_i = Y_i^T v on the closure of subdomain i (coarse term of the tangent);
// Y_i is stored column by column (Y[k * nc + c]), so the lanes read along c.
// The closure values of v are gathered into LDS once per block, so that the
// dot products stream Y_i alone, four loads per lane in flight.
// Grid (nsub, Q): one wavefront per coarse function, spread over Q blocks.
__global__ void __launch_bounds__(NLS_BLOCK)
k_coarse_ty(DevCoarse C, const double* __restrict__ v) {
    extern __shared__ double sv[];
    const int i = blockIdx.x;
    const int cb = C.off_c[i], nc = C.off_c[i + 1] - cb;
    const int k0 = C.off_k[i], nk = C.off_k[i + 1] - k0;
    const double* y = C.ybuf + C.off_phi[i];
    for (int c = threadIdx.x; c < nc; c += blockDim.x) sv[c] = v[C.cnode[cb + c]];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int k = wv + nw * blockIdx.y; k < nk; k += nw * gridDim.y) {
        const double* yk = y + (int64_t)k * nc;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int c = lane;
        for (; c + 192 < nc; c += 256) {
            a0 += yk[c] * sv[c];
            a1 += yk[c + 64] * sv[c + 64];
            a2 += yk[c + 128] * sv[c + 128];
            a3 += yk[c + 192] * sv[c + 192];
        }
        for (; c < nc; c += 64) a0 += yk[c] * sv[c];
        const double acc = wave_sum((a0 + a1) + (a2 + a3));
        if (lane == 0) C.gblk[k0 + k] = acc;
    }
}

// sum over t in [t0, t1) of val[src[t]], in that order: the first 16
// indices and values are loaded before any is added, so the loads overlap
// instead of each waiting for the one before
__device__ __forceinline__ double sum_pieces(const double* __restrict__ val,
                                             const int* __restrict__ src, int t0, int t1) {
    constexpr int GM = 16;
    if (t1 <= t0) return 0.0;
    int ix[GM];
#pragma unroll
    for (int q = 0; q < GM; ++q) ix[q] = src[min(t0 + q, t1 - 1)];
    double v[GM];
#pragma unroll
    for (int q = 0; q < GM; ++q) v[q] = val[ix[q]];
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < GM; ++q)
        if (t0 + q < t1) acc += v[q];
    for (int t = t0 + GM; t < t1; ++t) acc += val[src[t]];
    return acc;
}

// Deterministic assembly: rhs (band order) from the gblk pieces, and, if
// with_matrix, the CSR values of A0 from the Galerkin blocks.  Also writes
// ||rhs||_2 to scal[0] (single block).
// Block 0 forms rhs and its norm; with_matrix, blocks 1.. form the CSR
// values, one entry per thread.
__global__ void __launch_bounds__(NLS_BLOCK)
k_coarse_assemble(DevCoarse C, int with_matrix) {
    __shared__ double red[24];
    if (blockIdx.x > 0) {
        const int s = (blockIdx.x - 1) * blockDim.x + threadIdx.x;
        if (with_matrix && s < C.a0ptr[C.n0])
            C.a0val[s] = sum_pieces(C.ablk, C.a0src, C.a0src_ptr[s], C.a0src_ptr[s + 1]);
        return;
    }
    double ss = 0.0;
    for (int k = threadIdx.x; k < C.n0; k += blockDim.x) {
        const double acc = sum_pieces(C.gblk, C.gsrc, C.gsrc_ptr[k], C.gsrc_ptr[k + 1]);
        C.rhs[C.perm[k]] = acc;
        ss += acc * acc;
    }
    ss = block_sum(ss, red);
    if (threadIdx.x == 0) C.scal[0] = sqrt(ss);
}

// One workgroup per diagonal block of A0 (independent problems give one
// block each): (factor and) solve A0 d = rhs in place (band order).
// A factorisation carries the right-hand side along (its forward
// substitution), so only the backward substitution remains; the solves run
// on the whole workgroup with the LU's window (free by then) as staging.
template <int NPL>
__global__ void __launch_bounds__(NLS_BLOCK)
k_coarse_lu(DevCoarse C, int factor, int lds_bytes) {
    extern __shared__ double smem[];
    __shared__ int sflag[20];
    const int b = blockIdx.x;
    const int off = C.boff[b], n = C.boff[b + 1] - off, kl = C.bkl[b], ku = C.bku[b];
    double* x = smem;
    double* mult = x + n;
    double* W = mult + ((kl > 1 ? kl : 1) + 1);
    const int stage_bytes = lds_bytes - (int)((W - smem) * sizeof(double));
    double* U = C.a0U + C.offU[b];
    double* L = C.a0L + C.offL[b];
    int* piv = C.a0piv + off;
    for (int k = threadIdx.x; k < n; k += blockDim.x) x[k] = C.rhs[off + k];
    __syncthreads();
    if (factor) {
        if (band_lu_auto<double>(n, kl, ku, C.a0ptr + off, C.a0col, C.a0val, W, mult, sflag, U, L,
                                 piv, off, 0, x)) {
            if (threadIdx.x == 0) atomicOr(C.flag, 2);
        }
        __syncthreads();
    }
    band_solve_group<double, NPL>(n, kl, ku, U, L, piv, x, W, stage_bytes, factor != 0);
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x) C.rhs[off + k] = x[k];
}

// c += d (d in band order); scal[1] = max|d|, scal[2] = max|c| (new c).
__global__ void __launch_bounds__(NLS_BLOCK) k_coarse_update(DevCoarse C) {
    __shared__ double red[24];
    double dm = 0.0, cmx = 0.0;
    for (int k = threadIdx.x; k < C.n0; k += blockDim.x) {
        const double d = C.rhs[C.perm[k]];
        const double c = C.c[k] + d;
        C.c[k] = c;
        dm = fmax(dm, fabs(d));
        cmx = fmax(cmx, fabs(c));
    }
    dm = block_max(dm, red);
    cmx = block_max(cmx, red);
    if (threadIdx.x == 0) {
        C.scal[1] = dm;
        C.scal[2] = cmx;
    }
}

// cout[k] = rhs[perm[k]] (band order back to coarse ids).
__global__ void k_coarse_scatter(DevCoarse C, const double* __restrict__ src, double* __restrict__ cout) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < C.n0) cout[k] = src[C.perm[k]];
}

// ----------------------------------------------------------------------------
// Vector kernels (GMRES).  partial sums per block, then a fixed-order sum.
// ----------------------------------------------------------------------------
// partial[b m + j] = V_j . w over block b's chunk: each wavefront takes its
// own vectors j (wv, wv + 4, ...) over the whole chunk, four independent
// loads per lane in flight, and reduces them itself (fixed order).
__global__ void __launch_bounds__(NLS_BLOCK)
k_mdot_partial(const double* __restrict__ V, int64_t ld, int m, const double* __restrict__ w,
               int n, double* __restrict__ partial) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int chunk = (n + gridDim.x - 1) / gridDim.x;
    const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    for (int j = wv; j < m; j += nw) {
        const double* vj = V + (int64_t)j * ld;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int t = lo + lane;
        for (; t + 192 < hi; t += 256) {
            a0 += vj[t] * w[t];
            a1 += vj[t + 64] * w[t + 64];
            a2 += vj[t + 128] * w[t + 128];
            a3 += vj[t + 192] * w[t + 192];
        }
        for (; t < hi; t += 64) a0 += vj[t] * w[t];
        const double sum = wave_sum((a0 + a1) + (a2 + a3));
        if (lane == 0) partial[(int64_t)blockIdx.x * m + j] = sum;
    }
}

__global__ void __launch_bounds__(256)
k_mdot_final(const double* __restrict__ partial, int nb, int m, double* __restrict__ out) {
    __shared__ double red[24];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += partial[(int64_t)b * m + j];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[j] = s;
}

// w -= sign * sum_j h[j] V[j]  (sign = +1)   or  w += sum_j h[j] V[j] (sign = -1)
__global__ void k_maxpy(const double* __restrict__ V, int64_t ld, int m, const double* __restrict__ h,
                        double* __restrict__ w, int n, double sign) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double acc = 0.0;
    for (int j = 0; j < m; ++j) acc += h[j] * V[(int64_t)j * ld + t];
    w[t] -= sign * acc;
}

// w -= sum_j h[j] V[j] and the partial sums of ||w||^2 over the same block
// chunks as k_mdot_partial (so k_mdot_final with m = 1 completes the norm).
__global__ void __launch_bounds__(NLS_BLOCK)
k_maxpy_norm(const double* __restrict__ V, int64_t ld, int m, const double* __restrict__ h,
             double* __restrict__ w, int n, double* __restrict__ partial) {
    __shared__ double red[24];
    const int chunk = (n + gridDim.x - 1) / gridDim.x;
    const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double ss = 0.0;
    for (int t = lo + threadIdx.x; t < hi; t += blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < m; ++j) acc += h[j] * V[(int64_t)j * ld + t];
        const double x = w[t] - acc;
        w[t] = x;
        ss += x * x;
    }
    ss = block_sum(ss, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = ss;
}

// ---------------------------------------------------------------------------
// Arnoldi step kernels that finish the previous reduction themselves: every
// block adds up the partial sums of the dot products in the same fixed order
// (one wavefront per entry), so all blocks hold identical totals and no
// separate final launch is needed; block 0 also stores the totals.
// ---------------------------------------------------------------------------
__device__ void gmres_givens_step(const GmresDev& G, int j);

__device__ __forceinline__ void block_totals(const double* __restrict__ partial, int nb, int m,
                                             double* hs, double* out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int j = wv; j < m; j += nw) {
        double s = 0.0;
        for (int b = lane; b < nb; b += 64) s += partial[(int64_t)b * m + j];
        s = wave_sum(s);
        if (lane == 0) {
            hs[j] = s;
            if (blockIdx.x == 0) out[j] = s;
        }
    }
    __syncthreads();
}

// h = totals of partial; w -= V h on this block's chunk (the chunks of
// k_mdot_partial with gridDim.x blocks), then the chunk's partial dot
// products of the updated w with V into partial2: the update and the next
// k_mdot_partial in one launch, with the same operations per element and
// per partial sum as two separate launches
__global__ void __launch_bounds__(NLS_BLOCK)
k_maxpy_mdot_totals(const double* __restrict__ V, int64_t ld, int m,
                    const double* __restrict__ partial, int nb, double* __restrict__ hout,
                    double* __restrict__ w, int n, double* __restrict__ partial2) {
    extern __shared__ double hs[];
    block_totals(partial, nb, m, hs, hout);
    const int chunk = (n + gridDim.x - 1) / gridDim.x;
    const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    for (int t = lo + threadIdx.x; t < hi; t += blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < m; ++j) acc += hs[j] * V[(int64_t)j * ld + t];
        w[t] -= acc;
    }
    __threadfence_block();
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int j = wv; j < m; j += nw) {
        const double* vj = V + (int64_t)j * ld;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int t = lo + lane;
        for (; t + 192 < hi; t += 256) {
            a0 += vj[t] * w[t];
            a1 += vj[t + 64] * w[t + 64];
            a2 += vj[t + 128] * w[t + 128];
            a3 += vj[t + 192] * w[t + 192];
        }
        for (; t < hi; t += 64) a0 += vj[t] * w[t];
        const double sum = wave_sum((a0 + a1) + (a2 + a3));
        if (lane == 0) partial2[(int64_t)blockIdx.x * m + j] = sum;
    }
}

// h = totals of partial; w -= V h and partial sums of ||w||^2 into pnorm
// (the chunks of k_mdot_partial with gridDim.x blocks)
__global__ void __launch_bounds__(NLS_BLOCK)
k_maxpy_norm_totals(const double* __restrict__ V, int64_t ld, int m,
                    const double* __restrict__ partial, int nb, double* __restrict__ hout,
                    double* __restrict__ w, int n, double* __restrict__ pnorm) {
    extern __shared__ double hs[];
    __shared__ double red[24];
    block_totals(partial, nb, m, hs, hout);
    const int chunk = (n + gridDim.x - 1) / gridDim.x;
    const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double ss = 0.0;
    for (int t = lo + threadIdx.x; t < hi; t += blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < m; ++j) acc += hs[j] * V[(int64_t)j * ld + t];
        const double x = w[t] - acc;
        w[t] = x;
        ss += x * x;
    }
    ss = block_sum(ss, red);
    if (threadIdx.x == 0) pnorm[blockIdx.x] = ss;
}

// ||w||^2 = total of pnorm (nb); y = w / ||w||; block 0 stores ||w||^2 and
// its first thread applies rotation j of the Arnoldi column
__global__ void __launch_bounds__(NLS_BLOCK)
k_scale_givens_totals(const double* __restrict__ x, double* __restrict__ y, int n,
                      const double* __restrict__ pnorm, int nb, GmresDev G, int j) {
    __shared__ double tot;
    if (threadIdx.x < 64) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += 64) s += pnorm[b];
        s = wave_sum(s);
        if (threadIdx.x == 0) {
            tot = s;
            if (blockIdx.x == 0) {
                G.hn2[0] = s;
                gmres_givens_step(G, j);
            }
        }
    }
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double d = sqrt(tot);
    y[t] = (d > 0.0) ? x[t] / d : 0.0;
}

// rhs[perm[k]] = sum of the coarse blocks' entries of row k (no norm).
__global__ void k_coarse_gather(DevCoarse C) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= C.n0) return;
    C.rhs[C.perm[k]] = sum_pieces(C.gblk, C.gsrc, C.gsrc_ptr[k], C.gsrc_ptr[k + 1]);
}

__global__ void k_scale_by(const double* __restrict__ x, const double* __restrict__ dsq,
                           double* __restrict__ y, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double d = sqrt(*dsq);
    y[t] = (d > 0.0) ? x[t] / d : 0.0;
}

__global__ void k_axpy(double a, const double* __restrict__ x, double* __restrict__ y, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] += a * x[t];
}


__global__ void __launch_bounds__(NLS_BLOCK)
k_max_abs_partial(const double* __restrict__ x, int n, double* __restrict__ partial) {
    __shared__ double red[24];
    double m = 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
        m = fmax(m, fabs(x[t]));
    m = block_max(m, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ void k_max_final(const double* __restrict__ partial, int nb, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double m = 0.0;
    for (int b = 0; b < nb; ++b) m = fmax(m, partial[b]);
    *out = m;
}

__global__ void k_any_status(const int* __restrict__ st, int n, int* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int first = -1, code = 0;
    for (int i = 0; i < n; ++i)
        if (st[i] != 0) { first = i; code = st[i]; break; }
    out[0] = first;
    out[1] = code;
}

// Column j of the Arnoldi process on the device: H(:,j) = h1 + h2 (the two
// classical Gram-Schmidt passes), H(j+1,j) = ||w||; the previous rotations
// are applied, rotation j is formed and the residual vector g updated.
// Columns after the cycle has converged (st[0] != 0) are ignored.
__device__ void gmres_givens_step(const GmresDev& G, int j) {
    if (G.st[0] != 0) return;
    const int m = G.m;
    double* H = G.H;
    // the entry that rotation i leaves in row i + 1 is carried in a register
    // into rotation i + 1 (same arithmetic as storing and reloading it)
    double a = G.h1[0] + G.h2[0];
    for (int i = 0; i < j; ++i) {
        const double b = G.h1[i + 1] + G.h2[i + 1];
        H[i * m + j] = G.cs[i] * a + G.sn[i] * b;
        a = -G.sn[i] * a + G.cs[i] * b;
    }
    const double b = sqrt(G.hn2[0]);
    const double den = hypot(a, b);
    const double c = den > 0.0 ? a / den : 1.0, sn = den > 0.0 ? b / den : 0.0;
    G.cs[j] = c;
    G.sn[j] = sn;
    H[j * m + j] = den;
    H[(j + 1) * m + j] = 0.0;
    const double gj = G.g[j];
    G.g[j + 1] = -sn * gj;
    G.g[j] = c * gj;
    G.st[1] = j + 1;
    const double r = fabs(G.g[j + 1]);
    if (!(r == r) || isinf(r)) G.st[0] = -(j + 1);
    else if (r <= G.tol[0]) G.st[0] = j + 1;
}



inline int nblocks(int n, int b = NLS_BLOCK) { return (n + b - 1) / b; }

template <typename K>
hipError_t set_lds(K kernel, int bytes) {
    if (bytes > 64 * 1024)
        return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return hipSuccess;
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_p1_setup(const DevMesh& M, const double* xy, const double* elem_coef,
                           const double* elem_load, double* G6, double* kappa, double* eload,
                           int* bad, hipStream_t s) {
    if (M.E == 0) return hipSuccess;
    k_p1_setup<<<nblocks(M.E), NLS_BLOCK, 0, s>>>(M.E, M.conn, xy, elem_coef, elem_load, G6,
                                                  kappa, eload, bad);
    return hipGetLastError();
}

hipError_t launch_assemble_load(const DevMesh& M, double* bload, hipStream_t s) {
    k_assemble_load<<<nblocks(M.N), NLS_BLOCK, 0, s>>>(M, bload);
    return hipGetLastError();
}

hipError_t launch_global_residual(const DevMesh& M, const double* u, double* F, hipStream_t s) {
    if (M.kind == NLS_PROBLEM_NEOHOOKE)
        k_global_residual_nh<<<nblocks(M.ndof), NLS_BLOCK, 0, s>>>(M, u, F);
    else
        k_global_residual<<<nblocks(M.N), NLS_BLOCK, 0, s>>>(M, u, F);
    return hipGetLastError();
}

hipError_t launch_local_newton(const DevMesh& M, const DevMaps& P, const DevLocal& L,
                               const NewtonParams& np, const double* u, int nblk, int lds_bytes,
                               int npl, hipStream_t s) {
    hipError_t e;
#define NLS_LN(NPL, EL)                                                              \
    e = set_lds(k_local_newton<NPL, EL>, lds_bytes);                                 \
    if (e != hipSuccess) return e;                                                   \
    k_local_newton<NPL, EL><<<nblk, NLS_BLOCK, lds_bytes, s>>>(M, P, L, np, u, lds_bytes);
    if (M.kind == NLS_PROBLEM_NEOHOOKE) {
        if (npl <= 1) { NLS_LN(1, true) } else if (npl == 2) { NLS_LN(2, true) } else { NLS_LN(4, true) }
    } else {
        if (npl <= 1) { NLS_LN(1, false) } else if (npl == 2) { NLS_LN(2, false) } else { NLS_LN(4, false) }
    }
#undef NLS_LN
    return hipGetLastError();
}

hipError_t launch_local_assemble(const DevMesh& M, const DevMaps& P, const double* u, double* r,
                                 double* jval, int max_rows, int lds_bytes, hipStream_t s) {
    // blocks per subdomain, and 8 XCD slots each holding ceil(nsub / 8)
    // subdomains' worth of blocks
    const int Q = (max_rows + 255) / 256;
    const int grid = 8 * Q * ((P.nsub + 7) / 8);
    hipError_t e;
    if (M.kind == NLS_PROBLEM_NEOHOOKE) {
        e = set_lds(k_local_assemble<true>, lds_bytes);
        if (e != hipSuccess) return e;
        k_local_assemble<true><<<grid, 256, lds_bytes, s>>>(M, P, u, r, jval, Q);
    } else {
        e = set_lds(k_local_assemble<false>, lds_bytes);
        if (e != hipSuccess) return e;
        k_local_assemble<false><<<grid, 256, lds_bytes, s>>>(M, P, u, r, jval, Q);
    }
    return hipGetLastError();
}

hipError_t launch_tangent_local(const DevMesh& M, const DevMaps& P, const DevLocal& L,
                                const NewtonParams& np, const double* v, int lds_bytes, int npl,
                                hipStream_t s, int restrict_rhs) {
    hipError_t e;
#define NLS_TL(NPL)                                                                  \
    e = set_lds(k_tangent_local<NPL>, lds_bytes);                                    \
    if (e != hipSuccess) return e;                                                   \
    k_tangent_local<NPL><<<P.nsub, NLS_BLOCK, lds_bytes, s>>>(M, P, L, np, v, restrict_rhs, lds_bytes);
    if (npl <= 1) { NLS_TL(1) } else if (npl == 2) { NLS_TL(2) } else { NLS_TL(4) }
#undef NLS_TL
    return hipGetLastError();
}

hipError_t launch_prolong(const DevMesh& M, const DevMaps& P, const double* T,
                          const DevCoarse* C, const double* cvec, double* out, const double* addv,
                          hipStream_t s) {
    DevCoarse dummy{};
    k_prolong<<<nblocks(M.ndof), NLS_BLOCK, 0, s>>>(M.ndof, P.own_pidx, T, addv, C ? *C : dummy,
                                                 C ? 1 : 0, cvec, out);
    return hipGetLastError();
}

hipError_t launch_global_jv(const DevMesh& M, const double* u, const double* v, double* out,
                            hipStream_t s) {
    if (M.kind == NLS_PROBLEM_NEOHOOKE)
        k_global_jv_nh<<<nblocks(M.ndof), NLS_BLOCK, 0, s>>>(M, u, v, out);
    else
        k_global_jv<<<nblocks(M.N), NLS_BLOCK, 0, s>>>(M, u, v, out);
    return hipGetLastError();
}

hipError_t launch_coarse_phit(const DevCoarse& C, const double* r, hipStream_t s) {
    k_coarse_phit<<<C.nsub, NLS_BLOCK, 0, s>>>(C, r);
    return hipGetLastError();
}

hipError_t launch_local_factor(const DevMesh& M, const DevMaps& P, const DevLocal& L,
                               const NewtonParams& np, const double* u, int nblk, int lds_bytes,
                               hipStream_t s, const double* xloc, const double* gloc) {
    hipError_t e;
    if (M.kind == NLS_PROBLEM_NEOHOOKE) {
        e = set_lds(k_local_factor<true>, lds_bytes);
        if (e != hipSuccess) return e;
        k_local_factor<true><<<nblk, NLS_BLOCK, lds_bytes, s>>>(M, P, L, np, u, xloc, gloc);
    } else {
        e = set_lds(k_local_factor<false>, lds_bytes);
        if (e != hipSuccess) return e;
        k_local_factor<false><<<nblk, NLS_BLOCK, lds_bytes, s>>>(M, P, L, np, u, xloc, gloc);
    }
    return hipGetLastError();
}

hipError_t launch_sub_coarse(const DevMesh& M, const DevCoarse& C, const double* cvec,
                             const double* v, double* out, hipStream_t s) {
    k_sub_coarse<<<nblocks(M.ndof), NLS_BLOCK, 0, s>>>(M.ndof, C, cvec, v, out);
    return hipGetLastError();
}

hipError_t launch_gdsw_extend(const DevMesh& M, const DevCoarse& C, const double* ulin,
                              int lds_bytes, int npl, hipStream_t s) {
    hipError_t e;
#define NLS_GE(NPL, EL)                                                              \
    e = set_lds(k_gdsw_extend<NPL, EL>, lds_bytes);                                  \
    if (e != hipSuccess) return e;                                                   \
    k_gdsw_extend<NPL, EL><<<C.nsub, NLS_BLOCK, lds_bytes, s>>>(M, C, ulin);
    if (M.kind == NLS_PROBLEM_NEOHOOKE) {
        if (npl <= 1) { NLS_GE(1, true) } else if (npl == 2) { NLS_GE(2, true) } else { NLS_GE(4, true) }
    } else {
        if (npl <= 1) { NLS_GE(1, false) } else if (npl == 2) { NLS_GE(2, false) } else { NLS_GE(4, false) }
    }
#undef NLS_GE
    return hipGetLastError();
}

hipError_t launch_coarse_w(const DevMesh& M, const DevCoarse& C, const double* u, double* w,
                           hipStream_t s) {
    k_coarse_w<<<nblocks(M.ndof), NLS_BLOCK, 0, s>>>(M.ndof, C, u, w);
    return hipGetLastError();
}

hipError_t launch_coarse_q(const DevMesh& M, const DevCoarse& C, const double* w, const double* v,
                           int mode, int lds_bytes, hipStream_t s) {
    if (M.kind == NLS_PROBLEM_NEOHOOKE) {
        hipError_t e = set_lds(k_coarse_q<true>, lds_bytes);
        if (e != hipSuccess) return e;
        k_coarse_q<true><<<C.nsub, NLS_BLOCK, lds_bytes, s>>>(M, C, w, v, mode);
    } else {
        hipError_t e = set_lds(k_coarse_q<false>, lds_bytes);
        if (e != hipSuccess) return e;
        k_coarse_q<false><<<C.nsub, NLS_BLOCK, lds_bytes, s>>>(M, C, w, v, mode);
    }
    return hipGetLastError();
}

hipError_t launch_coarse_galerkin(const DevMesh& M, const DevCoarse& C, const double* w,
                                  int with_y, hipStream_t s) {
    // up to four workgroups per subdomain when there are fewer subdomains
    // than CUs
    const int q = C.nsub >= 256 ? 1 : (C.nsub >= 128 ? 2 : 4);
    const dim3 grid(C.nsub, q);
    if (M.kind == NLS_PROBLEM_NEOHOOKE)
        k_coarse_galerkin<true><<<grid, NLS_BLOCK, 0, s>>>(M, C, w, with_y);
    else
        k_coarse_galerkin<false><<<grid, NLS_BLOCK, 0, s>>>(M, C, w, with_y);
    k_coarse_galerkin_sum<<<grid, NLS_BLOCK, 0, s>>>(C);
    return hipGetLastError();
}

hipError_t launch_coarse_ty(const DevCoarse& C, const double* v, int lds_bytes, hipStream_t s) {
    // up to four blocks per subdomain when there are fewer subdomains than CUs
    const dim3 grid(C.nsub, C.nsub >= 256 ? 1 : (C.nsub >= 128 ? 2 : 4));
    k_coarse_ty<<<grid, NLS_BLOCK, lds_bytes, s>>>(C, v);
    return hipGetLastError();
}

hipError_t prepare_coarse_ty(int lds_bytes) { return set_lds(k_coarse_ty, lds_bytes); }

hipError_t launch_coarse_assemble(const DevCoarse& C, int with_matrix, hipStream_t s) {
    const int nnz = with_matrix ? C.nnz0 : 0;
    k_coarse_assemble<<<1 + (nnz + NLS_BLOCK - 1) / NLS_BLOCK, NLS_BLOCK, 0, s>>>(C, with_matrix);
    return hipGetLastError();
}

hipError_t launch_coarse_lu(const DevCoarse& C, int factor, int lds_bytes, int npl, hipStream_t s) {
    hipError_t e;
#define NLS_CL(NPL)                                                                  \
    e = set_lds(k_coarse_lu<NPL>, lds_bytes);                                        \
    if (e != hipSuccess) return e;                                                   \
    k_coarse_lu<NPL><<<C.nblk, NLS_BLOCK, lds_bytes, s>>>(C, factor, lds_bytes);
    if (npl <= 1) { NLS_CL(1) } else if (npl == 2) { NLS_CL(2) } else { NLS_CL(4) }
#undef NLS_CL
    return hipGetLastError();
}

hipError_t prepare_coarse_lu(int lds_bytes, int npl) {
    if (npl <= 1) return set_lds(k_coarse_lu<1>, lds_bytes);
    if (npl == 2) return set_lds(k_coarse_lu<2>, lds_bytes);
    return set_lds(k_coarse_lu<4>, lds_bytes);
}

hipError_t launch_coarse_update(const DevCoarse& C, hipStream_t s) {
    k_coarse_update<<<1, NLS_BLOCK, 0, s>>>(C);
    return hipGetLastError();
}

hipError_t launch_coarse_scatter(const DevCoarse& C, const double* src, double* cout, hipStream_t s) {
    k_coarse_scatter<<<nblocks(C.n0), NLS_BLOCK, 0, s>>>(C, src ? src : C.rhs, cout);
    return hipGetLastError();
}

// window buckets (KL, KW) of the multi-RHS solve
#define NLS_MR_BUCKETS(X) X(16, 32) X(24, 48) X(32, 64) X(40, 80) X(48, 96) X(56, 112)

int mrhs_bucket_kl(int kl, int ku) {
    const int need = std::max(kl, (kl + ku + 1) / 2);
    const int b = (need + 7) / 8 * 8;
    return b < 16 ? 16 : b;
}

int mrhs_lds_bytes(int kl_bucket) { return 2 * MR_CH * (2 * kl_bucket + 1) * 8; }
int coarse_inverse_lds_bytes(int max_block, int max_ldu) {
    return (max_block * INV_CB + 2 * INV_S * max_ldu) * 8 + 2 * INV_S * 4;
}

hipError_t launch_tangent_prep(const DevMaps& P, const DevLocal& L, const DevTangent& Tg,
                               int kl_bucket, int max_ng, hipStream_t s) {
    dim3 grid(P.nsub, (max_ng + MR_THREADS - 1) / MR_THREADS);
    const int lds = mrhs_lds_bytes(kl_bucket);
#define NLS_TP(A, B)                                                                      if (kl_bucket == A) {                                                                     k_tangent_prep<A, B><<<grid, MR_THREADS, lds, s>>>(P, L, Tg);                         return hipGetLastError();                                                         }
    NLS_MR_BUCKETS(NLS_TP)
#undef NLS_TP
    return hipErrorInvalidValue;
}

hipError_t launch_tangent_blocked(const DevMaps& P, const DevLocal& L, const DevTangent& Tg,
                                  int nblk, int nkk, int max_ng, hipStream_t s) {
    if (nblk <= 0 || nkk < 1 || nkk > 28) return hipErrorInvalidValue;
    k_tangent_blocks<<<nblk, 64, 0, s>>>(P, L, Tg);
    dim3 grid(P.nsub, (max_ng + 15) / 16);
    // nkk: k-steps of 4 band columns in the backward strip
    if (nkk <= 12)
        k_tangent_mfma<12><<<grid, 64, 0, s>>>(P, L, Tg);
    else if (nkk <= 18)
        k_tangent_mfma<18><<<grid, 64, 0, s>>>(P, L, Tg);
    else if (nkk <= 24)
        k_tangent_mfma<24><<<grid, 64, 0, s>>>(P, L, Tg);
    else
        k_tangent_mfma<28><<<grid, 64, 0, s>>>(P, L, Tg);
    return hipGetLastError();
}

hipError_t launch_tangent_gemv(const DevMaps& P, const DevTangent& Tg, const double* v, double* z,
                               int max_ng, bool stream_w, hipStream_t s) {
    // four workgroups per subdomain (eight with fewer subdomains than CUs,
    // whose patches are larger): one owned row per thread, so that enough
    // loads of W are in flight per CU
    dim3 grid(P.nsub, P.nsub < 256 ? 8 : 4);
    if (stream_w)
        k_tangent_gemv<true><<<grid, 256, max_ng * 8, s>>>(P, Tg, v, z);
    else
        k_tangent_gemv<false><<<grid, 256, max_ng * 8, s>>>(P, Tg, v, z);
    return hipGetLastError();
}

hipError_t launch_coarse_inverse(const DevCoarse& C, int max_block, int max_ldu, hipStream_t s) {
    if (C.inv_nblk > 0) {
        k_coarse_inv_blocks<<<C.inv_nblk, 64, 0, s>>>(C);
        const dim3 grid(C.nblk, (max_block + 15) / 16);
        if (C.inv_nkk <= 12)
            k_coarse_inv_mfma<12><<<grid, 64, 0, s>>>(C);
        else if (C.inv_nkk <= 18)
            k_coarse_inv_mfma<18><<<grid, 64, 0, s>>>(C);
        else if (C.inv_nkk <= 24)
            k_coarse_inv_mfma<24><<<grid, 64, 0, s>>>(C);
        else
            k_coarse_inv_mfma<28><<<grid, 64, 0, s>>>(C);
        return hipGetLastError();
    }
    if (max_ldu > INV_MAXW) return hipErrorInvalidValue;
    const dim3 nb((max_block + INV_CB - 1) / INV_CB, C.nblk);
    const int lds = coarse_inverse_lds_bytes(max_block, max_ldu);
    hipError_t e = set_lds(k_coarse_inverse, lds);
    if (e != hipSuccess) return e;
    k_coarse_inverse<<<nb, INV_THREADS, lds, s>>>(C, max_ldu);
    return hipGetLastError();
}


hipError_t launch_coarse_apply_inverse(const DevCoarse& C, const double* x, double* y, hipStream_t s) {
    k_coarse_apply_inverse<<<(C.n0 + 3) / 4, 256, 0, s>>>(C, x, y);
    return hipGetLastError();
}

hipError_t launch_mdot(const double* V, int64_t ld, int m, const double* w, int n,
                       double* partial, double* out, int nb, hipStream_t s) {
    k_mdot_partial<<<nb, NLS_BLOCK, 0, s>>>(V, ld, m, w, n, partial);
    k_mdot_final<<<m, 256, 0, s>>>(partial, nb, m, out);
    return hipGetLastError();
}

hipError_t launch_maxpy(const double* V, int64_t ld, int m, const double* h, double* w, int n,
                        double sign, hipStream_t s) {
    k_maxpy<<<nblocks(n), NLS_BLOCK, 0, s>>>(V, ld, m, h, w, n, sign);
    return hipGetLastError();
}

hipError_t launch_arnoldi_gs(const double* V, int64_t ld, int m, double* w, int n, double* partial,
                             double* pnorm, double* h1, double* h2, const GmresDev& G, int j,
                             double* vnext, int nb, hipStream_t s, double* partial2) {
    const int lds = m * (int)sizeof(double);
    k_mdot_partial<<<nb, NLS_BLOCK, 0, s>>>(V, ld, m, w, n, partial);
    k_maxpy_mdot_totals<<<nb, NLS_BLOCK, lds, s>>>(V, ld, m, partial, nb, h1, w, n, partial2);
    k_maxpy_norm_totals<<<nb, NLS_BLOCK, lds, s>>>(V, ld, m, partial2, nb, h2, w, n, pnorm);
    k_scale_givens_totals<<<nblocks(n), NLS_BLOCK, 0, s>>>(w, vnext, n, pnorm, nb, G, j);
    return hipGetLastError();
}

hipError_t launch_maxpy_norm(const double* V, int64_t ld, int m, const double* h, double* w, int n,
                             double* partial, double* out, int nb, hipStream_t s) {
    k_maxpy_norm<<<nb, NLS_BLOCK, 0, s>>>(V, ld, m, h, w, n, partial);
    k_mdot_final<<<1, 256, 0, s>>>(partial, nb, 1, out);
    return hipGetLastError();
}

hipError_t launch_coarse_gather(const DevCoarse& C, hipStream_t s) {
    k_coarse_gather<<<nblocks(C.n0), NLS_BLOCK, 0, s>>>(C);
    return hipGetLastError();
}

hipError_t launch_scale_by(const double* x, const double* dsq, double* y, int n, hipStream_t s) {
    k_scale_by<<<nblocks(n), NLS_BLOCK, 0, s>>>(x, dsq, y, n);
    return hipGetLastError();
}

hipError_t launch_axpy(double a, const double* x, double* y, int n, hipStream_t s) {
    k_axpy<<<nblocks(n), NLS_BLOCK, 0, s>>>(a, x, y, n);
    return hipGetLastError();
}


hipError_t launch_max_abs(const double* x, int n, double* partial, double* out, int nb,
                          hipStream_t s) {
    k_max_abs_partial<<<nb, NLS_BLOCK, 0, s>>>(x, n, partial);
    k_max_final<<<1, 64, 0, s>>>(partial, nb, out);
    return hipGetLastError();
}

hipError_t launch_any_status(const int* status, int n, int* out, hipStream_t s) {
    k_any_status<<<1, 64, 0, s>>>(status, n, out);
    return hipGetLastError();
}


