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

#include <climits>
#include <cmath>

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
__device__ double block_sum(double v, double* red) {
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

__device__ double block_max(double v, double* red) {
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
__device__ void local_residual(const DevMesh& M, const DevMaps& P, int n, int rowbase,
                               int ebase, const double* vp, double* rb) {
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        const int row = rowbase + a;
        const int g = P.l2g[row];
        if (M.dflag[g]) {
            rb[a] = vp[a] - M.dval[g];
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

// Jacobian rows [J_ii | B_i] into the CSR values jval (slots fixed at setup).
__device__ void local_jacobian(const DevMesh& M, const DevMaps& P, int n, int rowbase,
                               int ebase, const double* vp, double* __restrict__ jval) {
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        const int row = rowbase + a;
        const int g = P.l2g[row];
        const int js = P.jptr[row], je = P.jptr[row + 1];
        for (int s = js; s < je; ++s) jval[s] = 0.0;
        if (M.dflag[g]) {
            for (int s = js; s < je; ++s)
                if (P.jcol[s] == a) jval[s] = 1.0;
            continue;
        }
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
            const double s = gr[0] * uu[0] + gr[1] * uu[1] + gr[2] * uu[2];
            const double kap = M.kappa[ge];
            const double coef = kap * (1.0 + M.beta * m);
            const double rk = M.beta * kap * s * (1.0 / 6.0);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double K = coef * gr[c] + rk * (U + uu[c]);
                for (int t = js; t < je; ++t)
                    if (P.jcol[t] == nd[c]) { jval[t] += K; break; }
            }
        }
    }
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
__device__ int band_lu(int n, int kl, int ku, const int* __restrict__ rptr,
                       const int* __restrict__ cols, const double* __restrict__ vals,
                       T* W, T* mult, int* sflag, T* __restrict__ Uf, T* __restrict__ Lf,
                       int* __restrict__ piv) {
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
            const int c = cols[s];
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
                const int c = cols[s];
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

// ----------------------------------------------------------------------------
// Band triangular solves with the factors of band_lu, executed by ONE
// wavefront (threads 0..63), right-hand side b in LDS (FP64).  NPL values per
// lane cover bands up to 64*NPL.  The factor columns of S steps are fetched
// ahead into registers so that HBM latency is paid once per chunk.
// ----------------------------------------------------------------------------
template <typename T, int NPL>
__device__ void band_solve_wave(int n, int kl, int ku, const T* __restrict__ Uf,
                                const T* __restrict__ Lf, const int* __restrict__ piv,
                                double* b) {
    constexpr int S = 8;
    const int lane = threadIdx.x & 63;
    const int ldu = kl + ku + 1, ldl = kl > 1 ? kl : 1;
    for (int k0 = 0; k0 < n; k0 += S) {
        double lv[S][NPL];
        int pv[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int k = k0 + s;
            const int lim = (k < n) ? min(kl, n - 1 - k) : 0;
            pv[s] = (k < n) ? piv[k] : k;
#pragma unroll
            for (int q = 0; q < NPL; ++q) {
                const int j = lane + 64 * q;
                lv[s][q] = (j < lim) ? (double)Lf[(size_t)k * ldl + j] : 0.0;
            }
        }
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
    for (int k0 = n - 1; k0 >= 0; k0 -= S) {
        double uv[S][NPL];
        double dg[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int k = k0 - s;
            const int lim = (k >= 0) ? min(kl + ku, k) : 0;
            dg[s] = (k >= 0) ? (double)Uf[(size_t)k * ldu] : 1.0;
#pragma unroll
            for (int q = 0; q < NPL; ++q) {
                const int j = lane + 64 * q;
                uv[s][q] = (j < lim) ? (double)Uf[(size_t)k * ldu + 1 + j] : 0.0;
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int k = k0 - s;
            if (k >= 0) {
                if (lane == 0) b[k] = b[k] / dg[s];
                wave_sync();
                const double bk = b[k];
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

template <int NPL>
__device__ void band_solve_any(bool f32, int n, int kl, int ku, const double* Ud,
                               const double* Ld, const float* Us, const float* Ls,
                               const int* piv, double* b) {
    if (f32) band_solve_wave<float, NPL>(n, kl, ku, Us, Ls, piv, b);
    else band_solve_wave<double, NPL>(n, kl, ku, Ud, Ld, piv, b);
}

// Solve J d = rb in place (rb in LDS).  FP64 factors: one band solve.  FP32
// factors: iterative refinement with FP64 residuals r0 - J d computed from
// the FP64 CSR values (columns < n), until ||res|| <= ir_rtol ||r0||.
template <int NPL>
__device__ void local_linear_solve(const DevMaps& P, const DevLocal& L, const NewtonParams& np,
                                   int i, int n, int rowbase, double* rb, double* r0,
                                   double* dl, double* red) {
    const int kl = P.kl[i], ku = P.ku[i];
    const double* Ud = L.Uf + P.off_u[i];
    const double* Ld = L.Lf + P.off_l[i];
    const float* Us = np.mixed ? L.Uf32 + P.off_u[i] : nullptr;
    const float* Ls = np.mixed ? L.Lf32 + P.off_l[i] : nullptr;
    const int* piv = L.piv + rowbase;
    if (!np.mixed) {
        if (threadIdx.x < 64) band_solve_any<NPL>(false, n, kl, ku, Ud, Ld, Us, Ls, piv, rb);
        __syncthreads();
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
        if (threadIdx.x < 64) band_solve_any<NPL>(true, n, kl, ku, Ud, Ld, Us, Ls, piv, rb);
        __syncthreads();
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
__device__ int local_factor(const DevMaps& P, const DevLocal& L, const NewtonParams& np, int i,
                            int n, int rowbase, void* W, void* mult, int* sflag) {
    const int kl = P.kl[i], ku = P.ku[i];
    const int* rptr = P.jptr + rowbase;
    if (np.mixed)
        return band_lu<float>(n, kl, ku, rptr, P.jcol, L.jval, (float*)W, (float*)mult, sflag,
                              L.Uf32 + P.off_u[i], L.Lf32 + P.off_l[i], L.piv + rowbase);
    return band_lu<double>(n, kl, ku, rptr, P.jcol, L.jval, (double*)W, (double*)mult, sflag,
                           L.Uf + P.off_u[i], L.Lf + P.off_l[i], L.piv + rowbase);
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
template <int NPL>
__global__ void __launch_bounds__(NLS_BLOCK)
k_local_newton(DevMesh M, DevMaps P, DevLocal L, NewtonParams np, const double* __restrict__ u) {
    extern __shared__ double smem[];
    __shared__ int sflag[4];
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
    __syncthreads();
    local_residual(M, P, n, rowbase, ebase, vp, rb);
    double ss = 0.0;
    for (int a = threadIdx.x; a < n; a += blockDim.x) ss += rb[a] * rb[a];
    double rn = sqrt(block_sum(ss, red));
    const double tol = fmax(np.rtol * rn, np.abs_tol * sqrt((double)n));
    int its = 0, status = 0;
    double dprev = -1.0;
    for (;;) {
        if (!(rn == rn) || isinf(rn)) { status = 2; break; }
        if (rn <= tol) break;
        if (dprev >= 0.0) {
            double xm = 0.0;
            for (int a = threadIdx.x; a < n; a += blockDim.x) xm = fmax(xm, fabs(vp[a]));
            xm = block_max(xm, red);
            if (dprev <= np.stagnation * xm) break;
        }
        if (its == np.maxit) { status = 1; break; }
        local_jacobian(M, P, n, rowbase, ebase, vp, L.jval);
        __syncthreads();
        if (local_factor(P, L, np, i, n, rowbase, W, mult, sflag)) { status = 3; break; }
        local_linear_solve<NPL>(P, L, np, i, n, rowbase, rb, r0, dl, red);
        double dm = 0.0;
        for (int a = threadIdx.x; a < n; a += blockDim.x) {
            vp[a] -= rb[a];
            dm = fmax(dm, fabs(rb[a]));
        }
        dprev = block_max(dm, red);
        ++its;
        local_residual(M, P, n, rowbase, ebase, vp, rb);
        ss = 0.0;
        for (int a = threadIdx.x; a < n; a += blockDim.x) ss += rb[a] * rb[a];
        rn = sqrt(block_sum(ss, red));
    }
    if (status == 0) {
        local_jacobian(M, P, n, rowbase, ebase, vp, L.jval);
        __syncthreads();
        if (local_factor(P, L, np, i, n, rowbase, W, mult, sflag)) status = 3;
    }
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        const int row = rowbase + a;
        L.xstar[row] = vp[a];
        L.T[row] = u[P.l2g[row]] - vp[a];
    }
    if (threadIdx.x == 0) {
        L.its[i] = its;
        L.status[i] = status;
    }
}

// Local part of the exact tangent: z_i = J_ii^{-1} (B_i v_Gamma_i), with J,
// B at the converged local state (eq. 6 with R_i DF(u_i) v = J R_i v + B v_G).
template <int NPL>
__global__ void __launch_bounds__(NLS_BLOCK)
k_tangent_local(DevMesh M, DevMaps P, DevLocal L, NewtonParams np, const double* __restrict__ v) {
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
        for (int s = P.jptr[row]; s < P.jptr[row + 1]; ++s) {
            const int c = P.jcol[s];
            if (c >= n) acc += L.jval[s] * v[P.g2g[gbase + c - n]];
        }
        rb[a] = acc;
    }
    __syncthreads();
    local_linear_solve<NPL>(P, L, np, i, n, rowbase, rb, r0, dl, red);
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

// Harmonic extension Phi_I = -A_II^{-1} A_IG Phi_G with A = DF(0) = kappa G
// (one workgroup per subdomain; setup only).
template <int NPL>
__global__ void __launch_bounds__(NLS_BLOCK)
k_gdsw_extend(DevMesh M, DevCoarse C) {
    extern __shared__ double smem[];
    __shared__ int sflag[4];
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
        ph[t] = (C.ctype[cb + a] == 1 && C.ccomp[cb + a] == k) ? 1.0 : 0.0;
    }
    if (ni == 0 || nk == 0) return;
    double* rhs = smem;
    double* red = rhs + ni;
    double* mult = red + 24;
    double* W = mult + ((kl > 1 ? kl : 1) + 1);
    // A_II values
    for (int r = threadIdx.x; r < ni; r += blockDim.x) {
        const int ca = C.inode[ib + r];
        const int js = C.iptr[ib + r], je = C.iptr[ib + r + 1];
        for (int s = js; s < je; ++s) C.ival[s] = 0.0;
        for (int q = C.cinc_ptr[cb + ca]; q < C.cinc_ptr[cb + ca + 1]; ++q) {
            const int code = C.cinc[q];
            const int e = eb + (code >> 2), pos = code & 3;
            double gr[3];
            const int ge = C.ne_gid[e];
            g_row(M.G6 + 6 * (size_t)ge, pos, gr[0], gr[1], gr[2]);
            for (int c = 0; c < 3; ++c) {
                const int cc = C.iidx[cb + C.ne_conn[3 * e + c]];
                if (cc < 0) continue;
                for (int s = js; s < je; ++s)
                    if (C.icol[s] == cc) { C.ival[s] += M.kappa[ge] * gr[c]; break; }
            }
        }
    }
    __syncthreads();
    if (band_lu<double>(ni, kl, ku, C.iptr + ib, C.icol, C.ival, W, mult, sflag,
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
                double gr[3];
                const int ge = C.ne_gid[e];
                g_row(M.G6 + 6 * (size_t)ge, pos, gr[0], gr[1], gr[2]);
                for (int c = 0; c < 3; ++c) {
                    const int cn = cb + C.ne_conn[3 * e + c];
                    if (C.ctype[cn] == 1 && C.ccomp[cn] == k) acc -= M.kappa[ge] * gr[c];
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

// w = u - Phi c at every node (owner's block).
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

// Per subdomain: gblk_i = Phi_i^T q_i where, on closure nodes,
//   mode 0: q = sum over part-i elements of the element residual at w
//           (so that sum_i gblk_i = Phi^T F(w));
//   mode 1: q = sum over part-i elements of K_T(w) v_T
//           (so that sum_i gblk_i = Phi^T DF(w) v).
__global__ void __launch_bounds__(NLS_BLOCK)
k_coarse_q(DevMesh M, DevCoarse C, const double* __restrict__ w, const double* __restrict__ v, int mode) {
    extern __shared__ double smem[];
    const int i = blockIdx.x;
    const int cb = C.off_c[i], nc = C.off_c[i + 1] - cb;
    const int k0 = C.off_k[i], nk = C.off_k[i + 1] - k0;
    const int eb = C.off_ne[i];
    double* q = smem;
    for (int a = threadIdx.x; a < nc; a += blockDim.x) {
        double acc = 0.0;
        if (C.ctype[cb + a] != 2) {
            for (int t = C.cinc_ptr[cb + a]; t < C.cinc_ptr[cb + a + 1]; ++t) {
                const int code = C.cinc[t];
                const int e = eb + (code >> 2), pos = code & 3;
                const int ge = C.ne_gid[e];
                double uu[3], vv[3];
                for (int c = 0; c < 3; ++c) {
                    const int gn = C.cnode[cb + C.ne_conn[3 * e + c]];
                    uu[c] = w[gn];
                    vv[c] = mode ? v[gn] : 0.0;
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
                    for (int c = 0; c < 3; ++c) acc += (coef * gr[c] + rk * (U + uu[c])) * vv[c];
                }
            }
        }
        q[a] = acc;
    }
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

// Per subdomain Galerkin block A_i = Phi_i^T K_i(w) Phi_i (K_i: part-i elements).
__global__ void __launch_bounds__(NLS_BLOCK)
k_coarse_galerkin(DevMesh M, DevCoarse C, const double* __restrict__ w) {
    const int i = blockIdx.x;
    const int cb = C.off_c[i], nc = C.off_c[i + 1] - cb;
    const int k0 = C.off_k[i], nk = C.off_k[i + 1] - k0;
    const int eb = C.off_ne[i];
    const double* ph = C.phi + C.off_phi[i];
    double* z = C.zbuf + C.off_phi[i];
    for (int a = threadIdx.x; a < nc; a += blockDim.x) {
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
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int kk = wv; kk < nk * nk; kk += nw) {
        const int k = kk / nk, l = kk - k * nk;
        double acc = 0.0;
        for (int a = lane; a < nc; a += 64) acc += ph[(int64_t)a * nk + k] * z[(int64_t)a * nk + l];
        acc = wave_sum(acc);
        if (lane == 0) C.ablk[C.off_kk[i] + kk] = acc;
    }
}

// Deterministic assembly: rhs (band order) from the gblk pieces, and, if
// with_matrix, the CSR values of A0 from the Galerkin blocks.  Also writes
// ||rhs||_2 to scal[0] (single block).
__global__ void __launch_bounds__(NLS_BLOCK)
k_coarse_assemble(DevCoarse C, int with_matrix) {
    __shared__ double red[24];
    double ss = 0.0;
    for (int k = threadIdx.x; k < C.n0; k += blockDim.x) {
        double acc = 0.0;
        for (int t = C.gsrc_ptr[k]; t < C.gsrc_ptr[k + 1]; ++t) acc += C.gblk[C.gsrc[t]];
        C.rhs[C.perm[k]] = acc;
        ss += acc * acc;
    }
    if (with_matrix) {
        const int nnz = C.a0ptr[C.n0];
        for (int s = threadIdx.x; s < nnz; s += blockDim.x) {
            double acc = 0.0;
            for (int t = C.a0src_ptr[s]; t < C.a0src_ptr[s + 1]; ++t) acc += C.ablk[C.a0src[t]];
            C.a0val[s] = acc;
        }
    }
    ss = block_sum(ss, red);
    if (threadIdx.x == 0) C.scal[0] = sqrt(ss);
}

// Single workgroup: (factor A0 and) solve A0 d = rhs in place (band order).
template <int NPL>
__global__ void __launch_bounds__(NLS_BLOCK)
k_coarse_lu(DevCoarse C, int factor) {
    extern __shared__ double smem[];
    __shared__ int sflag[4];
    const int n = C.n0, kl = C.a0kl, ku = C.a0ku;
    double* b = smem;
    double* mult = b + n;
    double* W = mult + ((kl > 1 ? kl : 1) + 1);
    if (factor) {
        if (band_lu<double>(n, kl, ku, C.a0ptr, C.a0col, C.a0val, W, mult, sflag, C.a0U, C.a0L,
                            C.a0piv)) {
            if (threadIdx.x == 0) atomicOr(C.flag, 2);
        }
    }
    for (int k = threadIdx.x; k < n; k += blockDim.x) b[k] = C.rhs[k];
    __syncthreads();
    if (threadIdx.x < 64) band_solve_wave<double, NPL>(n, kl, ku, C.a0U, C.a0L, C.a0piv, b);
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x) C.rhs[k] = b[k];
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
__global__ void k_coarse_scatter(DevCoarse C, double* __restrict__ cout) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < C.n0) cout[k] = C.rhs[C.perm[k]];
}

// ----------------------------------------------------------------------------
// Vector kernels (GMRES).  partial sums per block, then a fixed-order sum.
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(NLS_BLOCK)
k_mdot_partial(const double* __restrict__ V, int64_t ld, int m, const double* __restrict__ w,
               int n, double* __restrict__ partial) {
    __shared__ double red[4 * 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int chunk = (n + gridDim.x - 1) / gridDim.x;
    const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    for (int j0 = 0; j0 < m; j0 += 64) {
        const int jn = min(64, m - j0);
        for (int jj = 0; jj < jn; ++jj) {
            const double* vj = V + (int64_t)(j0 + jj) * ld;
            double acc = 0.0;
            for (int t = lo + threadIdx.x; t < hi; t += blockDim.x) acc += vj[t] * w[t];
            acc = wave_sum(acc);
            if (lane == 0) red[wv * 64 + jj] = acc;
        }
        __syncthreads();
        if (threadIdx.x < jn) {
            double s = 0.0;
            for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += red[q * 64 + threadIdx.x];
            partial[(int64_t)blockIdx.x * m + j0 + threadIdx.x] = s;
        }
        __syncthreads();
    }
}

__global__ void k_mdot_final(const double* __restrict__ partial, int nb, int m, double* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[(int64_t)b * m + j];
    out[j] = s;
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

__global__ void k_add_inplace(const double* __restrict__ x, double* __restrict__ y, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] += x[t];
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
    k_global_residual<<<nblocks(M.N), NLS_BLOCK, 0, s>>>(M, u, F);
    return hipGetLastError();
}

hipError_t launch_local_newton(const DevMesh& M, const DevMaps& P, const DevLocal& L,
                               const NewtonParams& np, const double* u, int lds_bytes,
                               int npl, hipStream_t s) {
    hipError_t e;
#define NLS_LN(NPL)                                                                  \
    e = set_lds(k_local_newton<NPL>, lds_bytes);                                     \
    if (e != hipSuccess) return e;                                                   \
    k_local_newton<NPL><<<P.nsub, NLS_BLOCK, lds_bytes, s>>>(M, P, L, np, u);
    if (npl <= 1) { NLS_LN(1) } else if (npl == 2) { NLS_LN(2) } else { NLS_LN(4) }
#undef NLS_LN
    return hipGetLastError();
}

hipError_t launch_tangent_local(const DevMesh& M, const DevMaps& P, const DevLocal& L,
                                const NewtonParams& np, const double* v, int lds_bytes, int npl,
                                hipStream_t s) {
    hipError_t e;
#define NLS_TL(NPL)                                                                  \
    e = set_lds(k_tangent_local<NPL>, lds_bytes);                                    \
    if (e != hipSuccess) return e;                                                   \
    k_tangent_local<NPL><<<P.nsub, NLS_BLOCK, lds_bytes, s>>>(M, P, L, np, v);
    if (npl <= 1) { NLS_TL(1) } else if (npl == 2) { NLS_TL(2) } else { NLS_TL(4) }
#undef NLS_TL
    return hipGetLastError();
}

hipError_t launch_prolong(const DevMesh& M, const DevMaps& P, const double* T,
                          const DevCoarse* C, const double* cvec, double* out, const double* addv,
                          hipStream_t s) {
    DevCoarse dummy{};
    k_prolong<<<nblocks(M.N), NLS_BLOCK, 0, s>>>(M.N, P.own_pidx, T, addv, C ? *C : dummy,
                                                 C ? 1 : 0, cvec, out);
    return hipGetLastError();
}

hipError_t launch_gdsw_extend(const DevMesh& M, const DevCoarse& C, int lds_bytes, int npl,
                              hipStream_t s) {
    hipError_t e;
#define NLS_GE(NPL)                                                                  \
    e = set_lds(k_gdsw_extend<NPL>, lds_bytes);                                      \
    if (e != hipSuccess) return e;                                                   \
    k_gdsw_extend<NPL><<<C.nsub, NLS_BLOCK, lds_bytes, s>>>(M, C);
    if (npl <= 1) { NLS_GE(1) } else if (npl == 2) { NLS_GE(2) } else { NLS_GE(4) }
#undef NLS_GE
    return hipGetLastError();
}

hipError_t launch_coarse_w(const DevMesh& M, const DevCoarse& C, const double* u, double* w,
                           hipStream_t s) {
    k_coarse_w<<<nblocks(M.N), NLS_BLOCK, 0, s>>>(M.N, C, u, w);
    return hipGetLastError();
}

hipError_t launch_coarse_q(const DevMesh& M, const DevCoarse& C, const double* w, const double* v,
                           int mode, int lds_bytes, hipStream_t s) {
    hipError_t e = set_lds(k_coarse_q, lds_bytes);
    if (e != hipSuccess) return e;
    k_coarse_q<<<C.nsub, NLS_BLOCK, lds_bytes, s>>>(M, C, w, v, mode);
    return hipGetLastError();
}

hipError_t launch_coarse_galerkin(const DevMesh& M, const DevCoarse& C, const double* w,
                                  hipStream_t s) {
    k_coarse_galerkin<<<C.nsub, NLS_BLOCK, 0, s>>>(M, C, w);
    return hipGetLastError();
}

hipError_t launch_coarse_assemble(const DevCoarse& C, int with_matrix, hipStream_t s) {
    k_coarse_assemble<<<1, NLS_BLOCK, 0, s>>>(C, with_matrix);
    return hipGetLastError();
}

hipError_t launch_coarse_lu(const DevCoarse& C, int factor, int lds_bytes, int npl, hipStream_t s) {
    hipError_t e;
#define NLS_CL(NPL)                                                                  \
    e = set_lds(k_coarse_lu<NPL>, lds_bytes);                                        \
    if (e != hipSuccess) return e;                                                   \
    k_coarse_lu<NPL><<<1, NLS_BLOCK, lds_bytes, s>>>(C, factor);
    if (npl <= 1) { NLS_CL(1) } else if (npl == 2) { NLS_CL(2) } else { NLS_CL(4) }
#undef NLS_CL
    return hipGetLastError();
}

hipError_t launch_coarse_update(const DevCoarse& C, hipStream_t s) {
    k_coarse_update<<<1, NLS_BLOCK, 0, s>>>(C);
    return hipGetLastError();
}

hipError_t launch_coarse_scatter(const DevCoarse& C, double* cout, hipStream_t s) {
    k_coarse_scatter<<<nblocks(C.n0), NLS_BLOCK, 0, s>>>(C, cout);
    return hipGetLastError();
}

hipError_t launch_mdot(const double* V, int64_t ld, int m, const double* w, int n,
                       double* partial, double* out, int nb, hipStream_t s) {
    k_mdot_partial<<<nb, NLS_BLOCK, 0, s>>>(V, ld, m, w, n, partial);
    k_mdot_final<<<nblocks(m, 64), 64, 0, s>>>(partial, nb, m, out);
    return hipGetLastError();
}

hipError_t launch_maxpy(const double* V, int64_t ld, int m, const double* h, double* w, int n,
                        double sign, hipStream_t s) {
    k_maxpy<<<nblocks(n), NLS_BLOCK, 0, s>>>(V, ld, m, h, w, n, sign);
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

hipError_t launch_add_inplace(const double* x, double* y, int n, hipStream_t s) {
    k_add_inplace<<<nblocks(n), NLS_BLOCK, 0, s>>>(x, y, n);
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
