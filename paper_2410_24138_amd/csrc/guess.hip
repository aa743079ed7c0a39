// HIP kernels of the learned initial guess of the local Newton solves:
// sampling of the patch features, the transfinite lifting, training
// targets, and the network's bfloat16 matrix-core forward/backward with
// FP32 accumulation and its Adam update.
//
// The paper starts each inner Newton iteration (eq. 4) from R_i u; this part
// only proposes a start, which the local Newton kernel accepts when its
// residual is below that of R_i u.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "guess_device.h"

namespace {

__device__ __forceinline__ uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float gelu(float z) {
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_prime(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ---------------------------------------------------------------- sampling
__device__ __forceinline__ double sample(const DevGuessTables& T, int i, int k, const double* f) {
    const size_t b = ((size_t)i * NLS_G_IN + k) * 3;
    return T.sw[b] * f[T.snode[b]] + T.sw[b + 1] * f[T.snode[b + 1]] +
           T.sw[b + 2] * f[T.snode[b + 2]];
}

// Side function s (0 bottom, 1 right, 2 top, 3 left) at parameter t: linear
// between the NS samples of the side; the last interval ends at the first
// sample of the next side (the corner).
template <int NS>
__device__ __forceinline__ double side(const double* tr, int sd, double t) {
    const double pos = t * NS;
    int j = (int)floor(pos);
    j = j < 0 ? 0 : (j > NS - 1 ? NS - 1 : j);
    const double w = pos - j;
    const int nx = (j < NS - 1) ? sd * NS + j + 1 : ((sd + 1) & 3) * NS;
    return (1.0 - w) * tr[sd * NS + j] + w * tr[nx];
}

// Transfinite (Coons) interpolant of the sampled perimeter (NS samples per
// side) at unit (xi, eta).
template <int NS = NLS_G_SIDE>
__device__ __forceinline__ double coons(const double* tr, double xi, double eta) {
    const double g0 = side<NS>(tr, 0, xi), g1 = side<NS>(tr, 1, eta);
    const double g2 = side<NS>(tr, 2, 1.0 - xi), g3 = side<NS>(tr, 3, 1.0 - eta);
    const double c00 = tr[0], c10 = tr[NS], c11 = tr[2 * NS], c01 = tr[3 * NS];
    return (1.0 - eta) * g0 + eta * g2 + (1.0 - xi) * g3 + xi * g1 -
           ((1.0 - xi) * (1.0 - eta) * c00 + xi * (1.0 - eta) * c10 + xi * eta * c11 +
            (1.0 - xi) * eta * c01);
}

// Bilinear interpolant of the GX x GY reference-node values c[q*GX + p].
template <int GX = NLS_G_GRID, int GY = NLS_G_GRID>
__device__ __forceinline__ double bilinear(const float* c, double xi, double eta) {
    const double px = xi * (GX - 1), py = eta * (GY - 1);
    int p0 = (int)floor(px), q0 = (int)floor(py);
    p0 = p0 < 0 ? 0 : (p0 > GX - 2 ? GX - 2 : p0);
    q0 = q0 < 0 ? 0 : (q0 > GY - 2 ? GY - 2 : q0);
    const double a = px - p0, b = py - q0;
    const float* r0 = c + q0 * GX + p0;
    const float* r1 = r0 + GX;
    return (1.0 - a) * (1.0 - b) * r0[0] + a * (1.0 - b) * r0[1] + (1.0 - a) * b * r1[0] +
           a * b * r1[1];
}

// ------------------------------------------------- elasticity (Q1, d = 2)
// Component c of the dof field f (node-major, two per node) at sample k.
__device__ __forceinline__ double sample_e(const DevGuessTables& T, int i, int k,
                                           const double* f, int c) {
    const size_t b = ((size_t)i * NLS_GE_NSAMP + k) * 4;
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) v += T.sw[b + q] * f[2 * T.snode[b + q] + c];
    return v;
}

// Features: u_x, u_y at the 32 perimeter points, then f_x, f_y (external
// nodal forces) at the 128 points on the right side of the box.
__global__ void __launch_bounds__(NLS_G_IN)
k_guess_features_e(DevGuessTables T, const double* __restrict__ u, const double* __restrict__ fload,
                   const float* __restrict__ xm, const float* __restrict__ xs,
                   float* __restrict__ xraw, uint16_t* __restrict__ xbf) {
    const int i = blockIdx.x, k = threadIdx.x;
    double v;
    if (k < 2 * NLS_GE_TRACE) {
        v = sample_e(T, i, k % NLS_GE_TRACE, u, k / NLS_GE_TRACE);
    } else {
        const int kk = k - 2 * NLS_GE_TRACE;
        v = sample_e(T, i, NLS_GE_TRACE + kk % NLS_GE_LOAD, fload, kk / NLS_GE_LOAD);
    }
    const size_t o = (size_t)i * NLS_G_IN + k;
    if (xraw) xraw[o] = (float)v;
    if (xbf) xbf[o] = f2bf((float)((v - (double)xm[k]) / (double)xs[k]));
}

// x_pred on the V dofs: per component Coons of its 32 trace samples +
// bilinear interpolant of its 128 coefficients; Dirichlet dofs exact.
__global__ void __launch_bounds__(256)
k_guess_lift_e(DevMaps P, DevGuessTables T, DevMesh M, const double* __restrict__ xy,
               const double* __restrict__ u, const float* __restrict__ coef,
               double* __restrict__ xpred) {
    __shared__ double tr[2 * NLS_GE_TRACE];
    __shared__ float cf[NLS_G_OUT];
    const int i = blockIdx.x;
    if (threadIdx.x < 2 * NLS_GE_TRACE)
        tr[threadIdx.x] = sample_e(T, i, threadIdx.x % NLS_GE_TRACE, u, threadIdx.x / NLS_GE_TRACE);
    for (int k = threadIdx.x; k < NLS_G_OUT; k += blockDim.x) cf[k] = coef[(size_t)i * NLS_G_OUT + k];
    __syncthreads();
    const double x0 = T.box[4 * i], y0 = T.box[4 * i + 1];
    const double W = T.box[4 * i + 2] - x0, H = T.box[4 * i + 3] - y0;
    const int rb = P.off_n[i], n = P.off_n[i + 1] - rb;
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        const int dof = P.l2g[rb + a], g = dof >> 1, c = dof & 1;
        double v;
        if (M.dflag[dof]) {
            v = M.dval[dof];
        } else {
            const double xi = (xy[2 * g] - x0) / W, eta = (xy[2 * g + 1] - y0) / H;
            v = coons<NLS_GE_SIDE>(tr + c * NLS_GE_TRACE, xi, eta) +
                bilinear<NLS_GE_GX, NLS_GE_GY>(cf + c * NLS_GE_NGRID, xi, eta);
        }
        xpred[rb + a] = v;
    }
}

// Training target: per component (v(x*) - Coons) at the 16 x 8 reference
// nodes, v(x*) = x* on the V dofs and u elsewhere.
__global__ void __launch_bounds__(NLS_G_OUT)
k_guess_target_e(DevGuessTables T, const double* __restrict__ u, const double* __restrict__ xstar,
                 float* __restrict__ traw) {
    __shared__ double tr[2 * NLS_GE_TRACE];
    const int i = blockIdx.x, k = threadIdx.x;
    if (k < 2 * NLS_GE_TRACE) tr[k] = sample_e(T, i, k % NLS_GE_TRACE, u, k / NLS_GE_TRACE);
    __syncthreads();
    const int c = k / NLS_GE_NGRID, q = k % NLS_GE_NGRID;
    const size_t b = ((size_t)i * NLS_GE_NSAMP + NLS_GE_TRACE + NLS_GE_LOAD + q) * 4;
    const size_t bl = ((size_t)i * NLS_GE_NGRID + q) * 4;
    double v = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int loc = T.sloc[bl + t];
        v += T.sw[b + t] * (loc >= 0 ? xstar[loc + c] : u[2 * T.snode[b + t] + c]);
    }
    const int p = q % NLS_GE_GX, qq = q / NLS_GE_GX;
    const double xi = (double)p / (NLS_GE_GX - 1), eta = (double)qq / (NLS_GE_GY - 1);
    traw[(size_t)i * NLS_G_OUT + k] =
        (float)(v - coons<NLS_GE_SIDE>(tr + c * NLS_GE_TRACE, xi, eta));
}

// f^_g = mean of the edge-midpoint load samples over the (element, edge)
// pairs through node g; 1 without samples.
__global__ void k_nodal_load(DevMesh M, const double* __restrict__ fmid, double* __restrict__ fhat) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= M.N) return;
    if (!fmid) {
        fhat[g] = 1.0;
        return;
    }
    double acc = 0.0;
    int cnt = 0;
    for (int k = M.nptr[g]; k < M.nptr[g + 1]; ++k) {
        const int e = M.nel[k] >> 2, a = M.nel[k] & 3;
        acc += fmid[3 * e + a] + fmid[3 * e + (a + 2) % 3];
        cnt += 2;
    }
    fhat[g] = cnt ? acc / cnt : 0.0;
}

// Features of subdomain i: 64 perimeter samples of u, 256 grid samples of
// the nodal load.  Raw FP32 copy and/or standardised bfloat16 copy.
__global__ void __launch_bounds__(NLS_G_IN)
k_guess_features(DevGuessTables T, const double* __restrict__ u, const double* __restrict__ fhat,
                 const float* __restrict__ xm, const float* __restrict__ xs,
                 float* __restrict__ xraw, uint16_t* __restrict__ xbf) {
    const int i = blockIdx.x, k = threadIdx.x;
    const double v = sample(T, i, k, k < NLS_G_TRACE ? u : fhat);
    const size_t o = (size_t)i * NLS_G_IN + k;
    if (xraw) xraw[o] = (float)v;
    if (xbf) xbf[o] = f2bf((float)((v - (double)xm[k]) / (double)xs[k]));
}

// x_pred on V_i: Coons(trace of u) + bilinear(coef); Dirichlet rows exact.
__global__ void __launch_bounds__(256)
k_guess_lift(DevMaps P, DevGuessTables T, DevMesh M, const double* __restrict__ xy,
             const double* __restrict__ u, const float* __restrict__ coef,
             double* __restrict__ xpred) {
    __shared__ double tr[NLS_G_TRACE];
    __shared__ float cf[NLS_G_NGRID];
    const int i = blockIdx.x;
    if (threadIdx.x < NLS_G_TRACE) tr[threadIdx.x] = sample(T, i, threadIdx.x, u);
    for (int k = threadIdx.x; k < NLS_G_NGRID; k += blockDim.x)
        cf[k] = coef[(size_t)i * NLS_G_NGRID + k];
    __syncthreads();
    const double x0 = T.box[4 * i], y0 = T.box[4 * i + 1];
    const double W = T.box[4 * i + 2] - x0, H = T.box[4 * i + 3] - y0;
    const int rb = P.off_n[i], n = P.off_n[i + 1] - rb;
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        const int g = P.l2g[rb + a];
        double v;
        if (M.dflag[g]) {
            v = M.dval[g];
        } else {
            const double xi = (xy[2 * g] - x0) / W, eta = (xy[2 * g + 1] - y0) / H;
            v = coons(tr, xi, eta) + bilinear(cf, xi, eta);
        }
        xpred[rb + a] = v;
    }
}

// Training target of subdomain i: (v(x*) - Coons) at the 256 reference
// nodes, v(x*) = x* on V_i and u elsewhere.
__global__ void __launch_bounds__(NLS_G_NGRID)
k_guess_target(DevGuessTables T, const double* __restrict__ u, const double* __restrict__ xstar,
               float* __restrict__ traw) {
    __shared__ double tr[NLS_G_TRACE];
    const int i = blockIdx.x, k = threadIdx.x;
    if (k < NLS_G_TRACE) tr[k] = sample(T, i, k, u);
    __syncthreads();
    const size_t b = ((size_t)i * NLS_G_IN + NLS_G_TRACE + k) * 3;
    const size_t bl = ((size_t)i * NLS_G_NGRID + k) * 3;
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int loc = T.sloc[bl + c];
        v += T.sw[b + c] * (loc >= 0 ? xstar[loc] : u[T.snode[b + c]]);
    }
    const int p = k % NLS_G_GRID, q = k / NLS_G_GRID;
    const double xi = (double)p / (NLS_G_GRID - 1), eta = (double)q / (NLS_G_GRID - 1);
    traw[(size_t)i * NLS_G_NGRID + k] = (float)(v - coons(tr, xi, eta));
}

// ------------------------------------------------------- bf16 matrix cores
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int GBM = 64, GBN = 64, GBK = 32, GLD = GBK + 8;

// 64 x 64 output tile per workgroup of four waves; each wave owns a 32 x 32
// quarter as 2 x 2 blocks of the 16x16x16 bf16 MFMA.  A and B tiles are
// staged in LDS with k contiguous, so every lane reads its 4 consecutive k
// values of one row of A and one column of B.  Ragged edges read zeros.
__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
    __shared__ uint16_t As[GBM * GLD];
    __shared__ uint16_t Bs[GBN * GLD];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int lr = lane & 15, lk = 4 * (lane >> 4);
    for (int k0 = 0; k0 < g.K; k0 += GBK) {
        for (int e = tid; e < GBM * GBK; e += 256) {
            const int mm = e / GBK, kk = e % GBK;
            const int gm = m0 + mm, gk = k0 + kk;
            As[mm * GLD + kk] = (gm < g.M && gk < g.K) ? g.A[gm * g.sam + gk * g.sak] : (uint16_t)0;
        }
        for (int e = tid; e < GBN * GBK; e += 256) {
            const int nn = e % GBN, kk = e / GBN;
            const int gn = n0 + nn, gk = k0 + kk;
            Bs[nn * GLD + kk] = (gn < g.N && gk < g.K) ? g.B[gk * g.sbk + gn * g.sbn] : (uint16_t)0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GBK; kk += 16) {
            bf16x4 av[2], bv[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const uint16_t* pa = &As[(wm * 32 + t * 16 + lr) * GLD + kk + lk];
                const uint16_t* pb = &Bs[(wn * 32 + t * 16 + lr) * GLD + kk + lk];
                av[t] = bf16x4{(short)pa[0], (short)pa[1], (short)pa[2], (short)pa[3]};
                bv[t] = bf16x4{(short)pb[0], (short)pb[1], (short)pb[2], (short)pb[3]};
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = m0 + wm * 32 + a * 16 + lk + j;
                const int col = n0 + wn * 32 + b * 16 + lr;
                if (row >= g.M || col >= g.N) continue;
                const float v = acc[a][b][j];
                switch (g.epi) {
                case EPI_STORE:
                    g.out[(size_t)row * g.ldo + col] = v;
                    break;
                case EPI_BIAS_GELU: {
                    const float z = v + g.bias[col];
                    if (g.out) g.out[(size_t)row * g.ldo + col] = z;
                    g.outb[(size_t)row * g.ldob + col] = f2bf(gelu(z));
                    break;
                }
                case EPI_BIAS: {
                    float z = v + g.bias[col];
                    if (g.oscale) z = z * g.oscale[col] + g.oshift[col];
                    g.out[(size_t)row * g.ldo + col] = z;
                    break;
                }
                default: {
                    const float d = v * gelu_prime(g.aux[(size_t)row * g.ldaux + col]);
                    g.out[(size_t)row * g.ldo + col] = d;
                    g.outb[(size_t)row * g.ldob + col] = f2bf(d);
                    break;
                }
                }
            }
}

// ------------------------------------------------------------- training
// Column means and deviations of X (n x cols) in FP64; deviations at or
// below 1e-6 max(max deviation, 1) are replaced by 1.
__global__ void k_fit_norm(const float* __restrict__ X, int64_t n, int cols, float* mean,
                           float* dev) {
    __shared__ double red[1024];
    const int c = threadIdx.x;
    double m = 0.0, s = 0.0;
    if (c < cols) {
        for (int64_t r = 0; r < n; ++r) m += (double)X[r * cols + c];
        m /= (double)(n > 0 ? n : 1);
        for (int64_t r = 0; r < n; ++r) {
            const double d = (double)X[r * cols + c] - m;
            s += d * d;
        }
        s = sqrt(s / (double)(n > 0 ? n : 1));
    }
    red[c] = (c < cols) ? s : 0.0;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (c < h) red[c] = fmax(red[c], red[c + h]);
        __syncthreads();
    }
    const double smax = red[0];
    if (c < cols) {
        mean[c] = (float)m;
        dev[c] = (float)((s <= 1e-6 * fmax(smax, 1.0)) ? 1.0 : s);
    }
}

// Rows idx[r] (or r) of the raw inputs and targets, standardised: inputs to
// bfloat16, targets in FP32.  norm = [xm(320) xs(320) ym(256) ys(256)].
__global__ void __launch_bounds__(NLS_G_IN)
k_gather_batch(const float* __restrict__ X, const float* __restrict__ T, const int* __restrict__ idx,
               const float* __restrict__ norm, uint16_t* __restrict__ xb, float* __restrict__ tn) {
    const int r = blockIdx.x, k = threadIdx.x;
    const int64_t src = idx ? (int64_t)idx[r] : (int64_t)r;
    const float* xm = norm;
    const float* xs = norm + NLS_G_IN;
    const float* ym = norm + 2 * NLS_G_IN;
    const float* ys = ym + NLS_G_OUT;
    xb[(size_t)r * NLS_G_IN + k] = f2bf((X[src * NLS_G_IN + k] - xm[k]) / xs[k]);
    if (T && k < NLS_G_OUT) tn[(size_t)r * NLS_G_OUT + k] = (T[src * NLS_G_OUT + k] - ym[k]) / ys[k];
}

// dZ = 2 (Y - Tn) / (rows * 256); per-block partial sums of (Y - Tn)^2.
__global__ void __launch_bounds__(256)
k_mse_grad(const float* __restrict__ Y, const float* __restrict__ Tn, int64_t total, float scale,
           float* __restrict__ dz, uint16_t* __restrict__ dzb, double* __restrict__ partial) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const float d = Y[e] - Tn[e];
        s += (double)d * (double)d;
        const float v = scale * d;
        dz[e] = v;
        dzb[e] = f2bf(v);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_mse_final(const double* __restrict__ partial, int nb, double inv_total,
                            double* __restrict__ loss_acc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[b];
    loss_acc[0] += s * inv_total;
    loss_acc[1] += 1.0;
}

__global__ void k_colsum(const float* __restrict__ dz, int rows, int cols, float* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int r = 0; r < rows; ++r) s += dz[(size_t)r * cols + c];
    out[c] = s;
}

// Adam (Kingma and Ba) with bias corrections c1 = 1/(1-b1^t),
// c2 = 1/(1-b2^t); refreshes the bfloat16 copy of the parameters.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, uint16_t* __restrict__ wb, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    const float wn = w[p] - lr * (mp * c1) / (sqrtf(vp * c2) + eps);
    w[p] = wn;
    wb[p] = f2bf(wn);
}

__global__ void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) y[p] = f2bf(x[p]);
}

// counts[0] += subdomains that started from the prediction, counts[1] +=
// those that fell back to R_i u (start codes 1 and 2).
__global__ void k_count_starts(const int* __restrict__ start, int n, int* __restrict__ counts) {
    __shared__ int c1[256], c2[256];
    int a = 0, b = 0;
    for (int i = threadIdx.x; i < n; i += 256) {
        a += start[i] == 1;
        b += start[i] == 2;
    }
    c1[threadIdx.x] = a;
    c2[threadIdx.x] = b;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            c1[threadIdx.x] += c1[threadIdx.x + h];
            c2[threadIdx.x] += c2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        counts[0] = c1[0];
        counts[1] = c2[0];
    }
}

// flag[0] = 1 if any of idx[0..n) lies outside [0, limit).
__global__ void k_check_indices(const int* __restrict__ idx, int64_t n, int64_t limit,
                                int* __restrict__ flag) {
    int bad = 0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        bad |= (idx[p] < 0 || (int64_t)idx[p] >= limit);
    if (__any(bad) && (threadIdx.x & 63) == 0) flag[0] = 1;
}

}  // namespace

// ----------------------------------------------------------------- launchers
hipError_t launch_check_indices(const int* idx, int64_t n, int64_t limit, int* flag,
                                hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int nb = (int)((n + 255) / 256);
    if (nb > 1024) nb = 1024;
    k_check_indices<<<nb, 256, 0, s>>>(idx, n, limit, flag);
    return hipGetLastError();
}

hipError_t launch_gemm_bf16(const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    dim3 grid((g.N + GBN - 1) / GBN, (g.M + GBM - 1) / GBM);
    k_gemm_bf16<<<grid, 256, 0, s>>>(g);
    return hipGetLastError();
}

hipError_t launch_nodal_load(const DevMesh& M, const double* fmid, double* fhat, hipStream_t s) {
    if (M.N <= 0) return hipSuccess;
    k_nodal_load<<<(M.N + 255) / 256, 256, 0, s>>>(M, fmid, fhat);
    return hipGetLastError();
}

hipError_t launch_guess_features(const DevGuessTables& T, int nrows, const double* u,
                                 const double* fhat, const float* xm, const float* xs,
                                 float* xraw, uint16_t* xbf, hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    if (T.elast)
        k_guess_features_e<<<nrows, NLS_G_IN, 0, s>>>(T, u, fhat, xm, xs, xraw, xbf);
    else
        k_guess_features<<<nrows, NLS_G_IN, 0, s>>>(T, u, fhat, xm, xs, xraw, xbf);
    return hipGetLastError();
}

hipError_t launch_guess_lift(const DevMaps& P, const DevGuessTables& T, const DevMesh& M,
                             const double* xy, const double* u, const float* coef,
                             double* xpred, hipStream_t s) {
    if (T.nsub <= 0) return hipSuccess;
    if (T.elast)
        k_guess_lift_e<<<T.nsub, 256, 0, s>>>(P, T, M, xy, u, coef, xpred);
    else
        k_guess_lift<<<T.nsub, 256, 0, s>>>(P, T, M, xy, u, coef, xpred);
    return hipGetLastError();
}

hipError_t launch_guess_target(const DevGuessTables& T, int nrows, const double* u,
                               const double* xstar, float* traw, hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    if (T.elast)
        k_guess_target_e<<<nrows, NLS_G_OUT, 0, s>>>(T, u, xstar, traw);
    else
        k_guess_target<<<nrows, NLS_G_NGRID, 0, s>>>(T, u, xstar, traw);
    return hipGetLastError();
}

hipError_t launch_fit_norm(const float* X, int64_t n, int cols, float* mean, float* dev,
                           hipStream_t s) {
    if (cols <= 0 || cols > 1024) return hipErrorInvalidValue;
    int bs = 1;
    while (bs < cols) bs <<= 1;
    k_fit_norm<<<1, bs, 0, s>>>(X, n, cols, mean, dev);
    return hipGetLastError();
}

hipError_t launch_gather_batch(const float* X, const float* T, const int* idx, int rows,
                               const float* norm, uint16_t* xb, float* tn, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    k_gather_batch<<<rows, NLS_G_IN, 0, s>>>(X, T, idx, norm, xb, tn);
    return hipGetLastError();
}

hipError_t launch_mse_grad(const float* Y, const float* Tn, int rows, float* dz, uint16_t* dzb,
                           double* partial, double* loss_acc, hipStream_t s) {
    const int64_t total = (int64_t)rows * NLS_G_OUT;
    if (total <= 0) return hipSuccess;
    int nb = (int)((total + 255) / 256);
    if (nb > 256) nb = 256;
    k_mse_grad<<<nb, 256, 0, s>>>(Y, Tn, total, 2.0f / (float)total, dz, dzb, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_mse_final<<<1, 64, 0, s>>>(partial, nb, 1.0 / (double)total, loss_acc);
    return hipGetLastError();
}

hipError_t launch_colsum(const float* dz, int rows, int cols, float* out, hipStream_t s) {
    if (cols <= 0) return hipSuccess;
    k_colsum<<<(cols + 255) / 256, 256, 0, s>>>(dz, rows, cols, out);
    return hipGetLastError();
}

hipError_t launch_adam(float* w, const float* g, float* m, float* v, uint16_t* wb, int64_t n,
                       float lr, float b1, float b2, float eps, float c1, float c2,
                       hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_adam<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(w, g, m, v, wb, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_to_bf16<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, y, n);
    return hipGetLastError();
}

hipError_t launch_count_starts(const int* start, int n, int* counts, hipStream_t s) {
    k_count_starts<<<1, 256, 0, s>>>(start, n, counts);
    return hipGetLastError();
}
