// Device-side views and launchers of the learned initial guess.  Internal,
// not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "nls_device.h"

// Network and sampling sizes: 64 perimeter samples (16 per side), a 16 x 16
// reference grid, affine layers 320 -> 256 -> 256 -> 256 -> 256.
#define NLS_G_SIDE 16
#define NLS_G_TRACE 64
#define NLS_G_GRID 16
#define NLS_G_NGRID 256
#define NLS_G_IN 320
#define NLS_G_WIDTH 256
#define NLS_G_OUT 256
#define NLS_G_NPARAM 279552

// Offsets (floats) of the layer weights W_l [out][in] and biases b_l in the
// flat parameter vector W1 b1 W2 b2 W3 b3 W4 b4.
#define NLS_G_OFF_W1 0
#define NLS_G_OFF_B1 81920
#define NLS_G_OFF_W2 82176
#define NLS_G_OFF_B2 147712
#define NLS_G_OFF_W3 147968
#define NLS_G_OFF_B3 213504
#define NLS_G_OFF_W4 213760
#define NLS_G_OFF_B4 279296

// Elasticity (two dofs per node, Q1): 8 perimeter samples per side (32),
// 128 load samples on the right side of the box, a 16 x 8 reference grid;
// inputs and outputs per component (x then y).
#define NLS_GE_SIDE 8
#define NLS_GE_TRACE 32
#define NLS_GE_LOAD 128
#define NLS_GE_GX 16
#define NLS_GE_GY 8
#define NLS_GE_NGRID 128
#define NLS_GE_NSAMP 288

struct DevGuessTables {
    int nsub;
    int elast;           // 0: scalar P1 layout, 1: elasticity Q1 layout
    const double* box;   // 4 per subdomain: x0, y0, x1, y1
    const int* snode;    // nsub x 320 x 3 (elasticity: nsub x 288 x 4): element nodes
    const double* sw;    // interpolation weights, same layout
    const int* sloc;     // nsub x 256 x 3 (elasticity: nsub x 128 x 4): packed V row of
                         //   a grid-sample node (of its x dof), or -1
};

enum GemmEpilogue {
    EPI_STORE = 0,      // out = acc
    EPI_BIAS_GELU = 1,  // z = acc + bias; out = z; outb = bf16(gelu(z))
    EPI_BIAS = 2,       // z = acc + bias; out = z, or z * oscale + oshift
    EPI_GELU_BWD = 3,   // d = acc * gelu'(aux); out = d; outb = bf16(d)
};

// C[M x N] = A[M x K] B[K x N], bfloat16 operands addressed through
// strides (element (m,k) of A at A[m*sam + k*sak]), FP32 accumulation.
struct GemmArgs {
    int M, N, K;
    const uint16_t* A;
    long sam, sak;
    const uint16_t* B;
    long sbk, sbn;
    int epi;
    const float* bias;
    float* out;
    int ldo;
    uint16_t* outb;
    int ldob;
    const float* aux;
    int ldaux;
    const float* oscale;
    const float* oshift;
};

hipError_t launch_gemm_bf16(const GemmArgs& g, hipStream_t s);
hipError_t launch_nodal_load(const DevMesh& M, const double* fmid, double* fhat, hipStream_t s);
hipError_t launch_guess_features(const DevGuessTables& T, int nrows, const double* u,
                                 const double* fhat, const float* xm, const float* xs,
                                 float* xraw, uint16_t* xbf, hipStream_t s);
hipError_t launch_guess_lift(const DevMaps& P, const DevGuessTables& T, const DevMesh& M,
                             const double* xy, const double* u, const float* coef,
                             double* xpred, hipStream_t s);
hipError_t launch_guess_target(const DevGuessTables& T, int nrows, const double* u,
                               const double* xstar, float* traw, hipStream_t s);
hipError_t launch_fit_norm(const float* X, int64_t n, int cols, float* mean, float* dev,
                           hipStream_t s);
hipError_t launch_gather_batch(const float* X, const float* T, const int* idx, int rows,
                               const float* norm, uint16_t* xb, float* tn, hipStream_t s);
hipError_t launch_mse_grad(const float* Y, const float* Tn, int rows, float* dz, uint16_t* dzb,
                           double* partial, double* loss_acc, hipStream_t s);
hipError_t launch_colsum(const float* dz, int rows, int cols, float* out, hipStream_t s);
hipError_t launch_adam(float* w, const float* g, float* m, float* v, uint16_t* wb, int64_t n,
                       float lr, float b1, float b2, float eps, float c1, float c2,
                       hipStream_t s);
hipError_t launch_to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t s);
hipError_t launch_check_indices(const int* idx, int64_t n, int64_t limit, int* flag,
                                hipStream_t s);
hipError_t launch_count_starts(const int* start, int n, int* counts, hipStream_t s);
