// The solver handle: host state, device buffers and the helpers every
// entry point of libnls uses.  Internal, not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "nls.h"
#include "nls_device.h"
#include "nls_internal.h"

struct GuessState;  // learned initial guess (guess_api.cpp)
void guess_state_free(GuessState* g);

enum BufGroup { G_MESH = 0, G_MAPS = 1, G_COARSE = 2, G_NGROUPS = 3 };

struct Timer {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
            .count();
    }
};

struct nls_handle {
    nls_options opt{};
    hipStream_t stream = nullptr;
    std::string err;
    HostMesh mesh;
    bool have_mesh = false, have_part = false, have_coarse = false, have_state = false;
    int kind = NLS_PROBLEM_DIFFUSION;
    double beta = 1.0;
    double mu = 0.0, lam = 0.0;                // elasticity
    std::vector<double> kappa_h, fmid_h;
    std::vector<double> fnode_h;               // nodal forces (elasticity), ndof
    std::vector<int> part_h;
    HostMaps maps;
    HostCoarse co;
    std::vector<void*> bufs[G_NGROUPS];
    DevMesh dm{};
    DevMaps dp{};
    DevLocal dl{};
    DevCoarse dc{};
    DevTangent dt{};
    bool tangent_w = false;       // W_i = J^{-1} B on owned rows (else per-apply solves)
    bool w_stream = false;        // W read with nontemporal loads (too large to stay cached)
    int tangent_bucket = 0, max_ng = 0;
    int tangent_nblk = 0, tangent_nkk = 0;  // > 0: W_i by the blocked matrix-core solve
    bool coarse_inv = false;      // explicit A0^{-1} for the tangent
    bool coarse_lu_valid = false; // a factorisation of A0 is held (chord steps)
    bool coarse_inv_valid = false; // a0inv is the inverse of that factorisation
    bool tangent_ready = false;   // prepare_tangent ran at the last evaluated point
    bool local_factored = false;  // J_ii and its LU at the last evaluation's x* are held
    bool nks_mode = false;        // GMRES operator is DF(u) M^{-1} (Newton-Krylov-Schwarz)
    const double* nks_u = nullptr; // the NKS iterate the preconditioner was factored at
    int coarse_ldu = 1, max_block = 0;  // widest coarse band (kl + ku + 1), largest diagonal block
    bool coarse_can_inv = false;        // the explicit inverse fits (LDS, band width)
    // size buckets of the local-solve launches: [start, end) in the launch
    // order, LDS bytes and solve width of each
    std::vector<int> bk_start, bk_end, bk_lds, bk_npl;
    std::vector<int> bk_var;      // LU variant of each bucket (see NewtonParams)
    bool tuned = false;           // NLS_FLAG_AUTOTUNE decisions taken
    double tune_ms[3] = {0.0, 0.0, 0.0};  // coarse: inverse, inverse apply, LU solve
    double* rhs2 = nullptr;
    NewtonParams np{};
    double b_inf = 0.0, phib_inf = 0.0;
    int npl_local = 1, lds_local = 0, lds_tangent = 0;
    int npl_coarse = 1, lds_coarse_lu = 0, lds_coarse_q = 0;
    // GMRES / outer workspace
    int m = 0;
    double *V = nullptr, *wv = nullptr, *hbuf = nullptr, *hbuf2 = nullptr, *hn2 = nullptr,
           *partial = nullptr, *Fx = nullptr, *du = nullptr, *tmp = nullptr, *zbuf = nullptr, *ctmp = nullptr,
           *ydev = nullptr, *ubuf = nullptr;
    int* stat2 = nullptr;
    int nb_dot = 0;
    // pinned host memory for the small device-to-host reads of the driver
    // (status words, norms, iteration counts): bytes [0, 256) for the main
    // stream, [256, 512) the coarse stream, [512, 1024) the GMRES graph
    // stream, from 1024 the per-subdomain inner iteration counts
    void* pin = nullptr;
    size_t pin_bytes = 0;
    // problem data kept on the device for nls_set_load
    const double *d_xy = nullptr, *d_coef = nullptr;
    double* d_fmid = nullptr;
    int* d_bad = nullptr;
    double *d_part = nullptr, *d_mx = nullptr;
    // learned initial guess (null until first used)
    GuessState* guess = nullptr;
    // GMRES cycles with device-side rotations; blocks of gblock Arnoldi
    // steps captured once as HIP graphs and replayed on gstream
    hipStream_t gstream = nullptr;
    // second stream of NLS_FLAG_OVERLAP (coarse Newton beside the local
    // solves, coarse term of the tangent beside its local term); cev[0..1]
    // order the evaluation and tangent preparation, cev[2..3] the fork and
    // join inside a tangent product
    hipStream_t cstream = nullptr;
    // size buckets of the local kernels after the first run on streams of
    // their own, forked from and joined back into the launching stream
    std::vector<hipStream_t> bstream;
    std::vector<hipEvent_t> bev;
    hipEvent_t cev[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t gev[2] = {nullptr, nullptr};
    std::vector<hipGraphExec_t> gexec;
    double *Hd = nullptr, *csd = nullptr, *snd = nullptr, *gd = nullptr, *gtol = nullptr;
    int* gst = nullptr;
    int gblock = 4;
    void drop_graphs() {
        for (auto e : gexec)
            if (e) (void)hipGraphExecDestroy(e);
        gexec.clear();
    }
    std::vector<int> its_h;
    nls_stats* st = nullptr;  // stats of the running solve (may be null)
    // event pairs of profiled launches (kind 0: local Newton, 1: tangent)
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;
    bool profiling() const { return (opt.flags & NLS_FLAG_PROFILE) != 0 && st != nullptr; }
    hipEvent_t take_event() {
        if (!ev_pool.empty()) {
            hipEvent_t e = ev_pool.back();
            ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    void collect_events() {
        for (auto& u : ev_used) {
            float ms = 0.f;
            (void)hipEventSynchronize(u.second.second);
            (void)hipEventElapsedTime(&ms, u.second.first, u.second.second);
            if (st) {
                if (u.first == 0) { st->n_local_launches++; st->ms_local_kernel += ms; }
                else { st->n_tangent_launches++; st->ms_tangent_kernel += ms; }
            }
            ev_pool.push_back(u.second.first);
            ev_pool.push_back(u.second.second);
        }
        ev_used.clear();
    }

    ~nls_handle() {
        guess_state_free(guess);
        drop_graphs();
        for (auto e : gev)
            if (e) (void)hipEventDestroy(e);
        if (gstream) (void)hipStreamDestroy(gstream);
        if (pin) (void)hipHostFree(pin);
        if (cstream) (void)hipStreamDestroy(cstream);
        for (hipStream_t q : bstream) (void)hipStreamDestroy(q);
        for (hipEvent_t e : bev) (void)hipEventDestroy(e);
        for (hipEvent_t& e : cev)
            if (e) (void)hipEventDestroy(e);
        for (auto& g : bufs)
            for (void* p : g) (void)hipFree(p);
        for (auto& u : ev_used) {
            (void)hipEventDestroy(u.second.first);
            (void)hipEventDestroy(u.second.second);
        }
        for (auto e : ev_pool) (void)hipEventDestroy(e);
    }
    void free_group(int g) {
        for (void* p : bufs[g]) (void)hipFree(p);
        bufs[g].clear();
    }
    template <class T>
    int alloc(int group, T** out, size_t count) {
        void* p = nullptr;
        size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        if (hipMalloc(&p, bytes) != hipSuccess) {
            err = "device allocation of " + std::to_string(bytes) + " bytes failed";
            *out = nullptr;
            return NLS_ENOMEM;
        }
        bufs[group].push_back(p);
        *out = (T*)p;
        return NLS_OK;
    }
    template <class T>
    int upload(int group, T** out, const std::vector<T>& h) {
        int rc = alloc(group, out, h.size());
        if (rc) return rc;
        if (!h.empty() &&
            hipMemcpyAsync(*out, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, stream) !=
                hipSuccess) {
            err = "host-to-device copy failed";
            return NLS_EHIP;
        }
        return NLS_OK;
    }
};

#define HIPCHK(x)                                                          \
    do {                                                                   \
        hipError_t e_ = (x);                                               \
        if (e_ != hipSuccess) {                                            \
            h->err = std::string(#x) + ": " + hipGetErrorString(e_);       \
            return NLS_EHIP;                                               \
        }                                                                  \
    } while (0)
#define RC(x)                   \
    do {                        \
        int rc_ = (x);          \
        if (rc_ != NLS_OK) return rc_; \
    } while (0)

inline int fail(nls_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

inline int sync(nls_handle* h) {
    HIPCHK(hipStreamSynchronize(h->stream));
    return NLS_OK;
}

