// C ABI of the learned initial guess of the local Newton solves: the network
// (320 -> 256 -> 256 -> 256 -> 256, GELU, bfloat16 matrix-core products
// with FP32 accumulation, FP32 master weights), its training by Adam on
// (features, target) pairs captured from the solver's own converged local
// solves, and the hooks the local level calls around its fused launch.
//
// Features of subdomain i: 64 samples of u on the perimeter of the patch box
// and 256 samples of the nodal load on a 16 x 16 reference grid.  Network
// output: 256 coefficients on that grid; the predicted start is the
// transfinite lifting of the perimeter samples plus their bilinear
// interpolant.  Targets: (v(x*) - lifting) on the grid, where v(x*) is the
// state of eq. (4) at the converged local solution.
#include <cmath>
#include <mutex>

#include "guess_device.h"
#include "handle.h"

namespace {
constexpr int NORM_FLOATS = 2 * NLS_G_IN + 2 * NLS_G_OUT;
const long OFF_W[4] = {NLS_G_OFF_W1, NLS_G_OFF_W2, NLS_G_OFF_W3, NLS_G_OFF_W4};
const long OFF_B[4] = {NLS_G_OFF_B1, NLS_G_OFF_B2, NLS_G_OFF_B3, NLS_G_OFF_B4};
}  // namespace

struct GuessState {
    enum { B_TABLES = 0, B_MODEL, B_INFER, B_CAPTURE, B_BATCH, B_N };
    std::vector<void*> bufs[B_N];
    // sampling tables of the current partition
    bool tables = false;
    DevGuessTables T{};
    double* fhat = nullptr;
    // model: FP32 master weights, Adam moments, gradient, bfloat16 copy,
    // normalisation [xm xs ym ys]
    bool have_model = false;
    float *w = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *norm = nullptr;
    uint16_t* wb = nullptr;
    int64_t t = 0;
    double* lacc = nullptr;   // [sum of step losses, steps]
    double* part = nullptr;   // 256 partial sums
    int* counts = nullptr;    // start statistics
    // inference over the subdomains
    int inf_rows = 0;
    uint16_t *xin = nullptr, *a0 = nullptr, *a1 = nullptr;
    float* y = nullptr;
    double* xpred = nullptr;
    bool enabled = false;
    // within a solve: evaluations left without inference after one whose
    // predictions the judge took for fewer than 1 in 20 subdomains, and
    // whether the current evaluation consulted the network
    int skip = 0;
    bool consulted = false;
    // captured training pairs
    float *cx = nullptr, *ct = nullptr;
    int64_t cap = 0, count = 0;
    // batch buffers (training and test hooks)
    int tb = 0;
    uint16_t *tx = nullptr, *ta[3] = {nullptr, nullptr, nullptr}, *dzb[2] = {nullptr, nullptr};
    float *tz[3] = {nullptr, nullptr, nullptr}, *ty = nullptr, *ttn = nullptr,
          *dz[2] = {nullptr, nullptr};

    void free_group(int gi) {
        for (void* p : bufs[gi]) (void)hipFree(p);
        bufs[gi].clear();
    }
    ~GuessState() {
        for (int gi = 0; gi < B_N; ++gi) free_group(gi);
    }
};

void guess_state_free(GuessState* g) { delete g; }

template <class T>
static int galloc(nls_handle* h, int group, T** out, size_t count) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (hipMalloc(&p, bytes) != hipSuccess) {
        *out = nullptr;
        return fail(h, NLS_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    h->guess->bufs[group].push_back(p);
    *out = (T*)p;
    return NLS_OK;
}

static GuessState* state(nls_handle* h) {
    if (!h->guess) h->guess = new GuessState();
    return h->guess;
}

// --------------------------------------------------------------- tables
static int ensure_tables(nls_handle* h) {
    GuessState* g = state(h);
    if (g->tables) return NLS_OK;
    if (!h->have_part) return fail(h, NLS_ESTATE, "nls_set_partition first");
    const bool elast = h->kind == NLS_PROBLEM_NEOHOOKE;
    if (elast ? (h->mesh.d != 2 || h->mesh.nv != 4) : (h->mesh.d != 1 || h->mesh.nv != 3))
        return fail(h, NLS_EINVAL, "the learned guess needs P1 diffusion or Q1 elasticity");
    HostGuess hg;
    std::string err;
    int rc = nls_build_guess_tables(h->mesh, h->maps, hg, err);
    if (rc) return fail(h, rc, err);
    g->free_group(GuessState::B_TABLES);
    int *snode, *sloc;
    double *sw, *box;
    RC(galloc(h, GuessState::B_TABLES, &snode, hg.snode.size()));
    RC(galloc(h, GuessState::B_TABLES, &sloc, hg.sloc.size()));
    RC(galloc(h, GuessState::B_TABLES, &sw, hg.sw.size()));
    RC(galloc(h, GuessState::B_TABLES, &box, hg.box.size()));
    if (!elast) RC(galloc(h, GuessState::B_TABLES, &g->fhat, (size_t)h->mesh.N));
    HIPCHK(hipMemcpyAsync(snode, hg.snode.data(), hg.snode.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(sloc, hg.sloc.data(), hg.sloc.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(sw, hg.sw.data(), hg.sw.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(box, hg.box.data(), hg.box.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
    g->T.nsub = h->maps.nsub;
    g->T.elast = elast ? 1 : 0;
    g->T.box = box;
    g->T.snode = snode;
    g->T.sw = sw;
    g->T.sloc = sloc;
    if (!elast)
        HIPCHK(launch_nodal_load(h->dm, h->fmid_h.empty() ? nullptr : h->d_fmid, g->fhat, h->stream));
    RC(sync(h));
    g->tables = true;
    return NLS_OK;
}

// Called when the partition changes: tables and per-subdomain buffers go,
// the model and the captured pairs stay.
void guess_invalidate(nls_handle* h) {
    if (!h->guess) return;
    GuessState* g = h->guess;
    g->free_group(GuessState::B_TABLES);
    g->free_group(GuessState::B_INFER);
    g->tables = false;
    g->inf_rows = 0;
    g->T = DevGuessTables{};
}

int guess_refresh_load(nls_handle* h) {
    GuessState* g = h->guess;
    if (!g || !g->tables || g->T.elast) return NLS_OK;
    HIPCHK(launch_nodal_load(h->dm, h->fmid_h.empty() ? nullptr : h->d_fmid, g->fhat, h->stream));
    return NLS_OK;
}

// --------------------------------------------------------------- network
static int ensure_batch(nls_handle* h, int rows) {
    GuessState* g = state(h);
    if (g->tb >= rows) return NLS_OK;
    g->free_group(GuessState::B_BATCH);
    const size_t r = (size_t)rows;
    RC(galloc(h, GuessState::B_BATCH, &g->tx, r * NLS_G_IN));
    for (int l = 0; l < 3; ++l) {
        RC(galloc(h, GuessState::B_BATCH, &g->ta[l], r * NLS_G_WIDTH));
        RC(galloc(h, GuessState::B_BATCH, &g->tz[l], r * NLS_G_WIDTH));
    }
    for (int l = 0; l < 2; ++l) {
        RC(galloc(h, GuessState::B_BATCH, &g->dz[l], r * NLS_G_WIDTH));
        RC(galloc(h, GuessState::B_BATCH, &g->dzb[l], r * NLS_G_WIDTH));
    }
    RC(galloc(h, GuessState::B_BATCH, &g->ty, r * NLS_G_OUT));
    RC(galloc(h, GuessState::B_BATCH, &g->ttn, r * NLS_G_OUT));
    g->tb = rows;
    return NLS_OK;
}

// Four affine layers on standardised bfloat16 inputs x0 (rows x 320).
// z (optional) receives the FP32 pre-activations of layers 1-3, a the
// bfloat16 activations; y the output, un-standardised when unstd.
static int forward(nls_handle* h, const uint16_t* x0, int rows, float* const* z,
                   uint16_t* const* a, float* y, bool unstd) {
    GuessState* g = h->guess;
    for (int l = 0; l < 4; ++l) {
        const int in = l == 0 ? NLS_G_IN : NLS_G_WIDTH;
        GemmArgs ga{};
        ga.M = rows;
        ga.N = NLS_G_WIDTH;
        ga.K = in;
        ga.A = l == 0 ? x0 : a[l - 1];
        ga.sam = in;
        ga.sak = 1;
        ga.B = g->wb + OFF_W[l];
        ga.sbk = 1;
        ga.sbn = in;
        ga.bias = g->w + OFF_B[l];
        if (l < 3) {
            ga.epi = EPI_BIAS_GELU;
            ga.out = z ? z[l] : nullptr;
            ga.ldo = NLS_G_WIDTH;
            ga.outb = a[l];
            ga.ldob = NLS_G_WIDTH;
        } else {
            ga.epi = EPI_BIAS;
            ga.out = y;
            ga.ldo = NLS_G_OUT;
            if (unstd) {
                ga.oscale = g->norm + 2 * NLS_G_IN + NLS_G_OUT;
                ga.oshift = g->norm + 2 * NLS_G_IN;
            }
        }
        HIPCHK(launch_gemm_bf16(ga, h->stream));
    }
    return NLS_OK;
}

// MSE gradient of the batch in the batch buffers (ty against ttn) into
// g->grad; the step loss is added to lacc.
static int backward(nls_handle* h, const uint16_t* x0, int rows) {
    GuessState* g = h->guess;
    HIPCHK(launch_mse_grad(g->ty, g->ttn, rows, g->dz[0], g->dzb[0], g->part, g->lacc, h->stream));
    int cur = 0;
    for (int l = 3; l >= 0; --l) {
        const int in = l == 0 ? NLS_G_IN : NLS_G_WIDTH;
        GemmArgs gw{};
        gw.M = NLS_G_WIDTH;
        gw.N = in;
        gw.K = rows;
        gw.A = g->dzb[cur];
        gw.sam = 1;
        gw.sak = NLS_G_WIDTH;
        gw.B = l == 0 ? x0 : g->ta[l - 1];
        gw.sbk = in;
        gw.sbn = 1;
        gw.epi = EPI_STORE;
        gw.out = g->grad + OFF_W[l];
        gw.ldo = in;
        HIPCHK(launch_gemm_bf16(gw, h->stream));
        HIPCHK(launch_colsum(g->dz[cur], rows, NLS_G_WIDTH, g->grad + OFF_B[l], h->stream));
        if (l > 0) {
            GemmArgs gd{};
            gd.M = rows;
            gd.N = NLS_G_WIDTH;
            gd.K = NLS_G_WIDTH;
            gd.A = g->dzb[cur];
            gd.sam = NLS_G_WIDTH;
            gd.sak = 1;
            gd.B = g->wb + OFF_W[l];
            gd.sbk = NLS_G_WIDTH;
            gd.sbn = 1;
            gd.epi = EPI_GELU_BWD;
            gd.aux = g->tz[l - 1];
            gd.ldaux = NLS_G_WIDTH;
            gd.out = g->dz[1 - cur];
            gd.ldo = NLS_G_WIDTH;
            gd.outb = g->dzb[1 - cur];
            gd.ldob = NLS_G_WIDTH;
            HIPCHK(launch_gemm_bf16(gd, h->stream));
            cur = 1 - cur;
        }
    }
    return NLS_OK;
}

static int need_model(nls_handle* h) {
    if (!h->guess || !h->guess->have_model) return fail(h, NLS_ESTATE, "no network: nls_guess_set_model first");
    return NLS_OK;
}

// The nodal load field the features sample: f^ (diffusion), or the external
// nodal forces with Dirichlet dofs zeroed (elasticity), kept current by the
// load setters.
static const double* load_field(const nls_handle* h) {
    return h->guess->T.elast ? h->dm.bload : h->guess->fhat;
}

// ------------------------------------------------------- evaluate hooks
bool guess_enabled(const nls_handle* h) { return h->guess && h->guess->enabled; }

// Inference gating restarts with every solve.
void guess_new_solve(nls_handle* h) {
    if (h->guess) {
        h->guess->skip = 0;
        h->guess->consulted = false;
    }
}

// Evaluations a solve runs without inference after one whose predictions
// were almost all rejected (the start is then R_i u, as without a network).
#define NLS_GUESS_SKIP 2

// Predicted starts of every subdomain at u (packed like the V rows).
int guess_prepare(nls_handle* h, const double* u, const double** xpred) {
    GuessState* g = h->guess;
    g->consulted = false;
    if (h->st && g->skip > 0) {
        --g->skip;
        *xpred = nullptr;
        return NLS_OK;
    }
    g->consulted = true;
    RC(ensure_tables(h));
    const int ns = h->maps.nsub;
    if (g->inf_rows < ns) {
        g->free_group(GuessState::B_INFER);
        RC(galloc(h, GuessState::B_INFER, &g->xin, (size_t)ns * NLS_G_IN));
        RC(galloc(h, GuessState::B_INFER, &g->a0, (size_t)ns * NLS_G_WIDTH));
        RC(galloc(h, GuessState::B_INFER, &g->a1, (size_t)ns * NLS_G_WIDTH));
        RC(galloc(h, GuessState::B_INFER, &g->y, (size_t)ns * NLS_G_OUT));
        RC(galloc(h, GuessState::B_INFER, &g->xpred, (size_t)h->maps.off_n.back()));
        g->inf_rows = ns;
    }
    HIPCHK(launch_guess_features(g->T, ns, u, load_field(h), g->norm, g->norm + NLS_G_IN, nullptr,
                                 g->xin, h->stream));
    uint16_t* acts[3] = {g->a0, g->a1, g->a0};
    RC(forward(h, g->xin, ns, nullptr, acts, g->y, true));
    HIPCHK(launch_guess_lift(h->dp, g->T, h->dm, h->d_xy, u, g->y, g->xpred, h->stream));
    *xpred = g->xpred;
    return NLS_OK;
}

// After successful local solves at u: capture (features, target) pairs and
// count how the subdomains started.
int guess_after_local(nls_handle* h, const double* u) {
    GuessState* g = h->guess;
    if (!g) return NLS_OK;
    const int ns = h->maps.nsub;
    if (g->cap > 0 && g->count < g->cap) {
        RC(ensure_tables(h));
        const int rows = (int)std::min<int64_t>(ns, g->cap - g->count);
        HIPCHK(launch_guess_features(g->T, rows, u, load_field(h), nullptr, nullptr,
                                     g->cx + g->count * NLS_G_IN, nullptr, h->stream));
        HIPCHK(launch_guess_target(g->T, rows, u, h->dl.xstar, g->ct + g->count * NLS_G_OUT,
                                   h->stream));
        g->count += rows;
    }
    if (g->enabled && h->st && g->counts && g->consulted) {
        int c[2] = {0, 0};
        HIPCHK(launch_count_starts(h->dl.start, ns, g->counts, h->stream));
        HIPCHK(hipMemcpyAsync(c, g->counts, sizeof(c), hipMemcpyDeviceToHost, h->stream));
        RC(sync(h));
        h->st->guess_used += c[0];
        h->st->guess_fallback += c[1];
        if (20 * c[0] < ns) g->skip = NLS_GUESS_SKIP;
    }
    return NLS_OK;
}

// ------------------------------------------------------------------ ABI
extern "C" int nls_guess_set_model(nls_handle* h, const float* params, int64_t n_params,
                                   const float* norm) {
    if (!h || !params) return NLS_EINVAL;
    if (n_params != NLS_G_NPARAM)
        return fail(h, NLS_EINVAL, "the network has " + std::to_string(NLS_G_NPARAM) + " parameters");
    for (int64_t k = 0; k < n_params; ++k)
        if (!std::isfinite(params[k])) return fail(h, NLS_EINVAL, "parameters must be finite");
    std::vector<float> nm(NORM_FLOATS);
    if (norm) {
        nm.assign(norm, norm + NORM_FLOATS);
        for (int k = 0; k < NORM_FLOATS; ++k)
            if (!std::isfinite(nm[k])) return fail(h, NLS_EINVAL, "normalisation must be finite");
        for (int k = NLS_G_IN; k < 2 * NLS_G_IN; ++k)
            if (!(nm[k] > 0.f)) return fail(h, NLS_EINVAL, "input deviations must be positive");
        for (int k = 2 * NLS_G_IN + NLS_G_OUT; k < NORM_FLOATS; ++k)
            if (!(nm[k] > 0.f)) return fail(h, NLS_EINVAL, "output deviations must be positive");
    } else {
        std::fill(nm.begin(), nm.end(), 0.f);
        std::fill(nm.begin() + NLS_G_IN, nm.begin() + 2 * NLS_G_IN, 1.f);
        std::fill(nm.begin() + 2 * NLS_G_IN + NLS_G_OUT, nm.end(), 1.f);
    }
    HIPCHK(hipSetDevice(h->opt.device));
    GuessState* g = state(h);
    if (!g->have_model) {
        RC(galloc(h, GuessState::B_MODEL, &g->w, NLS_G_NPARAM));
        RC(galloc(h, GuessState::B_MODEL, &g->m, NLS_G_NPARAM));
        RC(galloc(h, GuessState::B_MODEL, &g->v, NLS_G_NPARAM));
        RC(galloc(h, GuessState::B_MODEL, &g->grad, NLS_G_NPARAM));
        RC(galloc(h, GuessState::B_MODEL, &g->wb, NLS_G_NPARAM));
        RC(galloc(h, GuessState::B_MODEL, &g->norm, NORM_FLOATS));
        RC(galloc(h, GuessState::B_MODEL, &g->lacc, 2));
        RC(galloc(h, GuessState::B_MODEL, &g->part, 256));
        RC(galloc(h, GuessState::B_MODEL, &g->counts, 2));
    }
    HIPCHK(hipMemcpyAsync(g->w, params, NLS_G_NPARAM * sizeof(float), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(g->norm, nm.data(), NORM_FLOATS * sizeof(float), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemsetAsync(g->m, 0, NLS_G_NPARAM * sizeof(float), h->stream));
    HIPCHK(hipMemsetAsync(g->v, 0, NLS_G_NPARAM * sizeof(float), h->stream));
    HIPCHK(launch_to_bf16(g->w, g->wb, NLS_G_NPARAM, h->stream));
    RC(sync(h));
    g->t = 0;
    g->have_model = true;
    return NLS_OK;
}

extern "C" int nls_guess_get_model(nls_handle* h, float* params, float* norm) {
    if (!h) return NLS_EINVAL;
    RC(need_model(h));
    GuessState* g = h->guess;
    if (params)
        HIPCHK(hipMemcpyAsync(params, g->w, NLS_G_NPARAM * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    if (norm)
        HIPCHK(hipMemcpyAsync(norm, g->norm, NORM_FLOATS * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    return sync(h);
}

extern "C" int nls_guess_enable(nls_handle* h, int enable) {
    if (!h) return NLS_EINVAL;
    if (enable) RC(need_model(h));
    if (h->guess) h->guess->enabled = enable != 0;
    h->have_state = false;
    return NLS_OK;
}

extern "C" int nls_guess_capture(nls_handle* h, int64_t capacity) {
    if (!h || capacity < 0) return NLS_EINVAL;
    HIPCHK(hipSetDevice(h->opt.device));
    GuessState* g = state(h);
    g->free_group(GuessState::B_CAPTURE);
    g->cx = g->ct = nullptr;
    g->cap = g->count = 0;
    if (capacity > 0) {
        RC(galloc(h, GuessState::B_CAPTURE, &g->cx, (size_t)capacity * NLS_G_IN));
        RC(galloc(h, GuessState::B_CAPTURE, &g->ct, (size_t)capacity * NLS_G_OUT));
        g->cap = capacity;
    }
    return NLS_OK;
}

extern "C" int nls_guess_captured(nls_handle* h, float* X, float* T, int64_t max_rows,
                                  int64_t* n_rows) {
    if (!h || !n_rows || max_rows < 0) return NLS_EINVAL;
    GuessState* g = h->guess;
    const int64_t have = g ? g->count : 0;
    const int64_t r = std::min(have, max_rows);
    *n_rows = (X || T) ? r : have;
    if (r > 0 && X)
        HIPCHK(hipMemcpyAsync(X, g->cx, r * NLS_G_IN * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    if (r > 0 && T)
        HIPCHK(hipMemcpyAsync(T, g->ct, r * NLS_G_OUT * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    return sync(h);
}

extern "C" int nls_guess_features(nls_handle* h, const double* u, float* X) {
    if (!h || !u || !X) return NLS_EINVAL;
    HIPCHK(hipSetDevice(h->opt.device));
    RC(ensure_tables(h));
    GuessState* g = h->guess;
    HIPCHK(launch_guess_features(g->T, h->maps.nsub, u, load_field(h), nullptr, nullptr, X, nullptr, h->stream));
    return sync(h);
}

extern "C" int nls_guess_lift(nls_handle* h, const double* u, const float* coef, double* xpred) {
    if (!h || !u || !coef || !xpred) return NLS_EINVAL;
    HIPCHK(hipSetDevice(h->opt.device));
    RC(ensure_tables(h));
    HIPCHK(launch_guess_lift(h->dp, h->guess->T, h->dm, h->d_xy, u, coef, xpred, h->stream));
    return sync(h);
}

extern "C" int nls_guess_predict(nls_handle* h, const float* X, int64_t n, float* Y) {
    if (!h || n < 0 || (n > 0 && (!X || !Y))) return NLS_EINVAL;
    if (n > (1 << 20)) return fail(h, NLS_ELIMIT, "at most 2^20 rows per call");
    RC(need_model(h));
    HIPCHK(hipSetDevice(h->opt.device));
    if (n == 0) return NLS_OK;
    GuessState* g = h->guess;
    RC(ensure_batch(h, (int)n));
    HIPCHK(launch_gather_batch(X, nullptr, nullptr, (int)n, g->norm, g->tx, nullptr, h->stream));
    RC(forward(h, g->tx, (int)n, nullptr, g->ta, Y, true));
    return sync(h);
}

// ------------------------------------------- allocation-free inference
// Working storage of nls_guess_predict_noalloc: a file-scope device array
// (each GPU holds its own copy until the process ends), so that the call
// allocates nothing.  Layout: the standardised bfloat16 inputs (rows x 320),
// then two bfloat16 activation buffers (rows x 256) that layers 1-3 write in
// turn.  Every call on a GPU shares that GPU's copy; nothing in it needs to
// start at zero (each call writes what it reads).
namespace {
constexpr int NOALLOC_ROWS = NLS_GUESS_NOALLOC_ROWS;
constexpr size_t SCRATCH_IN = (size_t)NOALLOC_ROWS * NLS_G_IN;      // bfloat16 elements
constexpr size_t SCRATCH_ACT = (size_t)NOALLOC_ROWS * NLS_G_WIDTH;  // per activation buffer
constexpr size_t SCRATCH_BYTES = (SCRATCH_IN + 2 * SCRATCH_ACT) * sizeof(uint16_t);
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_dev[SCRATCH_MAX_DEVICES] = {};  // device address of scratch, per device
}  // namespace

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

// Device address of this GPU's scratch array, looked up once per device
// with that device current (called by nls_create).  In host code the name
// scratch is not a device address; only the looked-up pointer is used.
int guess_scratch_setup(int device, std::string& err) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) {
        err = "device ordinal out of range";
        return NLS_EINVAL;
    }
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_dev[device]) return NLS_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return NLS_EHIP;
    }
    scratch_dev[device] = p;
    return NLS_OK;
}

extern "C" int nls_guess_predict_noalloc(nls_handle* h, const float* X, int64_t n, float* Y) {
    if (!h || n < 0 || (n > 0 && (!X || !Y))) return NLS_EINVAL;
    if (n > NOALLOC_ROWS)
        return fail(h, NLS_ELIMIT, "nls_guess_predict_noalloc takes at most " +
                                       std::to_string(NOALLOC_ROWS) + " rows per call");
    RC(need_model(h));
    const int dev = h->opt.device;
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES || !scratch_dev[dev])
        return fail(h, NLS_ESTATE, "no scratch address for this device");
    HIPCHK(hipSetDevice(dev));
    if (n == 0) return NLS_OK;
    GuessState* g = h->guess;
    uint16_t* tx = (uint16_t*)scratch_dev[dev];
    uint16_t* a0 = tx + SCRATCH_IN;
    uint16_t* a1 = a0 + SCRATCH_ACT;
    uint16_t* const act[3] = {a0, a1, a0};  // layer l reads act[l-1], writes act[l]
    HIPCHK(launch_gather_batch(X, nullptr, nullptr, (int)n, g->norm, tx, nullptr, h->stream));
    RC(forward(h, tx, (int)n, nullptr, act, Y, true));
    HIPCHK(hipGetLastError());
    return NLS_OK;
}

extern "C" int nls_guess_loss_grad(nls_handle* h, const float* X, const float* T, int64_t n,
                                   float* grad, double* loss) {
    if (!h || !X || !T || n <= 0) return NLS_EINVAL;
    if (n > 65536) return fail(h, NLS_ELIMIT, "at most 65536 rows per call");
    RC(need_model(h));
    HIPCHK(hipSetDevice(h->opt.device));
    GuessState* g = h->guess;
    RC(ensure_batch(h, (int)n));
    HIPCHK(launch_gather_batch(X, T, nullptr, (int)n, g->norm, g->tx, g->ttn, h->stream));
    RC(forward(h, g->tx, (int)n, g->tz, g->ta, g->ty, false));
    HIPCHK(hipMemsetAsync(g->lacc, 0, 2 * sizeof(double), h->stream));
    RC(backward(h, g->tx, (int)n));
    if (grad)
        HIPCHK(hipMemcpyAsync(grad, g->grad, NLS_G_NPARAM * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    double la[2] = {0.0, 0.0};
    HIPCHK(hipMemcpyAsync(la, g->lacc, sizeof(la), hipMemcpyDeviceToHost, h->stream));
    RC(sync(h));
    if (loss) *loss = la[0];
    return NLS_OK;
}

extern "C" int nls_guess_train(nls_handle* h, const nls_train_opts* o, const float* X,
                               const float* T, int64_t n, const int32_t* order,
                               nls_train_stats* st) {
    if (!h || !o || !X || !T || n <= 0) return NLS_EINVAL;
    if (o->epochs < 0 || o->batch <= 0 || o->batch > 65536 || !(o->lr > 0.0) ||
        !(o->beta1 >= 0.0 && o->beta1 < 1.0) || !(o->beta2 >= 0.0 && o->beta2 < 1.0) ||
        !(o->eps > 0.0))
        return fail(h, NLS_EINVAL, "bad training options");
    RC(need_model(h));
    HIPCHK(hipSetDevice(h->opt.device));
    GuessState* g = h->guess;
    Timer tm;
    if (order) {
        int bad = 0;
        HIPCHK(hipMemsetAsync(g->counts, 0, sizeof(int), h->stream));
        HIPCHK(launch_check_indices(order, (int64_t)o->epochs * n, n, g->counts, h->stream));
        HIPCHK(hipMemcpyAsync(&bad, g->counts, sizeof(int), hipMemcpyDeviceToHost, h->stream));
        RC(sync(h));
        if (bad) return fail(h, NLS_EINVAL, "order holds an index outside [0, n)");
    }
    if (o->flags & NLS_TRAIN_FIT_NORM) {
        HIPCHK(launch_fit_norm(X, n, NLS_G_IN, g->norm, g->norm + NLS_G_IN, h->stream));
        HIPCHK(launch_fit_norm(T, n, NLS_G_OUT, g->norm + 2 * NLS_G_IN,
                               g->norm + 2 * NLS_G_IN + NLS_G_OUT, h->stream));
    }
    const int B = (int)std::min<int64_t>(o->batch, n);
    RC(ensure_batch(h, B));
    const int64_t steps_per_epoch = (n + B - 1) / B;
    const int64_t total = steps_per_epoch * (int64_t)o->epochs;
    int64_t step = 0;
    if (st) std::memset(st, 0, sizeof(*st));
    for (int e = 0; e < o->epochs; ++e) {
        HIPCHK(hipMemsetAsync(g->lacc, 0, 2 * sizeof(double), h->stream));
        for (int64_t s = 0; s < steps_per_epoch; ++s, ++step) {
            const int rows = (int)std::min<int64_t>(B, n - s * B);
            if (order)
                HIPCHK(launch_gather_batch(X, T, order + (int64_t)e * n + s * B, rows, g->norm,
                                           g->tx, g->ttn, h->stream));
            else
                HIPCHK(launch_gather_batch(X + s * B * NLS_G_IN, T + s * B * NLS_G_OUT, nullptr,
                                           rows, g->norm, g->tx, g->ttn, h->stream));
            RC(forward(h, g->tx, rows, g->tz, g->ta, g->ty, false));
            RC(backward(h, g->tx, rows));
            g->t += 1;
            double lr = o->lr;
            if (o->flags & NLS_TRAIN_COSINE)
                lr = o->lr * 0.5 * (1.0 + std::cos(M_PI * (double)step / (double)std::max<int64_t>(total, 1)));
            const double c1 = 1.0 / (1.0 - std::pow(o->beta1, (double)g->t));
            const double c2 = 1.0 / (1.0 - std::pow(o->beta2, (double)g->t));
            HIPCHK(launch_adam(g->w, g->grad, g->m, g->v, g->wb, NLS_G_NPARAM, (float)lr,
                               (float)o->beta1, (float)o->beta2, (float)o->eps, (float)c1,
                               (float)c2, h->stream));
        }
        double la[2] = {0.0, 0.0};
        HIPCHK(hipMemcpyAsync(la, g->lacc, sizeof(la), hipMemcpyDeviceToHost, h->stream));
        RC(sync(h));
        const double el = la[1] > 0 ? la[0] / la[1] : 0.0;
        if (!std::isfinite(el)) return fail(h, NLS_ENAN, "non-finite training loss");
        if (st) {
            if (e < NLS_MAX_EPOCHS) st->epoch_loss[e] = el;
            st->final_loss = el;
        }
    }
    RC(sync(h));
    if (st) {
        st->steps = step;
        st->ms = tm.ms();
    }
    return NLS_OK;
}
