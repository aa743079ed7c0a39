// C ABI of libnls: handle, setup, and the outer Newton-GMRES driver of
// two-level nonlinear restricted additive Schwarz (paper, Section 2).
//
// The driver runs on the host thread and launches every numerical step as
// a HIP kernel on the handle's stream:
//   F_x(u)   local nonlinear solves (one fused launch over all subdomains),
//            coarse Newton iteration (eq. 9), restricted prolongation and
//            additive combination (eqs. 5, 8, 10);
//   tangent  y = v + sum_i P~_i J_ii^{-1} B_i v_Gi + Phi A0^{-1} Phi^T DF(u_0) v
//            (eqs. 6, 7, 12, using R_i DF(u_i) v = J_ii R_i v + B_i v_Gi);
//   GMRES    restarted, classical Gram-Schmidt with one reorthogonalisation,
//            Givens rotations on the host (a few scalars per iteration);
//   Newton   u <- u - du (eq. 13).
#include <hip/hip_runtime.h>

#include <atomic>
#include <memory>
#include <numeric>
#include <thread>

#include "handle.h"

void guess_invalidate(nls_handle* h);
int guess_scratch_setup(int device, std::string& err);

// ---------------------------------------------------------------------------
extern "C" int nls_default_options(nls_options* o) {
    if (!o) return NLS_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->device = 0;
    o->stream = nullptr;
    o->precision = NLS_PREC_FP64;
    o->coupling = NLS_ONE_LEVEL;
    o->outer_rtol = 1e-8;
    o->outer_maxit = 50;
    o->inner_rtol = 1e-12;
    o->inner_eta = 1e-10;
    o->stagnation = 1e-14;
    o->inner_maxit = 30;
    o->gmres_rtol = 1e-6;
    o->gmres_maxit = 1000;
    o->gmres_restart = 50;
    o->flags = 0;
    return NLS_OK;
}

extern "C" int nls_create(const nls_options* opt, nls_handle** out) {
    if (opt && (opt->lu_variant < 0 || opt->lu_variant > 3)) return NLS_EINVAL;
    if (!opt || !out) return NLS_EINVAL;
    if (opt->precision != NLS_PREC_FP64 && opt->precision != NLS_PREC_FP32_IR &&
        opt->precision != NLS_PREC_BF16_IR)
        return NLS_EINVAL;
    if (opt->coupling != NLS_ONE_LEVEL && opt->coupling != NLS_ADDITIVE &&
        opt->coupling != NLS_HYBRID)
        return NLS_EINVAL;
    if (opt->gmres_restart < 1 || opt->gmres_maxit < 1 || opt->outer_maxit < 0 ||
        opt->outer_maxit > NLS_MAX_OUTER || opt->inner_maxit < 1)
        return NLS_EINVAL;
    if (hipSetDevice(opt->device) != hipSuccess) return NLS_EHIP;
    {
        std::string err;
        if (guess_scratch_setup(opt->device, err) != NLS_OK) return NLS_EHIP;
    }
    auto* h = new (std::nothrow) nls_handle();
    if (!h) return NLS_ENOMEM;
    h->opt = *opt;
    h->stream = (hipStream_t)opt->stream;
    *out = h;
    return NLS_OK;
}

extern "C" int nls_destroy(nls_handle* h) {
    if (!h) return NLS_OK;
    (void)hipSetDevice(h->opt.device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    delete h;
    return NLS_OK;
}

extern "C" int nls_set_mesh(nls_handle* h, int elem_kind, int64_t n_nodes, const double* xy,
                            int64_t n_elems, const int32_t* conn) {
    if (!h) return NLS_EINVAL;
    if (elem_kind != NLS_ELEM_P1_TRI && elem_kind != NLS_ELEM_Q1_QUAD)
        return fail(h, NLS_EINVAL, "element kind must be P1 triangles or Q1 quadrilaterals");
    if (n_nodes <= 0 || n_elems <= 0 || !xy || !conn || n_nodes > (1 << 27) ||
        n_elems > (1 << 27))
        return fail(h, NLS_EINVAL, "bad mesh sizes or null arrays");
    HostMesh m;
    m.N = (int)n_nodes;
    m.E = (int)n_elems;
    m.nv = elem_kind == NLS_ELEM_Q1_QUAD ? 4 : 3;
    m.xy.assign(xy, xy + 2 * n_nodes);
    m.conn.assign(conn, conn + (size_t)m.nv * n_elems);
    std::string err;
    int rc = nls_build_node_incidence(m, err);
    if (rc) return fail(h, rc, err);
    if (m.nv == 4) {
        // counter-clockwise: every corner turns left
        for (int e = 0; e < m.E; ++e)
            for (int a = 0; a < 4; ++a) {
                const int p = m.conn[4 * e + a], q = m.conn[4 * e + (a + 1) % 4],
                          r = m.conn[4 * e + (a + 3) % 4];
                const double ux = m.xy[2 * q] - m.xy[2 * p], uy = m.xy[2 * q + 1] - m.xy[2 * p + 1];
                const double vx = m.xy[2 * r] - m.xy[2 * p], vy = m.xy[2 * r + 1] - m.xy[2 * p + 1];
                if (!(ux * vy - uy * vx > 0.0))
                    return fail(h, NLS_EINVAL, "a quadrilateral is clockwise, degenerate or not convex");
            }
    }
    m.dflag.assign(m.N, 0);
    m.dval.assign(m.N, 0.0);
    h->mesh = std::move(m);
    h->have_mesh = true;
    h->have_part = h->have_coarse = h->have_state = false;
    h->kappa_h.clear();
    h->fmid_h.clear();
    h->beta = 1.0;
    return NLS_OK;
}

extern "C" int nls_set_mesh_structured(nls_handle* h, int elem_kind, int32_t nx, int32_t ny,
                                       double lx, double ly) {
    if (!h) return NLS_EINVAL;
    if (elem_kind != NLS_ELEM_P1_TRI && elem_kind != NLS_ELEM_Q1_QUAD)
        return fail(h, NLS_EINVAL, "element kind must be P1 triangles or Q1 quadrilaterals");
    if (nx < 1 || ny < 1 || !(lx > 0.0) || !(ly > 0.0) || !std::isfinite(lx) || !std::isfinite(ly))
        return fail(h, NLS_EINVAL, "need nx, ny >= 1 and positive finite lengths");
    const int64_t nn = (int64_t)(nx + 1) * (ny + 1);
    const int64_t ne = (int64_t)nx * ny * (elem_kind == NLS_ELEM_P1_TRI ? 2 : 1);
    if (nn > (1 << 27) || ne > (1 << 27)) return fail(h, NLS_EINVAL, "mesh too large");
    std::vector<double> xy(2 * (size_t)nn);
    const double hx = lx / nx, hy = ly / ny;
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            const size_t g = (size_t)j * (nx + 1) + i;
            xy[2 * g] = (double)i * hx;
            xy[2 * g + 1] = (double)j * hy;
        }
    const int nv = elem_kind == NLS_ELEM_P1_TRI ? 3 : 4;
    std::vector<int32_t> conn((size_t)nv * ne);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const int32_t n00 = j * (nx + 1) + i, n10 = n00 + 1, n11 = n00 + nx + 2, n01 = n00 + nx + 1;
            const size_t c = (size_t)j * nx + i;
            if (nv == 3) {
                int32_t* t = &conn[6 * c];
                t[0] = n00; t[1] = n10; t[2] = n11;
                t[3] = n00; t[4] = n11; t[5] = n01;
            } else {
                int32_t* q = &conn[4 * c];
                q[0] = n00; q[1] = n10; q[2] = n11; q[3] = n01;
            }
        }
    return nls_set_mesh(h, elem_kind, nn, xy.data(), ne, conn.data());
}

extern "C" int nls_set_problem(nls_handle* h, int kind, const double* params,
                               const double* elem_coef, const double* elem_load) {
    if (!h) return NLS_EINVAL;
    if (!h->have_mesh) return fail(h, NLS_ESTATE, "nls_set_mesh first");
    if (kind != NLS_PROBLEM_DIFFUSION && kind != NLS_PROBLEM_NEOHOOKE)
        return fail(h, NLS_EINVAL, "unknown problem kind");
    if (kind == NLS_PROBLEM_NEOHOOKE) {
        if (h->mesh.nv != 4) return fail(h, NLS_EINVAL, "elasticity needs a Q1 mesh");
        if (!params || !(params[0] > 0.0) || !std::isfinite(params[0]) || !std::isfinite(params[1]))
            return fail(h, NLS_EINVAL, "need finite Lame parameters with mu > 0");
        if (elem_coef || elem_load)
            return fail(h, NLS_EINVAL, "elasticity takes nodal loads (nls_set_nodal_load)");
        h->kind = kind;
        h->mu = params[0];
        h->lam = params[1];
        h->kappa_h.clear();
        h->fmid_h.clear();
        h->mesh.d = 2;
        h->fnode_h.assign((size_t)h->mesh.ndof(), 0.0);
        h->mesh.dflag.assign(h->mesh.ndof(), 0);
        h->mesh.dval.assign(h->mesh.ndof(), 0.0);
        h->have_part = h->have_coarse = h->have_state = false;
        return NLS_OK;
    }
    if (h->mesh.nv != 3) return fail(h, NLS_EINVAL, "diffusion needs a P1 mesh");
    if (h->mesh.d != 1) {
        h->mesh.d = 1;
        h->mesh.dflag.assign(h->mesh.N, 0);
        h->mesh.dval.assign(h->mesh.N, 0.0);
    }
    h->fnode_h.clear();
    h->kind = kind;
    h->beta = params ? params[0] : 1.0;
    if (!std::isfinite(h->beta)) return fail(h, NLS_EINVAL, "beta must be finite");
    const int E = h->mesh.E;
    if (elem_coef) {
        h->kappa_h.assign(elem_coef, elem_coef + E);
        for (double k : h->kappa_h)
            if (!(k > 0.0) || !std::isfinite(k))
                return fail(h, NLS_EINVAL, "element coefficients must be positive and finite");
    } else {
        h->kappa_h.clear();
    }
    if (elem_load) {
        h->fmid_h.assign(elem_load, elem_load + 3 * (size_t)E);
    } else {
        h->fmid_h.clear();
    }
    h->have_part = h->have_coarse = h->have_state = false;
    return NLS_OK;
}

extern "C" int nls_set_dirichlet(nls_handle* h, int64_t n, const int64_t* nodes,
                                 const double* values) {
    if (!h) return NLS_EINVAL;
    if (!h->have_mesh) return fail(h, NLS_ESTATE, "nls_set_mesh first");
    if (n < 0 || (n > 0 && (!nodes || !values))) return fail(h, NLS_EINVAL, "bad Dirichlet arrays");
    std::fill(h->mesh.dflag.begin(), h->mesh.dflag.end(), 0);
    std::fill(h->mesh.dval.begin(), h->mesh.dval.end(), 0.0);
    for (int64_t k = 0; k < n; ++k) {
        if (nodes[k] < 0 || nodes[k] >= h->mesh.ndof()) return fail(h, NLS_EINVAL, "Dirichlet dof out of range");
        h->mesh.dflag[nodes[k]] = 1;
        h->mesh.dval[nodes[k]] = values[k];
    }
    h->have_part = h->have_coarse = h->have_state = false;
    return NLS_OK;
}

static int upload_problem(nls_handle* h) {
    const HostMesh& m = h->mesh;
    h->free_group(G_MESH);
    DevMesh d{};
    d.N = m.N;
    d.E = m.E;
    d.kind = h->kind;
    d.nv = m.nv;
    d.d = m.d;
    d.ndof = m.ndof();
    d.beta = h->beta;
    d.mu = h->mu;
    d.lam = h->lam;
    const int nv = m.nv, nd = m.ndof();
    int *conn, *nptr, *nel;
    double *xy, *G6 = nullptr, *kap = nullptr, *eload = nullptr, *bload, *dval, *coef = nullptr,
           *fmid = nullptr;
    unsigned char* dflag;
    std::vector<int> nelc(m.nel.size());
    for (int g = 0; g < m.N; ++g)
        for (int k = m.nptr[g]; k < m.nptr[g + 1]; ++k) {
            int e = m.nel[k], pos = 0;
            for (int v = 0; v < nv; ++v)
                if (m.conn[nv * e + v] == g) pos = v;
            nelc[k] = (e << 2) | pos;
        }
    RC(h->upload(G_MESH, &conn, m.conn));
    RC(h->upload(G_MESH, &nptr, m.nptr));
    RC(h->upload(G_MESH, &nel, nelc));
    RC(h->upload(G_MESH, &xy, m.xy));
    RC(h->upload(G_MESH, &dflag, m.dflag));
    RC(h->upload(G_MESH, &dval, m.dval));
    RC(h->alloc(G_MESH, &bload, nd));
    int* bad;
    double *part, *mx;
    int nb = 256;
    RC(h->alloc(G_MESH, &bad, 1));
    RC(h->alloc(G_MESH, &part, nb));
    RC(h->alloc(G_MESH, &mx, 1));
    d.conn = conn;
    d.xy = xy;
    d.nptr = nptr;
    d.nel = nel;
    d.bload = bload;
    d.dflag = dflag;
    d.dval = dval;
    HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), h->stream));
    if (h->kind == NLS_PROBLEM_DIFFUSION) {
        if (!h->kappa_h.empty()) RC(h->upload(G_MESH, &coef, h->kappa_h));
        if (!h->fmid_h.empty()) RC(h->upload(G_MESH, &fmid, h->fmid_h));
        RC(h->alloc(G_MESH, &G6, 6 * (size_t)m.E));
        RC(h->alloc(G_MESH, &kap, m.E));
        RC(h->alloc(G_MESH, &eload, 3 * (size_t)m.E));
        d.G6 = G6;
        d.kappa = kap;
        d.eload = eload;
        HIPCHK(launch_p1_setup(d, xy, coef, fmid, G6, kap, eload, bad, h->stream));
        HIPCHK(launch_assemble_load(d, bload, h->stream));
    } else {
        // nodal forces, zero on Dirichlet dofs
        std::vector<double> f(h->fnode_h);
        for (int k = 0; k < nd; ++k)
            if (m.dflag[k]) f[k] = 0.0;
        HIPCHK(hipMemcpyAsync(bload, f.data(), nd * sizeof(double), hipMemcpyHostToDevice, h->stream));
    }
    HIPCHK(launch_max_abs(bload, nd, part, mx, nb, h->stream));
    h->d_xy = xy;
    h->d_coef = coef;
    h->d_fmid = fmid;
    h->d_bad = bad;
    h->d_part = part;
    h->d_mx = mx;
    int bad_h = 0;
    HIPCHK(hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(&h->b_inf, mx, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    RC(sync(h));
    if (bad_h) return fail(h, NLS_EINVAL, "an element is clockwise or degenerate");
    h->dm = d;
    return NLS_OK;
}

// LDS bytes of the fused local Newton kernel for subdomain i with LU variant v:
// patch values, residual/step (and refinement vectors in mixed mode),
// reduction scratch, multipliers, and the band window of the factorisation
// (FP64 in every mode: the factorisation at the converged state is FP64).
static int local_lds_key(const HostMaps& M, int i, bool mixed, int v) {
    const int n = M.off_n[i + 1] - M.off_n[i], ng = M.off_g[i + 1] - M.off_g[i];
    const int dbl = (n + ng) + n + (mixed ? 2 * n : 0) + 24 + std::max(M.kl[i], 1) + 1;
    int w = band_window_doubles_v(M.kl[i], M.ku[i], v);
    if (w < 0) w = band_window_doubles_v(M.kl[i], M.ku[i], 3);
    return dbl * 8 + w * 8;
}

static int npl_for(int band) { return band <= 64 ? 1 : (band <= 128 ? 2 : 4); }

// LDS bytes that stage 64 steps of FP64 factor entries for the band solves:
// two buffers of 64 columns, each column in slot order (NPL + 1 slots of 64
// entries) with its pivot or reciprocal diagonal.
static int solve_stage_bytes(int kl, int ku) {
    const int slots = npl_for(std::max(kl, kl + ku)) + 1;
    return 2 * 64 * (slots * 64 * 8 + 8);
}

// LDS bytes of a launch: the working set above, with the window region
// grown (up to the 160 KB of a compute unit, less 1 KB for the kernels'
// static LDS) so that it also holds the band solves' staging buffers.  The
// kernel is limited to one workgroup per compute unit by its registers, so
// the extra LDS costs no occupancy.
static const int kLdsGrowCap = 159 * 1024;
static int local_lds_bytes(const HostMaps& M, int i, bool mixed, int v) {
    const int key = local_lds_key(M, i, mixed, v);
    const int n = M.off_n[i + 1] - M.off_n[i], ng = M.off_g[i + 1] - M.off_g[i];
    const int base = ((n + ng) + n + (mixed ? 2 * n : 0) + 24 + std::max(M.kl[i], 1) + 1) * 8;
    const int want = base + solve_stage_bytes(M.kl[i], M.ku[i]);
    return std::max(key, std::min(want, kLdsGrowCap));
}

extern "C" int nls_set_partition(nls_handle* h, int32_t n_sub, const int32_t* elem_part,
                                 int32_t overlap) {
    if (!h) return NLS_EINVAL;
    if (!h->have_mesh) return fail(h, NLS_ESTATE, "nls_set_mesh first");
    if (!elem_part) return fail(h, NLS_EINVAL, "elem_part is null");
    HIPCHK(hipSetDevice(h->opt.device));
    h->have_part = h->have_coarse = h->have_state = false;
    guess_invalidate(h);
    h->drop_graphs();
    h->tuned = false;
    h->free_group(G_MAPS);
    h->free_group(G_COARSE);
    RC(upload_problem(h));
    std::string err;
    int rc = nls_build_maps(h->mesh, elem_part, n_sub, overlap, h->maps, err);
    if (rc) return fail(h, rc, err);
    h->part_h.assign(elem_part, elem_part + h->mesh.E);
    const HostMaps& M = h->maps;
    const bool mixed = h->opt.precision != NLS_PREC_FP64;
    // kernel limits
    int maxband = 0, maxkl = 0, maxn = 0, maxng = 0;
    for (int i = 0; i < M.nsub; ++i) {
        maxkl = std::max(maxkl, M.kl[i]);
        maxband = std::max(maxband, M.kl[i] + M.ku[i]);
        maxn = std::max(maxn, M.off_n[i + 1] - M.off_n[i]);
        maxng = std::max(maxng, M.off_g[i + 1] - M.off_g[i]);
    }
    if (maxkl > 127 || maxband > 256)
        return fail(h, NLS_ELIMIT, "local band too wide (kl <= 127, kl+ku <= 256)");
    int lds = 0;
    const int var0 = h->opt.lu_variant;
    for (int i = 0; i < M.nsub; ++i) lds = std::max(lds, local_lds_key(M, i, mixed, var0));
    if (lds > 160 * 1024) return fail(h, NLS_ELIMIT, "subdomain too large for the LDS working set");
    h->lds_local = lds;
    // launch order: largest LDS first; size buckets of equal occupancy (WGs
    // per CU allowed by LDS), one launch each
    std::vector<int> sub_lds(M.nsub), sub_band(M.nsub);
    for (int i = 0; i < M.nsub; ++i) {
        sub_lds[i] = local_lds_key(M, i, mixed, var0);
        sub_band[i] = std::max(M.kl[i], M.kl[i] + M.ku[i]);
    }
    std::vector<int> lorder(M.nsub);
    std::iota(lorder.begin(), lorder.end(), 0);
    std::stable_sort(lorder.begin(), lorder.end(), [&](int a, int b) { return sub_lds[a] > sub_lds[b]; });
    h->maps.order = lorder;
    h->bk_start.clear(); h->bk_end.clear(); h->bk_lds.clear(); h->bk_npl.clear();
    h->bk_var.clear();
    h->tuned = false;
    auto occ = [](int bytes) { return std::min(8, std::max(1, (160 * 1024) / std::max(bytes, 1))); };
    for (int p = 0; p < M.nsub;) {
        int q = p, band = 0;
        while (q < M.nsub && occ(sub_lds[lorder[q]]) == occ(sub_lds[lorder[p]])) {
            band = std::max(band, sub_band[lorder[q]]);
            ++q;
        }
        int blds = 0;
        for (int t = p; t < q; ++t) blds = std::max(blds, local_lds_bytes(M, lorder[t], mixed, var0));
        h->bk_start.push_back(p);
        h->bk_end.push_back(q);
        h->bk_lds.push_back(blds);
        h->bk_npl.push_back(npl_for(band));
        h->bk_var.push_back(var0);
        p = q;
    }
    int stage = 0;
    for (int i = 0; i < M.nsub; ++i) stage = std::max(stage, solve_stage_bytes(M.kl[i], M.ku[i]));
    const int tan_min = (maxn + (mixed ? 2 * maxn : 0) + 24) * 8;
    h->lds_tangent = std::max(tan_min, std::min(tan_min + stage, kLdsGrowCap));
    h->npl_local = npl_for(std::max(maxkl, maxband));
    // tables
    DevMaps d{};
    d.nsub = M.nsub;
    int *off_n, *off_g, *off_e, *l2g, *g2g, *pe_conn, *pe_gid, *rinc_ptr, *rinc, *jptr, *jcol,
        *kl, *ku, *order, *own;
    int64_t *off_u, *off_l;
    RC(h->upload(G_MAPS, &off_n, M.off_n));
    RC(h->upload(G_MAPS, &off_g, M.off_g));
    RC(h->upload(G_MAPS, &off_e, M.off_e));
    RC(h->upload(G_MAPS, &l2g, M.l2g));
    RC(h->upload(G_MAPS, &g2g, M.g2g));
    RC(h->upload(G_MAPS, &pe_conn, M.pe_conn));
    RC(h->upload(G_MAPS, &pe_gid, M.pe_gid));
    RC(h->upload(G_MAPS, &rinc_ptr, M.rinc_ptr));
    RC(h->upload(G_MAPS, &rinc, M.rinc));
    RC(h->upload(G_MAPS, &jptr, M.jptr));
    RC(h->upload(G_MAPS, &jcol, M.jcol));
    RC(h->upload(G_MAPS, &kl, M.kl));
    RC(h->upload(G_MAPS, &ku, M.ku));
    RC(h->upload(G_MAPS, &order, h->maps.order));
    RC(h->upload(G_MAPS, &own, M.own_pidx));
    RC(h->upload(G_MAPS, &off_u, M.off_u));
    RC(h->upload(G_MAPS, &off_l, M.off_l));
    d.off_n = off_n; d.off_g = off_g; d.off_e = off_e; d.l2g = l2g; d.g2g = g2g;
    d.pe_conn = pe_conn; d.pe_gid = pe_gid; d.rinc_ptr = rinc_ptr; d.rinc = rinc;
    d.jptr = jptr; d.jcol = jcol; d.kl = kl; d.ku = ku; d.order = order; d.own_pidx = own;
    d.off_u = off_u; d.off_l = off_l;
    h->dp = d;
    // local state
    DevLocal L{};
    const size_t nrows = M.l2g.size();
    RC(h->alloc(G_MAPS, &L.jval, M.jcol.size()));
    // factor arrays carry 1024 elements of padding: the multi-RHS solve reads
    // up to its window size past a column's band (masked)
    RC(h->alloc(G_MAPS, &L.Uf, (size_t)M.factor_u_total + 1024));
    RC(h->alloc(G_MAPS, &L.Lf, (size_t)M.factor_l_total + 1024));
    if (mixed) {
        RC(h->alloc(G_MAPS, &L.Uf32, (size_t)M.factor_u_total));
        RC(h->alloc(G_MAPS, &L.Lf32, (size_t)M.factor_l_total));
    }
    RC(h->alloc(G_MAPS, &L.piv, nrows));
    RC(h->alloc(G_MAPS, &L.xstar, nrows));
    RC(h->alloc(G_MAPS, &L.ghost, std::max<size_t>(M.g2g.size(), 1)));
    RC(h->alloc(G_MAPS, &L.T, nrows));
    RC(h->alloc(G_MAPS, &L.z, nrows));
    RC(h->alloc(G_MAPS, &L.its, M.nsub));
    RC(h->alloc(G_MAPS, &L.status, M.nsub));
    RC(h->alloc(G_MAPS, &L.start, M.nsub));
    h->dl = L;
    h->its_h.assign(M.nsub, 0);
    {
        const size_t need = 1024 + sizeof(int) * (size_t)M.nsub;
        if (need > h->pin_bytes) {
            if (h->pin) HIPCHK(hipHostFree(h->pin));
            h->pin = nullptr;
            h->pin_bytes = 0;
            if (hipHostMalloc(&h->pin, need, hipHostMallocDefault) != hipSuccess)
                return fail(h, NLS_ENOMEM, "pinned host allocation failed");
            h->pin_bytes = need;
        }
    }
    // exact-tangent blocks W_i = (J_ii^{-1} B_i)[owned rows, :]
    {
        int bucket = 0;
        h->max_ng = 0;
        for (int i = 0; i < M.nsub; ++i) {
            bucket = std::max(bucket, mrhs_bucket_kl(M.kl[i], M.ku[i]));
            h->max_ng = std::max(h->max_ng, M.off_g[i + 1] - M.off_g[i]);
        }
        h->tangent_bucket = bucket;
        h->tangent_w = bucket <= 56 && M.max_bcol <= NLS_MAX_BCOL && h->max_ng * 8 <= 64 * 1024;
        if (h->tangent_w) {
            DevTangent T{};
            int *bptr, *brow, *bslot, *off_own, *ownrow, *rowown;
            int64_t *off_W, *off_F;
            RC(h->upload(G_MAPS, &bptr, M.bptr));
            RC(h->upload(G_MAPS, &brow, M.brow));
            RC(h->upload(G_MAPS, &bslot, M.bslot));
            RC(h->upload(G_MAPS, &off_own, M.off_own));
            RC(h->upload(G_MAPS, &ownrow, M.ownrow));
            RC(h->upload(G_MAPS, &rowown, M.rowown));
            RC(h->upload(G_MAPS, &off_W, M.off_W));
            RC(h->upload(G_MAPS, &off_F, M.off_F));
            T.bptr = bptr; T.brow = brow; T.bslot = bslot; T.off_own = off_own;
            T.ownrow = ownrow; T.rowown = rowown; T.off_W = off_W; T.off_F = off_F;
            RC(h->alloc(G_MAPS, &T.W, (size_t)M.off_W.back()));
            // W above 192 MiB cannot stay in MI355X's 256 MiB last-level
            // cache between products: stream it past the cache instead
            h->w_stream = (size_t)M.off_W.back() * sizeof(double) > ((size_t)192 << 20);
            RC(h->alloc(G_MAPS, &T.fwd, (size_t)M.off_F.back()));
            // the blocked solve holds the window of 16 + kl rows in four
            // row tiles and the backward strip of 16 + kl + ku rows in its
            // LDS ring
            int max_kl = 0, max_kw = 0;
            for (int i = 0; i < M.nsub; ++i) {
                max_kl = std::max(max_kl, M.kl[i]);
                max_kw = std::max(max_kw, M.kl[i] + M.ku[i]);
            }
            h->tangent_nblk = 0;
            h->tangent_nkk = 0;
            if (max_kl <= 48 && max_kw <= 112 && !(h->opt.flags & NLS_FLAG_TANGENT_SWEEP)) {
                std::vector<int> off_blk(1, 0), blk_sub;
                for (int i = 0; i < M.nsub; ++i) {
                    const int nb = (M.off_n[i + 1] - M.off_n[i] + 15) / 16;
                    for (int b = 0; b < nb; ++b) blk_sub.push_back(i);
                    off_blk.push_back(off_blk.back() + nb);
                }
                const size_t nblk = blk_sub.size();
                int *d_off_blk, *d_blk_sub;
                RC(h->upload(G_MAPS, &d_off_blk, off_blk));
                RC(h->upload(G_MAPS, &d_blk_sub, blk_sub));
                T.off_blk = d_off_blk;
                T.blk_sub = d_blk_sub;
                RC(h->alloc(G_MAPS, &T.tsig, nblk * 64));
                RC(h->alloc(G_MAPS, &T.tG, nblk * 1024));
                RC(h->alloc(G_MAPS, &T.tUi, nblk * 256));
                h->tangent_nblk = (int)nblk;
                h->tangent_nkk = (max_kw + 3) / 4;
            }
            h->dt = T;
        }
    }
    // Newton parameters
    NewtonParams np{};
    np.rtol = h->opt.inner_rtol;
    np.abs_tol = h->opt.inner_eta * h->b_inf;
    np.stagnation = h->opt.stagnation;
    np.maxit = h->opt.inner_maxit;
    np.mixed = h->opt.precision == NLS_PREC_BF16_IR ? 2 : (mixed ? 1 : 0);
    np.ir_maxit = np.mixed == 2 ? 30 : 10;
    np.ir_rtol = 1e-10;  // a Newton step needs no more; residuals stay FP64
    np.lu_variant = var0;
    np.keep_factor = 1;
    h->np = np;
    // GMRES workspace
    const int N = h->mesh.ndof();
    h->m = h->opt.gmres_restart;
    h->nb_dot = std::min(256, std::max(1, (N + 511) / 512));  // blocks of the vector reductions
    RC(h->alloc(G_MAPS, &h->V, (size_t)(h->m + 1) * N));
    RC(h->alloc(G_MAPS, &h->wv, N));
    RC(h->alloc(G_MAPS, &h->hbuf, h->m + 2));
    RC(h->alloc(G_MAPS, &h->hbuf2, h->m + 2));
    RC(h->alloc(G_MAPS, &h->hn2, 4));
    // nb x (m + 1) partial sums, nb norm partials, and a second nb x (m + 1)
    RC(h->alloc(G_MAPS, &h->partial, (size_t)h->nb_dot * (2 * (h->m + 1) + 1)));
    RC(h->alloc(G_MAPS, &h->Fx, N));
    RC(h->alloc(G_MAPS, &h->du, N));
    RC(h->alloc(G_MAPS, &h->tmp, N));
    RC(h->alloc(G_MAPS, &h->zbuf, N));
    RC(h->alloc(G_MAPS, &h->ydev, h->m + 2));
    RC(h->alloc(G_MAPS, &h->ubuf, N));
    RC(h->alloc(G_MAPS, &h->stat2, 2));
    RC(h->alloc(G_MAPS, &h->Hd, (size_t)(h->m + 1) * h->m));
    RC(h->alloc(G_MAPS, &h->csd, h->m));
    RC(h->alloc(G_MAPS, &h->snd, h->m));
    RC(h->alloc(G_MAPS, &h->gd, h->m + 1));
    RC(h->alloc(G_MAPS, &h->gtol, 1));
    RC(h->alloc(G_MAPS, &h->gst, 2));
    RC(sync(h));
    h->have_part = true;
    return NLS_OK;
}

// ------------------------------------------------------------ coarse space
// ||Phi^T b||_inf, the scale of the coarse stopping rule: G(c) at u = 0,
// c = 0 equals Phi^T F(0) = -Phi^T b.
static int coarse_rhs_scale(nls_handle* h) {
    DevCoarse& d = h->dc;
    HIPCHK(hipMemsetAsync(d.w, 0, sizeof(double) * h->mesh.ndof(), h->stream));
    HIPCHK(launch_coarse_q(h->dm, d, d.w, nullptr, 0, h->lds_coarse_q, h->stream));
    HIPCHK(launch_coarse_assemble(d, 0, h->stream));
    HIPCHK(launch_max_abs(d.rhs, h->co.n0, h->d_part, h->d_mx, 64, h->stream));
    HIPCHK(hipMemcpyAsync(&h->phib_inf, h->d_mx, sizeof(double), hipMemcpyDeviceToHost,
                          h->stream));
    return sync(h);
}

extern "C" int nls_build_coarse(nls_handle* h, int kind, const double* u_lin) {
    if (h) h->tuned = false;
    if (h) h->drop_graphs();
    if (!h) return NLS_EINVAL;
    if (!h->have_part) return fail(h, NLS_ESTATE, "nls_set_partition first");
    HIPCHK(hipSetDevice(h->opt.device));
    h->free_group(G_COARSE);
    h->have_coarse = false;
    h->have_state = false;
    if (kind == NLS_COARSE_NONE) return NLS_OK;
    if (kind != NLS_COARSE_GDSW && kind != NLS_COARSE_RGDSW)
        return fail(h, NLS_EINVAL, "unknown coarse space kind");
    if (u_lin)
        for (int k = 0; k < h->mesh.ndof(); ++k)
            if (!std::isfinite(u_lin[k])) return fail(h, NLS_EINVAL, "u_lin must be finite");
    std::string err;
    int rc = nls_build_coarse_symbolic(h->mesh, h->part_h.data(), h->maps.nsub, kind, h->co, err);
    if (rc) return fail(h, rc, err);
    const HostCoarse& C = h->co;
    if (C.n0 == 0) return NLS_OK;  // a single subdomain has no interface
    if (C.a0kl > 127 || C.a0kl + C.a0ku > 256)
        return fail(h, NLS_ELIMIT, "coarse matrix band too wide");
    int maxikl = 0, maxiband = 0, maxnc = 0;
    for (int i = 0; i < h->maps.nsub; ++i) {
        maxikl = std::max(maxikl, C.ikl[i]);
        maxiband = std::max(maxiband, C.ikl[i] + C.iku[i]);
        maxnc = std::max(maxnc, C.off_c[i + 1] - C.off_c[i]);
    }
    if (maxikl > 127 || maxiband > 256)
        return fail(h, NLS_ELIMIT, "interior band too wide");
    const int lds_gdsw = C.max_ilds_doubles * 8 + 64;
    int maxb = 0;
    for (size_t b = 0; b + 1 < C.boff.size(); ++b) maxb = std::max(maxb, C.boff[b + 1] - C.boff[b]);
    h->lds_coarse_lu = (maxb + std::max(C.a0kl, 1) + 1 + band_window_doubles(C.a0kl, C.a0ku)) * 8;
    // room for the solve's staged factor columns beyond the LU's window
    h->lds_coarse_lu = std::max(h->lds_coarse_lu,
                                std::min(h->lds_coarse_lu + solve_stage_bytes(C.a0kl, C.a0ku),
                                         kLdsGrowCap));
    h->lds_coarse_q = maxnc * 8;
    if (lds_gdsw > 160 * 1024 || h->lds_coarse_lu > 160 * 1024 || h->lds_coarse_q > 160 * 1024)
        return fail(h, NLS_ELIMIT, "coarse working set exceeds LDS");
    HIPCHK(prepare_coarse_ty(h->lds_coarse_q));
    h->npl_coarse = npl_for(std::max(C.a0kl, C.a0kl + C.a0ku));
    DevCoarse d{};
    d.n0 = C.n0;
    d.nsub = h->maps.nsub;
    d.a0kl = C.a0kl;
    d.a0ku = C.a0ku;
    double* cval;
    int *off_c, *cnode, *ctype, *off_k, *klist, *cfun, *off_ne, *ne_conn, *ne_gid, *cinc_ptr,
        *cinc, *iidx, *off_ni, *inode, *iptr, *icol, *ikl, *iku, *perm, *a0ptr, *a0col,
        *a0src_ptr, *a0src, *gsrc_ptr, *gsrc, *cpos, *cown;
    int64_t *off_phi, *off_iu, *off_il, *off_kk;
    RC(h->upload(G_COARSE, &off_c, C.off_c));
    RC(h->upload(G_COARSE, &cnode, C.cnode));
    RC(h->upload(G_COARSE, &ctype, C.ctype));
    RC(h->upload(G_COARSE, &off_k, C.off_k));
    RC(h->upload(G_COARSE, &klist, C.klist));
    RC(h->upload(G_COARSE, &cfun, C.cfun));
    RC(h->upload(G_COARSE, &cval, C.cval));
    RC(h->upload(G_COARSE, &off_ne, C.off_ne));
    RC(h->upload(G_COARSE, &ne_conn, C.ne_conn));
    RC(h->upload(G_COARSE, &ne_gid, C.ne_gid));
    RC(h->upload(G_COARSE, &cinc_ptr, C.cinc_ptr));
    RC(h->upload(G_COARSE, &cinc, C.cinc));
    RC(h->upload(G_COARSE, &iidx, C.iidx));
    RC(h->upload(G_COARSE, &off_ni, C.off_ni));
    RC(h->upload(G_COARSE, &inode, C.inode));
    RC(h->upload(G_COARSE, &iptr, C.iptr));
    RC(h->upload(G_COARSE, &icol, C.icol));
    RC(h->upload(G_COARSE, &ikl, C.ikl));
    RC(h->upload(G_COARSE, &iku, C.iku));
    RC(h->upload(G_COARSE, &perm, C.perm));
    RC(h->upload(G_COARSE, &a0ptr, C.a0ptr));
    RC(h->upload(G_COARSE, &a0col, C.a0col));
    RC(h->upload(G_COARSE, &a0src_ptr, C.a0src_ptr));
    RC(h->upload(G_COARSE, &a0src, C.a0src));
    RC(h->upload(G_COARSE, &gsrc_ptr, C.gsrc_ptr));
    RC(h->upload(G_COARSE, &gsrc, C.gsrc));
    RC(h->upload(G_COARSE, &cpos, C.cpos));
    RC(h->upload(G_COARSE, &cown, C.cown));
    RC(h->upload(G_COARSE, &off_phi, C.off_phi));
    RC(h->upload(G_COARSE, &off_iu, C.off_iu));
    RC(h->upload(G_COARSE, &off_il, C.off_il));
    RC(h->upload(G_COARSE, &off_kk, C.off_kk));
    {
        int *boff, *bkl, *bku, *rblk;
        int64_t *offU, *offL, *offI;
        RC(h->upload(G_COARSE, &boff, C.boff));
        RC(h->upload(G_COARSE, &bkl, C.bkl));
        RC(h->upload(G_COARSE, &bku, C.bku));
        RC(h->upload(G_COARSE, &rblk, C.rblk));
        RC(h->upload(G_COARSE, &offU, C.offU));
        RC(h->upload(G_COARSE, &offL, C.offL));
        RC(h->upload(G_COARSE, &offI, C.offI));
        d.nblk = (int)C.bkl.size();
        d.boff = boff; d.bkl = bkl; d.bku = bku; d.rblk = rblk;
        d.offU = offU; d.offL = offL; d.offI = offI;
        h->max_block = 0;
        for (int b = 0; b < d.nblk; ++b) h->max_block = std::max(h->max_block, C.boff[b + 1] - C.boff[b]);
    }
    d.off_c = off_c; d.cnode = cnode; d.ctype = ctype; d.off_k = off_k; d.klist = klist;
    d.cfun = cfun; d.cval = cval; d.off_ne = off_ne; d.ne_conn = ne_conn; d.ne_gid = ne_gid;
    d.cinc_ptr = cinc_ptr; d.cinc = cinc; d.iidx = iidx; d.off_ni = off_ni; d.inode = inode;
    d.iptr = iptr; d.icol = icol; d.ikl = ikl; d.iku = iku; d.perm = perm; d.a0ptr = a0ptr; d.nnz0 = C.a0ptr.back();
    d.a0col = a0col; d.a0src_ptr = a0src_ptr; d.a0src = a0src; d.gsrc_ptr = gsrc_ptr;
    d.gsrc = gsrc; d.cpos = cpos; d.cown = cown; d.off_phi = off_phi; d.off_iu = off_iu;
    d.off_il = off_il; d.off_kk = off_kk;
    const int64_t nphi = C.off_phi.back();
    RC(h->alloc(G_COARSE, &d.phi, (size_t)nphi));
    RC(h->alloc(G_COARSE, &d.zbuf, (size_t)nphi));
    RC(h->alloc(G_COARSE, &d.ybuf, (size_t)nphi));
    RC(h->alloc(G_COARSE, &d.ival, C.icol.size()));
    RC(h->alloc(G_COARSE, &d.iU, (size_t)C.iu_total));
    RC(h->alloc(G_COARSE, &d.iL, (size_t)C.il_total));
    RC(h->alloc(G_COARSE, &d.ipiv, C.inode.size()));
    RC(h->alloc(G_COARSE, &d.gblk, C.klist.size()));
    RC(h->alloc(G_COARSE, &d.ablk, (size_t)C.off_kk.back()));
    RC(h->alloc(G_COARSE, &d.a0val, C.a0col.size()));
    RC(h->alloc(G_COARSE, &d.a0U, (size_t)C.offU.back() + 1024));
    RC(h->alloc(G_COARSE, &d.a0L, (size_t)C.offL.back() + 1024));
    RC(h->alloc(G_COARSE, &d.a0piv, C.n0));
    RC(h->alloc(G_COARSE, &d.rhs, C.n0));
    RC(h->alloc(G_COARSE, &d.c, C.n0));
    RC(h->alloc(G_COARSE, &d.w, h->mesh.ndof()));
    RC(h->alloc(G_COARSE, &d.scal, 4));
    RC(h->alloc(G_COARSE, &d.flag, 1));
    RC(h->alloc(G_COARSE, &h->ctmp, C.n0));
    RC(h->alloc(G_COARSE, &h->rhs2, C.n0));
    h->coarse_ldu = 1;
    for (size_t b = 0; b < C.bkl.size(); ++b) h->coarse_ldu = std::max(h->coarse_ldu, C.bkl[b] + C.bku[b] + 1);
    h->coarse_can_inv = h->coarse_ldu <= 511 &&
                        coarse_inverse_lds_bytes(h->max_block, h->coarse_ldu) <= 160 * 1024 &&
                        !(h->opt.flags & NLS_FLAG_COARSE_LU_APPLY);
    h->coarse_inv = h->coarse_can_inv;
    h->coarse_lu_valid = false;
    h->coarse_inv_valid = false;
    if (h->coarse_inv) RC(h->alloc(G_COARSE, &d.a0inv, (size_t)C.offI.back()));
    // A0^{-1} by the blocked solve on the matrix cores where every diagonal
    // block's band allows it (kl <= 48, kl + ku <= 112)
    d.inv_nblk = 0;
    d.inv_nkk = 0;
    if (h->coarse_inv && !(h->opt.flags & NLS_FLAG_TANGENT_SWEEP)) {
        bool fits = true;
        int nkk = 1;
        for (size_t b = 0; b < C.bkl.size(); ++b) {
            fits = fits && C.bkl[b] <= 48 && C.bkl[b] + C.bku[b] <= 112;
            nkk = std::max(nkk, (C.bkl[b] + C.bku[b] + 3) / 4);
        }
        if (fits) {
            std::vector<int> off(1, 0);
            std::vector<int64_t> offY(1, 0);
            for (size_t b = 0; b + 1 < C.boff.size(); ++b) {
                const int nbk = (C.boff[b + 1] - C.boff[b] + 15) / 16;
                off.push_back(off.back() + nbk);
                offY.push_back(offY.back() + (int64_t)nbk * nbk * 256);
            }
            int* d_off;
            int64_t* d_offY;
            RC(h->upload(G_COARSE, &d_off, off));
            RC(h->upload(G_COARSE, &d_offY, offY));
            d.inv_off = d_off;
            d.inv_offY = d_offY;
            RC(h->alloc(G_COARSE, &d.inv_sig, (size_t)off.back() * 64));
            RC(h->alloc(G_COARSE, &d.inv_G, (size_t)off.back() * 1024));
            RC(h->alloc(G_COARSE, &d.inv_Ui, (size_t)off.back() * 256));
            RC(h->alloc(G_COARSE, &d.inv_Y, (size_t)offY.back()));
            d.inv_nblk = off.back();
            d.inv_nkk = nkk;
        }
    }
    HIPCHK(hipMemsetAsync(d.flag, 0, sizeof(int), h->stream));
    h->dc = d;
    // the linearisation point of the extension (C9: u = 0 unless given)
    double* ulin = nullptr;
    if (u_lin) {
        RC(h->alloc(G_COARSE, &ulin, (size_t)h->mesh.ndof()));
        HIPCHK(hipMemcpyAsync(ulin, u_lin, sizeof(double) * h->mesh.ndof(), hipMemcpyHostToDevice,
                              h->stream));
    }
    HIPCHK(launch_gdsw_extend(h->dm, d, ulin, lds_gdsw, npl_for(std::max(maxikl, maxiband)),
                              h->stream));
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, d.flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    RC(sync(h));
    if (flag) return fail(h, NLS_ESINGULAR, "zero pivot in an interior block of the extension");
    RC(coarse_rhs_scale(h));
    h->have_coarse = true;
    return NLS_OK;
}

// New load samples on the same mesh, coefficients and partition: the maps,
// the band structure and the GDSW basis (extended with DF at u = 0, which
// does not involve f) are kept; the element loads, b, ||b||_inf and
// ||Phi^T b||_inf are recomputed.
int guess_refresh_load(nls_handle* h);

static int upload_nodal_load(nls_handle* h, const double* f);

extern "C" int nls_set_nodal_load(nls_handle* h, const double* f) {
    if (!h || !f) return NLS_EINVAL;
    if (h->kind != NLS_PROBLEM_NEOHOOKE) return fail(h, NLS_EINVAL, "the problem's load is not nodal");
    const int nd = h->mesh.ndof();
    for (int k = 0; k < nd; ++k)
        if (!std::isfinite(f[k])) return fail(h, NLS_EINVAL, "nodal forces must be finite");
    h->fnode_h.assign(f, f + nd);
    if (!h->have_part) return NLS_OK;  // uploaded with the partition
    return upload_nodal_load(h, h->fnode_h.data());
}

// Device copy of nodal forces f (Dirichlet entries zeroed) and the load
// scales of the stopping rules.
static int upload_nodal_load(nls_handle* h, const double* f) {
    const int nd = h->mesh.ndof();
    HIPCHK(hipSetDevice(h->opt.device));
    std::vector<double> fz(f, f + nd);
    for (int k = 0; k < nd; ++k)
        if (h->mesh.dflag[k]) fz[k] = 0.0;
    DevMesh& d = h->dm;
    HIPCHK(hipMemcpyAsync(const_cast<double*>(d.bload), fz.data(), nd * sizeof(double),
                          hipMemcpyHostToDevice, h->stream));
    HIPCHK(launch_max_abs(d.bload, nd, h->d_part, h->d_mx, 256, h->stream));
    HIPCHK(hipMemcpyAsync(&h->b_inf, h->d_mx, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    RC(sync(h));
    h->np.abs_tol = h->opt.inner_eta * h->b_inf;
    if (h->have_coarse) RC(coarse_rhs_scale(h));
    h->have_state = false;
    return NLS_OK;
}

extern "C" int nls_set_load(nls_handle* h, const double* elem_load) {
    if (!h) return NLS_EINVAL;
    if (!h->have_part) return fail(h, NLS_ESTATE, "nls_set_partition first");
    if (h->kind != NLS_PROBLEM_DIFFUSION) return fail(h, NLS_EINVAL, "use nls_set_nodal_load");
    HIPCHK(hipSetDevice(h->opt.device));
    const int E = h->mesh.E;
    if (elem_load) {
        for (size_t k = 0; k < 3 * (size_t)E; ++k)
            if (!std::isfinite(elem_load[k])) return fail(h, NLS_EINVAL, "load samples must be finite");
        h->fmid_h.assign(elem_load, elem_load + 3 * (size_t)E);
        if (!h->d_fmid) RC(h->alloc(G_MESH, &h->d_fmid, 3 * (size_t)E));
        HIPCHK(hipMemcpyAsync(h->d_fmid, elem_load, 3 * (size_t)E * sizeof(double),
                              hipMemcpyHostToDevice, h->stream));
    } else {
        h->fmid_h.clear();
    }
    DevMesh& d = h->dm;
    HIPCHK(hipMemsetAsync(h->d_bad, 0, sizeof(int), h->stream));
    HIPCHK(launch_p1_setup(d, h->d_xy, h->d_coef, elem_load ? h->d_fmid : nullptr,
                           const_cast<double*>(d.G6), const_cast<double*>(d.kappa),
                           const_cast<double*>(d.eload), h->d_bad, h->stream));
    HIPCHK(launch_assemble_load(d, const_cast<double*>(d.bload), h->stream));
    HIPCHK(launch_max_abs(d.bload, h->mesh.ndof(), h->d_part, h->d_mx, 256, h->stream));
    HIPCHK(hipMemcpyAsync(&h->b_inf, h->d_mx, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    RC(sync(h));
    h->np.abs_tol = h->opt.inner_eta * h->b_inf;
    if (h->have_coarse) RC(coarse_rhs_scale(h));
    if (h->guess) RC(guess_refresh_load(h));
    h->have_state = false;
    return NLS_OK;
}

// learned initial guess (guess_api.cpp)
bool guess_enabled(const nls_handle* h);
int guess_prepare(nls_handle* h, const double* u, const double** xpred);
int guess_after_local(nls_handle* h, const double* u);
void guess_new_solve(nls_handle* h);

// ------------------------------------------------------------ evaluation
static bool two_level(nls_handle* h) {
    return h->opt.coupling != NLS_ONE_LEVEL && h->have_coarse && h->co.n0 > 0;
}

// Regions of the pinned host buffer (see nls_handle::pin).
static double* pin_main(nls_handle* h) { return (double*)h->pin; }
static double* pin_coarse(nls_handle* h) { return (double*)((char*)h->pin + 256); }
static int* pin_graph(nls_handle* h) { return (int*)((char*)h->pin + 512); }
static int* pin_its(nls_handle* h) { return (int*)((char*)h->pin + 1024); }

// The size buckets of a local kernel run concurrently: bucket 0 on s, bucket
// b > 0 on a stream of its own that waits for s first, and s waits for them
// all at the join (the buckets touch disjoint subdomains).
static int bucket_fork(nls_handle* h, hipStream_t s) {
    const size_t nb = h->bk_start.size();
    if (nb <= 1) return NLS_OK;
    while (h->bstream.size() + 1 < nb) {
        hipStream_t q = nullptr;
        HIPCHK(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
        h->bstream.push_back(q);
    }
    while (h->bev.size() < nb) {
        hipEvent_t e = nullptr;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        h->bev.push_back(e);
    }
    HIPCHK(hipEventRecord(h->bev[0], s));
    for (size_t b = 1; b < nb; ++b) HIPCHK(hipStreamWaitEvent(h->bstream[b - 1], h->bev[0], 0));
    return NLS_OK;
}

static hipStream_t bucket_stream(const nls_handle* h, size_t b, hipStream_t s) {
    return b == 0 ? s : h->bstream[b - 1];
}

static int bucket_join(nls_handle* h, hipStream_t s) {
    const size_t nb = h->bk_start.size();
    for (size_t b = 1; b < nb; ++b) {
        HIPCHK(hipEventRecord(h->bev[b], h->bstream[b - 1]));
        HIPCHK(hipStreamWaitEvent(s, h->bev[b], 0));
    }
    return NLS_OK;
}

// The second stream of NLS_FLAG_OVERLAP and its two events, created on first
// use.
static int ensure_cstream(nls_handle* h) {
    if (h->cstream) return NLS_OK;
    HIPCHK(hipStreamCreateWithFlags(&h->cstream, hipStreamNonBlocking));
    for (hipEvent_t& e : h->cev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return NLS_OK;
}

// Coarse Newton iteration for T_0(u) (eq. 9): c <- c + A0^{-1} Phi^T F(u - Phi c)
// from c = 0; keeps LU(A0) at the converged c and u_0 = u - Phi c in dc.w.
// T_0(u) (eq. 9): Newton on G(c) = Phi^T F(u - Phi c) = 0 from c = 0.  With
// NLS_FLAG_COARSE_CHORD the steps reuse the last factorisation of A0 (from
// the previous tangent, or the first step's) and refactor only when the
// residual fails to halve: a different iteration, whose T_0 agrees with
// Newton's to the coarse stopping tolerance, not to the rounding level.
// A0 and its LU at the converged c*, which only the tangent needs, are
// formed by prepare_tangent.
static int coarse_solve(nls_handle* h, const double* u, int* its_out, hipStream_t cs) {
    DevCoarse& d = h->dc;
    const int n0 = d.n0;
    const bool chord = (h->opt.flags & NLS_FLAG_COARSE_CHORD) != 0;
    HIPCHK(hipMemsetAsync(d.c, 0, sizeof(double) * n0, cs));
    HIPCHK(hipMemsetAsync(d.flag, 0, sizeof(int), cs));
    double tol = 0.0, dprev = -1.0, cmax = 0.0, gprev = 0.0;
    int its = 0;
    bool have_lu = chord && h->coarse_lu_valid;
    for (;;) {
        HIPCHK(launch_coarse_w(h->dm, d, u, d.w, cs));
        HIPCHK(launch_coarse_q(h->dm, d, d.w, nullptr, 0, h->lds_coarse_q, cs));
        HIPCHK(launch_coarse_assemble(d, 0, cs));
        double* pc = pin_coarse(h);
        HIPCHK(hipMemcpyAsync(pc, d.scal, sizeof(double), hipMemcpyDeviceToHost, cs));
        HIPCHK(hipStreamSynchronize(cs));
        const double gn = pc[0];
        if (its == 0)
            tol = std::max(h->opt.inner_rtol * gn, h->opt.inner_eta * h->phib_inf * std::sqrt((double)n0));
        if (!std::isfinite(gn)) {
            HIPCHK(hipMemcpyAsync(pc + 4, d.flag, sizeof(int), hipMemcpyDeviceToHost, cs));
            HIPCHK(hipStreamSynchronize(cs));
            if (*(const int*)(pc + 4) & 2)
                return fail(h, NLS_EDETF, "det F <= 0 in the coarse residual");
            return fail(h, NLS_ENAN, "coarse residual is not finite");
        }
        if (gn <= tol) break;
        if (dprev >= 0.0 && dprev <= h->opt.stagnation * cmax) break;
        if (its == h->opt.inner_maxit) return fail(h, NLS_ELOCAL, "coarse Newton did not converge");
        const bool refactor = !have_lu || (its > 0 && gn > 0.5 * gprev);
        if (refactor) {
            HIPCHK(launch_coarse_galerkin(h->dm, d, d.w, 0, cs));
            HIPCHK(launch_coarse_assemble(d, 1, cs));
            HIPCHK(launch_coarse_lu(d, 1, h->lds_coarse_lu, h->npl_coarse, cs));
            h->coarse_inv_valid = false;
        } else if (h->coarse_inv_valid) {
            // chord step with the explicit inverse of the same factorisation
            HIPCHK(launch_coarse_apply_inverse(d, d.rhs, h->rhs2, cs));
            HIPCHK(hipMemcpyAsync(d.rhs, h->rhs2, sizeof(double) * n0, hipMemcpyDeviceToDevice, cs));
        } else {
            HIPCHK(launch_coarse_lu(d, 0, h->lds_coarse_lu, h->npl_coarse, cs));
        }
        have_lu = chord;
        HIPCHK(launch_coarse_update(d, cs));
        HIPCHK(hipMemcpyAsync(pc, d.scal, 3 * sizeof(double), hipMemcpyDeviceToHost, cs));
        HIPCHK(hipMemcpyAsync(pc + 4, d.flag, sizeof(int), hipMemcpyDeviceToHost, cs));
        HIPCHK(hipStreamSynchronize(cs));
        if (*(const int*)(pc + 4)) return fail(h, NLS_ESINGULAR, "zero pivot in the coarse matrix");
        dprev = pc[1];
        cmax = pc[2];
        gprev = gn;
        ++its;
    }
    if (its_out) *its_out = its;
    return NLS_OK;
}

static int dot_host(nls_handle* h, const double* x, const double* y, int n, double* out) {
    HIPCHK(launch_mdot(x, n, 1, y, n, h->partial, h->hn2 + 2, h->nb_dot, h->stream));
    HIPCHK(hipMemcpyAsync(pin_main(h), h->hn2 + 2, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    RC(sync(h));
    *out = pin_main(h)[0];
    return NLS_OK;
}

// The coarse Newton solve and its phase time: counted as coarse time when
// it runs in series, as overlap time when it runs beside the local solves
// (hidden = true; the inner phase's wall time already spans it), so that
// inner + coarse + GMRES + other is the solve time.
static int coarse_phase(nls_handle* h, const double* u, hipStream_t cs, bool hidden = false) {
    Timer tc;
    int cits = 0;
    RC(coarse_solve(h, u, &cits, cs));
    HIPCHK(hipStreamSynchronize(cs));
    if (h->st) {
        (hidden ? h->st->ms_overlap : h->st->ms_coarse) += tc.ms();
        h->st->coarse_its_total += cits;
    }
    return NLS_OK;
}

// F_x(u) into Fx (device); keeps local and coarse states for the tangent.
// Hybrid coupling (eq. 11): T_0(u) first, and the local problems are solved
// at u_0 = u - P_0 T_0(u), which the coarse solve leaves in dc.w.
static int evaluate(nls_handle* h, const double* u, double* Fx) {
    h->have_state = false;
    const bool hybrid = h->opt.coupling == NLS_HYBRID && two_level(h);
    if (hybrid) {
        RC(coarse_phase(h, u, h->stream));
        u = h->dc.w;
    }
    // Additive coupling with NLS_FLAG_OVERLAP: T_0(u) depends on u only, so
    // the coarse Newton solve runs on a second stream while the local solves
    // run; its small kernels fit beside the local workgroups on each CU.
    const bool overlap = two_level(h) && !hybrid && (h->opt.flags & NLS_FLAG_OVERLAP);
    if (overlap) {
        RC(ensure_cstream(h));
        HIPCHK(hipEventRecord(h->cev[0], h->stream));  // u is final on the main stream
        HIPCHK(hipStreamWaitEvent(h->cstream, h->cev[0], 0));
    }
    Timer t;
    NewtonParams np = h->np;
    np.xpred = nullptr;
    np.keep_factor = 0;  // J_ii and its LU at x* are formed by prepare_tangent
    h->local_factored = false;
    if (guess_enabled(h)) RC(guess_prepare(h, u, &np.xpred));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (h->profiling()) {
        e0 = h->take_event();
        e1 = h->take_event();
        HIPCHK(hipEventRecord(e0, h->stream));
    }
    RC(bucket_fork(h, h->stream));
    for (size_t b = 0; b < h->bk_start.size(); ++b) {
        DevMaps pb = h->dp;
        pb.order = h->dp.order + h->bk_start[b];
        np.lu_variant = h->bk_var[b];
        HIPCHK(launch_local_newton(h->dm, pb, h->dl, np, u, h->bk_end[b] - h->bk_start[b],
                                   h->bk_lds[b], h->bk_npl[b], bucket_stream(h, b, h->stream)));
    }
    RC(bucket_join(h, h->stream));
    if (e0) {
        HIPCHK(hipEventRecord(e1, h->stream));
        h->ev_used.push_back({0, {e0, e1}});
    }
    HIPCHK(launch_any_status(h->dl.status, h->maps.nsub, h->stat2, h->stream));
    int st2[2];
    if (overlap) {
        const int rc = coarse_phase(h, u, h->cstream, true);
        HIPCHK(hipEventRecord(h->cev[1], h->cstream));
        HIPCHK(hipStreamWaitEvent(h->stream, h->cev[1], 0));
        if (rc) {
            (void)sync(h);
            return rc;
        }
    }
    HIPCHK(hipMemcpyAsync(pin_main(h), h->stat2, 2 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(pin_its(h), h->dl.its, h->maps.nsub * sizeof(int),
                          hipMemcpyDeviceToHost, h->stream));
    RC(sync(h));
    st2[0] = ((const int*)pin_main(h))[0];
    st2[1] = ((const int*)pin_main(h))[1];
    std::copy(pin_its(h), pin_its(h) + h->maps.nsub, h->its_h.begin());
    if (h->st) {
        h->st->ms_inner += t.ms();
        for (int v : h->its_h) {
            h->st->inner_its_total += v;
            h->st->inner_its_max = std::max(h->st->inner_its_max, v);
        }
        h->st->local_solves += h->maps.nsub;
    }
    if (st2[0] >= 0) {
        if (h->st) h->st->failed_subdomain = st2[0];
        if (st2[1] == 2) return fail(h, NLS_ENAN, "non-finite local residual in subdomain " + std::to_string(st2[0]));
        if (st2[1] == 4)
            return fail(h, NLS_EDETF, "det F <= 0 in the local residual of subdomain " + std::to_string(st2[0]));
        if (st2[1] == 3) return fail(h, NLS_ESINGULAR, "zero pivot in subdomain " + std::to_string(st2[0]));
        return fail(h, NLS_ELOCAL, "local Newton failed in subdomain " + std::to_string(st2[0]));
    }
    RC(guess_after_local(h, u));
    if (two_level(h)) {
        if (!hybrid && !overlap) RC(coarse_phase(h, u, h->stream));
        HIPCHK(launch_prolong(h->dm, h->dp, h->dl.T, &h->dc, h->dc.c, Fx, nullptr, h->stream));
    } else {
        HIPCHK(launch_prolong(h->dm, h->dp, h->dl.T, nullptr, nullptr, Fx, nullptr, h->stream));
    }
    h->have_state = true;
    h->tangent_ready = false;
    return NLS_OK;
}

// A0 at the converged c* (Galerkin product with the rows Y_i for the
// tangent), its LU and, where chosen, its inverse, enqueued on stream s.
static int coarse_tangent_enqueue(nls_handle* h, hipStream_t s) {
    DevCoarse& d = h->dc;
    HIPCHK(launch_coarse_galerkin(h->dm, d, d.w, 1, s));
    HIPCHK(launch_coarse_assemble(d, 1, s));
    HIPCHK(launch_coarse_lu(d, 1, h->lds_coarse_lu, h->npl_coarse, s));
    if (h->coarse_inv) HIPCHK(launch_coarse_inverse(d, h->max_block, h->coarse_ldu, s));
    return NLS_OK;
}

// The factorisations the tangent (eqs. 7, 12) needs at the last evaluated
// point: J_ii^{-1} B_i per subdomain, and A0 with its LU (and inverse) at the
// converged c*.  Formed on first use, so the evaluation that ends the outer
// iteration pays for none of them.  With NLS_FLAG_OVERLAP the coarse part
// (which depends on c* only) runs on the second stream beside the local
// factorisations.
static int prepare_tangent(nls_handle* h) {
    if (h->tangent_ready) return NLS_OK;
    if (!h->have_state) return fail(h, NLS_ESTATE, "no evaluated point (nls_eval_precond_residual)");
    const bool two = two_level(h);
    const bool ovl = two && (h->opt.flags & NLS_FLAG_OVERLAP);
    if (ovl) {
        RC(ensure_cstream(h));
        HIPCHK(hipEventRecord(h->cev[0], h->stream));  // the evaluated state is final
        HIPCHK(hipStreamWaitEvent(h->cstream, h->cev[0], 0));
        RC(coarse_tangent_enqueue(h, h->cstream));
    }
    // on an error of the local part, let the coarse stream drain first
    auto bail = [&](int rc) {
        if (ovl) (void)hipStreamSynchronize(h->cstream);
        return rc;
    };
    if (!h->local_factored) {
        // J_ii and its FP64 LU at the converged local states (eq. 6)
        Timer tf;
        NewtonParams np = h->np;
        const int rcf = bucket_fork(h, h->stream);
        if (rcf) return bail(rcf);
        for (size_t b = 0; b < h->bk_start.size(); ++b) {
            DevMaps pb = h->dp;
            pb.order = h->dp.order + h->bk_start[b];
            np.lu_variant = h->bk_var[b];
            const hipError_t e = launch_local_factor(h->dm, pb, h->dl, np, h->dl.xstar,
                                                     h->bk_end[b] - h->bk_start[b], h->bk_lds[b],
                                                     bucket_stream(h, b, h->stream), h->dl.xstar,
                                                     h->dl.ghost);
            if (e != hipSuccess) return bail(fail(h, NLS_EHIP, hipGetErrorString(e)));
        }
        const int rcj = bucket_join(h, h->stream);
        if (rcj) return bail(rcj);
        int st2[2];
        hipError_t e = launch_any_status(h->dl.status, h->maps.nsub, h->stat2, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(st2, h->stat2, 2 * sizeof(int), hipMemcpyDeviceToHost, h->stream);
        if (e != hipSuccess) return bail(fail(h, NLS_EHIP, hipGetErrorString(e)));
        const int rc = sync(h);
        if (rc) return bail(rc);
        if (st2[0] >= 0)
            return bail(fail(h, NLS_ESINGULAR, "zero pivot in subdomain " + std::to_string(st2[0]) +
                                                   " at its converged state"));
        h->local_factored = true;
        if (h->st) h->st->ms_inner += tf.ms();
    }
    if (h->tangent_w) {
        Timer tp;
        const hipError_t e =
            h->tangent_nblk > 0
                ? launch_tangent_blocked(h->dp, h->dl, h->dt, h->tangent_nblk, h->tangent_nkk,
                                         h->max_ng, h->stream)
                : launch_tangent_prep(h->dp, h->dl, h->dt, h->tangent_bucket, h->max_ng,
                                      h->stream);
        if (e != hipSuccess) return bail(fail(h, NLS_EHIP, hipGetErrorString(e)));
        const int rc = sync(h);
        if (rc) return bail(rc);
        if (h->st) h->st->ms_inner += tp.ms();
    }
    if (two) {
        // with the overlap, only the part of the coarse work that outlasts
        // the local part is counted here
        Timer tc;
        hipStream_t cs = ovl ? h->cstream : h->stream;
        if (!ovl) RC(coarse_tangent_enqueue(h, cs));
        DevCoarse& d = h->dc;
        int flag = 0;
        HIPCHK(hipMemcpyAsync(&flag, d.flag, sizeof(int), hipMemcpyDeviceToHost, cs));
        HIPCHK(hipStreamSynchronize(cs));
        h->coarse_lu_valid = true;
        h->coarse_inv_valid = h->coarse_inv;
        if (flag) return fail(h, NLS_ESINGULAR, "zero pivot in the coarse matrix");
        if (h->st) h->st->ms_coarse += tc.ms();
    }
    h->tangent_ready = true;
    return NLS_OK;
}

// ------------------------------------------------------------ autotuner
// Times each candidate with HIP events on the handle's stream (second of
// two runs) and keeps the fastest.
template <class F>
static int time_ms(nls_handle* h, F&& launch, float* ms) {
    hipEvent_t a = nullptr, b = nullptr;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    float best = 0.f;
    for (int rep = 0; rep < 2; ++rep) {
        HIPCHK(hipEventRecord(a, h->stream));
        int rc = launch();
        if (rc) {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            return rc;
        }
        HIPCHK(hipEventRecord(b, h->stream));
        HIPCHK(hipEventSynchronize(b));
        HIPCHK(hipEventElapsedTime(&best, a, b));
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = best;
    return NLS_OK;
}

// Per size bucket: the LU variants that hold the bucket's widest band
// (blocked NB=16, NB=8, unblocked), each timed as the bucket's fused local
// Newton launch at u; each variant sizes its own LDS, so a narrower window
// may also raise the workgroups per CU.  A mixed-precision handle times the
// buckets in both precisions and keeps the one with the smaller total.
static int autotune_local(nls_handle* h, const double* u) {
    const HostMaps& M = h->maps;
    // binary32 is timed against binary64; the bfloat16 trial runs as asked,
    // in the blocked forms that hold its matrix-core update
    const bool can_mixed = h->opt.precision == NLS_PREC_FP32_IR;
    const bool bf16 = h->opt.precision == NLS_PREC_BF16_IR;
    const int nprec = can_mixed ? 2 : 1;
    const size_t nbk = h->bk_start.size();
    std::vector<int> var[2], ldsv[2];
    double total[2] = {0.0, 0.0};
    for (int pm = 0; pm < nprec; ++pm) {
        const bool mixed = (can_mixed && pm == 0) || bf16;  // pass 0: the handle's precision
        for (size_t b = 0; b < nbk; ++b) {
            int kmax = 0;
            for (int p = h->bk_start[b]; p < h->bk_end[b]; ++p) kmax = std::max(kmax, M.kl[M.order[p]]);
            float best = 1e30f;
            int bv = 3, blds = 0;
            for (int p = h->bk_start[b]; p < h->bk_end[b]; ++p)
                blds = std::max(blds, local_lds_bytes(M, M.order[p], mixed, 3));
            for (int v = 1; v <= 3; ++v) {
                if (v == 3 && bf16 && kmax + 8 <= 64) continue;
                if (v == 1 && kmax + 16 > 64) continue;
                if (v == 2 && kmax + 8 > 64) continue;
                int lds = 0;
                for (int p = h->bk_start[b]; p < h->bk_end[b]; ++p)
                    lds = std::max(lds, local_lds_bytes(M, M.order[p], mixed, v));
                if (lds > 160 * 1024) continue;
                NewtonParams np = h->np;
                np.xpred = nullptr;
                np.lu_variant = v;
                np.mixed = bf16 ? 2 : (mixed ? 1 : 0);
                // with the factorisation at x*, so that every subdomain's
                // time includes at least one LU even where Newton stops at once
                np.keep_factor = 1;
                DevMaps pb = h->dp;
                pb.order = h->dp.order + h->bk_start[b];
                const int nb = h->bk_end[b] - h->bk_start[b];
                float ms = 0.f;
                RC(time_ms(h, [&]() -> int {
                    HIPCHK(launch_local_newton(h->dm, pb, h->dl, np, u, nb, lds, h->bk_npl[b], h->stream));
                    return NLS_OK;
                }, &ms));
                if (ms < best) {
                    best = ms;
                    bv = v;
                    blds = lds;
                }
            }
            var[pm].push_back(bv);
            ldsv[pm].push_back(blds);
            total[pm] += best;
        }
    }
    const int pick = (nprec == 2 && total[1] < total[0]) ? 1 : 0;
    h->bk_var = var[pick];
    h->bk_lds = ldsv[pick];
    h->np.mixed = bf16 ? 2 : ((can_mixed && pick == 0) ? 1 : 0);
    return NLS_OK;
}

// Coarse term of the tangent: explicit A0^{-1} (formed once per evaluation,
// then a GEMV per GMRES step) against a band LU solve per step, priced with
// the measured kernel times at TUNE_STEPS steps per evaluation.
static constexpr int TUNE_STEPS = 20;
static int autotune_coarse(nls_handle* h) {
    if (!two_level(h) || !h->coarse_can_inv)
        return NLS_OK;
    RC(prepare_tangent(h));
    DevCoarse& d = h->dc;
    float t_inv = 0.f, t_apply = 0.f, t_lu = 0.f;
    RC(time_ms(h, [&]() -> int {
        HIPCHK(launch_coarse_inverse(d, h->max_block, h->coarse_ldu, h->stream));
        return NLS_OK;
    }, &t_inv));
    RC(time_ms(h, [&]() -> int {
        HIPCHK(launch_coarse_apply_inverse(d, d.rhs, h->rhs2, h->stream));
        return NLS_OK;
    }, &t_apply));
    RC(time_ms(h, [&]() -> int {
        HIPCHK(launch_coarse_lu(d, 0, h->lds_coarse_lu, h->npl_coarse, h->stream));
        return NLS_OK;
    }, &t_lu));
    const bool inv = t_inv + TUNE_STEPS * t_apply <= TUNE_STEPS * t_lu;
    if (inv != h->coarse_inv) {
        h->coarse_inv = inv;
        h->drop_graphs();
        if (inv) HIPCHK(launch_coarse_inverse(d, h->max_block, h->coarse_ldu, h->stream));
    }
    h->coarse_inv_valid = h->coarse_inv && h->tangent_ready;
    h->tune_ms[0] = t_inv;
    h->tune_ms[1] = t_apply;
    h->tune_ms[2] = t_lu;
    return sync(h);
}

// y = D F_x(u) v (eqs. 6, 7, 12) at the last evaluated point.
// Enqueued on s (the handle's stream by default); no host synchronisation,
// so the sequence can be captured into a graph (events only when eager).
static int nks_apply(nls_handle* h, const double* x, double* y, hipStream_t s);

static int tangent(nls_handle* h, const double* v, double* y, hipStream_t s = nullptr) {
    const bool eager = s == nullptr;
    if (eager) s = h->stream;
    if (h->nks_mode) return nks_apply(h, v, y, s);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (eager && h->profiling()) {
        e0 = h->take_event();
        e1 = h->take_event();
        HIPCHK(hipEventRecord(e0, s));
    }
    // coarse term q = Q_0 v = Phi A0^{-1} Phi^T DF(u_0) v, as coefficients in ctmp
    auto coarse_term = [&]() -> int {
        DevCoarse& d = h->dc;
        HIPCHK(launch_coarse_ty(d, v, h->lds_coarse_q, s));
        HIPCHK(launch_coarse_gather(d, s));
        if (h->coarse_inv) {
            HIPCHK(launch_coarse_apply_inverse(d, d.rhs, h->rhs2, s));
            HIPCHK(launch_coarse_scatter(d, h->rhs2, h->ctmp, s));
        } else {
            HIPCHK(launch_coarse_lu(d, 0, h->lds_coarse_lu, h->npl_coarse, s));
            HIPCHK(launch_coarse_scatter(d, nullptr, h->ctmp, s));
        }
        return NLS_OK;
    };
    // Hybrid (eq. 12): D F_h v = D F_1 (v - q) + q = v + sum_i P~_i J_ii^{-1}
    // B_i (v - q)_Gamma_i, so the local term acts on z = v - q.
    const bool hybrid = h->opt.coupling == NLS_HYBRID && two_level(h);
    const double* vloc = v;
    if (hybrid) {
        RC(coarse_term());
        HIPCHK(launch_sub_coarse(h->dm, h->dc, h->ctmp, v, h->zbuf, s));
        vloc = h->zbuf;
    }
    // Additive coupling with NLS_FLAG_OVERLAP: the coarse term runs on the
    // second stream beside the local term (a fork and a join, also when the
    // product is captured into a graph) and both meet in the prolongation.
    const bool fork = two_level(h) && !hybrid && (h->opt.flags & NLS_FLAG_OVERLAP);
    if (fork) {
        RC(ensure_cstream(h));
        HIPCHK(hipEventRecord(h->cev[2], s));
        HIPCHK(hipStreamWaitEvent(h->cstream, h->cev[2], 0));
        const hipStream_t s0 = s;
        s = h->cstream;
        const int rc = coarse_term();
        s = s0;
        RC(rc);
        HIPCHK(hipEventRecord(h->cev[3], h->cstream));
    }
    if (h->tangent_w)
        HIPCHK(launch_tangent_gemv(h->dp, h->dt, vloc, h->dl.z, h->max_ng, h->w_stream, s));
    else
        HIPCHK(launch_tangent_local(h->dm, h->dp, h->dl, h->np, vloc, h->lds_tangent, h->npl_local, s));
    if (e0) {
        HIPCHK(hipEventRecord(e1, s));
        h->ev_used.push_back({1, {e0, e1}});
    }
    if (two_level(h) && !hybrid) {
        if (fork)
            HIPCHK(hipStreamWaitEvent(s, h->cev[3], 0));
        else
            RC(coarse_term());
        HIPCHK(launch_prolong(h->dm, h->dp, h->dl.z, &h->dc, h->ctmp, y, v, s));
    } else {
        HIPCHK(launch_prolong(h->dm, h->dp, h->dl.z, nullptr, nullptr, y, v, s));
    }
    return NLS_OK;
}

// ---------------------------------------------------- graph-captured GMRES
static GmresDev gmres_dev(nls_handle* h) {
    GmresDev G{};
    G.H = h->Hd;
    G.cs = h->csd;
    G.sn = h->snd;
    G.g = h->gd;
    G.h1 = h->hbuf;
    G.h2 = h->hbuf2;
    G.hn2 = h->hn2;
    G.tol = h->gtol;
    G.st = h->gst;
    G.m = h->m;
    return G;
}

// Arnoldi step j on stream s: w = A v_j, two classical Gram-Schmidt passes,
// v_{j+1} = w / ||w||, then rotation j on the device.  No host contact.
static int arnoldi_step(nls_handle* h, int j, hipStream_t s) {
    const int N = h->mesh.ndof();
    const int64_t ld = N;
    double* vj = h->V + (int64_t)j * ld;
    double* vn = h->V + (int64_t)(j + 1) * ld;
    RC(tangent(h, vj, h->wv, s));
    // norm partial sums after the (m + 1) nb dot-product partials
    double* pnorm = h->partial + (int64_t)h->nb_dot * (h->m + 1);
    HIPCHK(launch_arnoldi_gs(h->V, ld, j + 1, h->wv, N, h->partial, pnorm, h->hbuf, h->hbuf2,
                             gmres_dev(h), j, vn, h->nb_dot, s, pnorm + h->nb_dot));
    return NLS_OK;
}

static bool graph_gmres_ok(const nls_handle* h) {
    return (h->opt.flags & NLS_FLAG_GRAPH) && h->tangent_w && !h->nks_mode;
}

// Steps [b*K, min((b+1)*K, m)) of a cycle as one graph, captured on first use.
static int block_graph(nls_handle* h, int b, hipGraphExec_t* out) {
    const int K = h->gblock;
    if ((int)h->gexec.size() <= b) h->gexec.resize(b + 1, nullptr);
    if (!h->gexec[b]) {
        // kernel attributes are set before capture, never inside it
        if (two_level(h) && !h->coarse_inv)
            HIPCHK(prepare_coarse_lu(h->lds_coarse_lu, h->npl_coarse));
        hipGraph_t graph = nullptr;
        HIPCHK(hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal));
        int rc = NLS_OK;
        for (int j = b * K; j < std::min((b + 1) * K, h->m) && rc == NLS_OK; ++j)
            rc = arnoldi_step(h, j, h->gstream);
        hipError_t ec = hipStreamEndCapture(h->gstream, &graph);
        if (rc != NLS_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        HIPCHK(ec);
        hipGraphExec_t ex = nullptr;
        hipError_t ei = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(ei);
        h->gexec[b] = ex;
    }
    *out = h->gexec[b];
    return NLS_OK;
}

// Restarted GMRES as gmres() below, with the Hessenberg rotations on the
// device and each block of gblock Arnoldi steps replayed as one graph; the
// host reads the convergence state once per block.  Steps of a block after
// convergence run but are not used.
static int gmres_graph(nls_handle* h, const double* b, double* x, int* its_out) {
    RC(prepare_tangent(h));
    const int N = h->mesh.ndof(), m = h->m, K = h->gblock;
    double bn2 = 0.0;
    RC(dot_host(h, b, b, N, &bn2));
    const double bn = std::sqrt(bn2);
    HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * N, h->stream));
    *its_out = 0;
    if (bn == 0.0) return NLS_OK;
    if (!h->gstream) {
        HIPCHK(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&h->gev[0], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&h->gev[1], hipEventDisableTiming));
    }
    const double tol = h->opt.gmres_rtol * bn;
    HIPCHK(hipMemcpyAsync(h->gtol, &tol, sizeof(double), hipMemcpyHostToDevice, h->stream));
    std::vector<double> H((size_t)(m + 1) * m), g(m + 1), y(m), g0(m + 1);
    int its = 0;
    bool first = true;
    while (its < h->opt.gmres_maxit) {
        double beta2;
        if (first) {
            HIPCHK(hipMemcpyAsync(h->V, b, sizeof(double) * N, hipMemcpyDeviceToDevice, h->stream));
            beta2 = bn2;
        } else {
            RC(tangent(h, x, h->tmp));
            HIPCHK(hipMemcpyAsync(h->V, b, sizeof(double) * N, hipMemcpyDeviceToDevice, h->stream));
            HIPCHK(launch_axpy(-1.0, h->tmp, h->V, N, h->stream));
            RC(dot_host(h, h->V, h->V, N, &beta2));
        }
        first = false;
        const double beta = std::sqrt(beta2);
        if (beta <= tol) break;
        HIPCHK(hipMemcpyAsync(h->hn2, &beta2, sizeof(double), hipMemcpyHostToDevice, h->stream));
        HIPCHK(launch_scale_by(h->V, h->hn2, h->V, N, h->stream));
        std::fill(g0.begin(), g0.end(), 0.0);
        g0[0] = beta;
        const int st0[2] = {0, 0};
        HIPCHK(hipMemcpyAsync(h->gd, g0.data(), (m + 1) * sizeof(double), hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->gst, st0, sizeof(st0), hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipEventRecord(h->gev[0], h->stream));
        HIPCHK(hipStreamWaitEvent(h->gstream, h->gev[0], 0));
        int j = 0, conv = 0;
        while (j < m) {
            const int budget = h->opt.gmres_maxit - its - j;
            if (budget <= 0) break;
            const int blk = j / K, jn = std::min((blk + 1) * K, m);
            if (j == blk * K && jn - j <= budget) {
                hipGraphExec_t ex = nullptr;
                RC(block_graph(h, blk, &ex));
                HIPCHK(hipGraphLaunch(ex, h->gstream));
            } else {
                for (int jj = j; jj < std::min(jn, j + budget); ++jj) RC(arnoldi_step(h, jj, h->gstream));
            }
            HIPCHK(hipMemcpyAsync(pin_graph(h), h->gst, 2 * sizeof(int), hipMemcpyDeviceToHost,
                                  h->gstream));
            HIPCHK(hipStreamSynchronize(h->gstream));
            const int st[2] = {pin_graph(h)[0], pin_graph(h)[1]};
            if (st[0] < 0) return fail(h, NLS_ENAN, "GMRES breakdown (non-finite)");
            if (st[0] > 0) {
                conv = st[0];
                j = conv;
                break;
            }
            j = st[1];
        }
        if (j == 0) break;
        HIPCHK(hipMemcpyAsync(H.data(), h->Hd, H.size() * sizeof(double), hipMemcpyDeviceToHost, h->gstream));
        HIPCHK(hipMemcpyAsync(g.data(), h->gd, (m + 1) * sizeof(double), hipMemcpyDeviceToHost, h->gstream));
        HIPCHK(hipStreamSynchronize(h->gstream));
        for (int i = j - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < j; ++k) s -= H[(size_t)i * m + k] * y[k];
            y[i] = s / H[(size_t)i * m + i];
        }
        HIPCHK(hipMemcpyAsync(h->ydev, y.data(), j * sizeof(double), hipMemcpyHostToDevice, h->gstream));
        HIPCHK(launch_maxpy(h->V, N, j, h->ydev, x, N, -1.0, h->gstream));
        HIPCHK(hipEventRecord(h->gev[1], h->gstream));
        HIPCHK(hipStreamWaitEvent(h->stream, h->gev[1], 0));
        its += j;
        RC(sync(h));
        if (conv) break;
    }
    *its_out = its;
    return NLS_OK;
}

// Restarted GMRES(m) for D F_x(u) x = b from x = 0 (classical Gram-Schmidt
// with one reorthogonalisation).  Returns the iteration count in *its.
static int gmres(nls_handle* h, const double* b, double* x, int* its_out) {
    if (!h->nks_mode) RC(prepare_tangent(h));
    const int N = h->mesh.ndof(), m = h->m;
    const int64_t ld = N;
    double bn2 = 0.0;
    RC(dot_host(h, b, b, N, &bn2));
    const double bn = std::sqrt(bn2);
    HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * N, h->stream));
    int its = 0;
    *its_out = 0;
    if (bn == 0.0) return NLS_OK;
    const double rtol = h->opt.gmres_rtol;
    std::vector<double> H((m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), hh(m + 2), hh2(m + 2), y(m);
    bool first = true;
    while (its < h->opt.gmres_maxit) {
        double beta2;
        if (first) {
            HIPCHK(hipMemcpyAsync(h->V, b, sizeof(double) * N, hipMemcpyDeviceToDevice, h->stream));
            beta2 = bn2;
        } else {
            RC(tangent(h, x, h->tmp));
            HIPCHK(hipMemcpyAsync(h->V, b, sizeof(double) * N, hipMemcpyDeviceToDevice, h->stream));
            HIPCHK(launch_axpy(-1.0, h->tmp, h->V, N, h->stream));
            RC(dot_host(h, h->V, h->V, N, &beta2));
        }
        first = false;
        const double beta = std::sqrt(beta2);
        if (beta <= rtol * bn) break;
        HIPCHK(hipMemcpyAsync(h->hn2, &beta2, sizeof(double), hipMemcpyHostToDevice, h->stream));
        HIPCHK(launch_scale_by(h->V, h->hn2, h->V, N, h->stream));
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int j = 0;
        bool done = false;
        while (j < m && its < h->opt.gmres_maxit) {
            double* vj = h->V + (int64_t)j * ld;
            double* vn = h->V + (int64_t)(j + 1) * ld;
            RC(tangent(h, vj, h->wv));
            ++its;
            HIPCHK(launch_mdot(h->V, ld, j + 1, h->wv, N, h->partial, h->hbuf, h->nb_dot, h->stream));
            HIPCHK(launch_maxpy(h->V, ld, j + 1, h->hbuf, h->wv, N, 1.0, h->stream));
            HIPCHK(launch_mdot(h->V, ld, j + 1, h->wv, N, h->partial, h->hbuf2, h->nb_dot, h->stream));
            HIPCHK(launch_maxpy_norm(h->V, ld, j + 1, h->hbuf2, h->wv, N, h->partial, h->hn2,
                                     h->nb_dot, h->stream));
            HIPCHK(launch_scale_by(h->wv, h->hn2, vn, N, h->stream));
            double hn2;
            HIPCHK(hipMemcpyAsync(hh.data(), h->hbuf, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, h->stream));
            HIPCHK(hipMemcpyAsync(hh2.data(), h->hbuf2, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, h->stream));
            HIPCHK(hipMemcpyAsync(&hn2, h->hn2, sizeof(double), hipMemcpyDeviceToHost, h->stream));
            RC(sync(h));
            for (int i = 0; i <= j; ++i) H[i * m + j] = hh[i] + hh2[i];
            H[(j + 1) * m + j] = std::sqrt(hn2);
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
                H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
                H[i * m + j] = t;
            }
            const double den = std::hypot(H[j * m + j], H[(j + 1) * m + j]);
            cs[j] = den > 0.0 ? H[j * m + j] / den : 1.0;
            sn[j] = den > 0.0 ? H[(j + 1) * m + j] / den : 0.0;
            H[j * m + j] = den;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++j;
            if (!std::isfinite(g[j])) return fail(h, NLS_ENAN, "GMRES breakdown (non-finite)");
            if (std::fabs(g[j]) <= rtol * bn) { done = true; break; }
        }
        for (int i = j - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < j; ++k) s -= H[i * m + k] * y[k];
            y[i] = s / H[i * m + i];
        }
        HIPCHK(hipMemcpyAsync(h->ydev, y.data(), j * sizeof(double), hipMemcpyHostToDevice, h->stream));
        HIPCHK(launch_maxpy(h->V, ld, j, h->ydev, x, N, -1.0, h->stream));
        RC(sync(h));
        if (done) break;
    }
    *its_out = its;
    return NLS_OK;
}

static int solve_impl(nls_handle* h, double* u, int u_on_device, nls_stats* st);

// The full external load of the problem as set (nodal forces, or the load
// samples of the diffusion problem; f = 1 when none were given), the load
// scaled by sc on the device, and the set load again.
static std::vector<double> full_load(const nls_handle* h, bool* had_samples) {
    *had_samples = !h->fmid_h.empty();
    if (h->kind == NLS_PROBLEM_NEOHOOKE) return h->fnode_h;
    return *had_samples ? h->fmid_h : std::vector<double>(3 * (size_t)h->mesh.E, 1.0);
}

static int apply_load(nls_handle* h, const std::vector<double>& full, double sc) {
    std::vector<double> f(full.size());
    for (size_t j = 0; j < full.size(); ++j) f[j] = sc * full[j];
    return h->kind == NLS_PROBLEM_NEOHOOKE ? upload_nodal_load(h, f.data()) : nls_set_load(h, f.data());
}

static int restore_load(nls_handle* h, const std::vector<double>& full, bool had_samples) {
    if (h->kind == NLS_PROBLEM_NEOHOOKE) return upload_nodal_load(h, full.data());
    return nls_set_load(h, had_samples ? full.data() : nullptr);
}

extern "C" int nls_solve(nls_handle* h, double* u, int u_on_device, double load_factor,
                         nls_stats* st) {
    if (!h || !u) return NLS_EINVAL;
    if (!std::isfinite(load_factor)) return fail(h, NLS_EINVAL, "load_factor must be finite");
    if (load_factor == 1.0) return solve_impl(h, u, u_on_device, st);
    if (!h->have_part) return fail(h, NLS_ESTATE, "nls_set_partition first");
    HIPCHK(hipSetDevice(h->opt.device));
    bool had = false;
    const std::vector<double> full = full_load(h, &had);
    int rc = apply_load(h, full, load_factor);
    if (rc == NLS_OK) rc = solve_impl(h, u, u_on_device, st);
    const int r2 = restore_load(h, full, had);
    return rc ? rc : r2;
}

static int solve_impl(nls_handle* h, double* u, int u_on_device, nls_stats* st) {
    if (!h || !u) return NLS_EINVAL;
    if (!h->have_part) return fail(h, NLS_ESTATE, "nls_set_partition first");
    if (h->opt.coupling != NLS_ONE_LEVEL && !h->have_coarse)
        return fail(h, NLS_ESTATE, "two-level coupling needs nls_build_coarse");
    HIPCHK(hipSetDevice(h->opt.device));
    Timer ttot;
    nls_stats local{};
    nls_stats* S = st ? st : &local;
    std::memset(S, 0, sizeof(*S));
    S->failed_subdomain = -1;
    h->st = S;
    guess_new_solve(h);
    h->coarse_lu_valid = false;  // chord steps reuse factorisations within one solve only
    h->coarse_inv_valid = false;
    const int N = h->mesh.ndof();
    double* ud = u;
    if (!u_on_device) {
        ud = h->ubuf;
        HIPCHK(hipMemcpyAsync(ud, u, sizeof(double) * N, hipMemcpyHostToDevice, h->stream));
    }
    auto finish = [&](int code) {
        if (!u_on_device)
            (void)hipMemcpyAsync(u, ud, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream);
        (void)hipStreamSynchronize(h->stream);
        h->collect_events();
        S->ms_total = ttot.ms();
        S->ms_other = S->ms_total - S->ms_inner - S->ms_coarse - S->ms_gmres;
        h->st = nullptr;
        return code;
    };
    const bool tune = (h->opt.flags & NLS_FLAG_AUTOTUNE) && !h->tuned;
    int rc = tune ? autotune_local(h, ud) : NLS_OK;
    if (rc) return finish(rc);
    rc = evaluate(h, ud, h->Fx);
    if (rc) return finish(rc);
    if (tune) {
        rc = autotune_coarse(h);
        if (rc) return finish(rc);
        h->tuned = true;
    }
    double r2 = 0.0;
    rc = dot_host(h, h->Fx, h->Fx, N, &r2);
    if (rc) return finish(rc);
    const double r0 = std::sqrt(r2);
    S->res0 = r0;
    S->res_final = r0;
    if (!std::isfinite(r0)) return finish(fail(h, NLS_ENAN, "F_x(u_0) is not finite"));
    for (int k = 0;; ++k) {
        if (S->res_final <= h->opt.outer_rtol * r0) {
            S->converged = 1;
            break;
        }
        if (k == h->opt.outer_maxit) break;
        rc = prepare_tangent(h);
        if (rc) return finish(rc);
        Timer tg;
        int gits = 0;
        rc = graph_gmres_ok(h) ? gmres_graph(h, h->Fx, h->du, &gits) : gmres(h, h->Fx, h->du, &gits);
        S->ms_gmres += tg.ms();
        if (rc) return finish(rc);
        S->gmres_its[k] = gits;
        S->gmres_its_total += gits;
        rc = 0;
        if (launch_axpy(-1.0, h->du, ud, N, h->stream) != hipSuccess)
            return finish(fail(h, NLS_EHIP, "update failed"));
        rc = evaluate(h, ud, h->Fx);
        if (rc) return finish(rc);
        S->outer_its = k + 1;
        rc = dot_host(h, h->Fx, h->Fx, N, &r2);
        if (rc) return finish(rc);
        S->res_final = std::sqrt(r2);
        if (!std::isfinite(S->res_final)) return finish(fail(h, NLS_ENAN, "F_x is not finite"));
    }
    return finish(S->converged ? NLS_OK : NLS_ENOCONV);
}

// Independent solves (a batch of problems, each with its own handle): every
// handle runs its own outer Newton iteration (eq. 13) with its own stopping
// rule and status, driven by a host thread of its own (at most
// NLS_BATCH_THREADS at a time, taking handles in order), so that the work of
// handles on different streams runs on the device at the same time.
#define NLS_BATCH_THREADS 32
extern "C" int nls_solve_batch(nls_handle* const* hs, int n, double* const* us,
                               const int* u_on_device, nls_stats* sts, int* codes) {
    if (!hs || !us || !codes || n < 1) return NLS_EINVAL;
    for (int k = 0; k < n; ++k)
        if (!hs[k] || !us[k]) return NLS_EINVAL;
    {
        std::vector<nls_handle*> v(hs, hs + n);
        std::sort(v.begin(), v.end());
        if (std::adjacent_find(v.begin(), v.end()) != v.end()) return NLS_EINVAL;
    }
    std::atomic<int> next{0};
    auto work = [&]() {
        for (;;) {
            const int k = next.fetch_add(1);
            if (k >= n) break;
            codes[k] = nls_solve(hs[k], us[k], u_on_device ? u_on_device[k] : 0, 1.0,
                                 sts ? sts + k : nullptr);
        }
    };
    std::vector<std::thread> pool;
    const int nw = std::min(n, NLS_BATCH_THREADS);
    try {
        for (int w = 1; w < nw; ++w) pool.emplace_back(work);
    } catch (...) {
        // fewer threads: the ones started and this one take the rest
    }
    work();
    for (auto& t : pool) t.join();
    int rc = NLS_OK;
    for (int k = 0; k < n; ++k) {
        if (codes[k] < 0) return codes[k];
        if (codes[k] > 0) rc = NLS_ENOCONV;
    }
    return rc;
}

// Load stepping (continuation): the load at s / n_steps of its full value,
// s = 1..n_steps, each outer solve starting from the previous solution.
extern "C" int nls_solve_load_steps(nls_handle* h, double* u, int u_on_device, int n_steps,
                                    nls_stats* st) {
    if (!h || !u || n_steps < 1) return NLS_EINVAL;
    if (!h->have_part) return fail(h, NLS_ESTATE, "nls_set_partition first");
    HIPCHK(hipSetDevice(h->opt.device));
    bool had = false;
    const std::vector<double> full = full_load(h, &had);
    int rc = NLS_OK;
    for (int k = 1; k <= n_steps; ++k) {
        rc = apply_load(h, full, (double)k / (double)n_steps);
        if (rc) break;
        rc = solve_impl(h, u, u_on_device, st ? st + (k - 1) : nullptr);
        if (rc) break;
    }
    // the full load again (the stored problem is unchanged)
    const int r2 = restore_load(h, full, had);
    return rc ? rc : r2;
}

// ------------------------------------------------ Newton-Krylov-Schwarz
// y = DF(u) M^{-1} x with the linear Schwarz preconditioner M^{-1} x =
// sum_i P~_i J_ii(u)^{-1} R_i x (+ Phi A0(u)^{-1} Phi^T x) factored at the
// current iterate (h->nks_u); M^{-1} x is left in h->zbuf.
static int nks_precond(nls_handle* h, const double* x, hipStream_t s) {
    NewtonParams np = h->np;
    np.mixed = 0;
    HIPCHK(launch_tangent_local(h->dm, h->dp, h->dl, np, x, h->lds_tangent, h->npl_local, s, 1));
    if (two_level(h)) {
        DevCoarse& d = h->dc;
        HIPCHK(launch_coarse_phit(d, x, s));
        HIPCHK(launch_coarse_gather(d, s));
        if (h->coarse_inv) {
            HIPCHK(launch_coarse_apply_inverse(d, d.rhs, h->rhs2, s));
            HIPCHK(launch_coarse_scatter(d, h->rhs2, h->ctmp, s));
        } else {
            HIPCHK(launch_coarse_lu(d, 0, h->lds_coarse_lu, h->npl_coarse, s));
            HIPCHK(launch_coarse_scatter(d, nullptr, h->ctmp, s));
        }
        HIPCHK(launch_prolong(h->dm, h->dp, h->dl.z, &d, h->ctmp, h->zbuf, nullptr, s));
    } else {
        HIPCHK(launch_prolong(h->dm, h->dp, h->dl.z, nullptr, nullptr, h->zbuf, nullptr, s));
    }
    return NLS_OK;
}

static int nks_apply(nls_handle* h, const double* x, double* y, hipStream_t s) {
    RC(nks_precond(h, x, s));
    HIPCHK(launch_global_jv(h->dm, h->nks_u, h->zbuf, y, s));
    return NLS_OK;
}

// Factorisations of the preconditioner at u: J_ii(u) per subdomain (FP64
// band LU) and, on a two-level handle, A0(u) = Phi^T DF(u) Phi.
static int nks_factor(nls_handle* h, const double* u) {
    Timer t;
    NewtonParams np = h->np;
    np.mixed = 0;
    RC(bucket_fork(h, h->stream));
    for (size_t b = 0; b < h->bk_start.size(); ++b) {
        DevMaps pb = h->dp;
        pb.order = h->dp.order + h->bk_start[b];
        np.lu_variant = h->bk_var[b];
        HIPCHK(launch_local_factor(h->dm, pb, h->dl, np, u, h->bk_end[b] - h->bk_start[b],
                                   h->bk_lds[b], bucket_stream(h, b, h->stream)));
    }
    RC(bucket_join(h, h->stream));
    HIPCHK(launch_any_status(h->dl.status, h->maps.nsub, h->stat2, h->stream));
    int st2[2];
    HIPCHK(hipMemcpyAsync(st2, h->stat2, 2 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    RC(sync(h));
    if (h->st) h->st->ms_inner += t.ms();
    if (st2[0] >= 0) {
        if (h->st) h->st->failed_subdomain = st2[0];
        return fail(h, NLS_ESINGULAR, "zero pivot in subdomain " + std::to_string(st2[0]));
    }
    if (two_level(h)) {
        Timer tc;
        DevCoarse& d = h->dc;
        HIPCHK(launch_coarse_galerkin(h->dm, d, u, 0, h->stream));
        HIPCHK(launch_coarse_assemble(d, 1, h->stream));
        HIPCHK(launch_coarse_lu(d, 1, h->lds_coarse_lu, h->npl_coarse, h->stream));
        if (h->coarse_inv) HIPCHK(launch_coarse_inverse(d, h->max_block, h->coarse_ldu, h->stream));
        h->coarse_lu_valid = false;  // not the coarse Newton's matrix
        h->coarse_inv_valid = false;
        int flag = 0;
        HIPCHK(hipMemcpyAsync(&flag, d.flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
        RC(sync(h));
        if (flag) return fail(h, NLS_ESINGULAR, "zero pivot in the coarse matrix");
        if (h->st) h->st->ms_coarse += tc.ms();
    }
    return NLS_OK;
}

extern "C" int nls_solve_nks(nls_handle* h, double* u, int u_on_device, nls_stats* st) {
    if (!h || !u) return NLS_EINVAL;
    if (!h->have_part) return fail(h, NLS_ESTATE, "nls_set_partition first");
    if (h->opt.coupling != NLS_ONE_LEVEL && !h->have_coarse)
        return fail(h, NLS_ESTATE, "two-level coupling needs nls_build_coarse");
    HIPCHK(hipSetDevice(h->opt.device));
    Timer ttot;
    nls_stats local{};
    nls_stats* S = st ? st : &local;
    std::memset(S, 0, sizeof(*S));
    S->failed_subdomain = -1;
    h->st = S;
    h->have_state = false;  // the local factors and J values are overwritten
    const int N = h->mesh.ndof();
    double* ud = u;
    if (!u_on_device) {
        ud = h->ubuf;
        HIPCHK(hipMemcpyAsync(ud, u, sizeof(double) * N, hipMemcpyHostToDevice, h->stream));
    }
    h->nks_u = ud;
    auto finish = [&](int code) {
        h->nks_mode = false;
        h->nks_u = nullptr;
        if (!u_on_device)
            (void)hipMemcpyAsync(u, ud, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream);
        (void)hipStreamSynchronize(h->stream);
        S->ms_total = ttot.ms();
        S->ms_other = S->ms_total - S->ms_inner - S->ms_coarse - S->ms_gmres;
        h->st = nullptr;
        return code;
    };
    double r2 = 0.0;
    HIPCHK(launch_global_residual(h->dm, ud, h->Fx, h->stream));
    int rc = dot_host(h, h->Fx, h->Fx, N, &r2);
    if (rc) return finish(rc);
    const double r0 = std::sqrt(r2);
    S->res0 = S->res_final = r0;
    if (!std::isfinite(r0)) return finish(fail(h, NLS_ENAN, "F(u_0) is not finite"));
    for (int k = 0;; ++k) {
        if (S->res_final <= h->opt.outer_rtol * r0) {
            S->converged = 1;
            break;
        }
        if (k == h->opt.outer_maxit) break;
        rc = nks_factor(h, ud);
        if (rc) return finish(rc);
        Timer tg;
        int gits = 0;
        h->nks_mode = true;
        rc = gmres(h, h->Fx, h->du, &gits);  // right-preconditioned: du holds y
        if (rc == NLS_OK) rc = nks_precond(h, h->du, h->stream) ? NLS_EHIP : NLS_OK;
        h->nks_mode = false;
        S->ms_gmres += tg.ms();
        if (rc) return finish(rc);
        S->gmres_its[k] = gits;
        S->gmres_its_total += gits;
        if (launch_axpy(-1.0, h->zbuf, ud, N, h->stream) != hipSuccess)
            return finish(fail(h, NLS_EHIP, "update failed"));
        if (launch_global_residual(h->dm, ud, h->Fx, h->stream) != hipSuccess)
            return finish(fail(h, NLS_EHIP, "residual failed"));
        rc = dot_host(h, h->Fx, h->Fx, N, &r2);
        if (rc) return finish(rc);
        S->outer_its = k + 1;
        S->res_final = std::sqrt(r2);
        if (!std::isfinite(S->res_final)) return finish(fail(h, NLS_ENAN, "F(u) is not finite"));
    }
    return finish(S->converged ? NLS_OK : NLS_ENOCONV);
}

// ------------------------------------------------------------------- hooks
extern "C" int nls_eval_residual(nls_handle* h, const double* u, double* F) {
    if (!h || !u || !F) return NLS_EINVAL;
    if (!h->have_part) return fail(h, NLS_ESTATE, "nls_set_partition first");
    HIPCHK(hipSetDevice(h->opt.device));
    HIPCHK(launch_global_residual(h->dm, u, F, h->stream));
    return sync(h);
}

extern "C" int nls_eval_precond_residual(nls_handle* h, const double* u, double* Fx) {
    if (!h || !u || !Fx) return NLS_EINVAL;
    if (!h->have_part) return fail(h, NLS_ESTATE, "nls_set_partition first");
    if (h->opt.coupling != NLS_ONE_LEVEL && !h->have_coarse)
        return fail(h, NLS_ESTATE, "two-level coupling needs nls_build_coarse");
    HIPCHK(hipSetDevice(h->opt.device));
    h->coarse_lu_valid = false;
    h->coarse_inv_valid = false;
    RC(evaluate(h, u, Fx));
    return sync(h);
}

extern "C" int nls_apply_tangent(nls_handle* h, const double* v, double* y) {
    if (!h || !v || !y) return NLS_EINVAL;
    if (!h->have_state) return fail(h, NLS_ESTATE, "no evaluated point (nls_eval_precond_residual)");
    HIPCHK(hipSetDevice(h->opt.device));
    RC(prepare_tangent(h));
    RC(tangent(h, v, y));
    return sync(h);
}

extern "C" int nls_eval_local(nls_handle* h, const double* u, double* r, double* jval) {
    if (!h || !u || !r) return NLS_EINVAL;
    if (!h->have_part) return fail(h, NLS_ESTATE, "nls_set_partition first");
    HIPCHK(hipSetDevice(h->opt.device));
    const HostMaps& M = h->maps;
    int maxn = 0, maxp = 0;
    for (int i = 0; i < M.nsub; ++i) {
        const int n = M.off_n[i + 1] - M.off_n[i], ng = M.off_g[i + 1] - M.off_g[i];
        maxn = std::max(maxn, n);
        maxp = std::max(maxp, n + ng);
    }
    if (maxp * 8 > 160 * 1024) return fail(h, NLS_ELIMIT, "patch values exceed LDS");
    HIPCHK(launch_local_assemble(h->dm, h->dp, u, r, jval, maxn, maxp * 8, h->stream));
    return sync(h);
}

extern "C" int nls_get_local_pattern(nls_handle* h, int64_t* counts, int32_t* off_v,
                                     int32_t* row_dof, int32_t* off_g, int32_t* gamma_dof,
                                     int64_t* rowptr, int32_t* col) {
    if (!h) return NLS_EINVAL;
    if (!h->have_part) return fail(h, NLS_ESTATE, "nls_set_partition first");
    const HostMaps& M = h->maps;
    const int64_t nrows = M.off_n.back(), nnz = M.jcol.size(), ngam = M.off_g.back();
    if (counts) {
        counts[0] = nrows;
        counts[1] = nnz;
        counts[2] = ngam;
    }
    if (off_v) std::copy(M.off_n.begin(), M.off_n.end(), off_v);
    if (row_dof) std::copy(M.l2g.begin(), M.l2g.end(), row_dof);
    if (off_g) std::copy(M.off_g.begin(), M.off_g.end(), off_g);
    if (gamma_dof) std::copy(M.g2g.begin(), M.g2g.end(), gamma_dof);
    if (rowptr) std::copy(M.jptr.begin(), M.jptr.begin() + nrows + 1, rowptr);
    if (col) std::copy(M.jcol.begin(), M.jcol.end(), col);
    return NLS_OK;
}

extern "C" int nls_get_inner_iterations(nls_handle* h, int32_t* its) {
    if (!h || !its) return NLS_EINVAL;
    if (!h->have_part) return fail(h, NLS_ESTATE, "nls_set_partition first");
    for (int i = 0; i < h->maps.nsub; ++i) its[i] = h->its_h[i];
    return NLS_OK;
}

extern "C" int nls_get_sizes(nls_handle* h, int32_t* n_sub, int32_t* n_coarse, int32_t* nv) {
    if (!h) return NLS_EINVAL;
    if (!h->have_part) return fail(h, NLS_ESTATE, "nls_set_partition first");
    if (n_sub) *n_sub = h->maps.nsub;
    if (n_coarse) *n_coarse = h->have_coarse ? h->co.n0 : 0;
    if (nv)
        for (int i = 0; i < h->maps.nsub; ++i) nv[i] = h->maps.off_n[i + 1] - h->maps.off_n[i];
    return NLS_OK;
}

extern "C" int nls_get_coarse_basis(nls_handle* h, int64_t* nnz, int64_t* rowptr, int32_t* col,
                                    double* val) {
    if (!h || !nnz) return NLS_EINVAL;
    if (!h->have_coarse) return fail(h, NLS_ESTATE, "nls_build_coarse first");
    const HostCoarse& C = h->co;
    const int N = h->mesh.ndof();
    std::vector<double> phi(C.off_phi.back());
    if (!phi.empty()) {
        HIPCHK(hipMemcpyAsync(phi.data(), h->dc.phi, phi.size() * sizeof(double),
                              hipMemcpyDeviceToHost, h->stream));
        RC(sync(h));
    }
    // row g of Phi from the owner's block (the basis is single-valued)
    int64_t cnt = 0;
    std::vector<int64_t> rp(N + 1, 0);
    for (int g = 0; g < N; ++g) {
        const int o = C.cown[g];
        const int nk = C.off_k[o + 1] - C.off_k[o];
        const double* pr = phi.data() + C.off_phi[o] + (int64_t)(C.cpos[g] - C.off_c[o]) * nk;
        for (int l = 0; l < nk; ++l)
            if (pr[l] != 0.0) {
                if (rowptr) {
                    col[cnt] = C.klist[C.off_k[o] + l];
                    val[cnt] = pr[l];
                }
                ++cnt;
            }
        rp[g + 1] = cnt;
    }
    if (rowptr && cnt > *nnz) return fail(h, NLS_EINVAL, "nnz buffer too small");
    if (rowptr)
        for (int g = 0; g <= N; ++g) rowptr[g] = rp[g];
    *nnz = cnt;
    return NLS_OK;
}

extern "C" const char* nls_strerror(int code) {
    switch (code) {
        case NLS_OK: return "success";
        case NLS_ENOCONV: return "outer Newton iteration did not converge";
        case NLS_EINVAL: return "invalid argument";
        case NLS_EHIP: return "HIP runtime error";
        case NLS_ENOMEM: return "device allocation failed";
        case NLS_EPARTITION: return "invalid partition";
        case NLS_ESINGULAR: return "zero pivot";
        case NLS_ELOCAL: return "inner Newton iteration failed";
        case NLS_ENAN: return "non-finite value";
        case NLS_ESTATE: return "call out of order";
        case NLS_ELIMIT: return "size exceeds a kernel limit";
        default: return "unknown status";
    }
}

extern "C" const char* nls_last_error(nls_handle* h) {
    return h ? h->err.c_str() : "null handle";
}

extern "C" int nls_get_tuning(nls_handle* h, int32_t* n_buckets, int32_t* lu_variant,
                              int32_t* lds_bytes, int32_t* n_sub, int32_t* coarse_inverse,
                              double* coarse_ms, int32_t* local_precision) {
    if (!h) return NLS_EINVAL;
    if (!h->have_part) return fail(h, NLS_ESTATE, "nls_set_partition first");
    const int nb = (int)h->bk_start.size();
    if (n_buckets) *n_buckets = nb;
    for (int b = 0; b < nb; ++b) {
        if (lu_variant) lu_variant[b] = h->bk_var[b];
        if (lds_bytes) lds_bytes[b] = h->bk_lds[b];
        if (n_sub) n_sub[b] = h->bk_end[b] - h->bk_start[b];
    }
    if (coarse_inverse) *coarse_inverse = h->coarse_inv ? 1 : 0;
    if (coarse_ms)
        for (int k = 0; k < 3; ++k) coarse_ms[k] = h->tune_ms[k];
    if (local_precision)
        *local_precision = h->np.mixed == 2 ? NLS_PREC_BF16_IR
                                            : (h->np.mixed ? NLS_PREC_FP32_IR : NLS_PREC_FP64);
    return NLS_OK;
}
