// Host-side setup of libnls: overlapping subdomains, local orderings and
// band widths, restricted-prolongation owners, and the symbolic part of the
// GDSW coarse space.  Integer work only; every floating-point step of the
// method runs in the HIP kernels.
//
// Overlap (paper, Section 2, last paragraph): the overlapping partition is
// element based so that each subdomain assembles its own residual and
// tangent.  Each subdomain's element set is grown by `overlap` layers of
// elements that share a node with it.  V_i holds the patch nodes whose
// every element lies in the patch (so R_i F can be assembled from patch
// elements alone); the remaining patch nodes Gamma_i carry the current
// global values.  Restricted prolongation P~_i (eq. 8): node g belongs to
// the largest subdomain id among its elements.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <numeric>
#include <queue>

#include "nls.h"
#include "nls_internal.h"

int nls_build_node_incidence(HostMesh& m, std::string& err) {
    const int nv = m.nv;
    m.nptr.assign(m.N + 1, 0);
    for (int e = 0; e < m.E; ++e)
        for (int v = 0; v < nv; ++v) {
            int g = m.conn[nv * e + v];
            if (g < 0 || g >= m.N) {
                err = "element node index out of range";
                return NLS_EINVAL;
            }
            m.nptr[g + 1]++;
        }
    for (int g = 0; g < m.N; ++g) m.nptr[g + 1] += m.nptr[g];
    m.nel.assign(m.nptr[m.N], 0);
    std::vector<int> fill(m.nptr.begin(), m.nptr.end() - 1);
    for (int e = 0; e < m.E; ++e)
        for (int v = 0; v < nv; ++v) m.nel[fill[m.conn[nv * e + v]]++] = e;
    return NLS_OK;
}

static inline int vertex_pos(const HostMesh& m, int e, int g) {
    for (int v = 0; v < m.nv; ++v)
        if (m.conn[m.nv * e + v] == g) return v;
    return -1;
}

int nls_build_maps(const HostMesh& m, const int* part, int nsub, int overlap,
                   HostMaps& out, std::string& err) {
    const int N = m.N, E = m.E, nv = m.nv, dd = m.d;
    if (nsub <= 0 || overlap < 1) {
        err = "need n_sub >= 1 and overlap >= 1 (owned nodes must lie in V_i)";
        return NLS_EPARTITION;
    }
    std::vector<std::vector<int>> elems_of(nsub);
    for (int e = 0; e < E; ++e) {
        if (part[e] < 0 || part[e] >= nsub) {
            err = "elem_part entry out of range";
            return NLS_EINVAL;
        }
        elems_of[part[e]].push_back(e);
    }
    for (int i = 0; i < nsub; ++i)
        if (elems_of[i].empty()) {
            err = "subdomain " + std::to_string(i) + " is empty";
            return NLS_EPARTITION;
        }
    std::vector<int> owner(N, -1);
    for (int e = 0; e < E; ++e)
        for (int v = 0; v < nv; ++v) {
            int g = m.conn[nv * e + v];
            owner[g] = std::max(owner[g], part[e]);
        }

    HostMaps& M = out;
    M = HostMaps();
    M.nsub = nsub;
    M.off_n.assign(1, 0);
    M.off_g.assign(1, 0);
    M.off_e.assign(1, 0);
    M.rinc_ptr.assign(1, 0);
    M.jptr.assign(1, 0);
    M.own_pidx.assign((size_t)N * dd, -1);
    std::vector<char> inpatch(E, 0), nmark(N, 0);
    std::vector<int> cnt(N, 0), loc(N, -1), eloc(E, -1);

    for (int i = 0; i < nsub; ++i) {
        std::vector<int> pe = elems_of[i];
        for (int e : pe) inpatch[e] = 1;
        for (int layer = 0; layer < overlap; ++layer) {
            std::vector<int> nodes;
            for (int e : pe)
                for (int v = 0; v < nv; ++v) {
                    int g = m.conn[nv * e + v];
                    if (!nmark[g]) { nmark[g] = 1; nodes.push_back(g); }
                }
            std::vector<int> add;
            for (int g : nodes) {
                nmark[g] = 0;
                for (int k = m.nptr[g]; k < m.nptr[g + 1]; ++k) {
                    int e = m.nel[k];
                    if (!inpatch[e]) { inpatch[e] = 1; add.push_back(e); }
                }
            }
            pe.insert(pe.end(), add.begin(), add.end());
        }
        std::sort(pe.begin(), pe.end());
        std::vector<int> pnodes;
        for (int e : pe)
            for (int v = 0; v < nv; ++v) {
                int g = m.conn[nv * e + v];
                if (cnt[g]++ == 0) pnodes.push_back(g);
            }
        std::vector<int> V, G;
        for (int g : pnodes) {
            if (cnt[g] == m.nptr[g + 1] - m.nptr[g]) V.push_back(g);
            else G.push_back(g);
        }
        std::sort(V.begin(), V.end());
        std::sort(G.begin(), G.end());
        if (dd > 1 && !V.empty()) {
            // vector problems: the shorter side of the patch box varies
            // fastest, so the dof band of J_ii stays near d x (short side)
            double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
            for (int g : V) {
                x0 = std::min(x0, m.xy[2 * g]);
                x1 = std::max(x1, m.xy[2 * g]);
                y0 = std::min(y0, m.xy[2 * g + 1]);
                y1 = std::max(y1, m.xy[2 * g + 1]);
            }
            if (x1 - x0 > y1 - y0)
                std::stable_sort(V.begin(), V.end(), [&](int a, int b) {
                    if (m.xy[2 * a] != m.xy[2 * b]) return m.xy[2 * a] < m.xy[2 * b];
                    return m.xy[2 * a + 1] < m.xy[2 * b + 1];
                });
        }
        const int nn = (int)V.size(), n = dd * nn;
        for (int a = 0; a < nn; ++a) loc[V[a]] = a;
        for (int j = 0; j < (int)G.size(); ++j) loc[G[j]] = nn + j;
        for (int k = 0; k < (int)pe.size(); ++k) eloc[pe[k]] = k;
        for (int e : pe) {
            for (int v = 0; v < nv; ++v) M.pe_conn.push_back(loc[m.conn[nv * e + v]]);
            M.pe_gid.push_back(e);
        }
        int kl = 0, ku = 0;
        std::vector<int> cols, inc;
        for (int a = 0; a < nn; ++a) {
            int g = V[a];
            cols.clear();
            inc.clear();
            for (int k = m.nptr[g]; k < m.nptr[g + 1]; ++k) {
                int e = m.nel[k];
                inc.push_back((eloc[e] << 2) | vertex_pos(m, e, g));
                for (int v = 0; v < nv; ++v)
                    for (int c = 0; c < dd; ++c) cols.push_back(dd * loc[m.conn[nv * e + v]] + c);
            }
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
            for (int c = 0; c < dd; ++c) {
                const int row = dd * a + c;
                M.rinc.insert(M.rinc.end(), inc.begin(), inc.end());
                for (int col : cols) {
                    M.jcol.push_back(col);
                    if (col < n) {
                        kl = std::max(kl, row - col);
                        ku = std::max(ku, col - row);
                    }
                }
                M.rinc_ptr.push_back((int)M.rinc.size());
                M.jptr.push_back((int)M.jcol.size());
            }
        }
        const int rb = (int)M.l2g.size();
        for (int a = 0; a < nn; ++a)
            for (int c = 0; c < dd; ++c) {
                M.l2g.push_back(dd * V[a] + c);
                if (owner[V[a]] == i) M.own_pidx[(size_t)dd * V[a] + c] = rb + dd * a + c;
            }
        for (int g : G)
            for (int c = 0; c < dd; ++c) M.g2g.push_back(dd * g + c);
        M.off_n.push_back((int)M.l2g.size());
        M.off_g.push_back((int)M.g2g.size());
        M.off_e.push_back((int)M.pe_gid.size());
        M.kl.push_back(kl);
        M.ku.push_back(ku);
        for (int g : pnodes) { cnt[g] = 0; loc[g] = -1; }
        for (int e : pe) { eloc[e] = -1; inpatch[e] = 0; }
    }

    // owners: the owned nodes of subdomain o must lie in V_o
    for (int g = 0; g < N; ++g) {
        int o = owner[g];
        if (o < 0) {
            err = "node " + std::to_string(g) + " belongs to no element";
            return NLS_EINVAL;
        }
        if (M.own_pidx[(size_t)dd * g] < 0) {
            err = "subdomain " + std::to_string(o) + ": owned node " +
                  std::to_string(g) + " not in V_i";
            return NLS_EPARTITION;
        }
    }

    // B_i by columns (Gamma columns of the local CSR rows), owned rows
    M.bptr.assign(1, 0);
    M.off_own.assign(1, 0);
    M.rowown.assign(M.l2g.size(), -1);
    M.off_W.assign(1, 0);
    M.off_F.assign(1, 0);
    for (int i = 0; i < nsub; ++i) {
        const int rb = M.off_n[i], n = M.off_n[i + 1] - rb, ng = M.off_g[i + 1] - M.off_g[i];
        std::vector<std::vector<std::pair<int, int>>> colent(ng);
        for (int a = 0; a < n; ++a)
            for (int s = M.jptr[rb + a]; s < M.jptr[rb + a + 1]; ++s)
                if (M.jcol[s] >= n) colent[M.jcol[s] - n].push_back({a, s});
        for (int j = 0; j < ng; ++j) {
            for (auto& e : colent[j]) {
                M.brow.push_back(e.first);
                M.bslot.push_back(e.second);
            }
            M.max_bcol = std::max(M.max_bcol, (int)colent[j].size());
            M.bptr.push_back((int)M.brow.size());
        }
        int no = 0;
        for (int a = 0; a < n; ++a)
            if (owner[M.l2g[rb + a] / dd] == i) {
                M.rowown[rb + a] = no++;
                M.ownrow.push_back(a);
            }
        M.off_own.push_back((int)M.ownrow.size());
        M.off_W.push_back(M.off_W.back() + (int64_t)no * ng);
        M.off_F.push_back(M.off_F.back() + (int64_t)((n + 15) / 16 * 16) * ((ng + 15) / 16 * 16));
    }

    // factor storage and launch order
    M.off_u.assign(nsub + 1, 0);
    M.off_l.assign(nsub + 1, 0);
    M.lds_doubles.assign(nsub, 0);
    for (int i = 0; i < nsub; ++i) {
        int64_t n = M.off_n[i + 1] - M.off_n[i];
        int ng = M.off_g[i + 1] - M.off_g[i];
        M.off_u[i + 1] = M.off_u[i] + n * (M.kl[i] + M.ku[i] + 1);
        M.off_l[i + 1] = M.off_l[i] + n * std::max(M.kl[i], 1);
        M.lds_doubles[i] = local_lds_doubles((int)n, ng, M.kl[i], M.ku[i]);
        M.max_lds_doubles = std::max(M.max_lds_doubles, M.lds_doubles[i]);
    }
    M.factor_u_total = M.off_u[nsub];
    M.factor_l_total = M.off_l[nsub];
    M.order.resize(nsub);
    std::iota(M.order.begin(), M.order.end(), 0);
    std::stable_sort(M.order.begin(), M.order.end(), [&](int a, int b) {
        return M.lds_doubles[a] > M.lds_doubles[b];
    });
    return NLS_OK;
}

// Reverse Cuthill-McKee ordering of a symmetric pattern (adjacency lists).
static std::vector<int> rcm_order(const std::vector<std::vector<int>>& adj) {
    const int n = (int)adj.size();
    std::vector<int> order, deg(n);
    for (int i = 0; i < n; ++i) deg[i] = (int)adj[i].size();
    std::vector<char> seen(n, 0);
    std::vector<int> byDeg(n);
    std::iota(byDeg.begin(), byDeg.end(), 0);
    std::stable_sort(byDeg.begin(), byDeg.end(),
                     [&](int a, int b) { return deg[a] < deg[b]; });
    for (int s : byDeg) {
        if (seen[s]) continue;
        std::queue<int> q;
        q.push(s);
        seen[s] = 1;
        while (!q.empty()) {
            int v = q.front();
            q.pop();
            order.push_back(v);
            std::vector<int> nb;
            for (int w : adj[v])
                if (!seen[w]) { seen[w] = 1; nb.push_back(w); }
            std::stable_sort(nb.begin(), nb.end(),
                             [&](int a, int b) { return deg[a] < deg[b]; });
            for (int w : nb) q.push(w);
        }
    }
    std::reverse(order.begin(), order.end());
    return order;  // order[p] = vertex at position p
}

int nls_build_coarse_symbolic(const HostMesh& m, const int* part, int nsub, int kind,
                              HostCoarse& out, std::string& err) {
    const int N = m.N, E = m.E, nv = m.nv, dd = m.d;
    HostCoarse& C = out;
    C = HostCoarse();
    // subdomain sets of every node
    std::vector<std::vector<int>> sset(N);
    for (int g = 0; g < N; ++g) {
        for (int k = m.nptr[g]; k < m.nptr[g + 1]; ++k) sset[g].push_back(part[m.nel[k]]);
        std::sort(sset[g].begin(), sset[g].end());
        sset[g].erase(std::unique(sset[g].begin(), sset[g].end()), sset[g].end());
    }
    // a node is a Dirichlet node when any of its dofs is
    std::vector<char> ndir(N, 0), iface(N, 0);
    for (int g = 0; g < N; ++g) {
        for (int c = 0; c < dd; ++c) ndir[g] |= m.dflag[(size_t)dd * g + c];
        iface[g] = sset[g].size() >= 2 && !ndir[g];
    }
    // classes keyed by the subdomain set, split into connected components
    std::map<std::vector<int>, int> key_id;
    std::vector<int> cls(N, -1);
    for (int g = 0; g < N; ++g)
        if (iface[g]) {
            auto it = key_id.find(sset[g]);
            if (it == key_id.end()) it = key_id.emplace(sset[g], (int)key_id.size()).first;
            cls[g] = it->second;
        }
    C.comp_of.assign(N, -1);
    std::vector<std::vector<int>> comps;
    for (int g = 0; g < N; ++g) {
        if (cls[g] < 0 || C.comp_of[g] >= 0) continue;
        int cid = (int)comps.size();
        comps.emplace_back();
        std::queue<int> q;
        q.push(g);
        C.comp_of[g] = cid;
        while (!q.empty()) {
            int v = q.front();
            q.pop();
            comps[cid].push_back(v);
            for (int k = m.nptr[v]; k < m.nptr[v + 1]; ++k) {
                int e = m.nel[k];
                // neighbours along element edges (consecutive nodes)
                const int p = vertex_pos(m, e, v);
                for (int t : {(p + 1) % nv, (p + nv - 1) % nv}) {
                    int w = m.conn[nv * e + t];
                    if (cls[w] == cls[g] && C.comp_of[w] < 0) {
                        C.comp_of[w] = cid;
                        q.push(w);
                    }
                }
            }
        }
        std::sort(comps[cid].begin(), comps[cid].end());
    }
    // order components by their smallest node (canonical)
    std::vector<int> cperm(comps.size());
    std::iota(cperm.begin(), cperm.end(), 0);
    std::sort(cperm.begin(), cperm.end(),
              [&](int a, int b) { return comps[a][0] < comps[b][0]; });
    std::vector<int> rank(comps.size());
    for (int r = 0; r < (int)cperm.size(); ++r) rank[cperm[r]] = r;
    C.comps.resize(comps.size());
    for (int c = 0; c < (int)comps.size(); ++c) C.comps[rank[c]] = comps[c];
    for (int g = 0; g < N; ++g)
        if (C.comp_of[g] >= 0) C.comp_of[g] = rank[C.comp_of[g]];
    // interface values of the coarse functions at every interface dof:
    // (function id, value) pairs
    const int ncomps = (int)C.comps.size();
    std::vector<std::vector<std::pair<int, double>>> ifv((size_t)N * dd);
    std::vector<double> cxc(ncomps, 0.0), cyc(ncomps, 0.0);
    auto centroid = [&](int c) {
        cxc[c] = cyc[c] = 0.0;
        for (int g : C.comps[c]) {
            cxc[c] += m.xy[2 * g];
            cyc[c] += m.xy[2 * g + 1];
        }
        cxc[c] /= (double)C.comps[c].size();
        cyc[c] /= (double)C.comps[c].size();
    };
    // the functions of one coarse node (base fb, center c) at node g with
    // weight w: scalar w; elasticity translations w and rotation w * r_c(g)
    auto put = [&](int g, int fb, int nf, double w, double x0, double y0) {
        if (dd == 1) {
            ifv[g].push_back({fb, w});
            return;
        }
        const double r[2] = {-(m.xy[2 * g + 1] - y0), m.xy[2 * g] - x0};
        for (int c = 0; c < 2; ++c) {
            ifv[2 * (size_t)g + c].push_back({fb + c, w});
            if (nf == 3 && r[c] != 0.0) ifv[2 * (size_t)g + c].push_back({fb + 2, w * r[c]});
        }
    };
    C.fun_base.assign(ncomps, -1);
    C.nfun.assign(ncomps, 0);
    int nfuns = 0;
    if (kind != NLS_COARSE_RGDSW) {
        // GDSW: every component; scalar 1 function, elasticity the two
        // translations and, on components of >= 2 nodes, the rotation
        for (int c = 0; c < ncomps; ++c) {
            C.fun_base[c] = nfuns;
            C.nfun[c] = dd == 1 ? 1 : (C.comps[c].size() >= 2 ? 3 : 2);
            nfuns += C.nfun[c];
            if (C.nfun[c] == 3) centroid(c);
            for (int g : C.comps[c]) put(g, C.fun_base[c], C.nfun[c], 1.0, cxc[c], cyc[c]);
        }
    } else {
        // RGDSW option 2.2: coarse nodes are the crosspoint components
        // (>= 3 subdomains) and edge components without ancestor
        // crosspoints; other edge nodes take inverse-distance weights of
        // their ancestors, a Dirichlet node ending the edge counting as an
        // ancestor of value 0
        std::vector<std::vector<int>> anc(ncomps);
        std::vector<char> isvert(ncomps, 0);
        for (int c = 0; c < ncomps; ++c) isvert[c] = sset[C.comps[c][0]].size() >= 3;
        for (int c = 0; c < ncomps; ++c) {
            if (isvert[c]) continue;
            const auto& se = sset[C.comps[c][0]];
            for (int v = 0; v < ncomps; ++v)
                if (isvert[v] && std::includes(sset[C.comps[v][0]].begin(), sset[C.comps[v][0]].end(),
                                               se.begin(), se.end()))
                    anc[c].push_back(v);
        }
        const int nf = dd == 1 ? 1 : 3;
        for (int c = 0; c < ncomps; ++c) {   // canonical order: smallest node
            if (!isvert[c] && !anc[c].empty()) continue;
            C.fun_base[c] = nfuns;
            C.nfun[c] = nf;
            nfuns += nf;
            centroid(c);
            for (int g : C.comps[c]) put(g, C.fun_base[c], nf, 1.0, cxc[c], cyc[c]);
        }
        for (int c = 0; c < ncomps; ++c) {
            if (isvert[c] || anc[c].empty()) continue;
            const auto& se = sset[C.comps[c][0]];
            std::vector<int> dends;
            for (int g : C.comps[c])
                for (int k = m.nptr[g]; k < m.nptr[g + 1]; ++k) {
                    const int e = m.nel[k], p = vertex_pos(m, e, g);
                    for (int t : {(p + 1) % nv, (p + nv - 1) % nv}) {
                        const int w = m.conn[nv * e + t];
                        if (ndir[w] && std::includes(sset[w].begin(), sset[w].end(), se.begin(), se.end()))
                            dends.push_back(w);
                    }
                }
            std::sort(dends.begin(), dends.end());
            dends.erase(std::unique(dends.begin(), dends.end()), dends.end());
            for (int g : C.comps[c]) {
                const double gx = m.xy[2 * g], gy = m.xy[2 * g + 1];
                double den = 0.0;
                std::vector<double> inv(anc[c].size());
                for (size_t a = 0; a < anc[c].size(); ++a) {
                    const int v = anc[c][a];
                    inv[a] = 1.0 / std::hypot(gx - cxc[v], gy - cyc[v]);
                    den += inv[a];
                }
                for (int w : dends) den += 1.0 / std::hypot(gx - m.xy[2 * w], gy - m.xy[2 * w + 1]);
                for (size_t a = 0; a < anc[c].size(); ++a) {
                    const int v = anc[c][a];
                    put(g, C.fun_base[v], nf, inv[a] / den, cxc[v], cyc[v]);
                }
            }
        }
    }
    C.n0 = nfuns;
    for (auto& l : ifv)
        if ((int)l.size() > NLS_CFUN) {
            err = "an interface dof carries more than NLS_CFUN coarse functions";
            return NLS_ELIMIT;
        }

    std::vector<std::vector<int>> elems_of(nsub);
    for (int e = 0; e < E; ++e) elems_of[part[e]].push_back(e);

    C.off_c.assign(1, 0);
    C.off_k.assign(1, 0);
    C.off_phi.assign(1, 0);
    C.off_ne.assign(1, 0);
    C.off_ni.assign(1, 0);
    C.cinc_ptr.assign(1, 0);
    C.iptr.assign(1, 0);
    C.off_iu.assign(1, 0);
    C.off_il.assign(1, 0);
    C.off_kk.assign(1, 0);
    std::vector<int> cl(N, -1), el(E, -1);
    for (int i = 0; i < nsub; ++i) {
        std::vector<int> nodes;
        for (int e : elems_of[i])
            for (int v = 0; v < nv; ++v) nodes.push_back(m.conn[nv * e + v]);
        std::sort(nodes.begin(), nodes.end());
        nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
        for (int a = 0; a < (int)nodes.size(); ++a) cl[nodes[a]] = a;
        for (int k = 0; k < (int)elems_of[i].size(); ++k) el[elems_of[i][k]] = k;
        std::vector<int> K;
        for (int g : nodes)
            if (iface[g])
                for (int c = 0; c < dd; ++c)
                    for (auto& fv : ifv[(size_t)dd * g + c]) K.push_back(fv.first);
        std::sort(K.begin(), K.end());
        K.erase(std::unique(K.begin(), K.end()), K.end());
        auto kpos = [&](int f) { return (int)(std::lower_bound(K.begin(), K.end(), f) - K.begin()); };
        C.max_k = std::max(C.max_k, (int)K.size());
        int ni = 0;
        std::vector<int> inter;   // closure dof index of each interior row
        for (int a = 0; a < (int)nodes.size(); ++a) {
            const int g = nodes[a];
            const int t = ndir[g] ? 2 : (iface[g] ? 1 : (sset[g].size() == 1 ? 0 : 2));
            std::vector<int> ci;
            for (int k = m.nptr[g]; k < m.nptr[g + 1]; ++k) {
                int e = m.nel[k];
                if (part[e] == i) ci.push_back((el[e] << 2) | vertex_pos(m, e, g));
            }
            for (int c = 0; c < dd; ++c) {
                C.cnode.push_back(dd * g + c);
                C.ctype.push_back(t);
                const auto& fl = ifv[(size_t)dd * g + c];
                for (int q = 0; q < NLS_CFUN; ++q) {
                    const bool has = t == 1 && q < (int)fl.size();
                    C.cfun.push_back(has ? kpos(fl[q].first) : -1);
                    C.cval.push_back(has ? fl[q].second : 0.0);
                }
                C.iidx.push_back(t == 0 ? ni : -1);
                if (t == 0) { inter.push_back(dd * a + c); ++ni; }
                C.cinc.insert(C.cinc.end(), ci.begin(), ci.end());
                C.cinc_ptr.push_back((int)C.cinc.size());
            }
        }
        for (int e : elems_of[i]) {
            for (int v = 0; v < nv; ++v) C.ne_conn.push_back(cl[m.conn[nv * e + v]]);
            C.ne_gid.push_back(e);
        }
        // interior CSR and band of A_II
        int kl = 0, ku = 0;
        const int cbase = C.off_c.back();
        std::vector<int> cols;
        for (int r = 0; r < ni; ++r) {
            const int g = nodes[inter[r] / dd];
            cols.clear();
            for (int k = m.nptr[g]; k < m.nptr[g + 1]; ++k) {
                int e = m.nel[k];
                for (int v = 0; v < nv; ++v)
                    for (int c = 0; c < dd; ++c) {
                        int col = C.iidx[cbase + dd * cl[m.conn[nv * e + v]] + c];
                        if (col >= 0) cols.push_back(col);
                    }
            }
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
            for (int c : cols) {
                C.icol.push_back(c);
                kl = std::max(kl, r - c);
                ku = std::max(ku, c - r);
            }
            C.iptr.push_back((int)C.icol.size());
            C.inode.push_back(inter[r]);
        }
        C.ikl.push_back(kl);
        C.iku.push_back(ku);
        C.off_iu.push_back(C.off_iu.back() + (int64_t)ni * (kl + ku + 1));
        C.off_il.push_back(C.off_il.back() + (int64_t)ni * std::max(kl, 1));
        int ld = interior_lds_doubles(ni, kl, ku, (int)K.size());
        C.ilds_doubles.push_back(ld);
        C.max_ilds_doubles = std::max(C.max_ilds_doubles, ld);
        C.klist.insert(C.klist.end(), K.begin(), K.end());
        C.off_c.push_back((int)C.cnode.size());
        C.off_k.push_back((int)C.klist.size());
        C.off_phi.push_back(C.off_phi.back() + (int64_t)nodes.size() * dd * K.size());
        C.off_ne.push_back((int)C.ne_gid.size());
        C.off_ni.push_back((int)C.inode.size());
        C.off_kk.push_back(C.off_kk.back() + (int64_t)K.size() * K.size());
        for (int g : nodes) cl[g] = -1;
        for (int e : elems_of[i]) el[e] = -1;
    }
    C.iu_total = C.off_iu.back();
    C.il_total = C.off_il.back();

    // owner closure positions for prolongation of coarse vectors (per dof)
    C.cpos.assign((size_t)N * dd, -1);
    C.cown.assign((size_t)N * dd, -1);
    for (int g = 0; g < N; ++g) {
        int o = -1;
        for (int k = m.nptr[g]; k < m.nptr[g + 1]; ++k) o = std::max(o, part[m.nel[k]]);
        for (int c = 0; c < dd; ++c) {
            const int gd = dd * g + c;
            auto b = C.cnode.begin() + C.off_c[o], en = C.cnode.begin() + C.off_c[o + 1];
            auto it = std::lower_bound(b, en, gd);
            C.cown[gd] = o;
            C.cpos[gd] = (int)(it - C.cnode.begin());
        }
    }

    // Galerkin pattern, banded ordering and deterministic source lists
    const int n0 = C.n0;
    std::vector<std::vector<int>> adj(n0);
    std::map<std::pair<int, int>, std::vector<int>> src;
    std::vector<std::vector<int>> gs(n0);
    for (int i = 0; i < nsub; ++i) {
        int k0 = C.off_k[i], nk = C.off_k[i + 1] - k0;
        for (int p = 0; p < nk; ++p) {
            int kp = C.klist[k0 + p];
            gs[kp].push_back(k0 + p);
            for (int q = 0; q < nk; ++q) {
                int kq = C.klist[k0 + q];
                src[{kp, kq}].push_back((int)(C.off_kk[i] + (int64_t)p * nk + q));
                if (kp != kq) adj[kp].push_back(kq);
            }
        }
    }
    for (auto& a : adj) {
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
    }
    // banded ordering of A0: reverse Cuthill-McKee, or the canonical order
    // (components by smallest node) when that is narrower
    std::vector<int> ord = n0 ? rcm_order(adj) : std::vector<int>();
    std::vector<int> prcm(n0), pnat(n0);
    for (int p = 0; p < n0; ++p) { prcm[ord[p]] = p; pnat[p] = p; }
    auto width = [&](const std::vector<int>& pm) {
        int w = 0;
        for (int k = 0; k < n0; ++k)
            for (int l : adj[k]) w = std::max(w, std::abs(pm[k] - pm[l]));
        return w;
    };
    std::vector<int> perm0 = width(prcm) < width(pnat) ? prcm : pnat;
    // independent problems give a block-diagonal A0: make every connected
    // component contiguous in band order (relative order kept) and factor
    // the blocks separately
    std::vector<int> comp(n0, -1);
    int ncomp = 0;
    {
        std::vector<int> pos2k(n0);
        for (int k = 0; k < n0; ++k) pos2k[perm0[k]] = k;
        for (int p = 0; p < n0; ++p) {
            const int k0 = pos2k[p];
            if (comp[k0] >= 0) continue;
            std::queue<int> q;
            q.push(k0);
            comp[k0] = ncomp;
            while (!q.empty()) {
                const int v = q.front();
                q.pop();
                for (int w : adj[v])
                    if (comp[w] < 0) { comp[w] = ncomp; q.push(w); }
            }
            ++ncomp;
        }
        std::vector<int> bypos(n0);
        std::iota(bypos.begin(), bypos.end(), 0);  // band positions
        std::stable_sort(bypos.begin(), bypos.end(),
                         [&](int a, int b) { return comp[pos2k[a]] < comp[pos2k[b]]; });
        C.perm.assign(n0, 0);
        for (int p = 0; p < n0; ++p) C.perm[pos2k[bypos[p]]] = p;
    }
    C.boff.assign(ncomp + 1, 0);
    for (int k = 0; k < n0; ++k) C.boff[comp[k] + 1]++;
    for (int b = 0; b < ncomp; ++b) C.boff[b + 1] += C.boff[b];
    C.bkl.assign(ncomp, 0);
    C.bku.assign(ncomp, 0);
    C.rblk.assign(n0, 0);
    for (int k = 0; k < n0; ++k) C.rblk[C.perm[k]] = comp[k];
    std::vector<std::vector<std::pair<int, std::vector<int>*>>> rows(n0);
    for (auto& kv : src) {
        int r = C.perm[kv.first.first], c = C.perm[kv.first.second];
        rows[r].push_back({c, &kv.second});
        const int b = C.rblk[r];
        C.bkl[b] = std::max(C.bkl[b], r - c);
        C.bku[b] = std::max(C.bku[b], c - r);
    }
    C.offU.assign(ncomp + 1, 0);
    C.offL.assign(ncomp + 1, 0);
    C.offI.assign(ncomp + 1, 0);
    for (int b = 0; b < ncomp; ++b) {
        const int64_t nb = C.boff[b + 1] - C.boff[b];
        C.offU[b + 1] = C.offU[b] + nb * (C.bkl[b] + C.bku[b] + 1);
        C.offL[b + 1] = C.offL[b] + nb * std::max(C.bkl[b], 1);
        C.offI[b + 1] = C.offI[b] + nb * nb;
        C.a0kl = std::max(C.a0kl, C.bkl[b]);
        C.a0ku = std::max(C.a0ku, C.bku[b]);
    }
    C.a0ptr.assign(1, 0);
    C.a0src_ptr.assign(1, 0);
    for (int r = 0; r < n0; ++r) {
        std::sort(rows[r].begin(), rows[r].end(),
                  [](const auto& a, const auto& b) { return a.first < b.first; });
        for (auto& e : rows[r]) {
            C.a0col.push_back(e.first);
            C.a0src.insert(C.a0src.end(), e.second->begin(), e.second->end());
            C.a0src_ptr.push_back((int)C.a0src.size());
        }
        C.a0ptr.push_back((int)C.a0col.size());
    }
    C.gsrc_ptr.assign(1, 0);
    for (int k = 0; k < n0; ++k) {
        C.gsrc.insert(C.gsrc.end(), gs[k].begin(), gs[k].end());
        C.gsrc_ptr.push_back((int)C.gsrc.size());
    }
    (void)err;
    return NLS_OK;
}

// ---------------------------------------------------------------- inspection
// ---------------------------------------------------------------------------
// Learned initial guess: patch boxes and sampling tables.
//
// Each sample is the linear interpolant of a global nodal field in the mesh
// element containing the sample point: among the candidate elements the one
// with the largest smallest barycentric coordinate (on a shared edge either
// neighbour gives the same value up to rounding).  The candidates come from
// a uniform bucket grid over the mesh; a point whose bucket holds no element
// containing it widens the search ring by ring (points outside the mesh end
// with the nearest element, i.e. linear extrapolation).
// ---------------------------------------------------------------------------
namespace {
struct BucketGrid {
    double x0, y0, hx, hy;
    int nx, ny;
    std::vector<int> ptr, elems;
};

void barycentric(const HostMesh& m, int e, double px, double py, double lam[3]) {
    const int a = m.conn[3 * e], b = m.conn[3 * e + 1], c = m.conn[3 * e + 2];
    const double ax = m.xy[2 * a], ay = m.xy[2 * a + 1];
    const double bx = m.xy[2 * b], by = m.xy[2 * b + 1];
    const double cx = m.xy[2 * c], cy = m.xy[2 * c + 1];
    const double det = (bx - ax) * (cy - ay) - (cx - ax) * (by - ay);
    const double dx = px - ax, dy = py - ay;
    const double l1 = (dx * (cy - ay) - dy * (cx - ax)) / det;
    const double l2 = ((bx - ax) * dy - (by - ay) * dx) / det;
    lam[0] = 1.0 - l1 - l2;
    lam[1] = l1;
    lam[2] = l2;
}

BucketGrid build_buckets(const HostMesh& m) {
    BucketGrid g;
    double xmin = m.xy[0], xmax = m.xy[0], ymin = m.xy[1], ymax = m.xy[1];
    for (int v = 0; v < m.N; ++v) {
        xmin = std::min(xmin, m.xy[2 * v]);
        xmax = std::max(xmax, m.xy[2 * v]);
        ymin = std::min(ymin, m.xy[2 * v + 1]);
        ymax = std::max(ymax, m.xy[2 * v + 1]);
    }
    const int nb = std::max(1, (int)std::sqrt((double)m.E / 4.0));
    g.nx = g.ny = nb;
    g.x0 = xmin;
    g.y0 = ymin;
    g.hx = std::max(xmax - xmin, 1e-300) / nb;
    g.hy = std::max(ymax - ymin, 1e-300) / nb;
    auto cell = [&](double v, double o, double h, int n) {
        return std::min(n - 1, std::max(0, (int)std::floor((v - o) / h)));
    };
    std::vector<int> cnt((size_t)nb * nb + 1, 0);
    std::vector<int> lo(4 * (size_t)m.E);
    for (int e = 0; e < m.E; ++e) {
        double ex0 = 1e300, ex1 = -1e300, ey0 = 1e300, ey1 = -1e300;
        for (int k = 0; k < m.nv; ++k) {
            const int v = m.conn[m.nv * e + k];
            ex0 = std::min(ex0, m.xy[2 * v]);
            ex1 = std::max(ex1, m.xy[2 * v]);
            ey0 = std::min(ey0, m.xy[2 * v + 1]);
            ey1 = std::max(ey1, m.xy[2 * v + 1]);
        }
        int* L = &lo[4 * (size_t)e];
        L[0] = cell(ex0, g.x0, g.hx, nb);
        L[1] = cell(ex1, g.x0, g.hx, nb);
        L[2] = cell(ey0, g.y0, g.hy, nb);
        L[3] = cell(ey1, g.y0, g.hy, nb);
        for (int j = L[2]; j <= L[3]; ++j)
            for (int i = L[0]; i <= L[1]; ++i) cnt[(size_t)j * nb + i + 1]++;
    }
    for (size_t k = 1; k < cnt.size(); ++k) cnt[k] += cnt[k - 1];
    g.ptr = cnt;
    g.elems.resize(cnt.back());
    std::vector<int> fill(cnt.begin(), cnt.end() - 1);
    for (int e = 0; e < m.E; ++e) {
        const int* L = &lo[4 * (size_t)e];
        for (int j = L[2]; j <= L[3]; ++j)
            for (int i = L[0]; i <= L[1]; ++i) g.elems[fill[(size_t)j * nb + i]++] = e;
    }
    return g;
}

// Reference coordinates of (px, py) in quadrilateral e: Newton's method on
// the bilinear element map x(xi, eta) = p from the centre (corners counter-
// clockwise at (0,0), (1,0), (1,1), (0,1)); the bilinear weights of the
// corners into w, and min(xi, 1 - xi, eta, 1 - eta) returned.
double q1_weights(const HostMesh& m, int e, double px, double py, double w[4]) {
    double X[4], Y[4];
    for (int k = 0; k < 4; ++k) {
        X[k] = m.xy[2 * m.conn[4 * e + k]];
        Y[k] = m.xy[2 * m.conn[4 * e + k] + 1];
    }
    double xi = 0.5, eta = 0.5;
    for (int it = 0; it < 30; ++it) {
        const double N[4] = {(1 - xi) * (1 - eta), xi * (1 - eta), xi * eta, (1 - xi) * eta};
        const double dxi[4] = {-(1 - eta), 1 - eta, eta, -eta};
        const double deta[4] = {-(1 - xi), -xi, xi, 1 - xi};
        double rx = -px, ry = -py, a = 0, b = 0, c = 0, d = 0;
        for (int k = 0; k < 4; ++k) {
            rx += N[k] * X[k];
            ry += N[k] * Y[k];
            a += dxi[k] * X[k];
            b += deta[k] * X[k];
            c += dxi[k] * Y[k];
            d += deta[k] * Y[k];
        }
        const double det = a * d - b * c;
        const double sx = (d * rx - b * ry) / det, sy = (-c * rx + a * ry) / det;
        xi -= sx;
        eta -= sy;
        if (std::max(std::abs(sx), std::abs(sy)) < 1e-15) break;
    }
    w[0] = (1 - xi) * (1 - eta);
    w[1] = xi * (1 - eta);
    w[2] = xi * eta;
    w[3] = (1 - xi) * eta;
    return std::min(std::min(xi, 1 - xi), std::min(eta, 1 - eta));
}

// Element containing (px, py) and its interpolation weights: barycentric
// (P1, w[3] = 0) or bilinear (Q1); the element whose weights are largest at
// their smallest wins, ties to the lower element id.
int locate(const HostMesh& m, const BucketGrid& g, double px, double py, double w[4]) {
    const int ci = std::min(g.nx - 1, std::max(0, (int)std::floor((px - g.x0) / g.hx)));
    const int cj = std::min(g.ny - 1, std::max(0, (int)std::floor((py - g.y0) / g.hy)));
    int best = -1;
    double bmin = -1e300;
    const int rmax = std::max(g.nx, g.ny);
    for (int r = 0; r <= rmax; ++r) {
        for (int j = cj - r; j <= cj + r; ++j) {
            if (j < 0 || j >= g.ny) continue;
            for (int i = ci - r; i <= ci + r; ++i) {
                if (i < 0 || i >= g.nx) continue;
                if (std::max(std::abs(i - ci), std::abs(j - cj)) != r) continue;
                const size_t b = (size_t)j * g.nx + i;
                for (int k = g.ptr[b]; k < g.ptr[b + 1]; ++k) {
                    const int e = g.elems[k];
                    double lam[4] = {0.0, 0.0, 0.0, 0.0};
                    double mn;
                    if (m.nv == 4) {
                        mn = q1_weights(m, e, px, py, lam);
                    } else {
                        barycentric(m, e, px, py, lam);
                        mn = std::min(lam[0], std::min(lam[1], lam[2]));
                    }
                    if (mn > bmin || (mn == bmin && e < best)) {
                        bmin = mn;
                        best = e;
                        for (int v = 0; v < 4; ++v) w[v] = lam[v];
                    }
                }
            }
        }
        if (best >= 0 && bmin >= -1e-12) break;
    }
    return best;
}
}  // namespace

// Elasticity (Q1, two dofs per node): 32 perimeter points (8 per side), 128
// points on the right side of the box, the 16 x 8 reference nodes; four
// nodes and bilinear weights per sample; for the reference nodes the packed
// V row of each element node's x dof in the subdomain, or -1.
static int build_guess_tables_q1(const HostMesh& m, const HostMaps& M, const BucketGrid& grid,
                                 HostGuess& out, std::string& err) {
    constexpr int NS = 8, NT = 32, NL = 128, GX = 16, GY = 8, NSAMP = 288;
    const int nsub = M.nsub;
    out.nper = 4;
    out.nsamp = NSAMP;
    out.ngrid = GX * GY;
    out.box.assign(4 * (size_t)nsub, 0.0);
    out.snode.assign((size_t)nsub * NSAMP * 4, 0);
    out.sw.assign((size_t)nsub * NSAMP * 4, 0.0);
    out.sloc.assign((size_t)nsub * GX * GY * 4, -1);
    std::vector<int> rowof(m.N, -1);
    for (int i = 0; i < nsub; ++i) {
        double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
        auto take = [&](int dof) {
            const int g = dof / 2;
            x0 = std::min(x0, m.xy[2 * g]);
            x1 = std::max(x1, m.xy[2 * g]);
            y0 = std::min(y0, m.xy[2 * g + 1]);
            y1 = std::max(y1, m.xy[2 * g + 1]);
        };
        for (int r = M.off_n[i]; r < M.off_n[i + 1]; ++r) take(M.l2g[r]);
        for (int r = M.off_g[i]; r < M.off_g[i + 1]; ++r) take(M.g2g[r]);
        const double W = x1 - x0, H = y1 - y0;
        if (!(W > 0.0) || !(H > 0.0)) {
            err = "subdomain " + std::to_string(i) + " has a degenerate patch box";
            return NLS_EPARTITION;
        }
        double* bx = &out.box[4 * (size_t)i];
        bx[0] = x0;
        bx[1] = y0;
        bx[2] = x1;
        bx[3] = y1;
        for (int r = M.off_n[i]; r < M.off_n[i + 1]; ++r)
            if (M.l2g[r] % 2 == 0) rowof[M.l2g[r] / 2] = r;
        for (int k = 0; k < NSAMP; ++k) {
            double px, py;
            if (k < NT) {
                const int sd = k / NS;
                const double t = (double)(k % NS) / NS;
                if (sd == 0) { px = x0 + t * W; py = y0; }
                else if (sd == 1) { px = x1; py = y0 + t * H; }
                else if (sd == 2) { px = x1 - t * W; py = y1; }
                else { px = x0; py = y1 - t * H; }
            } else if (k < NT + NL) {
                px = x1;
                py = y0 + ((double)(k - NT) / (NL - 1)) * H;
            } else {
                const int q = (k - NT - NL) / GX, p = (k - NT - NL) % GX;
                px = x0 + ((double)p / (GX - 1)) * W;
                py = y0 + ((double)q / (GY - 1)) * H;
            }
            double w[4];
            const int e = locate(m, grid, px, py, w);
            const size_t o = ((size_t)i * NSAMP + k) * 4;
            for (int v = 0; v < 4; ++v) {
                const int g = m.conn[4 * e + v];
                out.snode[o + v] = g;
                out.sw[o + v] = w[v];
                if (k >= NT + NL)
                    out.sloc[((size_t)i * GX * GY + (k - NT - NL)) * 4 + v] = rowof[g];
            }
        }
        for (int r = M.off_n[i]; r < M.off_n[i + 1]; ++r)
            if (M.l2g[r] % 2 == 0) rowof[M.l2g[r] / 2] = -1;
    }
    return NLS_OK;
}

int nls_build_guess_tables(const HostMesh& m, const HostMaps& M, HostGuess& out,
                           std::string& err) {
    constexpr int NS = 16, NT = 64, NG = 16, NIN = 320;
    const int nsub = M.nsub;
    if (m.E == 0) {
        err = "empty mesh";
        return NLS_EINVAL;
    }
    const BucketGrid grid = build_buckets(m);
    if (m.nv == 4) return build_guess_tables_q1(m, M, grid, out, err);
    out.nper = 3;
    out.nsamp = NIN;
    out.ngrid = NG * NG;
    out.box.assign(4 * (size_t)nsub, 0.0);
    out.snode.assign((size_t)nsub * NIN * 3, 0);
    out.sw.assign((size_t)nsub * NIN * 3, 0.0);
    out.sloc.assign((size_t)nsub * (NIN - NT) * 3, -1);
    for (int i = 0; i < nsub; ++i) {
        double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
        auto take = [&](int g) {
            x0 = std::min(x0, m.xy[2 * g]);
            x1 = std::max(x1, m.xy[2 * g]);
            y0 = std::min(y0, m.xy[2 * g + 1]);
            y1 = std::max(y1, m.xy[2 * g + 1]);
        };
        for (int r = M.off_n[i]; r < M.off_n[i + 1]; ++r) take(M.l2g[r]);
        for (int r = M.off_g[i]; r < M.off_g[i + 1]; ++r) take(M.g2g[r]);
        const double W = x1 - x0, H = y1 - y0;
        if (!(W > 0.0) || !(H > 0.0)) {
            err = "subdomain " + std::to_string(i) + " has a degenerate patch box";
            return NLS_EPARTITION;
        }
        double* bx = &out.box[4 * (size_t)i];
        bx[0] = x0;
        bx[1] = y0;
        bx[2] = x1;
        bx[3] = y1;
        for (int k = 0; k < NIN; ++k) {
            double px, py;
            if (k < NT) {
                const int sd = k / NS;
                const double t = (double)(k % NS) / NS;
                if (sd == 0) { px = x0 + t * W; py = y0; }
                else if (sd == 1) { px = x1; py = y0 + t * H; }
                else if (sd == 2) { px = x1 - t * W; py = y1; }
                else { px = x0; py = y1 - t * H; }
            } else {
                const int q = (k - NT) / NG, p = (k - NT) % NG;
                px = x0 + ((double)p / (NG - 1)) * W;
                py = y0 + ((double)q / (NG - 1)) * H;
            }
            double w[4];
            const int e = locate(m, grid, px, py, w);
            const size_t o = ((size_t)i * NIN + k) * 3;
            for (int v = 0; v < 3; ++v) {
                const int g = m.conn[3 * e + v];
                out.snode[o + v] = g;
                out.sw[o + v] = w[v];
                if (k >= NT) {
                    // packed V row of g in subdomain i (l2g ascending per subdomain)
                    const int* b = M.l2g.data() + M.off_n[i];
                    const int* en = M.l2g.data() + M.off_n[i + 1];
                    const int* it = std::lower_bound(b, en, g);
                    out.sloc[((size_t)i * (NIN - NT) + (k - NT)) * 3 + v] =
                        (it != en && *it == g) ? M.off_n[i] + (int)(it - b) : -1;
                }
            }
        }
    }
    return NLS_OK;
}

static int inspect_mesh(int64_t n_nodes, int64_t n_elems, const int32_t* conn, HostMesh& m,
                        std::string& err) {
    if (n_nodes <= 0 || n_elems <= 0 || !conn) return NLS_EINVAL;
    m.N = (int)n_nodes;
    m.E = (int)n_elems;
    m.conn.assign(conn, conn + 3 * n_elems);
    m.dflag.assign(m.N, 0);
    m.dval.assign(m.N, 0.0);
    return nls_build_node_incidence(m, err);
}

extern "C" int nls_inspect_partition(int64_t n_nodes, int64_t n_elems, const int32_t* conn,
                                     int32_t n_sub, const int32_t* elem_part, int32_t overlap,
                                     int64_t* counts, int32_t* off_v, int32_t* v_nodes,
                                     int32_t* off_g, int32_t* g_nodes, int32_t* own_pos,
                                     int32_t* kl, int32_t* ku) {
    HostMesh m;
    std::string err;
    if (!elem_part) return NLS_EINVAL;
    int rc = inspect_mesh(n_nodes, n_elems, conn, m, err);
    if (rc) return rc;
    HostMaps M;
    rc = nls_build_maps(m, elem_part, n_sub, overlap, M, err);
    if (rc) return rc;
    if (counts) {
        counts[0] = (int64_t)M.l2g.size();
        counts[1] = (int64_t)M.g2g.size();
    }
    if (off_v) std::copy(M.off_n.begin(), M.off_n.end(), off_v);
    if (off_g) std::copy(M.off_g.begin(), M.off_g.end(), off_g);
    if (v_nodes) std::copy(M.l2g.begin(), M.l2g.end(), v_nodes);
    if (g_nodes) std::copy(M.g2g.begin(), M.g2g.end(), g_nodes);
    if (own_pos) std::copy(M.own_pidx.begin(), M.own_pidx.end(), own_pos);
    if (kl) std::copy(M.kl.begin(), M.kl.end(), kl);
    if (ku) std::copy(M.ku.begin(), M.ku.end(), ku);
    return NLS_OK;
}

extern "C" int nls_inspect_coarse(int64_t n_nodes, int64_t n_elems, const int32_t* conn,
                                  int32_t n_sub, const int32_t* elem_part, int64_t n_dir,
                                  const int64_t* dirichlet, int64_t* counts, int32_t* comp_off,
                                  int32_t* comp_nodes) {
    HostMesh m;
    std::string err;
    if (!elem_part || n_sub <= 0 || n_dir < 0 || (n_dir > 0 && !dirichlet)) return NLS_EINVAL;
    int rc = inspect_mesh(n_nodes, n_elems, conn, m, err);
    if (rc) return rc;
    for (int64_t k = 0; k < n_dir; ++k) {
        if (dirichlet[k] < 0 || dirichlet[k] >= n_nodes) return NLS_EINVAL;
        m.dflag[dirichlet[k]] = 1;
    }
    for (int64_t e = 0; e < n_elems; ++e)
        if (elem_part[e] < 0 || elem_part[e] >= n_sub) return NLS_EINVAL;
    HostCoarse C;
    rc = nls_build_coarse_symbolic(m, elem_part, n_sub, NLS_COARSE_GDSW, C, err);
    if (rc) return rc;
    int64_t tot = 0;
    for (auto& c : C.comps) tot += (int64_t)c.size();
    if (counts) {
        counts[0] = C.n0;
        counts[1] = tot;
    }
    if (comp_off && comp_nodes) {
        int64_t p = 0;
        comp_off[0] = 0;
        for (int k = 0; k < C.n0; ++k) {
            for (int g : C.comps[k]) comp_nodes[p++] = g;
            comp_off[k + 1] = (int32_t)p;
        }
    }
    return NLS_OK;
}
