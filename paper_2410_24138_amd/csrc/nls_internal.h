// Internal data structures of libnls shared by the host setup, the solver
// driver and the HIP kernels.  Not part of the public ABI.
#pragma once

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

// Band-window size of the LU kernels (ring buffers): blocked panels of NB
// columns need (NB+kl) x (NB+kl+ku); the unblocked form (kl+1) x (kl+ku+1).
// Blocked variants: (NB + kl) x (NB + kl + ku) window, NB x NB L11, 64 ints
// (32 doubles) for the panel's moved-row list and NB x (64 + NB) staged
// multipliers.
inline int band_window_doubles(int kl, int ku) {
    if (kl + 16 <= 64) return (16 + kl) * (16 + kl + ku) + 16 * 16 + 32 + 16 * 80;
    if (kl + 8 <= 64) return (8 + kl) * (8 + kl + ku) + 8 * 8 + 32 + 8 * 72;
    return (kl + 1) * (kl + ku + 1);
}
// Window of a forced LU variant: 1 blocked NB=16, 2 blocked NB=8,
// 3 unblocked, 0 the automatic choice above; -1 if the variant cannot hold kl.
inline int band_window_doubles_v(int kl, int ku, int v) {
    if (v == 0) return band_window_doubles(kl, ku);
    if (v == 1) return kl + 16 <= 64 ? (16 + kl) * (16 + kl + ku) + 16 * 16 + 32 + 16 * 80 : -1;
    if (v == 2) return kl + 8 <= 64 ? (8 + kl) * (8 + kl + ku) + 8 * 8 + 32 + 8 * 72 : -1;
    return (kl + 1) * (kl + ku + 1);
}
// LDS of the fused local Newton kernel, in doubles:
//   patch values (n + ng) | residual / step (n) | LU window | multipliers | scratch
inline int local_lds_doubles(int n, int ng, int kl, int ku) {
    return 2 * n + ng + band_window_doubles(kl, ku) + std::max(kl, 1) + 72;
}
// LDS of the interior (harmonic extension) kernel, in doubles.
inline int interior_lds_doubles(int ni, int kl, int ku, int nk) {
    (void)nk;
    return ni + band_window_doubles(kl, ku) + std::max(kl, 1) + 72;
}

// ---------------------------------------------------------------- host side

struct HostMesh {
    int N = 0;                     // nodes
    int E = 0;                     // elements
    int nv = 3;                    // nodes per element: 3 (P1 triangle), 4 (Q1 quad)
    int d = 1;                     // dofs per node (node-major, interleaved)
    std::vector<double> xy;        // 2N
    std::vector<int> conn;         // nv * E
    std::vector<int> nptr, nel;    // node -> incident elements (CSR, ascending)
    std::vector<unsigned char> dflag;  // N*d, 1 on Dirichlet dofs
    std::vector<double> dval;      // N*d
    int ndof() const { return N * d; }
};

// Overlapping subdomains and the tables the local kernels read.
// "Packed" arrays concatenate the per-subdomain arrays in subdomain order.
// Rows are dofs: row d*a + c is component c of the a-th node of V_i; the
// patch-local id of a node is its position in V_i, or n_V + its position
// in Gamma_i, and its dof c has local index d*id + c.
struct HostMaps {
    int nsub = 0;
    std::vector<int> off_n;        // nsub+1, offsets into packed V rows
    std::vector<int> off_g;        // nsub+1, offsets into packed Gamma nodes
    std::vector<int> off_e;        // nsub+1, offsets into packed patch elements
    std::vector<int> l2g;          // packed V_i global dof ids (node order of V_i:
                                   //   ascending, or along the shorter side of the
                                   //   patch box for vector problems)
    std::vector<int> g2g;          // packed Gamma_i global dof ids (nodes ascending)
    std::vector<int> pe_conn;      // nv per packed patch element, patch-local node ids
    std::vector<int> pe_gid;       // global element id of each packed patch element
    std::vector<int> rinc_ptr;     // packed V row -> [rinc_ptr, rinc_ptr+1) in rinc
    std::vector<int> rinc;         // (patch element local index << 2) | vertex position
    std::vector<int> jptr;         // packed V row -> CSR slots (global over all rows)
    std::vector<int> jcol;         // patch-local column of each slot (sorted per row)
    std::vector<int> kl, ku;       // band widths of J_ii per subdomain
    std::vector<int64_t> off_u;    // offset (doubles) of the U factor, n_i*(kl+ku+1)
    std::vector<int64_t> off_l;    // offset (doubles) of the L factor, n_i*max(kl,1)
    int64_t factor_u_total = 0, factor_l_total = 0;
    std::vector<int> own_pidx;     // N*d: packed V row of the owner's copy of dof g
    // exact-tangent tables: B_i by columns, owned rows of each subdomain
    std::vector<int> bptr;         // packed Gamma column -> [bptr, bptr+1) entries
    std::vector<int> brow;         // local row of each B entry (ascending per column)
    std::vector<int> bslot;        // CSR slot of the entry in jptr/jcol/jval
    int max_bcol = 0;              // longest B column
    std::vector<int> off_own;      // nsub+1: owned rows, packed
    std::vector<int> ownrow;       // packed owned index -> local V row
    std::vector<int> rowown;       // packed V row -> owned index in its subdomain, or -1
    std::vector<int64_t> off_W;    // nsub+1: |owned_i| x |Gamma_i| tangent blocks
    std::vector<int64_t> off_F;    // nsub+1: n_i x |Gamma_i| forward-sweep scratch
    std::vector<int> order;        // launch order of subdomains (largest first)
    std::vector<int> lds_doubles;  // per subdomain LDS need of the local Newton kernel
    int max_lds_doubles = 0;
};

// GDSW coarse space: symbolic part (host) plus the tables its kernels read.
// Closure arrays are per dof (d per closure node, node-major): closure dof
// d*a + c is component c of the a-th closure node.
struct HostCoarse {
    int n0 = 0;                            // coarse functions
    std::vector<std::vector<int>> comps;   // interface components, by smallest node
    std::vector<int> comp_of;              // N: component id or -1
    std::vector<int> fun_base, nfun;       // per component: its first function, count
                                           //   (1 scalar; 2 translations + rotation if
                                           //   the component has >= 2 nodes, elasticity)
    // per non-overlapping subdomain i
    std::vector<int> off_c;        // nsub+1: closure dofs (dofs of nodes of part-i elements)
    std::vector<int> cnode;        // packed closure dof global ids (ascending)
    std::vector<int> ctype;        // 0 interior, 1 interface, 2 Dirichlet/other
    std::vector<int> off_k;        // nsub+1: coarse functions touching subdomain i
    std::vector<int> klist;        // packed coarse ids (ascending per subdomain)
    std::vector<int> cfun;         // NLS_CFUN per packed closure dof: local positions in
    std::vector<double> cval;      //   K_i of the functions nonzero there (or -1), values
    std::vector<int64_t> off_phi;  // nsub+1: dense |C_i| x |K_i| blocks (row-major)
    std::vector<int> off_ne;       // nsub+1: elements of part i
    std::vector<int> ne_conn;      // nv per element, closure-local node positions
    std::vector<int> ne_gid;       // global element ids
    std::vector<int> cinc_ptr;     // packed closure node -> incident part-i elements
    std::vector<int> cinc;         // (element local index << 2) | vertex position
    std::vector<int> iidx;         // packed closure: interior-local index or -1
    std::vector<int> off_ni;       // nsub+1: interior rows
    std::vector<int> inode;        // packed interior row -> closure-local index
    std::vector<int> iptr, icol;   // interior CSR (interior-local columns)
    std::vector<int> ikl, iku;     // band widths of A_II
    std::vector<int64_t> off_iu, off_il;
    int64_t iu_total = 0, il_total = 0;
    std::vector<int> ilds_doubles; // LDS need of the extension kernel
    int max_ilds_doubles = 0;
    // Galerkin matrix A0 = Phi^T DF Phi in CSR over the banded ordering
    std::vector<int> perm;         // coarse id -> band position
    std::vector<int> a0ptr, a0col; // CSR in band positions
    std::vector<int> a0src_ptr;    // slot -> [ptr, ptr+1) of a0src
    std::vector<int> a0src;        // packed position in the per-subdomain blocks
    std::vector<int64_t> off_kk;   // nsub+1: offsets of the |K_i|^2 blocks
    std::vector<int> gsrc_ptr;     // coarse id -> contributions to Phi^T q
    std::vector<int> gsrc;         // packed position in the per-subdomain vectors
    int a0kl = 0, a0ku = 0;           // largest block band widths
    // diagonal blocks of A0 in band order (one per connected component)
    std::vector<int> boff, bkl, bku, rblk;
    std::vector<int64_t> offU, offL, offI;
    std::vector<int> cpos;         // N*d: packed closure index in the owner's block
    std::vector<int> cown;         // N*d: owner subdomain
    int max_k = 0;
};

// Sampling tables of the learned initial guess, per subdomain: the patch box
// and, for 64 perimeter points followed by the 256 reference-grid nodes, the
// mesh element containing the point (its three nodes and barycentric
// weights); for the grid nodes also the packed V row of each node in the
// subdomain, or -1.
// Elasticity (Q1): 288 samples (32 perimeter, 128 on the right side of the
// box, 16 x 8 reference nodes) of four nodes each; sloc holds the packed V
// row of the node's x dof.
struct HostGuess {
    int nper = 3, nsamp = 320, ngrid = 256;  // nodes per sample, samples, grid nodes
    std::vector<double> box;       // 4 per subdomain: x0, y0, x1, y1
    std::vector<int> snode;        // nsub x nsamp x nper
    std::vector<double> sw;        // nsub x nsamp x nper
    std::vector<int> sloc;         // nsub x ngrid x nper
};

// Most coarse functions nonzero at one interface dof: RGDSW elasticity on an
// edge between two crosspoints has a translation and a rotation of each.
#ifndef NLS_CFUN
#define NLS_CFUN 4
#endif

// Setup entry points (setup.cpp).  Return 0 or an NLS_* error with err set.
int nls_build_node_incidence(HostMesh& m, std::string& err);
int nls_build_maps(const HostMesh& m, const int* part, int nsub, int overlap,
                   HostMaps& out, std::string& err);
int nls_build_coarse_symbolic(const HostMesh& m, const int* part, int nsub, int kind,
                              HostCoarse& out, std::string& err);
int nls_build_guess_tables(const HostMesh& m, const HostMaps& maps, HostGuess& out,
                           std::string& err);
