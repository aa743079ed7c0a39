"""Two-level nonlinear restricted additive Schwarz (RASPEN), FP64 oracle.

Follows Section 2 of the paper:
  * local corrections T_i(u) solving R_i F(u - P_i T_i(u)) = 0 (eq. 4) by an
    inner Newton iteration on each overlapping subdomain;
  * one-level residual F_1(u) = sum_i P~_i T_i(u) (eq. 5) with restricted
    prolongations P~_i forming a partition of unity (eq. 8);
  * coarse correction T_0(u) solving R_0 F(u - P_0 T_0(u)) = 0 (eq. 9) with
    a GDSW coarse space (energy-minimising extension of interface indicator
    functions) and R_0 = P_0^T;
  * additive coupling F_a(u) = F_1(u) + P_0 T_0(u) (eq. 10);
  * hybrid coupling F_h(u) = F_1(u - P_0 T_0(u)) + P_0 T_0(u) (eq. 11): the
    coarse correction first, then the local corrections at the coarse-
    corrected point;
  * the exact tangents (eqs. 6, 7, 12) and the outer Newton iteration on the
    tangent system (eq. 13), solved by restarted GMRES.

Readings where the paper is silent (all are stated again where used):
  * overlap: delta layers of elements added by node adjacency;
  * V_i = nodes of the overlapping patch whose every element lies in the
    patch; the other patch nodes (Gamma_i) carry the current global values;
    Dirichlet nodes in V_i keep identity rows;
  * P~_i: node g is owned by the largest subdomain id among its elements and
    P~_i copies the owned entries only (a partition of unity, eq. 8);
  * the coarse basis is extended with DF at the linearisation point u = 0;
  * inner/coarse Newton start from T = 0 and stop when
    ||r||_2 <= max(rtol * rho_0, eta * ||b||_inf * sqrt(n)) or the last step
    was below 1e-14 of the iterate (rounding stagnation); at most 30 steps;
  * the exact tangent uses DF at the converged local states;
  * outer Newton: u <- u - du (eq. 13), full steps, stop when
    ||F_x(u_k)|| <= rtol ||F_x(u_0)||; GMRES restarted every 50 iterations,
    x_0 = 0, modified Gram-Schmidt, Givens rotations.

LU with partial pivoting is the linear solver of every step: in band form
(LAPACK gbtrf/gbtrs through SciPy) for the local Jacobians and the interior
blocks of the coarse basis, whose nonzeros lie in a band under the
ascending node order, dense (LAPACK getrf) for the coarse matrix.  GDSW components
are ordered by their smallest node index.  FP64 throughout.  Test
infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.linalg.lapack as lapack
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .p1 import P1Problem, p1_element


class LocalFailure(RuntimeError):
    """An inner (or coarse) Newton iteration did not meet its stopping rule."""


def _stop_tol(rho0, b_inf, n, rtol, eta):
    return max(rtol * rho0, eta * b_inf * np.sqrt(n))


def band_lu_factor(J):
    """LU with partial pivoting of a square matrix whose nonzeros lie within
    kl sub- and ku super-diagonals (LAPACK gbtrf; the row interchanges widen
    the upper band of U to kl + ku, which the storage leaves room for).
    Mathematically the same factorisation as dense getrf.  Returns the
    factors, pivots and band widths for band_lu_solve."""
    J = np.asarray(J, dtype=np.float64)
    n = J.shape[0]
    i, j = np.nonzero(J)
    kl = int(max(np.max(i - j), 0)) if len(i) else 0
    ku = int(max(np.max(j - i), 0)) if len(i) else 0
    ab = np.zeros((2 * kl + ku + 1, n))
    ab[kl + ku + i - j, j] = J[i, j]
    lub, piv, info = lapack.dgbtrf(ab, kl, ku)
    if info > 0:
        raise LocalFailure(f"zero pivot at column {info - 1}")
    return lub, piv, kl, ku


def band_lu_solve(fac, r):
    """Solve with the factors of band_lu_factor (LAPACK gbtrs); r is a
    vector or an n x k array of right-hand sides."""
    lub, piv, kl, ku = fac
    r = np.asarray(r, dtype=np.float64)
    x, info = lapack.dgbtrs(lub, kl, ku, r.reshape(len(r), -1), piv)
    if info != 0:
        raise ValueError(f"gbtrs: illegal argument {-info}")
    return x.reshape(r.shape)


class Schwarz:
    """RASPEN with optional GDSW coarse level for one problem (P1Problem or
    NHProblem: d dofs per node, element_local, residual, jacobian).

    coupling: "one_level" (F_1, eq. 5), "additive" (F_a, eq. 10) or
    "hybrid" (F_h, eq. 11).
    """

    def __init__(self, problem: P1Problem, coupling: str = "one_level",
                 inner_rtol=1e-12, inner_eta=1e-10, inner_maxit=30,
                 stagnation=1e-14, coarse="gdsw", coarse_lin=None):
        if coupling not in ("one_level", "additive", "hybrid"):
            raise ValueError(coupling)
        self.P = problem
        self.case = problem.case
        self.coupling = coupling
        self.inner_rtol = inner_rtol
        self.inner_eta = inner_eta
        self.inner_maxit = inner_maxit
        self.stagnation = stagnation
        self.b_inf = float(np.max(np.abs(problem.b))) if problem.ndof else 0.0
        self._build_maps()
        self.Phi = None
        if coarse not in ("gdsw", "rgdsw"):
            raise ValueError(coarse)
        self.coarse = coarse
        if coupling in ("additive", "hybrid"):
            self._build_gdsw(coarse_lin)
        self.state = None

    # ------------------------------------------------------------------ maps
    def _build_maps(self):
        """Overlapping subdomains and transfer operators (Section 2).

        The paper builds an element-based overlap from the dual graph; here
        the non-overlapping element set of each subdomain is grown by
        `overlap` layers of elements sharing a node with the current set.
        Maps are built on nodes and expanded to the problem's d dofs per
        node (node-major, interleaved); a node's dofs share its subdomains,
        its V/Gamma status and its owner.
        """
        P = self.P
        conn = P.conn
        nv = conn.shape[1]
        dd = P.d
        part = np.asarray(self.case["elem_part"], dtype=np.int64)
        n_sub = int(self.case["n_sub"])
        delta = int(self.case["overlap"])
        N, E = P.N, P.E
        self.part = part
        self.n_sub = n_sub
        self.d = dd
        inc = sp.csr_matrix((np.ones(nv * E), (conn.ravel(),
                             np.repeat(np.arange(E), nv))), shape=(N, E))
        self.inc = inc
        deg = np.asarray(inc.sum(axis=1)).ravel()
        owner = np.full(N, -1, dtype=np.int64)
        np.maximum.at(owner, conn.ravel(), np.repeat(part, nv))
        self.owner = owner
        # a node is a Dirichlet node when any of its dofs is
        self.node_dir = P.is_dir.reshape(N, dd).any(axis=1)

        def dofs(nodes):
            return (dd * np.asarray(nodes)[:, None] + np.arange(dd)).ravel()

        subs = []
        for i in range(n_sub):
            pe = (part == i).astype(np.float64)
            if not pe.any():
                raise ValueError(f"subdomain {i} is empty")
            for _ in range(delta):
                nodes = (inc @ pe) > 0
                pe = ((inc.T @ nodes.astype(np.float64)) > 0).astype(np.float64)
            cnt = inc @ pe
            in_patch = cnt > 0
            V = np.nonzero(in_patch & (cnt == deg))[0]
            Gam = np.nonzero(in_patch & (cnt != deg))[0]
            elems = np.nonzero(pe)[0]
            loc = np.full(N, -1, dtype=np.int64)
            loc[V] = np.arange(len(V))
            loc[Gam] = len(V) + np.arange(len(Gam))
            lconn = loc[conn[elems]]
            ldof = (dd * lconn[:, :, None] + np.arange(dd)).reshape(len(elems), nv * dd)
            Vd = dofs(V)
            subs.append({"V": V, "Gam": Gam, "elems": elems, "lconn": lconn,
                         "Vd": Vd, "Gd": dofs(Gam), "ldof": ldof,
                         "dirV": P.is_dir[Vd], "loc": loc})
        self.subs = subs
        # restricted prolongation P~_i: owned nodes and their positions in V_i
        own_loc = np.empty(N, dtype=np.int64)
        for i, s in enumerate(subs):
            owned = np.nonzero(owner == i)[0]
            li = s["loc"][owned]
            if np.any(li < 0) or np.any(li >= len(s["V"])):
                raise ValueError(f"subdomain {i}: owned nodes not in V_i "
                                 "(overlap must be >= 1)")
            own_loc[owned] = li
            s["owned"] = dofs(owned)
            s["owned_loc"] = dofs(li)
        self.own_loc = own_loc

    # ----------------------------------------------------------- local level
    def local_residual(self, i, x, trace):
        """r = R_i F(v) with v = u outside V_i and x on V_i (eq. 4).

        Assembled from the patch elements only; exact because every element
        touching a node of V_i lies in the patch.
        """
        s = self.subs[i]
        P = self.P
        v = np.concatenate([x, trace])
        r_e, _ = P.element_local(s["elems"], v[s["ldof"]])
        R = np.zeros(len(v))
        np.add.at(R, s["ldof"], r_e)
        r = R[:len(x)] - P.ext_load[s["Vd"]]
        d = s["dirV"]
        r[d] = x[d] - P.dir_value[s["Vd"][d]]
        return r

    def local_jacobian(self, i, x, trace):
        """J_ii = R_i DF(v) P_i and the coupling B_i = R_i DF(v) on Gamma_i."""
        s = self.subs[i]
        P = self.P
        nV = len(x)
        v = np.concatenate([x, trace])
        _, K = P.element_local(s["elems"], v[s["ldof"]])
        lc = s["ldof"]
        rows = np.broadcast_to(lc[:, :, None], K.shape).ravel()
        cols = np.broadcast_to(lc[:, None, :], K.shape).ravel()
        keep = rows < nV
        Jf = np.zeros((nV, len(v)))
        np.add.at(Jf, (rows[keep], cols[keep]), K.ravel()[keep])
        d = np.nonzero(s["dirV"])[0]
        Jf[d, :] = 0.0
        Jf[d, d] = 1.0
        return Jf[:, :nV].copy(), Jf[:, nV:].copy()

    def local_solve(self, i, u, x0=None, guess=None):
        """T_i(u) by Newton's method on R_i F(u - P_i T_i(u)) = 0 (eq. 4).

        Starts from x = R_i u (T_i = 0) unless x0 is given; the stopping rule
        is measured against rho_plain = ||R_i F(u)||.  Returns the converged
        local state, T_i(u) = R_i u - x*, and the LU of J_ii and B_i at x*
        (the exact tangent, eq. 6, needs DF at u_i = u - P_i T_i(u)).

        guess: a predicted start (learned initial guess).  It is taken only
        when its residual is finite and below rho_plain; if Newton from it
        fails, the solve restarts from R_i u.  "start" in the result is
        "plain", "guess" or "fallback".
        """
        s = self.subs[i]
        xu = u[s["Vd"]].copy()
        tr = u[s["Gd"]].copy()
        r = self.local_residual(i, xu, tr)
        rho_plain = float(np.linalg.norm(r))
        tol = _stop_tol(rho_plain, self.b_inf, len(xu), self.inner_rtol,
                        self.inner_eta)
        start = "plain"
        if guess is not None:
            xg = np.array(guess, dtype=np.float64)
            rg = self.local_residual(i, xg, tr)
            rho_g = float(np.linalg.norm(rg))
            if np.isfinite(rho_g) and rho_g < rho_plain:
                try:
                    out = self._newton(i, xg, rg, tr, tol)
                    return self._finish(i, xu, tr, out, rho_plain, "guess")
                except LocalFailure:
                    start = "fallback"
            else:
                start = "fallback"
        x = xu if x0 is None else np.array(x0, dtype=np.float64)
        if x0 is not None:
            r = self.local_residual(i, x, tr)
        out = self._newton(i, x, r, tr, tol)
        return self._finish(i, xu, tr, out, rho_plain, start)

    def _newton(self, i, x, r, tr, tol):
        """Inner Newton steps x <- x - J(x)^{-1} r(x) until the stopping rule."""
        its = 0
        dprev = None
        hist = [float(np.linalg.norm(r))]
        while True:
            rn = float(np.linalg.norm(r))
            if not np.isfinite(rn):
                raise LocalFailure(f"subdomain {i}: non-finite residual")
            if rn <= tol:
                break
            if dprev is not None and dprev <= self.stagnation * np.max(np.abs(x)):
                break
            if its == self.inner_maxit:
                raise LocalFailure(f"subdomain {i}: no convergence in "
                                   f"{its} Newton steps")
            J, _ = self.local_jacobian(i, x, tr)
            d = band_lu_solve(band_lu_factor(J), r)
            x = x - d
            its += 1
            dprev = float(np.max(np.abs(d)))
            r = self.local_residual(i, x, tr)
            hist.append(float(np.linalg.norm(r)))
        return x, its, hist

    def _finish(self, i, xu, tr, out, rho_plain, start):
        x, its, hist = out
        J, B = self.local_jacobian(i, x, tr)
        return {"x": x, "T": xu - x, "lu": band_lu_factor(J),
                "B": B, "its": its, "rho_plain": rho_plain, "hist": hist,
                "start": start}

    def F1(self, u, sols=None, guesses=None):
        """One-level RASPEN residual F_1(u)[g] = T_{o(g)}(u)[l(g)] (eqs. 5, 8)."""
        if sols is None:
            if guesses is None:
                guesses = [None] * self.n_sub
            sols = [self.local_solve(i, u, guess=guesses[i])
                    for i in range(self.n_sub)]
        Fx = np.empty(self.P.ndof)
        for s, sol in zip(self.subs, sols):
            Fx[s["owned"]] = sol["T"][s["owned_loc"]]
        return Fx, sols

    # ---------------------------------------------------------- coarse level
    def _build_gdsw(self, u_lin=None):
        """GDSW coarse basis Phi (ndof x n0) (Section 1 and 2).

        Interface nodes (not Dirichlet, adjacent to elements of >= 2
        subdomains) are grouped by the set of subdomains they touch and each
        group is split into connected components (vertices: >= 3 subdomains,
        edges: 2).  Each component contributes the problem's null-space
        vectors restricted to it (scalar problem: 1; elasticity: the two
        translations, plus the rotation about the component's centroid when
        it has two or more nodes), zero on the rest of the interface, and
        every function is extended into each subdomain interior by the
        discrete harmonic extension Phi_I = -A_II^{-1} A_IG Phi_G with
        A = DF(u_lin), u_lin = 0 unless the constructor's coarse_lin is
        given.
        """
        P = self.P
        N = P.N
        dd = P.d
        nd = P.ndof
        conn = P.conn
        nv = conn.shape[1]
        part = self.part
        NS = sp.csr_matrix((np.ones(nv * P.E), (conn.ravel(), np.repeat(part, nv))),
                           shape=(N, self.n_sub))
        NS.sort_indices()
        nsub = np.diff(NS.indptr)
        iface = (nsub >= 2) & ~self.node_dir
        keys = {}
        for g in np.nonzero(iface)[0]:
            k = tuple(NS.indices[NS.indptr[g]:NS.indptr[g + 1]].tolist())
            keys.setdefault(k, []).append(g)
        # mesh edges (consecutive element nodes) for connectivity of a class
        e = np.concatenate([conn[:, [a, (a + 1) % nv]] for a in range(nv)])
        adj = sp.csr_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(N, N))
        adj = ((adj + adj.T) > 0).tocsr()
        comps = []
        for k, nodes in keys.items():
            nodes = np.array(sorted(nodes))
            sub = adj[nodes][:, nodes]
            nc, lab = sp.csgraph.connected_components(sub, directed=False)
            for c in range(nc):
                comps.append((nodes[lab == c], len(k)))
        comps.sort(key=lambda t: int(t[0].min()))
        rows, cols, vals = [], [], []
        n0 = 0
        if self.coarse == "gdsw":
            for nodes, _ in comps:
                cd = (dd * nodes[:, None] + np.arange(dd)).ravel()
                for vec in P.nullspace(nodes):
                    nz = vec != 0.0
                    rows.append(cd[nz])
                    cols.append(np.full(int(nz.sum()), n0))
                    vals.append(vec[nz])
                    n0 += 1
        else:
            n0 = self._rgdsw_values(comps, NS, adj, rows, cols, vals)
        rows = np.concatenate(rows) if rows else np.zeros(0, int)
        cols = np.concatenate(cols) if cols else np.zeros(0, int)
        vals = np.concatenate(vals) if vals else np.zeros(0)
        PhiG = sp.csr_matrix((vals, (rows, cols)), shape=(nd, n0))
        self.components = comps
        u0 = np.zeros(nd) if u_lin is None else u_lin
        A = P.jacobian(u0)
        prow, pcol, pval = [rows], [cols], [vals]
        interior_node = (nsub == 1) & ~self.node_dir
        interior = np.repeat(interior_node, dd)
        self.interior_blocks = []
        for i in range(self.n_sub):
            el = np.nonzero(part == i)[0]
            clos = np.zeros(N, dtype=bool)
            clos[conn[el].ravel()] = True
            closd = np.repeat(clos, dd)
            I = np.nonzero(closd & interior)[0]
            bnd = np.nonzero(closd & ~interior)[0]
            if len(I) == 0:
                continue
            AII = A[I][:, I].toarray()
            rhs = -(A[I][:, bnd] @ PhiG[bnd]).toarray()
            # only the functions with interface values next to the interior
            # have nonzero right-hand sides (the others extend by zero)
            nzc = np.nonzero(np.any(rhs != 0.0, axis=0))[0]
            PhiI = band_lu_solve(band_lu_factor(AII), rhs[:, nzc])
            prow.append(np.repeat(I, len(nzc)))
            pcol.append(np.tile(nzc, len(I)))
            pval.append(PhiI.ravel())
            self.interior_blocks.append((i, I, bnd))
        self.Phi = sp.csr_matrix((np.concatenate(pval), (np.concatenate(prow),
                                  np.concatenate(pcol))), shape=(nd, n0))
        self.Phi.eliminate_zeros()
        self.PhiT = self.Phi.T.tocsr()
        self.n0 = n0
        self.phib_inf = float(np.max(np.abs(self.PhiT @ P.b))) if n0 else 0.0

    def _rgdsw_values(self, comps, NS, adj, rows, cols, vals):
        """Interface values of the RGDSW coarse space, option 2.2 with the
        paper's modification (Section 2).  Reading: the coarse nodes are the
        vertices (components shared by >= 3 subdomains); an edge component
        (2 subdomains) takes its values from its ancestor vertices (those
        whose subdomain set contains the edge's) with inverse Euclidean
        distance weights w_c(x) = d_c(x)^-1 / sum d(x)^-1, where a Dirichlet
        node ending the edge (adjacent to it, in both subdomains) enters the
        sum as an ancestor with value 0; an edge without ancestor vertices is
        a coarse node of its own (value 1).  Scalar problems: one function
        per coarse node; elasticity: translations and the rotation about the
        coarse node's position (w_c times the rigid mode)."""
        P = self.P
        dd = P.d
        xy = P.xy
        sets = [frozenset(NS.indices[NS.indptr[c[0][0]]:NS.indptr[c[0][0] + 1]].tolist())
                for c in comps]
        vert = [k for k, (nodes, ns) in enumerate(comps) if ns >= 3]
        anc = {}
        for k, (nodes, ns) in enumerate(comps):
            if ns >= 3:
                continue
            anc[k] = [v for v in vert if sets[v] >= sets[k]]
        # coarse nodes in canonical order (smallest node), with positions
        cnodes = [k for k in range(len(comps)) if comps[k][1] >= 3 or not anc[k]]
        cnodes.sort(key=lambda k: int(comps[k][0].min()))
        pos = {k: xy[comps[k][0]].mean(axis=0) for k in cnodes}
        nfun = 1 if dd == 1 else 3
        base = {k: nfun * r for r, k in enumerate(cnodes)}

        def put(node, fb, w, center):
            x, y = xy[node]
            if dd == 1:
                rows.append(np.array([node]))
                cols.append(np.array([fb]))
                vals.append(np.array([w]))
                return
            r = [-(y - center[1]), x - center[0]]
            for c in range(2):
                rows.append(np.array([2 * node + c, 2 * node + c]))
                cols.append(np.array([fb + c, fb + 2]))
                vals.append(np.array([w, w * r[c]]))

        for k in cnodes:
            for g in comps[k][0]:
                put(g, base[k], 1.0, pos[k])
        node_dir = self.node_dir
        for k, (nodes, ns) in enumerate(comps):
            if ns >= 3 or not anc[k]:
                continue
            # Dirichlet nodes ending this edge
            dends = set()
            for g in nodes:
                for w_ in adj.indices[adj.indptr[g]:adj.indptr[g + 1]]:
                    if node_dir[w_]:
                        sw = frozenset(NS.indices[NS.indptr[w_]:NS.indptr[w_ + 1]].tolist())
                        if sw >= sets[k]:
                            dends.add(int(w_))
            for g in nodes:
                inv = {v: 1.0 / np.linalg.norm(xy[g] - pos[v]) for v in anc[k]}
                den = sum(inv.values()) + sum(1.0 / np.linalg.norm(xy[g] - xy[dn]) for dn in dends)
                for v in anc[k]:
                    put(g, base[v], inv[v] / den, pos[v])
        self.coarse_nodes = cnodes
        return nfun * len(cnodes)

    def refresh_load(self):
        """Recompute the load scales of the stopping rules after the
        problem's load changed (load stepping)."""
        P = self.P
        self.b_inf = float(np.max(np.abs(P.b))) if P.ndof else 0.0
        if self.Phi is not None:
            self.phib_inf = float(np.max(np.abs(self.PhiT @ P.b))) if self.n0 else 0.0

    def coarse_solve(self, u):
        """T_0(u) by Newton on G(c) = Phi^T F(u - Phi c) = 0 (eq. 9, R_0 =
        P_0^T = Phi^T), from c = 0:  c <- c + A0^{-1} G(c) with the Galerkin
        matrix A0 = Phi^T DF(u - Phi c) Phi.  Keeps LU(A0) and DF at the
        converged point u_0 = u - Phi c* for the tangent (eq. 12)."""
        P = self.P
        Phi, PhiT = self.Phi, self.PhiT
        c = np.zeros(self.n0)
        w = u.copy()
        G = PhiT @ P.residual(w)
        rho = float(np.linalg.norm(G))
        tol = _stop_tol(rho, self.phib_inf, self.n0, self.inner_rtol,
                        self.inner_eta)
        its = 0
        dprev = None
        while True:
            gn = float(np.linalg.norm(G))
            if not np.isfinite(gn):
                raise LocalFailure("coarse: non-finite residual")
            if gn <= tol:
                break
            if dprev is not None and dprev <= self.stagnation * np.max(np.abs(c)):
                break
            if its == self.inner_maxit:
                raise LocalFailure("coarse: no convergence")
            A0 = (PhiT @ (P.jacobian(w) @ Phi)).toarray()
            d = sla.lu_solve(sla.lu_factor(A0, check_finite=False), G)
            c = c + d
            its += 1
            dprev = float(np.max(np.abs(d)))
            w = u - Phi @ c
            G = PhiT @ P.residual(w)
        DF0 = P.jacobian(w)
        A0 = (PhiT @ (DF0 @ Phi)).toarray()
        return {"c": c, "lu": sla.lu_factor(A0, check_finite=False),
                "DF0": DF0, "its": its, "A0": A0}

    # --------------------------------------------------------- combinations
    def evaluate(self, u, guesses=None, predictor=None):
        """F_x(u) for the configured coupling; keeps the state for the tangent.

        guesses: optional per-subdomain predicted starts (see local_solve);
        predictor: alternatively an object whose guesses(w) gives them at the
        point w where the local problems are solved."""
        co = None
        w = u
        if self.coupling == "hybrid":
            # eq. (11): T_0 first; the local corrections at u_0 = u - P_0 T_0(u)
            co = self.coarse_solve(u)
            w = u - self.Phi @ co["c"]
        if predictor is not None:
            guesses = predictor.guesses(w)
        Fx, sols = self.F1(w, guesses=guesses)
        if self.coupling == "additive":
            co = self.coarse_solve(u)
        if co is not None:
            Fx = Fx + self.Phi @ co["c"]
        self.state = {"u": w.copy(), "sols": sols, "coarse": co}
        return Fx

    def tangent(self, v):
        """D F_x(u) v at the last evaluated u, using R_i DF(u_i) v =
        J_ii R_i v + B_i v_Gamma and the partition of unity (eq. 8):
        D F_1 v = v + sum_i P~_i J_ii^{-1} B_i v_Gamma_i      (eqs. 6, 7),
        D F_a v = D F_1 v + q,  q = Q_0 v = Phi A0^{-1} Phi^T DF(u_0) v,
        D F_h v = D F_1 (v - q) + q                        (eq. 12), where
        D F_1 is taken at the local states of the last evaluation (at u_0
        for the hybrid coupling)."""
        st = self.state
        co = st["coarse"]
        q = None
        if co is not None:
            q = self.Phi @ sla.lu_solve(co["lu"], self.PhiT @ (co["DF0"] @ v))
        z = v - q if self.coupling == "hybrid" else v
        y = z.copy()
        for s, sol in zip(self.subs, st["sols"]):
            zz = band_lu_solve(sol["lu"], sol["B"] @ z[s["Gd"]])
            y[s["owned"]] += zz[s["owned_loc"]]
        if q is not None:
            y += q
        return y

    def tangent_literal(self, v):
        """The same tangent from its definition: with Q_i(w) = P~_i (R_i DF(w)
        P_i)^-1 R_i DF(w) and DF assembled globally at the local states
        u_i = u - P_i T_i(u) (eqs. 6, 7),
        additive: sum_i Q_i(u_i) v + Q_0(u_0) v,
        hybrid:   sum_i Q_i(v_i) (I - Q_0(u_0)) v + Q_0(u_0) v with
                  v_i = u_0 - P_i T_i(u_0) (eq. 12)."""
        st = self.state
        P = self.P
        co = st["coarse"]
        q = None
        if co is not None:
            q = self.Phi @ sla.lu_solve(co["lu"], self.PhiT @ (co["DF0"] @ v))
        z = v - q if self.coupling == "hybrid" else v
        y = np.zeros_like(v)
        for s, sol in zip(self.subs, st["sols"]):
            ui = st["u"].copy()
            ui[s["Vd"]] = sol["x"]
            w = (P.jacobian(ui) @ z)[s["Vd"]]
            zz = band_lu_solve(sol["lu"], w)
            y[s["owned"]] += zz[s["owned_loc"]]
        if q is not None:
            y += q
        return y

    def solve(self, u0=None, rtol=1e-8, maxit=50, gmres_rtol=1e-6,
              gmres_restart=50, gmres_maxit=1000, predictor=None):
        """Outer Newton on F_x(u) = 0: solve D F_x(u_k) du = F_x(u_k) (eq. 13)
        by GMRES and set u_{k+1} = u_k - du.

        predictor: optional object whose guesses(u) gives the learned starts
        of the local solves (oracle.guess.Predictor)."""
        def ev(u):
            return self.evaluate(u, predictor=predictor)
        u = np.zeros(self.P.ndof) if u0 is None else np.array(u0, dtype=np.float64)
        Fx = ev(u)
        r0 = float(np.linalg.norm(Fx))
        stats = {"outer": 0, "gmres": [], "inner": [], "coarse": [],
                 "res": [r0], "converged": False}
        stats["inner"].append(sum(s["its"] for s in self.state["sols"]))
        if self.state["coarse"] is not None:
            stats["coarse"].append(self.state["coarse"]["its"])
        for _ in range(maxit):
            if float(np.linalg.norm(Fx)) <= rtol * r0:
                stats["converged"] = True
                break
            du, its = gmres_mgs(self.tangent, Fx, rtol=gmres_rtol,
                                restart=gmres_restart, maxit=gmres_maxit)
            stats["gmres"].append(its)
            u = u - du
            Fx = ev(u)
            stats["outer"] += 1
            stats["res"].append(float(np.linalg.norm(Fx)))
            stats["inner"].append(sum(s["its"] for s in self.state["sols"]))
            if self.state["coarse"] is not None:
                stats["coarse"].append(self.state["coarse"]["its"])
        else:
            stats["converged"] = float(np.linalg.norm(Fx)) <= rtol * r0
        return u, stats

    def solve_load_steps(self, n_steps, u0=None, **kw):
        """Load stepping (continuation): the external load is raised to
        s / n_steps of its full value in steps s = 1..n_steps, each outer
        solve starting from the previous step's solution.  Returns the last
        solution and the per-step statistics."""
        u = np.zeros(self.P.ndof) if u0 is None else np.array(u0, dtype=np.float64)
        steps = []
        for st in range(1, n_steps + 1):
            self.P.set_load_scale(st / n_steps)
            self.refresh_load()
            u, stats = self.solve(u0=u, **kw)
            steps.append(stats)
            if not stats["converged"]:
                break
        return u, steps


def gmres_mgs(apply, b, rtol=1e-6, restart=50, maxit=1000):
    """Restarted GMRES(m) for apply(x) = b from x_0 = 0 (Saad-Schultz):
    Arnoldi with modified Gram-Schmidt, Givens rotations, stop when the
    residual estimate |g_{j+1}| <= rtol ||b||.  Returns (x, iterations)."""
    n = len(b)
    x = np.zeros(n)
    bn = float(np.linalg.norm(b))
    if bn == 0.0:
        return x, 0
    its = 0
    r = b.copy()
    while its < maxit:
        beta = float(np.linalg.norm(r))
        if beta <= rtol * bn:
            break
        m = restart
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j = 0
        done = False
        while j < m and its < maxit:
            w = apply(V[j])
            its += 1
            for i in range(j + 1):
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            j += 1
            if abs(g[j]) <= rtol * bn:
                done = True
                break
        y = sla.solve_triangular(H[:j, :j], g[:j])
        x = x + V[:j].T @ y
        if done:
            break
        r = b - apply(x)
    return x, its


def global_newton(problem, u0=None, maxit=50, dense=False):
    """Plain definition of the discrete solution u*: Newton's method on
    F(u) = 0 (eq. 3) with a direct solve of DF(u) du = F(u), run until the
    step is at the rounding level (|du|_inf <= 1e-13 |u|_inf) or F = 0."""
    u = np.zeros(problem.ndof) if u0 is None else np.array(u0, dtype=np.float64)
    its = 0
    for its in range(1, maxit + 1):
        F = problem.residual(u)
        if not np.any(F):
            break
        A = problem.jacobian(u)
        if dense:
            d = sla.lu_solve(sla.lu_factor(A.toarray()), F)
        else:
            d = spla.spsolve(A.tocsc(), F)
        u = u - d
        if np.max(np.abs(d)) <= 1e-13 * max(np.max(np.abs(u)), 1e-300):
            break
    return u, its
