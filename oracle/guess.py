"""Learned initial guess of the local Newton solves, FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper starts every inner Newton iteration for T_i(u) (eq. 4) from
x = R_i u.  The learned variant predicts a better start from data the local
problem already has; the paper has no such part, so every definition below is
a reading, stated once here and again where used:

  * patch box: the bounding box [x0,x1] x [y0,y1] of the patch nodes
    (V_i and Gamma_i); every sample below is the linear interpolant of a
    global nodal field in the mesh element containing the sample point;
  * trace features (64): u on the box perimeter, 16 samples per side at
    t = j/16 of the side, sides counter-clockwise from the lower-left corner
    (bottom, right, top, left);
  * load features (256): the nodal load f^_g, the mean of the edge-midpoint
    values of f over the (element, edge) pairs incident to node g, sampled
    at the 16 x 16 reference nodes (x0 + p W/15, y0 + q H/15), index
    q*16 + p;
  * lifting: the transfinite (Coons) interpolant of the side functions that
    interpolate the 64 samples linearly in t (the last interval of a side
    ends at the first sample of the next side, its corner);
  * prediction: x_pred = Coons + bilinear interpolant of 256 coefficients at
    the reference nodes, on V_i; Dirichlet nodes of V_i take their values;
  * training target: (v(x*) - Coons) at the reference nodes, where v(x*) is
    u outside V_i and x* on V_i (eq. 4), sampled like the load;
  * network: affine layers 320 -> 256 -> 256 -> 256 -> 256, GELU
    (x Phi(x), exact erf) after the first three; inputs and outputs
    standardised with stored means and deviations; MSE loss over all outputs;
    Adam (Kingma and Ba, 2015) with bias correction;
  * judge: start from x_pred only if ||R_i F(v(x_pred))||_2 < rho_plain =
    ||R_i F(u)||_2 and it is finite; the stopping rule stays relative to
    rho_plain; when Newton from x_pred fails the solve restarts from R_i u.

Elasticity (Q1, two displacement components; PatchGeometryNH), the same
320 inputs and 256 outputs laid out per component:
  * sampling: the bilinear (Q1) interpolant in the quadrilateral containing
    the point, local coordinates from the inverse of the element map;
  * trace features (64): u_x then u_y at 32 perimeter points, 8 per side at
    t = j/8, sides counter-clockwise from the lower-left corner;
  * load features (256): f_x then f_y, f the external nodal forces (zero on
    Dirichlet dofs), at 128 points (x1, y0 + j H/127) on the right side of
    the box (the loaded edge of the cantilever; zero when the box does not
    reach it);
  * output and target: per component the 16 x 8 reference nodes
    (x0 + p W/15, y0 + q H/7), index q*16 + p, x then y; lifting per
    component: Coons of its 32 trace samples + bilinear interpolant of its
    128 coefficients.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

N_SIDE = 16
N_TRACE = 4 * N_SIDE
GRID = 16
N_GRID = GRID * GRID
N_IN = N_TRACE + N_GRID
WIDTH = 256
N_OUT = N_GRID
DIMS = (N_IN, WIDTH, WIDTH, WIDTH, N_OUT)


# ------------------------------------------------------------ patch geometry
def nodal_load(problem) -> np.ndarray:
    """f^_g: mean of the midpoint samples of f on the element edges through
    node g (one term per incident element and edge); 1 when f = 1.
    Elasticity: the external nodal forces, zero on Dirichlet dofs."""
    if getattr(problem, "d", 1) == 2:
        f = np.array(problem.ext_load, dtype=np.float64)
        f[problem.is_dir] = 0.0
        return f
    case = problem.case
    fm = case.get("elem_load")
    if fm is None:
        return np.ones(problem.N)
    fm = np.asarray(fm, dtype=np.float64)
    conn = problem.conn
    acc = np.zeros(problem.N)
    cnt = np.zeros(problem.N)
    for a in range(3):
        # vertex a lies on edges (a, a+1) (index a) and (a+2, a) (index a+2)
        np.add.at(acc, conn[:, a], fm[:, a] + fm[:, (a + 2) % 3])
        np.add.at(cnt, conn[:, a], 2.0)
    return acc / cnt


def _barycentric(p, tri):
    """Barycentric coordinates of points p (k,2) in triangles tri (m,3,2)."""
    a, b, c = tri[:, 0], tri[:, 1], tri[:, 2]
    det = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) \
        - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1])
    dx = p[:, None, 0] - a[None, :, 0]
    dy = p[:, None, 1] - a[None, :, 1]
    l1 = (dx * (c[None, :, 1] - a[None, :, 1])
          - dy * (c[None, :, 0] - a[None, :, 0])) / det[None, :]
    l2 = ((b[None, :, 0] - a[None, :, 0]) * dy
          - (b[None, :, 1] - a[None, :, 1]) * dx) / det[None, :]
    return np.stack([1.0 - l1 - l2, l1, l2], axis=-1)


class PatchGeometry:
    """Box and sampling tables of one patch.

    Every sample (64 perimeter points, then the 256 reference nodes) is the
    linear interpolant of a global nodal field in the mesh element that
    contains the point (largest smallest barycentric coordinate, so a point
    on an edge may take either neighbour: the interpolant is continuous).
    Sampling the global field lets the box corners lie outside the patch,
    which happens when the overlap layers leave stair-stepped corners.
    """

    def __init__(self, S, i):
        s = S.subs[i]
        P = S.P
        xy = P.xy
        nodes = np.concatenate([s["V"], s["Gam"]])
        self.V = s["V"]
        pts = xy[nodes]
        self.x0, self.y0 = pts.min(axis=0)
        self.x1, self.y1 = pts.max(axis=0)
        W, H = self.x1 - self.x0, self.y1 - self.y0
        self.W, self.H = W, H
        self.eligible = bool(W > 0 and H > 0)
        if not self.eligible:
            return
        t = np.arange(N_SIDE) / N_SIDE
        x0, x1, y0, y1 = self.x0, self.x1, self.y0, self.y1
        per = np.concatenate([
            np.stack([x0 + t * W, np.full_like(t, y0)], 1),
            np.stack([np.full_like(t, x1), y0 + t * H], 1),
            np.stack([x1 - t * W, np.full_like(t, y1)], 1),
            np.stack([np.full_like(t, x0), y1 - t * H], 1)])
        p = np.arange(GRID) / (GRID - 1)
        self.grid_pts = np.stack(np.meshgrid(x0 + p * W, y0 + p * H, indexing="xy"),
                                 axis=-1).reshape(-1, 2)
        self.sample_pts = np.concatenate([per, self.grid_pts])
        # candidate elements: those whose bounding box meets the patch box
        tri = xy[P.conn]
        lo = tri.min(axis=1)
        hi = tri.max(axis=1)
        eps = 1e-12 * max(W, H)
        cand = np.nonzero((hi[:, 0] >= x0 - eps) & (lo[:, 0] <= x1 + eps)
                          & (hi[:, 1] >= y0 - eps) & (lo[:, 1] <= y1 + eps))[0]
        lam = _barycentric(self.sample_pts, tri[cand])
        best = np.argmax(lam.min(axis=-1), axis=1)
        self.samp_nodes = P.conn[cand[best]]              # (320, 3) global ids
        self.samp_w = lam[np.arange(len(best)), best]     # (320, 3)
        self.xi = (xy[s["V"], 0] - x0) / W
        self.eta = (xy[s["V"], 1] - y0) / H

    # -------------------------------------------------------------- features
    def _interp(self, nodal, rows):
        return (self.samp_w[rows] * nodal[self.samp_nodes[rows]]).sum(axis=1)

    def trace(self, u):
        return self._interp(u, slice(0, N_TRACE))

    def grid_sample(self, nodal):
        return self._interp(nodal, slice(N_TRACE, N_IN))

    def features(self, u, fhat):
        return np.concatenate([self.trace(u), self.grid_sample(fhat)])

    # --------------------------------------------------------------- lifting
    @staticmethod
    def _side(samples, sd, t, n_side=N_SIDE):
        pos = np.asarray(t) * n_side
        j = np.minimum(np.floor(pos).astype(np.int64), n_side - 1)
        w = pos - j
        v0 = samples[sd * n_side + j]
        nxt = np.where(j < n_side - 1, sd * n_side + j + 1,
                       ((sd + 1) % 4) * n_side)
        return (1.0 - w) * v0 + w * samples[nxt]

    @classmethod
    def coons(cls, samples, xi, eta, n_side=N_SIDE):
        """Transfinite interpolant of the sampled boundary at unit (xi, eta)
        (n_side samples per side)."""
        g0 = cls._side(samples, 0, xi, n_side)
        g1 = cls._side(samples, 1, eta, n_side)
        g2 = cls._side(samples, 2, 1.0 - xi, n_side)
        g3 = cls._side(samples, 3, 1.0 - eta, n_side)
        c00, c10, c11, c01 = (samples[0], samples[n_side],
                              samples[2 * n_side], samples[3 * n_side])
        return ((1 - eta) * g0 + eta * g2 + (1 - xi) * g3 + xi * g1
                - ((1 - xi) * (1 - eta) * c00 + xi * (1 - eta) * c10
                   + xi * eta * c11 + (1 - xi) * eta * c01))

    @staticmethod
    def bilinear(coef, xi, eta, gx=GRID, gy=GRID):
        """Bilinear interpolant of values at the gx x gy reference nodes
        (index q*gx + p) at unit (xi, eta)."""
        c = np.asarray(coef).reshape(gy, gx)    # [q, p]
        px = np.asarray(xi) * (gx - 1)
        py = np.asarray(eta) * (gy - 1)
        p0 = np.clip(np.floor(px).astype(np.int64), 0, gx - 2)
        q0 = np.clip(np.floor(py).astype(np.int64), 0, gy - 2)
        a = px - p0
        b = py - q0
        return ((1 - a) * (1 - b) * c[q0, p0] + a * (1 - b) * c[q0, p0 + 1]
                + (1 - a) * b * c[q0 + 1, p0] + a * b * c[q0 + 1, p0 + 1])

    def _grid_unit(self):
        p = np.arange(GRID) / (GRID - 1)
        xi, eta = np.meshgrid(p, p, indexing="xy")
        return xi.ravel(), eta.ravel()

    def lift(self, u, coef, dirV, dir_vals):
        """x_pred on V_i: Coons(trace) + bilinear(coef); Dirichlet rows exact."""
        tr = self.trace(u)
        x = self.coons(tr, self.xi, self.eta) + self.bilinear(coef, self.xi, self.eta)
        x = np.where(dirV, dir_vals, x)
        return x

    def target(self, u, xstar):
        """(v(x*) - Coons) at the reference nodes, where v(x*) is u outside V_i
        and x* on V_i (the state of eq. 4 at the local solution)."""
        v = np.array(u, dtype=np.float64)
        v[self.V] = xstar
        xi, eta = self._grid_unit()
        return self.grid_sample(v) - self.coons(self.trace(u), xi, eta)


# ------------------------------------------------- elasticity (Q1, d = 2)
NH_SIDE = 8
NH_TRACE = 4 * NH_SIDE        # perimeter points (two components each)
NH_LOAD = 128                 # points on the right side of the box
NH_GX, NH_GY = 16, 8
NH_NGRID = NH_GX * NH_GY      # reference nodes (two components each)


def q1_shape(xi, eta):
    """Bilinear shape functions of the counter-clockwise corners (0,0),
    (1,0), (1,1), (0,1) of the reference square."""
    return np.stack([(1 - xi) * (1 - eta), xi * (1 - eta), xi * eta, (1 - xi) * eta], axis=-1)


def q1_local(p, quad, iters=30):
    """Reference coordinates of points p (k,2) in quadrilaterals quad (m,4,2):
    Newton's method on x(xi, eta) = p for the bilinear element map, from
    the centre (exact after one step on parallelograms)."""
    k, m = len(p), len(quad)
    xi = np.full((k, m), 0.5)
    eta = np.full((k, m), 0.5)
    X = quad[None, :, :, 0]
    Y = quad[None, :, :, 1]
    for _ in range(iters):
        N = q1_shape(xi, eta)
        dxi = np.stack([-(1 - eta), 1 - eta, eta, -eta], axis=-1)
        deta = np.stack([-(1 - xi), -xi, xi, 1 - xi], axis=-1)
        rx = (N * X).sum(-1) - p[:, None, 0]
        ry = (N * Y).sum(-1) - p[:, None, 1]
        a, b = (dxi * X).sum(-1), (deta * X).sum(-1)
        c, d = (dxi * Y).sum(-1), (deta * Y).sum(-1)
        det = a * d - b * c
        sx = (d * rx - b * ry) / det
        sy = (-c * rx + a * ry) / det
        xi, eta = xi - sx, eta - sy
        if max(np.abs(sx).max(), np.abs(sy).max()) < 1e-15:
            break
    return xi, eta


class PatchGeometryNH:
    """Box and sampling tables of one elasticity patch (two components):
    32 perimeter points, 128 points on the right side of the box and the
    16 x 8 reference nodes, each sampled with the bilinear interpolant in
    the quadrilateral that contains it (largest smallest distance of its
    reference coordinates to the element's sides)."""

    def __init__(self, S, i):
        s = S.subs[i]
        P = S.P
        xy = P.xy
        nodes = np.concatenate([s["V"], s["Gam"]])
        self.V = s["V"]
        self.Vd = s["Vd"]
        pts = xy[nodes]
        self.x0, self.y0 = pts.min(axis=0)
        self.x1, self.y1 = pts.max(axis=0)
        W, H = self.x1 - self.x0, self.y1 - self.y0
        self.W, self.H = W, H
        self.eligible = bool(W > 0 and H > 0)
        if not self.eligible:
            return
        x0, x1, y0, y1 = self.x0, self.x1, self.y0, self.y1
        t = np.arange(NH_SIDE) / NH_SIDE
        per = np.concatenate([
            np.stack([x0 + t * W, np.full_like(t, y0)], 1),
            np.stack([np.full_like(t, x1), y0 + t * H], 1),
            np.stack([x1 - t * W, np.full_like(t, y1)], 1),
            np.stack([np.full_like(t, x0), y1 - t * H], 1)])
        r = np.arange(NH_LOAD) / (NH_LOAD - 1)
        right = np.stack([np.full_like(r, x1), y0 + r * H], 1)
        px = np.arange(NH_GX) / (NH_GX - 1)
        py = np.arange(NH_GY) / (NH_GY - 1)
        self.grid_pts = np.stack(np.meshgrid(x0 + px * W, y0 + py * H, indexing="xy"),
                                 axis=-1).reshape(-1, 2)
        self.sample_pts = np.concatenate([per, right, self.grid_pts])
        quad = xy[P.conn]
        lo, hi = quad.min(axis=1), quad.max(axis=1)
        eps = 1e-12 * max(W, H)
        cand = np.nonzero((hi[:, 0] >= x0 - eps) & (lo[:, 0] <= x1 + eps)
                          & (hi[:, 1] >= y0 - eps) & (lo[:, 1] <= y1 + eps))[0]
        xi, eta = q1_local(self.sample_pts, quad[cand])
        inside = np.minimum(np.minimum(xi, 1 - xi), np.minimum(eta, 1 - eta))
        best = np.argmax(inside, axis=1)
        k = np.arange(len(best))
        self.samp_nodes = P.conn[cand[best]]                       # (288, 4)
        self.samp_w = q1_shape(xi[k, best], eta[k, best])          # (288, 4)
        self.samp_inside = inside[k, best]
        self.xi = (xy[s["V"], 0] - x0) / W
        self.eta = (xy[s["V"], 1] - y0) / H

    def _interp(self, dofvec, rows, c):
        return (self.samp_w[rows] * dofvec[2 * self.samp_nodes[rows] + c]).sum(axis=1)

    def trace(self, u):
        rows = slice(0, NH_TRACE)
        return np.concatenate([self._interp(u, rows, 0), self._interp(u, rows, 1)])

    def load(self, f):
        rows = slice(NH_TRACE, NH_TRACE + NH_LOAD)
        return np.concatenate([self._interp(f, rows, 0), self._interp(f, rows, 1)])

    def grid_sample(self, v, c):
        return self._interp(v, slice(NH_TRACE + NH_LOAD, NH_TRACE + NH_LOAD + NH_NGRID), c)

    def features(self, u, f):
        return np.concatenate([self.trace(u), self.load(f)])

    def _grid_unit(self):
        px = np.arange(NH_GX) / (NH_GX - 1)
        py = np.arange(NH_GY) / (NH_GY - 1)
        xi, eta = np.meshgrid(px, py, indexing="xy")
        return xi.ravel(), eta.ravel()

    def lift(self, u, coef, dirV, dir_vals):
        """x_pred on the V dofs (x then y per node): per component Coons of its
        trace samples + bilinear interpolant of its 128 coefficients;
        Dirichlet dofs exact."""
        tr = self.trace(u)
        coef = np.asarray(coef, dtype=np.float64)
        x = np.empty(2 * len(self.V))
        for c in range(2):
            x[c::2] = (PatchGeometry.coons(tr[c * NH_TRACE:(c + 1) * NH_TRACE], self.xi,
                                           self.eta, NH_SIDE)
                       + PatchGeometry.bilinear(coef[c * NH_NGRID:(c + 1) * NH_NGRID],
                                                self.xi, self.eta, NH_GX, NH_GY))
        return np.where(dirV, dir_vals, x)

    def target(self, u, xstar):
        """Per component (v(x*) - Coons) at the 16 x 8 reference nodes, v(x*)
        = x* on the V dofs and u elsewhere; x then y."""
        v = np.array(u, dtype=np.float64)
        v[self.Vd] = xstar
        tr = self.trace(u)
        xi, eta = self._grid_unit()
        return np.concatenate([
            self.grid_sample(v, c) - PatchGeometry.coons(tr[c * NH_TRACE:(c + 1) * NH_TRACE],
                                                         xi, eta, NH_SIDE)
            for c in range(2)])


# ------------------------------------------------------------------ network
def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) \
        + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def unpack(flat, dims=DIMS):
    """Flat parameters (W1, b1, W2, b2, ...; W_l row-major [out][in])."""
    flat = np.asarray(flat, dtype=np.float64)
    out, o = [], 0
    for l in range(len(dims) - 1):
        ni, no = dims[l], dims[l + 1]
        W = flat[o:o + no * ni].reshape(no, ni)
        o += no * ni
        b = flat[o:o + no]
        o += no
        out.append((W, b))
    assert o == len(flat), (o, len(flat))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def n_params(dims=DIMS):
    return sum(dims[l] * dims[l + 1] + dims[l + 1] for l in range(len(dims) - 1))


def forward(flat, Xn, dims=DIMS):
    """Network on standardised inputs; returns (output, pre-activations,
    activations)."""
    layers = unpack(flat, dims)
    a = np.asarray(Xn, dtype=np.float64)
    zs, acts = [], [a]
    for l, (W, b) in enumerate(layers):
        z = a @ W.T + b
        zs.append(z)
        a = gelu(z) if l + 1 < len(layers) else z
        acts.append(a)
    return a, zs, acts


def loss_grad(flat, Xn, Tn, dims=DIMS):
    """MSE over all outputs of a batch and its gradient (flat, same order)."""
    y, zs, acts = forward(flat, Xn, dims)
    layers = unpack(flat, dims)
    B = y.shape[0]
    diff = y - Tn
    loss = float(np.mean(diff * diff))
    dz = 2.0 * diff / diff.size
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads[l] = (dz.T @ acts[l], dz.sum(axis=0))
        if l > 0:
            dz = (dz @ W) * gelu_prime(zs[l - 1])
    del B
    return loss, pack(grads)


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(x):
    """Round float32 values to bfloat16 (nearest, ties to even), as float64."""
    f = np.asarray(x, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    r = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def standardise_stats(X, floor=1e-6):
    """Column means and deviations; deviations below floor*max(dev, 1) -> 1."""
    X = np.asarray(X, dtype=np.float64)
    m = X.mean(axis=0)
    s = X.std(axis=0)
    s = np.where(s <= floor * max(float(s.max(initial=0.0)), 1.0), 1.0, s)
    return m, s


class Predictor:
    """Network prediction of local initial guesses (oracle side)."""

    def __init__(self, S, flat, norm):
        self.S = S
        self.flat = np.asarray(flat, dtype=np.float64)
        self.xm, self.xs, self.ym, self.ys = (np.asarray(a, np.float64) for a in norm)
        self.fhat = nodal_load(S.P)
        cls = PatchGeometryNH if S.P.d == 2 else PatchGeometry
        self.geo = [cls(S, i) for i in range(S.n_sub)]

    def features(self, u):
        return [g.features(u, self.fhat) if g.eligible else None for g in self.geo]

    def coefficients(self, u):
        feats = self.features(u)
        idx = [i for i, f in enumerate(feats) if f is not None]
        out = [None] * len(feats)
        if idx:
            X = np.stack([feats[i] for i in idx])
            y, _, _ = forward(self.flat, (X - self.xm) / self.xs)
            Y = y * self.ys + self.ym
            for k, i in enumerate(idx):
                out[i] = Y[k]
        return out

    def guesses(self, u):
        P = self.S.P
        res = []
        for i, c in enumerate(self.coefficients(u)):
            if c is None:
                res.append(None)
                continue
            s = self.S.subs[i]
            res.append(self.geo[i].lift(u, c, s["dirV"], P.dir_value[s["Vd"]]))
        return res
