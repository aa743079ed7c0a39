"""Pins of the oracle's learned-initial-guess parts against mathematics.

The sampling and lifting operators are pinned by exactness on the function
classes they must reproduce (linear and bilinear fields), the network by
central differences of its loss, special values of GELU and a library
bfloat16 rounding, Adam by its closed form under a constant gradient, and the
judge by what it must do with an exact and with a useless guess.
"""
import numpy as np
import pytest
from scipy.stats import norm

import synth
from oracle import P1Problem, Schwarz
from oracle import guess as G

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _schwarz(**kw):
    case = synth.small_case(**kw)
    return Schwarz(P1Problem(case), "one_level")


def _perimeter_points(geo):
    """Positions of the 64 trace samples, from the side parametrisation."""
    t = np.arange(G.N_SIDE) / G.N_SIDE
    x0, x1, y0, y1 = geo.x0, geo.x1, geo.y0, geo.y1
    W, H = x1 - x0, y1 - y0
    sides = [np.stack([x0 + t * W, np.full_like(t, y0)], 1),
             np.stack([np.full_like(t, x1), y0 + t * H], 1),
             np.stack([x1 - t * W, np.full_like(t, y1)], 1),
             np.stack([np.full_like(t, x0), y1 - t * H], 1)]
    return np.concatenate(sides)


def test_sample_points_located_in_their_elements():
    """Every sample point lies in (or on) the element it is interpolated in,
    including box corners cut off the patch by stair-stepped overlap."""
    S = _schwarz(n=12, boxes=3, overlap=2, uneven=True)
    xy = S.P.xy
    for i in range(S.n_sub):
        geo = G.PatchGeometry(S, i)
        assert geo.eligible
        np.testing.assert_allclose(geo.samp_w.sum(axis=1), 1.0, atol=1e-14)
        assert geo.samp_w.min() >= -1e-12
        rec = (geo.samp_w[:, :, None] * xy[geo.samp_nodes]).sum(axis=1)
        np.testing.assert_allclose(rec, geo.sample_pts, atol=1e-14)
        np.testing.assert_allclose(geo.sample_pts[:G.N_TRACE], _perimeter_points(geo),
                                   atol=0)


def test_trace_exact_for_linear_fields():
    S = _schwarz(n=13, boxes=3, overlap=2, uneven=True)
    xy = S.P.xy
    u = 0.3 + 1.7 * xy[:, 0] - 2.2 * xy[:, 1]
    for i in range(S.n_sub):
        geo = G.PatchGeometry(S, i)
        pts = _perimeter_points(geo)
        ref = 0.3 + 1.7 * pts[:, 0] - 2.2 * pts[:, 1]
        np.testing.assert_allclose(geo.trace(u), ref, rtol=0, atol=1e-14)


def test_coons_and_bilinear_reproduce_bilinear_functions():
    S = _schwarz(n=12, boxes=3, overlap=1)
    geo = G.PatchGeometry(S, 4)
    rng = np.random.default_rng(1)
    a, b, c, d = rng.normal(size=4)

    def f(x, y):
        return a + b * x + c * y + d * x * y

    pts = _perimeter_points(geo)
    samples = f(pts[:, 0], pts[:, 1])
    xi, eta = rng.uniform(size=(2, 200))
    x = geo.x0 + xi * geo.W
    y = geo.y0 + eta * geo.H
    np.testing.assert_allclose(G.PatchGeometry.coons(samples, xi, eta), f(x, y),
                               rtol=0, atol=1e-13)
    p = np.arange(G.GRID) / (G.GRID - 1)
    gx, gy = np.meshgrid(geo.x0 + p * geo.W, geo.y0 + p * geo.H, indexing="xy")
    coef = f(gx, gy).ravel()
    np.testing.assert_allclose(G.PatchGeometry.bilinear(coef, xi, eta), f(x, y),
                               rtol=0, atol=1e-13)
    # the Coons interpolant matches the boundary samples on the sides
    t = np.arange(G.N_SIDE) / G.N_SIDE
    np.testing.assert_allclose(G.PatchGeometry.coons(samples, t, 0 * t),
                               samples[:G.N_SIDE], atol=1e-14)


def test_grid_sampling_and_nodal_load_on_linear_data():
    S = _schwarz(n=12, boxes=3, overlap=2)
    xy = S.P.xy
    lin = 1.0 - 0.5 * xy[:, 0] + 0.25 * xy[:, 1]
    for i in (0, 4, 8):
        geo = G.PatchGeometry(S, i)
        ref = 1.0 - 0.5 * geo.grid_pts[:, 0] + 0.25 * geo.grid_pts[:, 1]
        np.testing.assert_allclose(geo.grid_sample(lin), ref, atol=1e-14)
    # midpoint samples of a linear f: the nodal mean is exact on interior
    # nodes of the grid (each node's edge star is point-symmetric)
    case = synth.diffusion_case(10, 10, synth.even_cuts(10, 2),
                                synth.even_cuts(10, 2), 1,
                                forcing=lambda p: 2.0 + p[..., 0] - 3.0 * p[..., 1])
    P = P1Problem(case)
    fh = G.nodal_load(P)
    inner = ~P.is_dir
    ref = 2.0 + P.xy[:, 0] - 3.0 * P.xy[:, 1]
    np.testing.assert_allclose(fh[inner], ref[inner], atol=1e-14)
    assert np.all(G.nodal_load(P1Problem(synth.small_case(n=6, boxes=2))) == 1.0)


def test_lift_and_target_vanish_on_linear_states():
    S = _schwarz(n=12, boxes=3, overlap=2, uneven=True)
    P = S.P
    u = 0.2 + 0.7 * P.xy[:, 0] + 0.4 * P.xy[:, 1]
    for i in range(S.n_sub):
        s = S.subs[i]
        geo = G.PatchGeometry(S, i)
        x = geo.lift(u, np.zeros(G.N_GRID), s["dirV"], P.dir_value[s["V"]])
        nd = ~s["dirV"]
        np.testing.assert_allclose(x[nd], u[s["V"]][nd], atol=1e-14)
        np.testing.assert_array_equal(x[s["dirV"]], P.dir_value[s["V"]][s["dirV"]])
        t = geo.target(u, u[s["V"]])
        assert np.abs(t).max() <= 1e-14


def test_gelu_special_values_and_derivative():
    z = np.array([-3.0, -1.0, -0.25, 0.0, 0.5, 1.0, 2.5])
    np.testing.assert_allclose(G.gelu(z), z * norm.cdf(z), rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(G.gelu_prime(z), norm.cdf(z) + z * norm.pdf(z),
                               rtol=1e-14, atol=1e-16)
    assert G.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, abs=1e-15)


def test_loss_gradient_matches_central_differences():
    dims = (12, 8, 8, 8, 6)
    rng = np.random.default_rng(5)
    flat = rng.normal(scale=0.4, size=G.n_params(dims))
    X = rng.normal(size=(7, 12))
    T = rng.normal(size=(7, 6))
    loss, g = G.loss_grad(flat, X, T, dims)
    eps = 1e-6
    fd = np.empty_like(flat)
    for k in range(len(flat)):
        e = np.zeros_like(flat)
        e[k] = eps
        fd[k] = (G.loss_grad(flat + e, X, T, dims)[0]
                 - G.loss_grad(flat - e, X, T, dims)[0]) / (2 * eps)
    np.testing.assert_allclose(g, fd, rtol=1e-7, atol=1e-9)
    assert loss == pytest.approx(np.mean((G.forward(flat, X, dims)[0] - T) ** 2))


def test_network_shape_and_parameter_count():
    assert G.n_params() == 279552
    flat = synth.mlp_init(0)
    assert flat.dtype == np.float32 and len(flat) == G.n_params()
    X, _ = synth.mlp_batch(1, 5)
    y, zs, acts = G.forward(flat, X)
    assert y.shape == (5, 256) and len(zs) == 4


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are g and g^2,
    so every step is exactly lr * g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    w = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    lr = 0.01
    for t in range(1, 6):
        w_new, m, v = G.adam_step(w, g, m, v, t, lr)
        np.testing.assert_allclose(w_new - w, -lr * g / (np.abs(g) + 1e-8),
                                   rtol=1e-12, atol=1e-18)
        w = w_new


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(2).normal(scale=50.0, size=4096).astype(np.float32)
    x[:8] = [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.140625, -2.5e-3, 65504.0]
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(G.bf16_round(x), ref)


def test_judge_exact_guess_and_useless_guess():
    S = Schwarz(P1Problem(synth.small_case(n=12, boxes=3, overlap=2, forcing_seed=3)),
                "one_level")
    u = np.zeros(S.P.N)
    for i in (0, 4):
        plain = S.local_solve(i, u)
        assert plain["start"] == "plain" and plain["its"] >= 1
        exact = S.local_solve(i, u, guess=plain["x"])
        assert exact["start"] == "guess" and exact["its"] == 0
        np.testing.assert_array_equal(exact["x"], plain["x"])
        bad = S.local_solve(i, u, guess=np.full(len(plain["x"]), 1e3))
        assert bad["start"] == "fallback" and bad["its"] == plain["its"]
        np.testing.assert_array_equal(bad["x"], plain["x"])
        near = S.local_solve(i, u, guess=plain["x"] * (1 + 1e-3))
        assert near["start"] == "guess"
        x_scale = np.abs(plain["x"]).max()
        assert np.abs(near["x"] - plain["x"]).max() <= 1e-10 * x_scale


def test_predictor_solve_reaches_plain_solution():
    """Any network (here an untrained one) leaves the solution unchanged:
    the judge and the unchanged stopping rule make it a start only."""
    case = synth.small_case(n=16, boxes=4, overlap=2, forcing_seed=1, two_level=True)
    S = Schwarz(P1Problem(case), "additive")
    u0, st0 = S.solve()
    flat = synth.mlp_init(7)
    normz = (np.zeros(G.N_IN), np.ones(G.N_IN), np.zeros(G.N_OUT),
             np.full(G.N_OUT, 1e-3))
    pred = G.Predictor(S, flat, normz)
    u1, st1 = S.solve(predictor=pred)
    assert st1["converged"] and st1["outer"] == st0["outer"]
    assert np.linalg.norm(u1 - u0) <= 1e-10 * np.linalg.norm(u0)


# ------------------------------------------------------------- elasticity
def _nh_schwarz(**kw):
    from oracle import NHProblem
    case = synth.small_elasticity_case(**kw)
    return Schwarz(NHProblem(case), "one_level")


def test_q1_inverse_map_recovers_reference_coordinates():
    """Newton's inverse of the bilinear element map on random convex
    quadrilaterals: x(xi, eta) of known (xi, eta) maps back to them."""
    rng = np.random.default_rng(5)
    base = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    quads = base[None] * rng.uniform(0.5, 2.0, size=(6, 1, 2)) \
        + rng.uniform(-0.15, 0.15, size=(6, 4, 2))
    ref = rng.uniform(0.0, 1.0, size=(10, 2))
    for q in quads:
        N = G.q1_shape(ref[:, 0], ref[:, 1])
        p = N @ q
        xi, eta = G.q1_local(p, q[None])
        np.testing.assert_allclose(xi[:, 0], ref[:, 0], atol=1e-13)
        np.testing.assert_allclose(eta[:, 0], ref[:, 1], atol=1e-13)


def test_nh_sampling_exact_for_bilinear_fields():
    """On rectangles the Q1 interpolant reproduces a + bx + cy + dxy, so
    every sample (trace, load and grid) of such a field is exact, each
    sample point lies in its element, and the weights sum to 1."""
    S = _nh_schwarz(nx=12, ny=8, boxes=(3, 2), overlap=2, traction=(0.0, -1.0))
    xy = S.P.xy
    fx = lambda p: 0.3 + 1.7 * p[:, 0] - 2.2 * p[:, 1] + 0.5 * p[:, 0] * p[:, 1]  # noqa: E731
    fy = lambda p: -1.1 + 0.4 * p[:, 0] + 0.9 * p[:, 1] - 0.7 * p[:, 0] * p[:, 1]  # noqa: E731
    u = np.empty(2 * len(xy))
    u[0::2], u[1::2] = fx(xy), fy(xy)
    for i in range(S.n_sub):
        geo = G.PatchGeometryNH(S, i)
        assert geo.eligible and geo.samp_inside.min() >= -1e-12
        np.testing.assert_allclose(geo.samp_w.sum(axis=1), 1.0, atol=1e-14)
        rec = (geo.samp_w[:, :, None] * xy[geo.samp_nodes]).sum(axis=1)
        np.testing.assert_allclose(rec, geo.sample_pts, atol=1e-13)
        pts = geo.sample_pts
        T = G.NH_TRACE
        np.testing.assert_allclose(geo.trace(u), np.concatenate([fx(pts[:T]), fy(pts[:T])]),
                                   atol=1e-13)
        L = slice(T, T + G.NH_LOAD)
        np.testing.assert_allclose(geo.load(u), np.concatenate([fx(pts[L]), fy(pts[L])]),
                                   atol=1e-13)
        np.testing.assert_allclose(geo.grid_sample(u, 1), fy(geo.grid_pts), atol=1e-13)


def test_nh_lift_and_target_on_bilinear_states():
    """For a bilinear displacement the Coons lifting of its trace (8 samples
    per side) is the field itself, so lift(u, 0) = u on the free V dofs and
    the target of x* = R_i u vanishes."""
    S = _nh_schwarz(nx=16, ny=8, boxes=(2, 2), overlap=1, traction=(0.0, -1.0))
    P = S.P
    xy = P.xy
    u = np.empty(P.ndof)
    u[0::2] = 0.1 - 0.3 * xy[:, 0] + 0.2 * xy[:, 1] + 0.05 * xy[:, 0] * xy[:, 1]
    u[1::2] = -0.2 + 0.1 * xy[:, 0] - 0.4 * xy[:, 0] * xy[:, 1]
    for i in range(S.n_sub):
        s = S.subs[i]
        geo = G.PatchGeometryNH(S, i)
        x = geo.lift(u, np.zeros(G.N_OUT), s["dirV"], P.dir_value[s["Vd"]])
        free = ~s["dirV"]
        np.testing.assert_allclose(x[free], u[s["Vd"]][free], atol=1e-13)
        np.testing.assert_array_equal(x[s["dirV"]], P.dir_value[s["Vd"]][s["dirV"]])
        np.testing.assert_allclose(geo.target(u, u[s["Vd"]]), 0.0, atol=1e-13)
        # bilinear coefficients are reproduced by the reference-grid interpolant
        xi, eta = geo._grid_unit()
        c = 0.7 - 0.2 * xi + 1.3 * eta + 0.4 * xi * eta
        coef = np.concatenate([c, -c])
        y = geo.lift(np.zeros(P.ndof), coef, np.zeros(len(x), bool), np.zeros(len(x)))
        ref = 0.7 - 0.2 * geo.xi + 1.3 * geo.eta + 0.4 * geo.xi * geo.eta
        np.testing.assert_allclose(y[0::2], ref, atol=1e-13)
        np.testing.assert_allclose(y[1::2], -ref, atol=1e-13)


def test_nh_load_features_sample_the_loaded_edge():
    """Load features: zero for boxes away from the loaded edge; on the edge
    the interpolant of the lumped traction t h (t h / 2 at the two end
    nodes), so t h wherever the sample lies between two interior nodes."""
    t = (0.0, -3.0)
    S = _nh_schwarz(nx=12, ny=6, boxes=(3, 2), overlap=1, traction=t)
    f = G.nodal_load(S.P)
    h = 1.0 / 6
    touched = 0
    for i in range(S.n_sub):
        geo = G.PatchGeometryNH(S, i)
        ld = geo.load(f)
        if geo.x1 < 2.0 - 1e-12:
            np.testing.assert_array_equal(ld, 0.0)
            continue
        touched += 1
        y = geo.sample_pts[G.NH_TRACE:G.NH_TRACE + G.NH_LOAD, 1]
        mid = (y >= h - 1e-12) & (y <= 1.0 - h + 1e-12)
        np.testing.assert_allclose(ld[:G.NH_LOAD][mid], t[0] * h, atol=1e-14)
        np.testing.assert_allclose(ld[G.NH_LOAD:][mid], t[1] * h, rtol=1e-13)
    assert touched == 2


def test_nh_predictor_solve_reaches_plain_solution():
    """Elasticity: an untrained network only changes the starts; the local
    solutions and the outer iteration are those of the plain method."""
    from oracle import NHProblem
    case = synth.small_elasticity_case(nx=16, ny=8, boxes=(2, 2), overlap=1,
                                       traction=(0.0, -2.0), two_level=True)
    S = Schwarz(NHProblem(case), "additive")
    u0, st0 = S.solve()
    normz = (np.zeros(G.N_IN), np.ones(G.N_IN), np.zeros(G.N_OUT), np.full(G.N_OUT, 1e-4))
    pred = G.Predictor(S, synth.mlp_init(9), normz)
    u1, st1 = S.solve(predictor=pred)
    assert st1["converged"] and st1["outer"] == st0["outer"]
    assert np.linalg.norm(u1 - u0) <= 1e-10 * np.linalg.norm(u0)
