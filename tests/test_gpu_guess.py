"""Learned initial guess: HIP path (through the C ABI) against the oracle.

Tolerances:
  * features, training targets: FP32 storage, 2e-6 of the largest magnitude;
  * lifting from given coefficients: FP64, 1e-12 of the largest magnitude;
  * network output: bfloat16 weights and activations with FP32 accumulation
    against the FP64 network with the same bfloat16-rounded weights: 2e-2
    of the largest output;
  * gradient: cosine >= 0.999 and relative 2-norm error <= 3e-2 against the
    FP64 gradient of the unrounded network;
  * local solutions with the learned start: 1e-10 relative (the start changes
    only the iterates, not the stopping rule, C27).
"""
import numpy as np
import pytest

import synth
from oracle import P1Problem, Schwarz
from oracle import guess as G
from tests._lib import ensure_built

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(case, **kw):
    from paper_2410_24138_amd import Solver
    return Solver(case, **kw)


def _np(t):
    return t.detach().cpu().numpy()


def _case(two_level=True):
    return synth.small_case(n=20, boxes=4, overlap=2, forcing_seed=5, coef_seed=3,
                            two_level=two_level, uneven=True)


def _probe(P, seed=1):
    rng = np.random.default_rng(seed)
    u = 0.02 * rng.standard_normal(P.N)
    u[P.is_dir] = P.dir_value[P.is_dir]
    return u


def _norm(seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.normal(size=320), rng.uniform(0.5, 2.0, 320),
                           rng.normal(size=256), rng.uniform(0.5, 2.0, 256)]).astype(np.float32)


def test_features_match_oracle():
    case = _case()
    P = P1Problem(case)
    S = Schwarz(P, "one_level")
    s = _solver(case)
    u = _probe(P)
    X = _np(s.guess_features(u))
    fhat = G.nodal_load(P)
    Xo = np.stack([G.PatchGeometry(S, i).features(u, fhat) for i in range(S.n_sub)])
    for sl in (slice(0, 64), slice(64, 320)):
        scale = np.abs(Xo[:, sl]).max()
        assert np.abs(X[:, sl] - Xo[:, sl]).max() <= 2e-6 * scale


def test_lift_matches_oracle():
    case = _case()
    P = P1Problem(case)
    S = Schwarz(P, "one_level")
    s = _solver(case)
    u = _probe(P, 2)
    coef = (0.01 * np.random.default_rng(3).standard_normal((S.n_sub, 256))).astype(np.float32)
    x = _np(s.guess_lift(u, coef))
    ref = np.concatenate([
        G.PatchGeometry(S, i).lift(u, coef[i].astype(np.float64), S.subs[i]["dirV"],
                                   P.dir_value[S.subs[i]["V"]])
        for i in range(S.n_sub)])
    assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()


def test_captured_pairs_match_oracle():
    case = _case()
    P = P1Problem(case)
    S = Schwarz(P, "one_level")
    s = _solver(case, coupling="one_level")
    u = _probe(P, 4)
    s.guess_capture(100)
    s.precond_residual(u)
    X, T = s.guess_captured()
    X, T = _np(X), _np(T)
    assert X.shape == (S.n_sub, 320) and T.shape == (S.n_sub, 256)
    S.evaluate(u)
    fhat = G.nodal_load(P)
    geos = [G.PatchGeometry(S, i) for i in range(S.n_sub)]
    Xo = np.stack([g.features(u, fhat) for g in geos])
    To = np.stack([g.target(u, sol["x"]) for g, sol in zip(geos, S.state["sols"])])
    assert np.abs(X - Xo).max() <= 2e-6 * np.abs(Xo).max()
    assert np.abs(T - To).max() <= 2e-6 * np.abs(To).max()
    # capacity bounds the store: a second evaluation appends, a third stops at 2.5 batches
    s.guess_capture(int(2.5 * S.n_sub))
    for _ in range(3):
        s.precond_residual(u)
    X2, _ = s.guess_captured()
    assert X2.shape[0] == int(2.5 * S.n_sub)


def test_forward_matches_oracle_with_bf16_weights():
    case = _case()
    s = _solver(case)
    params = synth.mlp_init(3)
    norm = _norm(5)
    s.guess_set_model(params, norm)
    X, _ = synth.mlp_batch(4, 300)          # ragged against the 64-row tiles
    Y = _np(s.guess_predict(X))
    xm, xs, ym, ys = norm[:320], norm[320:640], norm[640:896], norm[896:]
    y, _, _ = G.forward(G.bf16_round(params), (X - xm) / xs)
    Yo = y * ys + ym
    assert np.abs(Y - Yo).max() <= 2e-2 * np.abs(Yo).max()
    p2, n2 = s.guess_get_model()
    np.testing.assert_array_equal(p2, params)
    np.testing.assert_array_equal(n2, norm)


def test_gradient_matches_oracle():
    case = _case()
    s = _solver(case)
    params = synth.mlp_init(8)
    norm = _norm(9)
    s.guess_set_model(params, norm)
    X, T = synth.mlp_batch(10, 200)
    g, loss = s.guess_loss_grad(X, T)
    g = _np(g).astype(np.float64)
    xm, xs, ym, ys = norm[:320], norm[320:640], norm[640:896], norm[896:]
    lo, go = G.loss_grad(params.astype(np.float64), (X - xm) / xs, (T - ym) / ys)
    cos = g @ go / (np.linalg.norm(g) * np.linalg.norm(go))
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    assert cos >= 0.999 and rel <= 3e-2, (cos, rel)
    assert abs(loss - lo) <= 1e-2 * lo


def test_adam_first_step_follows_gradient_sign():
    """One Adam step from zero moments moves each weight by lr g/(|g|+eps):
    -lr sign(g) wherever the gradient is well above its rounding error."""
    case = _case()
    s = _solver(case)
    params = synth.mlp_init(11)
    norm = _norm(12)
    s.guess_set_model(params, norm)
    X, T = synth.mlp_batch(13, 128)
    xm, xs, ym, ys = norm[:320], norm[320:640], norm[640:896], norm[896:]
    _, go = G.loss_grad(params.astype(np.float64), (X - xm) / xs, (T - ym) / ys)
    lr = 1e-3
    st = s.guess_train(X, T, epochs=1, batch=128, lr=lr, fit_norm=False)
    assert st["steps"] == 1
    w1, n1 = s.guess_get_model()
    np.testing.assert_array_equal(n1, norm)
    step = (w1.astype(np.float64) - params) / lr
    big = np.abs(go) >= 0.05 * np.abs(go).max()
    assert big.sum() > 500
    assert np.abs(step[big] + np.sign(go[big])).max() <= 2e-3


def test_learned_start_keeps_the_solution():
    """Any network leaves T_i(u) and the outer iteration unchanged up to the
    stopping tolerance; every local solve reports how it started."""
    case = _case()
    P = P1Problem(case)
    S = Schwarz(P, "additive")
    u = _probe(P, 6) + 0.5 * S.solve()[0]
    Fx_ref = S.evaluate(u)
    s = _solver(case, coupling="additive")
    norm = np.concatenate([np.zeros(320), np.ones(320), np.zeros(256),
                           np.full(256, 1e-3)]).astype(np.float32)
    s.guess_set_model(synth.mlp_init(7), norm)
    s.guess_enable(True)
    Fx = _np(s.precond_residual(u))
    assert np.abs(Fx - Fx_ref).max() <= 1e-10 * np.abs(Fx_ref).max()
    u_ref, st_ref = S.solve()
    uu, st, rc = s.solve()
    assert rc == 0 and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(_np(uu) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)
    # evaluations after one with almost no accepted predictions skip inference
    assert 0 < st["guess_used"] + st["guess_fallback"] <= st["local_solves"]


def _strong_case(seed, n=32):
    m = synth.fourier_modes(seed, amp=300.0)
    return synth.diffusion_case(n, n, synth.even_cuts(n, 4), synth.even_cuts(n, 4), 2,
                                two_level=True,
                                forcing=lambda p: synth.fourier_eval(p, m),
                                name=f"strong_{seed}")


def test_trained_network_saves_inner_iterations():
    """Strongly nonlinear forcing (|u| ~ 1): train on local solves captured
    from 40 forcings, then solve a held-out forcing with and without the
    network.  Its starts must save inner iterations at u = 0 and leave the
    outer iteration and the solution unchanged."""
    base = _strong_case(5000)
    s = _solver(base)
    s.guess_capture(20000)
    for seed in range(5000, 5040):
        s.set_load(_strong_case(seed)["elem_load"])
        _, st, rc = s.solve()
        assert rc == 0
    X, T = s.guess_captured()
    n = X.shape[0]
    assert n >= 40 * 16
    s.guess_set_model(synth.mlp_init(1))
    order = synth.epoch_orders(2, n, 150)
    tr = s.guess_train(X, T, epochs=150, batch=128, lr=1e-3, order=order, cosine=True)
    assert tr["final_loss"] < 0.2 * tr["epoch_loss"][0], tr["epoch_loss"][::25]
    held = _strong_case(6000)
    s.set_load(held["elem_load"])
    s.guess_enable(False)
    u0, st0, _ = s.solve()
    s.precond_residual(np.zeros(len(held["xy"])))
    its_plain = s.inner_iterations()
    s.guess_enable(True)
    u1, st1, rc = s.solve()
    assert rc == 0 and st1["outer_its"] == st0["outer_its"]
    assert np.linalg.norm(_np(u1 - u0)) <= 1e-10 * np.linalg.norm(_np(u0))
    s.precond_residual(np.zeros(len(held["xy"])))
    its_learned = s.inner_iterations()
    print("inner its at u=0 plain", its_plain.sum(), "learned", its_learned.sum(),
          "solve plain", st0["inner_its_total"], "learned", st1["inner_its_total"],
          "used", st1["guess_used"], "fallback", st1["guess_fallback"])
    assert its_learned.sum() < its_plain.sum()
