"""Pins of the warm-start oracle (oracle/mlp_oracle.py) against facts that do
not come from the oracle itself: central finite differences of the loss,
the closed form of Adam under a constant gradient, exact reproduction of
bilinear functions by the interpolation and the coarse values returned by
restricting an interpolant.  Each pin also fails on a planted mistake."""
import numpy as np
import pytest

from oracle import mlp_oracle as MO


def _net(seed, n_in=5, w=7, n_out=3, B=6):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(MO.num_params(n_in, w, n_out)) * 0.6
    X = rng.standard_normal((B, n_in)) * 2.0 + 1.0
    Y = rng.standard_normal((B, n_out)) * 3.0 - 0.5
    norm = dict(in_mu=rng.standard_normal(n_in), in_sd=rng.uniform(0.5, 2.0, n_in),
                out_mu=rng.standard_normal(n_out), out_sd=rng.uniform(0.5, 2.0, n_out))
    return p, X, Y, norm, (n_in, w, n_out)


def _min_abs_preact(p, X, dims, norm):
    n_in, w, n_out = dims
    W1, b1, W2, b2, W3, b3, W4, b4 = MO.unflatten(p, *dims)
    xn = (X - norm["in_mu"]) / norm["in_sd"]
    a1 = xn @ W1.T + b1
    a2 = np.maximum(a1, 0) @ W2.T + b2
    a3 = np.maximum(a2, 0) @ W3.T + b3
    return min(np.abs(a1).min(), np.abs(a2).min(), np.abs(a3).min())


def _fd_grad(p, X, Y, dims, norm, h=1e-6):
    g = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        g[i] = (MO.loss(p + e, X, Y, *dims, **norm) - MO.loss(p - e, X, Y, *dims, **norm)) / (2 * h)
    return g


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    p, X, Y, norm, dims = _net(seed)
    # finite differences are exact up to O(h^2) only away from ReLU kinks
    assert _min_abs_preact(p, X, dims, norm) > 1e-4
    L, g = MO.loss_grad(p, X, Y, *dims, **norm)
    assert L == pytest.approx(MO.loss(p, X, Y, *dims, **norm), rel=1e-15)
    fd = _fd_grad(p, X, Y, dims, norm)
    assert np.max(np.abs(g - fd)) <= 1e-7 * max(1.0, np.max(np.abs(fd)))
    # some ReLUs are inactive, so the kink handling is exercised
    assert np.any(g == 0.0)


def test_planted_gradient_mistake_is_caught():
    p, X, Y, norm, dims = _net(0)
    L, g = MO.loss_grad(p, X, Y, *dims, **norm)
    fd = _fd_grad(p, X, Y, dims, norm)
    # a bias gradient with a dropped factor 2 (mean vs sum mix-up)
    n_in, w, n_out = dims
    off_b4 = MO.num_params(n_in, w, n_out) - n_out
    bad = g.copy()
    bad[off_b4:] *= 0.5
    assert np.max(np.abs(bad - fd)) > 1e-3


def test_loss_is_mean_squared_standardised_error():
    # single sample, identity-like network: W = 0, b4 chosen -> z = b4
    dims = (2, 3, 2)
    p = np.zeros(MO.num_params(*dims))
    p[-2:] = [1.0, -2.0]
    X = np.array([[0.3, 0.4]])
    Y = np.array([[5.0, 1.0]])
    mu, sd = np.array([1.0, 3.0]), np.array([2.0, 4.0])
    # standardised targets (2, -0.5); errors (-1, -1.5); mean square 1.625
    assert MO.loss(p, X, Y, *dims, out_mu=mu, out_sd=sd) == pytest.approx(1.625, rel=1e-15)
    y = MO.predict(p, X, *dims, out_mu=mu, out_sd=sd)
    assert np.allclose(y, [[3.0, -5.0]], rtol=0, atol=1e-15)


def test_adam_constant_gradient_closed_form():
    # With a constant gradient g the bias-corrected moments are exactly g and
    # g^2 at every step, so each update is -lr * g / (|g| + eps).
    rng = np.random.default_rng(4)
    g = rng.standard_normal(50)
    p0 = rng.standard_normal(50)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    lr, eps = 1e-2, 1e-8
    for step in range(1, 6):
        p, m, v = MO.adam_step(p, g, m, v, step, lr, 0.9, 0.999, eps)
        expect = p0 - step * lr * g / (np.abs(g) + eps)
        assert np.allclose(p, expect, rtol=0, atol=1e-12)


def test_adam_bias_correction_matters():
    g = np.array([0.5, -2.0])
    p, m, v = MO.adam_step(np.zeros(2), g, np.zeros(2), np.zeros(2), 1, 0.1)
    # first step moves every parameter by lr in the direction of -sign(g)
    assert np.allclose(p, [-0.1, 0.1], atol=1e-8)
    # without bias correction the first step would be 0.1 * 0.1 g/(sqrt(0.001)|g|)
    assert not np.allclose(p, -0.1 * 0.1 * g / (np.sqrt(0.001) * np.abs(g)), atol=1e-3)


@pytest.mark.parametrize("nx,nt", [(255, 64), (511, 128), (2047, 512)])
def test_interpolation_reproduces_bilinear_functions(nx, nt):
    # f(x, t) = a + b x + c t + d x t sampled on the coarse grid, the
    # boundaries and the initial level is reproduced at every fine point
    a, b, c, d = 0.7, -0.3, 1.9, 0.45
    f = lambda x, t: a + b * x + c * t + d * x * t
    T = 1.0
    xc, tc, ic, kc = MO.coarse_positions(nx, nt, T)
    coarse = f(xc[None, :], tc[:, None]).astype(np.float32).astype(np.float64)
    # use float32-representable coarse values: compare against the bilinear
    # interpolant of exactly those values, built independently per point
    h = 6.0 / (nx + 1)
    xf = -3.0 + (np.arange(nx) + 1) * h
    tf = (np.arange(nt) + 1) * T / nt
    u0 = f(xf, 0.0)
    gl = f(-3.0, tf)
    gr = f(3.0, tf)
    out = MO.interpolate(coarse.astype(np.float32), nx, nt, u0, gl, gr).reshape(nt, nx)
    exact = f(xf[None, :], tf[:, None])
    # coarse values carry float32 rounding (relative 6e-8 of |f| <= 6)
    assert np.max(np.abs(out - exact)) < 1e-6
    exact64 = MO.interpolate(f(xc[None, :], tc[:, None]), nx, nt, u0, gl, gr).reshape(nt, nx)
    assert np.max(np.abs(exact64 - exact)) < 1e-12


def test_restriction_of_interpolant_returns_coarse_values():
    nx, nt = 511, 128
    rng = np.random.default_rng(7)
    coarse = rng.standard_normal((64, 128)).astype(np.float32)
    x = MO.interpolate(coarse, nx, nt, rng.standard_normal(nx), rng.standard_normal(nt),
                       rng.standard_normal(nt))
    assert np.array_equal(MO.restrict(x, nx, nt), coarse)
    # the coarse nodes sit at the fine points the kernels use
    xc, tc, ic, kc = MO.coarse_positions(nx, nt, 1.0)
    assert ic[0] == 1 and ic[-1] == nx - 2 and np.all(np.diff(ic) == 4)
    assert kc[0] == 1 and kc[-1] == nt - 1 and np.all(np.diff(kc) == 2)


def test_planted_interpolation_mistake_is_caught():
    # swapped boundary data would break bilinear reproduction (with a coarse
    # ratio of 4 the first and last fine nodes lie in the boundary half-cells)
    nx, nt = 511, 128
    f = lambda x, t: 1.0 + 2.0 * x + 3.0 * t
    xc, tc, ic, kc = MO.coarse_positions(nx, nt, 1.0)
    h = 6.0 / (nx + 1)
    xf = -3.0 + (np.arange(nx) + 1) * h
    tf = (np.arange(nt) + 1) / nt
    good = MO.interpolate(f(xc[None, :], tc[:, None]), nx, nt, f(xf, 0.0), f(-3.0, tf),
                          f(3.0, tf))
    bad = MO.interpolate(f(xc[None, :], tc[:, None]), nx, nt, f(xf, 0.0), f(3.0, tf),
                         f(-3.0, tf))
    exact = f(xf[None, :], tf[:, None]).reshape(-1)
    assert np.max(np.abs(good - exact)) < 1e-12
    assert np.max(np.abs(bad - exact)) > 1.0


def test_bf16_rounding_matches_its_definition():
    # 8 significant bits, ties to even: 1 + 2^-8 is a tie between 1 and
    # 1 + 2^-7 -> 1 (even); 1 + 3*2^-8 ties between 1 + 2^-7 and 1 + 2^-6 ->
    # 1 + 2^-6; 1 + 2^-8 + 2^-20 rounds up
    a = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -20, 257.0, -3.0])
    assert np.array_equal(MO.bf16(a), [1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7, 256.0, -3.0])


def test_operand_rounding_is_exact_on_small_integers_and_visible_otherwise():
    p, X, Y, norm, dims = _net(5)
    Pi = np.rint(p * 2)
    Xi = np.rint(X)
    Li, gi = MO.loss_grad(Pi, Xi, np.rint(Y), *dims)
    Lr, gr = MO.loss_grad(Pi, Xi, np.rint(Y), *dims, rnd=MO.bf16)
    # integer operands below 256 are bf16 numbers, dz = 2 d / (B n_out)
    # with B n_out = 18 is not: compare the forward pass only
    zi, _ = MO.forward(Pi, Xi, *dims)
    zr, _ = MO.forward(Pi, Xi, *dims, rnd=MO.bf16)
    assert np.array_equal(zi, zr)
    z1, _ = MO.forward(p, X, *dims, **{k: norm[k] for k in ("in_mu", "in_sd")})
    z2, _ = MO.forward(p, X, *dims, **{k: norm[k] for k in ("in_mu", "in_sd")}, rnd=MO.bf16)
    rel = np.linalg.norm(z1 - z2) / np.linalg.norm(z1)
    assert 1e-4 < rel < 2e-2
