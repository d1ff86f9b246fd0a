"""Learned initial guess on the GPU: the network's kernels against the oracle
(forward and every gradient bit-exact on integer data, within the bf16
bound on random data), Adam, restriction and interpolation, the fallback
start, and what a network trained by the library's own kernels gains over
the zero start on held-out instances."""
import numpy as np
import pytest
import torch

from oracle import cn_oracle as O
from oracle import mlp_oracle as MO
from paper_2401_16113_amd import binding as B
from paper_2401_16113_amd import warmstart as WS
from paper_2401_16113_amd import workloads as W
from gpu_helpers import T, banner, rel_inf, solver

pytestmark = pytest.mark.gpu


def dev():
    return torch.device("cuda:0")


def f32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=dev())


def identity_norm(net):
    net.set_normalization(f32(np.zeros(net.n_in)), f32(np.ones(net.n_in)),
                          f32(np.zeros(net.n_out)), f32(np.ones(net.n_out)))


def signed_permutation(rng, n):
    P = np.zeros((n, n))
    P[np.arange(n), rng.permutation(n)] = rng.choice([-1.0, 1.0], size=n)
    return P


def integer_net(seed, n_in, w, n_out):
    """Parameters and inputs whose every product and partial sum (forward
    and backward) is exact in bf16 operands and float32 accumulation: entries
    in {-1, 0, 1}, hidden layers 2 and 3 signed permutations (so hidden
    values stay <= n_in + 4 in magnitude, well inside bf16's exact integers),
    small integer biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.integers(-1, 2, size=(w, n_in)).astype(np.float64)
    W2 = signed_permutation(rng, w)
    W3 = signed_permutation(rng, w)
    W4 = rng.integers(-1, 2, size=(n_out, w)).astype(np.float64)
    bs = [rng.integers(-2, 3, size=k).astype(np.float64) for k in (w, w, w, n_out)]
    p = np.concatenate([W1.ravel(), bs[0], W2.ravel(), bs[1], W3.ravel(), bs[2], W4.ravel(),
                        bs[3]])
    return p


@pytest.mark.parametrize("n_in,w,n_out,Bn", [(67, 96, 200, 37), (67, 128, 256, 64),
                                             (5, 64, 8192, 3)])
def test_forward_bit_exact_on_integer_data(n_in, w, n_out, Bn):
    banner(f"mlp forward exact {n_in}x{w}x{n_out} batch {Bn}")
    p = integer_net(1, n_in, w, n_out)
    X = np.random.default_rng(2).integers(-1, 2, size=(Bn, n_in)).astype(np.float64)
    net = B.Mlp(n_in, w, n_out, max(Bn, 8))
    assert net.num_params == MO.num_params(n_in, w, n_out)
    net.set_params(f32(p))
    identity_norm(net)
    Y = torch.empty((Bn, n_out), dtype=torch.float32, device=dev())
    net.forward(f32(X), Y)
    ref = MO.predict(p, X, n_in, w, n_out)
    assert np.array_equal(Y.cpu().numpy().astype(np.float64), ref)
    net.close()


def test_gradients_bit_exact_on_integer_data():
    """Every backward product (transposed operands, ReLU masks, bias sums)
    against the oracle's chain rule; targets differ from the outputs by -1, 0
    or 1 and B * n_out is a power of two, so the scaled error is exact."""
    n_in, w, n_out, Bn = 67, 96, 256, 32
    banner("mlp gradients exact")
    p = integer_net(3, n_in, w, n_out)
    rng = np.random.default_rng(4)
    X = rng.integers(-1, 2, size=(Bn, n_in)).astype(np.float64)
    z = MO.predict(p, X, n_in, w, n_out)
    Yt = z + rng.integers(-1, 2, size=z.shape)
    net = B.Mlp(n_in, w, n_out, Bn)
    net.set_params(f32(p))
    identity_norm(net)
    g = torch.empty(net.num_params, dtype=torch.float32, device=dev())
    loss = torch.empty(1, dtype=torch.float32, device=dev())
    net.loss_grad(f32(X), f32(Yt), grads=g, loss=loss)
    L, gref = MO.loss_grad(p, X, Yt, n_in, w, n_out)
    assert float(loss.cpu()) == L
    gg = g.cpu().numpy().astype(np.float64)
    assert np.count_nonzero(gref) > 1000
    assert np.array_equal(gg, gref), np.flatnonzero(gg != gref)[:10]
    net.close()


def _random_case(seed, n_in=67, w=128, n_out=256, Bn=64):
    rng = np.random.default_rng(seed)
    p = WS.init_params(seed, n_in, w, n_out).astype(np.float64)
    # a trained-like last layer (the initialiser shrinks it)
    k = MO.num_params(n_in, w, n_out) - n_out - n_out * w
    p[k:k + n_out * w] *= 10.0
    p[-n_out:] = rng.standard_normal(n_out) * 0.1
    X = rng.standard_normal((Bn, n_in)) * rng.uniform(0.1, 2.0, n_in) + rng.standard_normal(n_in)
    Yt = rng.standard_normal((Bn, n_out))
    norm = dict(in_mu=X.mean(0), in_sd=X.std(0), out_mu=rng.standard_normal(n_out) * 0.1,
                out_sd=rng.uniform(0.5, 2.0, n_out))
    # float32 values as the device holds them
    norm = {k: v.astype(np.float32).astype(np.float64) for k, v in norm.items()}
    return (p.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64),
            Yt.astype(np.float32).astype(np.float64), norm, (n_in, w, n_out))


@pytest.mark.parametrize("seed", [10, 11])
def test_gradients_match_oracle_on_random_data(seed):
    """Random data, two references.  (1) The oracle with every product operand
    rounded to bf16 as the kernels stage them: what remains is float32 versus
    float64 accumulation (~1e-6 relative per sum) and the rare operand that
    falls on the other side of a bf16 rounding boundary (one bf16 step,
    2^-8 relative, in isolated entries): relative Frobenius error <= 1e-3
    per tensor.  (2) The plain float64 oracle on the same bf16 weights,
    which shows the price of bf16 operands themselves: 2^-9 relative
    rounding per operand through four layers and back, ~5e-2 measured on the
    first layer's weights; bound 1e-1 with the direction kept (cosine >=
    0.995)."""
    banner(f"mlp gradients random seed {seed}")
    p, X, Yt, norm, dims = _random_case(seed)
    n_in, w, n_out = dims
    net = B.Mlp(n_in, w, n_out, X.shape[0])
    net.set_params(f32(p))
    net.set_normalization(f32(norm["in_mu"]), f32(norm["in_sd"]), f32(norm["out_mu"]),
                          f32(norm["out_sd"]))
    g = torch.empty(net.num_params, dtype=torch.float32, device=dev())
    loss = torch.empty(1, dtype=torch.float32, device=dev())
    net.loss_grad(f32(X), f32(Yt), grads=g, loss=loss)
    gg = g.cpu().numpy().astype(np.float64)
    shapes = MO.param_shapes(*dims)
    Lb, gb = MO.loss_grad(p, X, Yt, *dims, **norm, rnd=MO.bf16)
    assert abs(float(loss.cpu()) - Lb) <= 1e-5 * Lb
    L64, g64 = MO.loss_grad(MO.bf16(p), X, Yt, *dims, **norm)
    off = 0
    for s in shapes:
        k = int(np.prod(s))
        a = gg[off:off + k]
        for ref, tol, ctol in ((gb[off:off + k], 1e-3, 1 - 1e-6), (g64[off:off + k], 1e-1, 0.995)):
            rel = np.linalg.norm(a - ref) / np.linalg.norm(ref)
            cos = a @ ref / (np.linalg.norm(a) * np.linalg.norm(ref))
            assert rel <= tol and cos >= ctol, (s, tol, rel, cos)
        off += k
    # forward output on the same two premises (an activation that rounds to
    # the neighbouring bf16 value moves a whole output row by one bf16 step
    # of its contribution, so the first bound is 1e-3 too)
    Y = torch.empty((X.shape[0], n_out), dtype=torch.float32, device=dev())
    net.forward(f32(X), Y)
    y = Y.cpu().numpy()
    yb = MO.predict(p, X, *dims, **norm, rnd=MO.bf16)
    assert np.linalg.norm(y - yb) <= 1e-3 * np.linalg.norm(yb)
    y64 = MO.predict(MO.bf16(p), X, *dims, **norm)
    assert np.linalg.norm(y - y64) <= 2e-2 * np.linalg.norm(y64)
    net.close()


def test_adam_matches_oracle():
    banner("mlp adam")
    p, X, Yt, norm, dims = _random_case(12, w=64, n_out=128, Bn=32)
    net = B.Mlp(*dims, 32)
    net.set_params(f32(p))
    identity_norm(net)
    g = torch.empty(net.num_params, dtype=torch.float32, device=dev())
    m = np.zeros(p.size)
    v = np.zeros(p.size)
    pref = p.copy()
    lr = 1e-3
    for step in range(1, 4):
        net.loss_grad(f32(X), f32(Yt), grads=g)
        gg = g.cpu().numpy().astype(np.float64)
        net.adam_step(lr)
        pref, m, v = MO.adam_step(pref, gg, m, v, step, lr)
        out = torch.empty_like(g)
        net.get_params(out)
        # each step moves a parameter by at most ~lr; float32 arithmetic of
        # the update is accurate to ~1e-6 lr
        assert np.max(np.abs(out.cpu().numpy() - pref)) <= 1e-5 * lr + 2e-7 * np.abs(pref).max()
        pref = out.cpu().numpy().astype(np.float64)
    net.close()


def test_training_reduces_loss():
    """A few hundred Adam steps of the library's kernels fit a smooth map."""
    banner("mlp training")
    rng = np.random.default_rng(13)
    n_in, n_out, count = 8, 256, 512
    Xh = rng.uniform(-1, 1, size=(count, n_in))
    grid = np.linspace(0, 1, n_out)
    Yh = np.sin(np.outer(Xh[:, 0] + 0.5 * Xh[:, 1], 3 * grid)) + np.outer(Xh[:, 2], grid ** 2)
    X, Y = f32(Xh), f32(Yh)
    net = B.Mlp(n_in, 128, n_out, 64)
    net.set_params(torch.as_tensor(WS.init_params(0, n_in, 128, n_out), device=dev()))
    net.set_normalization(*WS.normalization(X, Y))
    loss = torch.empty(1, dtype=torch.float32, device=dev())
    first = None
    for ep in range(60):
        tot = 0.0
        for i in range(count // 64):
            net.loss_grad(X[i * 64:(i + 1) * 64], Y[i * 64:(i + 1) * 64], loss=loss)
            net.adam_step(2e-3)
            tot += float(loss.cpu())
        if first is None:
            first = tot
    assert tot < 0.05 * first, (first, tot)
    net.close()


def test_mlp_rejects_bad_calls():
    net = B.Mlp(4, 8, 4, 16)
    X = torch.zeros((17, 4), dtype=torch.float32, device=dev())
    Y = torch.zeros((17, 4), dtype=torch.float32, device=dev())
    with pytest.raises(B.CnError, match="max_batch"):
        net.forward(X, Y)
    with pytest.raises(B.CnError, match="Adam"):
        net.adam_step(-1.0)
    net.close()


@pytest.mark.parametrize("nx,nt", [(255, 64), (511, 128), (2047, 512)])
def test_restrict_and_interpolate_match_oracle(nx, nt):
    banner(f"restrict/interpolate {nx}x{nt}")
    rng = np.random.default_rng(nx + nt)
    count = 3
    coarse = rng.standard_normal((count, 64 * 128)).astype(np.float32)
    u0 = rng.standard_normal((count, nx))
    gl = rng.standard_normal((count, nt))
    gr = rng.standard_normal((count, nt))
    scale = rng.uniform(0.5, 2.0, count)
    x0 = torch.empty(count * nx * nt, dtype=torch.float64, device=dev())
    B.ws_interpolate(f32(coarse), count, nx, nt, T(u0.ravel()), T(gl.ravel()), T(gr.ravel()),
                     T(scale), x0)
    xs = x0.cpu().numpy().reshape(count, -1)
    for q in range(count):
        ref = MO.interpolate(coarse[q], nx, nt, u0[q], gl[q], gr[q], scale[q])
        assert np.max(np.abs(xs[q] - ref)) <= 1e-14 * np.max(np.abs(ref))
    xr = rng.standard_normal(count * nx * nt)
    inv = rng.uniform(0.5, 2.0, count)
    c = torch.empty((count, 8192), dtype=torch.float32, device=dev())
    B.ws_restrict(T(xr), count, nx, nt, T(inv), c)
    cs = c.cpu().numpy()
    for q in range(count):
        ref = MO.restrict(xr[q * nx * nt:(q + 1) * nx * nt], nx, nt, inv[q])
        assert np.array_equal(cs[q], ref.ravel())


def test_restrict_interpolate_reject_incompatible_grids():
    c = torch.zeros(8192, dtype=torch.float32, device=dev())
    x = torch.zeros(127 * 64, dtype=torch.float64, device=dev())
    one = torch.ones(1, dtype=torch.float64, device=dev())
    with pytest.raises(B.CnError, match="multiple of 128"):
        B.ws_restrict(x, 1, 127, 64, one, c)
    x = torch.zeros(255 * 60, dtype=torch.float64, device=dev())
    with pytest.raises(B.CnError, match="multiple of 64"):
        B.ws_restrict(x, 1, 255, 60, one, c)


def test_fallback_start_rejects_a_bad_guess():
    """use_x0 = 2: a guess with ||b - M x0|| >= ||b|| is replaced by zero
    (same iterations and result as the zero start), a good one is kept."""
    banner("fallback start")
    inst = W.config2(nx=511, nt=128, pc_prec="fp32")
    s = solver(inst, m_max=20)
    b = torch.empty(inst.n, dtype=torch.float64, device=dev())
    s.rhs(T(inst.u0), T(inst.f.reshape(-1)), b)
    x_zero = torch.zeros_like(b)
    r0 = s.solve(b, x_zero, m=20, rtol=1e-10)
    bad = T(np.random.default_rng(0).standard_normal(inst.n))
    r_bad = s.solve(b, bad, m=20, rtol=1e-10, use_x0=2)
    assert r_bad.x0_rejected == 1 and r_bad.iters == r0.iters
    assert rel_inf(bad.cpu().numpy(), x_zero.cpu().numpy()) <= 1e-12
    # plain use of the same bad guess is not rejected
    bad2 = T(np.random.default_rng(0).standard_normal(inst.n))
    r_plain = s.solve(b, bad2, m=20, rtol=1e-10, use_x0=1)
    assert r_plain.x0_rejected == 0 and r_plain.relres_true <= 1e-10
    # a good guess (the solution perturbed by 1e-3 relative) is kept
    good = x_zero.clone() * (1 + 1e-3 * T(np.random.default_rng(1).standard_normal(inst.n)))
    r_good = s.solve(b, good, m=20, rtol=1e-10, use_x0=2)
    assert r_good.x0_rejected == 0 and r_good.iters < r0.iters
    assert r_good.relres_true <= 1e-10
    s.close()


def test_learned_warm_start_gains_over_zero_start():
    """Data from plain solves, training on the GPU, then held-out instances
    solved from the network's guess and from zero: the warm start needs
    fewer iterations in total, every instance reaches the true relative
    residual 1e-8, and every solution matches the exact CN solution (both
    forms with error-controlled stopping at half the 1e-7 bar)."""
    banner("learned warm start 2047x512")
    torch.manual_seed(0)
    ptrain = W.config4_params(768, seed=40)
    ptest = W.config4_params(64, seed=41)
    X, Y, worst = WS.generate(ptrain, chunk=128)
    assert worst <= 1e-8
    net, hist = WS.train(X, Y, epochs=150, batch=128, lr=2e-3, seed=0)
    assert hist[-1] < 0.05 * hist[0], hist[::25]
    fb = WS.family_batch(ptest)
    _, tz, pz, _ = WS.solve_family(fb, err_tol=5e-8)
    x0, coarse = WS.initial_guess(net, fb)
    xw, tw, pw, _ = WS.solve_family(fb, x0=x0, warm=True, err_tol=5e-8)
    assert tz.status == B.CN_OK and tw.status == B.CN_OK
    iz = sum(r.iters for r in pz)
    iw = sum(r.iters for r in pw)
    rej = sum(r.x0_rejected for r in pw)
    print(f"zero start {iz} iterations, warm start {iw}, rejected guesses {rej}", flush=True)
    assert iw < iz and rej < len(pw) // 4
    assert all(r.relres_true <= 1e-8 for r in pw)
    # every held-out solution against the oracle's CN time stepping, to the
    # bar for warm-started mixed-precision forms (1e-7, relative max-norm)
    xs = xw.cpu().numpy()
    n = fb.nx * fb.nt
    worst = 0.0
    for q in range(fb.count):
        (_, lo, di, up, u0, f_col, _, _), _, _ = W.config4_rows(ptest[q], fb.nx, fb.nt)
        u = O.sequential_cn_banded(lo, di, up, float(ptest[q][3]), fb.nt, u0, f_col=f_col)
        worst = max(worst, rel_inf(xs[q * n:(q + 1) * n], u))
    print(f"max error of the warm-started solutions {worst:.2e}", flush=True)
    assert worst <= 1e-7
    net.close()


def test_predict_equals_forward_then_interpolate():
    """cn_ws_predict (chunked forward pass + interpolation in one call) gives
    bit for bit what the two separate calls give."""
    banner("ws predict")
    rng = np.random.default_rng(30)
    count, nx, nt = 5, 255, 64
    net = B.Mlp(67, 64, 8192, 2)   # max_batch 2: three chunks
    net.set_params(torch.as_tensor(WS.init_params(3, 67, 64, 8192), device=dev()))
    X = f32(rng.standard_normal((count, 67)))
    u0 = T(rng.standard_normal(count * nx))
    gl = T(rng.standard_normal(count * nt))
    gr = T(rng.standard_normal(count * nt))
    scale = T(rng.uniform(0.5, 2.0, count))
    coarse = torch.empty((count, 8192), dtype=torch.float32, device=dev())
    x0 = torch.empty(count * nx * nt, dtype=torch.float64, device=dev())
    net.predict(X, nx, nt, u0, gl, gr, scale, coarse, x0)
    c2 = torch.empty_like(coarse)
    for c0 in range(0, count, 2):
        net.forward(X[c0:c0 + 2], c2[c0:c0 + 2])
    x2 = torch.empty_like(x0)
    B.ws_interpolate(c2, count, nx, nt, u0, gl, gr, scale, x2)
    torch.cuda.synchronize()
    assert torch.equal(coarse, c2) and torch.equal(x0, x2)
    with pytest.raises(B.CnError, match="128 x 64"):
        B.Mlp(67, 64, 100, 2).predict(X, nx, nt, u0, gl, gr, scale, coarse, x0)
    net.close()


def test_predict_batch_equals_per_instance_predict():
    """cn_ws_predict_batch on an uneven batch (N_x in {255, 511, 1023}, N_t in
    {64, 128, 256}) gives, instance by instance, bit for bit what
    cn_ws_predict gives on each instance alone."""
    banner("ws predict over an uneven batch")
    rng = np.random.default_rng(31)
    shapes = [(255, 64), (1023, 128), (511, 256), (255, 128), (511, 64)]
    insts = [W.make_instance(nx, nt, T=1.0, r=0.03, K=1.0,
                             sigma_fn=lambda x: 0.2 + 0.0 * x, alpha=0.01) for nx, nt in shapes]
    bt = B.Batch([dict(a_lo=T(i.a_lo), a_di=T(i.a_di), a_up=T(i.a_up), nt=i.nt, T=i.T,
                       alpha=i.alpha, m_max=4) for i in insts], pc_prec="fp32")
    count = len(shapes)
    net = B.Mlp(67, 64, 8192, 2)   # max_batch 2: three chunks
    net.set_params(torch.as_tensor(WS.init_params(5, 67, 64, 8192), device=dev()))
    X = f32(rng.standard_normal((count, 67)))
    u0 = T(np.concatenate([rng.standard_normal(nx) for nx, _ in shapes]))
    gl = T(np.concatenate([rng.standard_normal(nt) for _, nt in shapes]))
    gr = T(np.concatenate([rng.standard_normal(nt) for _, nt in shapes]))
    scale = T(rng.uniform(0.5, 2.0, count))
    coarse = torch.empty((count, 8192), dtype=torch.float32, device=dev())
    x0 = torch.full((bt.n,), np.nan, dtype=torch.float64, device=dev())
    net.predict_batch(X, bt, u0, gl, gr, scale, coarse, x0)
    uo = go = 0
    for q, (nx, nt) in enumerate(shapes):
        c1 = torch.empty((1, 8192), dtype=torch.float32, device=dev())
        x1 = torch.empty(nx * nt, dtype=torch.float64, device=dev())
        net.predict(X[q:q + 1].contiguous(), nx, nt, u0[uo:uo + nx], gl[go:go + nt],
                    gr[go:go + nt], scale[q:q + 1], c1, x1)
        torch.cuda.synchronize()
        assert torch.equal(coarse[q:q + 1], c1)
        assert torch.equal(x0[bt.offsets[q]:bt.offsets[q + 1]], x1), q
        uo += nx
        go += nt
    # an instance whose grid does not fit the coarse grid is refused
    bad = B.Batch([dict(a_lo=T(insts[0].a_lo), a_di=T(insts[0].a_di), a_up=T(insts[0].a_up),
                        nt=32, T=1.0, alpha=0.01, m_max=4)], pc_prec="fp32")
    with pytest.raises(B.CnError, match="multiple of 64"):
        net.predict_batch(X[:1].contiguous(), bad, u0, gl, gr, scale, coarse, x0)
    net.close()
