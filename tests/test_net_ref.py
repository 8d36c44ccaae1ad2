"""Pins of the FP64 reference of the learned-guess network (oracle/net_ref.py).

Each test checks the reference against something other than itself: a
library routine (scipy's correlation, torch's bfloat16 conversion and
autograd), finite differences, or a closed form of Adam.
"""
import numpy as np
import pytest

from oracle import net_ref as R
from paper_1904_08510_amd import workloads as W


def small_params(seed=0, scale=1.0):
    ps = R.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    return [(Wt * scale, rng.standard_normal(b.shape) * 0.05) for Wt, b in ps]


def test_conv_matches_scipy_correlate():
    from scipy.signal import correlate
    rng = np.random.default_rng(1)
    x = rng.standard_normal((37, 3))
    Wt = rng.standard_normal((4, 5, 3))
    b = rng.standard_normal(4)
    y = R.conv(x, Wt, b)
    for co in range(4):
        ref = np.full(37, b[co])
        for ci in range(3):
            # y[i] = sum_j W[j] x[i + j - 2]: 'same' cross-correlation, zero padding
            ref += correlate(x[:, ci], Wt[co, :, ci], mode="same", method="direct")
        np.testing.assert_allclose(y[:, co], ref, rtol=1e-12, atol=1e-12)


def test_conv_edges_are_zero_padded():
    x = np.zeros((6, 1))
    x[0, 0] = 1.0
    Wt = np.zeros((1, 5, 1))
    Wt[0, 4, 0] = 1.0   # tap 4 reads cell i + 2
    y = R.conv(x, Wt, np.zeros(1))
    assert y[:, 0].tolist() == [0, 0, 0, 0, 0, 0]   # cell 0 is read by no output (i + 2 = 0 -> i = -2)
    Wt[0, 4, 0] = 0.0
    Wt[0, 0, 0] = 1.0   # tap 0 reads cell i - 2
    y = R.conv(x, Wt, np.zeros(1))
    assert y[:, 0].tolist() == [0, 0, 1, 0, 0, 0]


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.uniform(-8, 8, 20000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 65504.0, 3.0e38]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(R.bf16(x), ref)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    params = small_params(3)
    xs = [rng.standard_normal((n, 8)) for n in (7, 13)]
    ts = [rng.standard_normal((n, 2)) for n in (7, 13)]
    loss, grads = R.loss_and_grad(params, xs, ts)
    p0 = R.flat(params)
    g = R.flat(grads)
    idx = np.concatenate([rng.choice(R.nparams(), 60, replace=False),
                          [0, R.nparams() - 1, R.nparams() - 3]])
    h = 1e-6
    for i in idx:
        pp, pm = p0.copy(), p0.copy()
        pp[i] += h
        pm[i] -= h
        lp, _ = R.loss_and_grad(R.unflat(pp), xs, ts)
        lm, _ = R.loss_and_grad(R.unflat(pm), xs, ts)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (i, fd, g[i])


def test_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    params = small_params(4)
    xs = [rng.standard_normal((n, 8)) for n in (5, 40, 3)]
    ts = [rng.standard_normal((n, 2)) for n in (5, 40, 3)]
    loss, grads = R.loss_and_grad(params, xs, ts)
    tp = [(torch.tensor(Wt, requires_grad=True), torch.tensor(b, requires_grad=True)) for Wt, b in params]
    total = 0.0
    ncell = sum(x.shape[0] for x in xs)
    for x, t in zip(xs, ts):
        h = torch.tensor(x.T[None])
        for l, (Wt, b) in enumerate(tp):
            # torch conv1d is a cross-correlation: weight [cout, cin, k]
            h = torch.nn.functional.conv1d(h, Wt.permute(0, 2, 1), b, padding=2)
            if l < R.NLAYER - 1:
                h = torch.relu(h)
        total = total + ((h[0].T - torch.tensor(t)) ** 2).sum()
    total = total / ncell
    total.backward()
    assert abs(total.item() - loss) <= 1e-12 * abs(loss)
    for (Wt, b), (gW, gb) in zip(tp, grads):
        np.testing.assert_allclose(Wt.grad.numpy(), gW, rtol=1e-10, atol=1e-14)
        np.testing.assert_allclose(b.grad.numpy(), gb, rtol=1e-10, atol=1e-14)


def test_quantised_pass_stays_close_to_fp64():
    rng = np.random.default_rng(5)
    params = small_params(5)
    xs = [rng.standard_normal((50, 8))]
    ts = [rng.standard_normal((50, 2))]
    o64, _ = R.forward(params, xs[0])
    oq, _ = R.forward(params, xs[0], quant=True)
    assert np.linalg.norm(oq - o64) <= 0.05 * np.linalg.norm(o64)
    _, g64 = R.loss_and_grad(params, xs, ts)
    _, gq = R.loss_and_grad(params, xs, ts, quant=True)
    a, b = R.flat(g64), R.flat(gq)
    assert np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)) > 0.999


def test_adam_constant_gradient_closed_form():
    # with a constant gradient the bias-corrected moments are exactly g and
    # g^2, so every step moves each parameter by lr g / (|g| + eps)
    rng = np.random.default_rng(6)
    params = small_params(6)
    g = rng.standard_normal(R.nparams())
    grads = R.unflat(g)
    m = np.zeros(R.nparams())
    v = np.zeros(R.nparams())
    p = params
    lr, eps = 1e-3, 1e-8
    for step in range(1, 6):
        p, m, v = R.adam(p, grads, m, v, step, lr, eps=eps)
    expect = R.flat(params) - 5 * lr * g / (np.abs(g) + eps)
    np.testing.assert_allclose(R.flat(p), expect, rtol=1e-9, atol=1e-12)


def test_features_and_candidate_round_trip():
    col = W.flame_column(64, 300.0)
    ne_next = col.ne * 1.7 + 1e9
    phi_next = col.phi + 3.0
    s0, s1 = 0.1, 0.3
    t = R.targets(col, col.ne, col.phi, ne_next, phi_next, s0, s1)
    n2, p2 = R.candidate(col, col.ne, col.phi, t, s0, s1)
    # the targets are float32: the round trip is exact to that precision
    np.testing.assert_allclose(n2, ne_next, rtol=2e-5)
    np.testing.assert_allclose(p2, phi_next, rtol=1e-6)
    f = R.features(col, col.ne, col.phi)
    np.testing.assert_allclose(R.n_of(f[:, 0]), col.ne, rtol=1e-5)
    assert np.all(f[:, 6:] == 0.0)
    f2 = R.features(col, ne_next, phi_next, col.ne, col.phi)
    np.testing.assert_allclose(f2[:, 7], 3.0 / 300.0, rtol=1e-6)
    np.testing.assert_allclose(f2[:, 4], np.log10(0.02 / 64 / 1e-5), rtol=1e-6)
