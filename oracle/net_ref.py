"""FP64 numpy reference of the learned Newton-guess network.

TEST INFRASTRUCTURE ONLY: the tests use it to check the library's network
kernels (features, forward pass, loss, gradients, Adam step).  It shares no
code with them and is never imported by the library.

The network is not part of the paper's method: it predicts X^{n+1} of a
column from X^n (and X^{n-1}), the ion charge and the gas temperature, and
its prediction only serves as a Newton initial guess.

Architecture: six 1D convolutions, kernel 5, zero padding at the ends of
each column, channels 8 -> 64 -> 64 -> 64 -> 64 -> 64 -> 2, ReLU after the
first five.  Input channels per cell (n0 = 1e8 m^-3, a(n) = asinh(n/n0)/20,
phi_s = max(|phi_L|, |phi_R|, 1) V):
  0 a(n^n)        1 phi^n/phi_s      2 a(q)           3 (T - 1150)/850
  4 log10(h/1e-5) 5 (phi_R - phi_L)/1000
  6 a(n^n) - a(n^{n-1})              7 (phi^n - phi^{n-1})/phi_s  (0 without X^{n-1})
Outputs (o0, o1) are increments in units of the output scales (s0, s1):
a(n^{n+1}) = a(n^n) + s0 o0 and phi^{n+1} = phi^n + phi_s s1 o1.  The loss of
a batch is the mean over its cells of (o0 - t0)^2 + (o1 - t1)^2 with the
targets t the increments of the true X^{n+1} in the same units.

``quant=True`` rounds, as the matrix-core kernels store them, the inputs,
the weights, every hidden activation and every backpropagated activation
gradient to bfloat16 (round to nearest even, through float32); arithmetic
stays FP64 otherwise.
"""
from __future__ import annotations

import numpy as np

N0 = 1e8
CH = [8, 64, 64, 64, 64, 64, 2]
K = 5
NLAYER = 6


# ---------------------------------------------------------------------------
# bfloat16 rounding (round to nearest, ties to even, of the float32 value)
# ---------------------------------------------------------------------------

def bf16(x) -> np.ndarray:
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    out = (r.astype(np.uint32) << 16).view(np.float32)
    return out.astype(np.float64)


# ---------------------------------------------------------------------------
# features and targets
# ---------------------------------------------------------------------------

def a_of(n):
    return np.arcsinh(np.asarray(n, dtype=np.float64) / N0) / 20.0


def n_of(a):
    return N0 * np.sinh(20.0 * np.asarray(a, dtype=np.float64))


def phi_scale(phi_left, phi_right):
    return max(abs(phi_left), abs(phi_right), 1.0)


def features(col, ne, phi, ne_prev=None, phi_prev=None) -> np.ndarray:
    """[n, 8] input channels of one column (float32 values, as the kernels form them)."""
    n = col.n
    ps = phi_scale(col.phi_left, col.phi_right)
    an = a_of(ne)
    f = np.zeros((n, 8))
    f[:, 0] = an
    f[:, 1] = np.asarray(phi) / ps
    f[:, 2] = a_of(col.q)
    f[:, 3] = (np.asarray(col.temp) - 1150.0) / 850.0
    f[:, 4] = np.log10((col.length / n) / 1e-5)
    f[:, 5] = (col.phi_right - col.phi_left) / 1000.0
    if ne_prev is not None:
        f[:, 6] = an - a_of(ne_prev)
        f[:, 7] = (np.asarray(phi) - np.asarray(phi_prev)) / ps
    return f.astype(np.float32).astype(np.float64)


def targets(col, ne, phi, ne_next, phi_next, s0, s1) -> np.ndarray:
    ps = phi_scale(col.phi_left, col.phi_right)
    t = np.stack([(a_of(ne_next) - a_of(ne)) / s0,
                  (np.asarray(phi_next) - np.asarray(phi)) / (ps * s1)], axis=1)
    return t.astype(np.float32).astype(np.float64)


def candidate(col, ne, phi, out, s0, s1):
    """Next-state guess (n, phi) from the outputs [n, 2]."""
    ps = phi_scale(col.phi_left, col.phi_right)
    return n_of(a_of(ne) + s0 * out[:, 0]), np.asarray(phi) + ps * s1 * out[:, 1]


# ---------------------------------------------------------------------------
# parameters: list of (W [cout, K, cin], b [cout]); flat order W then b per layer
# ---------------------------------------------------------------------------

def init_params(seed=0):
    """He-normal hidden layers, a small output layer, zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for l in range(NLAYER):
        cin, cout = CH[l], CH[l + 1]
        std = np.sqrt(2.0 / (cin * K)) if l < NLAYER - 1 else 0.1 * np.sqrt(1.0 / (cin * K))
        params.append((rng.standard_normal((cout, K, cin)) * std, np.zeros(cout)))
    return params


def flat(params) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def unflat(v) -> list:
    v = np.asarray(v, dtype=np.float64)
    out, o = [], 0
    for l in range(NLAYER):
        cin, cout = CH[l], CH[l + 1]
        W = v[o:o + cout * K * cin].reshape(cout, K, cin)
        o += cout * K * cin
        b = v[o:o + cout]
        o += cout
        out.append((W.copy(), b.copy()))
    return out


def nparams() -> int:
    return sum(CH[l + 1] * K * CH[l] + CH[l + 1] for l in range(NLAYER))


# ---------------------------------------------------------------------------
# forward / backward (one column at a time, cells along axis 0)
# ---------------------------------------------------------------------------

def conv(x, W, b):
    """y[i, co] = b[co] + sum_{j, ci} W[co, j, ci] x[i + j - 2, ci], x = 0 outside."""
    n, cin = x.shape
    xp = np.zeros((n + K - 1, cin))
    xp[2:n + 2] = x
    y = np.tile(b, (n, 1)).astype(np.float64)
    for j in range(K):
        y += xp[j:j + n] @ W[:, j, :].T
    return y


def _q(x, quant):
    return bf16(x) if quant else x


def forward(params, x, quant=False):
    """(output [n, 2], inputs of the six layers)."""
    acts = [_q(x, quant)]
    h = acts[0]
    for l, (W, b) in enumerate(params):
        z = conv(h, _q(W, quant), b)
        if l < NLAYER - 1:
            h = _q(np.maximum(z, 0.0), quant)
            acts.append(h)
        else:
            h = z.astype(np.float32).astype(np.float64) if quant else z
    return h, acts


def loss_and_grad(params, cols_x, cols_t, quant=False):
    """Loss (mean over all cells of all columns of the summed squared
    output errors) and its gradient, a list like params."""
    ncell = sum(x.shape[0] for x in cols_x)
    grads = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    loss = 0.0
    for x, t in zip(cols_x, cols_t):
        out, acts = forward(params, x, quant)
        r = out - t
        loss += float(np.sum(r * r))
        if quant:
            d = bf16(np.float32(2.0) * r.astype(np.float32) * np.float32(1.0 / ncell))
        else:
            d = 2.0 * r / ncell
        for l in range(NLAYER - 1, -1, -1):
            W, b = params[l]
            Wq = _q(W, quant)
            a_in = acts[l]
            n = a_in.shape[0]
            gW, gb = grads[l]
            gb += d.sum(axis=0)
            ap = np.zeros((n + K - 1, a_in.shape[1]))
            ap[2:n + 2] = a_in
            for j in range(K):
                gW[:, j, :] += d.T @ ap[j:j + n]
            if l > 0:
                # input cell i + j - 2 feeds output cell i through tap j
                dp = np.zeros((n + K - 1, d.shape[1]))
                dp[2:n + 2] = d
                din = np.zeros_like(a_in)
                for j in range(K):
                    din += dp[K - 1 - j:K - 1 - j + n] @ Wq[:, j, :]
                d = _q(din * (a_in > 0.0), quant)
    return loss / ncell, grads


def adam(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; returns (params, m, v) with m, v flat arrays."""
    p = flat(params)
    g = flat(grads)
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    p = p - lr * mh / (np.sqrt(vh) + eps)
    return unflat(p), m, v
