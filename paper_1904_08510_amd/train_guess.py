"""Training driver of the learned Newton initial guess (a Python loop over
the C ABI; every kernel runs in libjfnk).

Data: batches of uneven flame columns drawn like the evaluation batch
(cells, voltage, ion peak and flame position from the same ranges) but with
the training seeds, each advanced by the solver itself for an episode of
backward-Euler steps from the start state.  One training example is a
(batch, step) pair: inputs X^k (and X^{k-1}), target X^{k+1}, all columns of
the batch at once.  torch holds the stored states in device memory.

    python -m paper_1904_08510_amd.train_guess --out guess.npz
"""
from __future__ import annotations

import argparse
import math
import time
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from . import jfnk, workloads as W

# output scales of the network (increments of a(n) and of phi / phi_s)
OUT_SCALE_NE = 0.1
OUT_SCALE_PHI = 0.3


@dataclass
class Episode:
    prob: object          # jfnk.DeviceProblem
    states: list          # [(ne, phi)] device tensors, X^0 .. X^steps
    ncols: int
    cells: int


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal hidden layers, a small output layer, zero biases (flat FP32)."""
    rng = np.random.default_rng(seed)
    ch = [8, 64, 64, 64, 64, 64, 2]
    out = []
    for l in range(6):
        cin, cout = ch[l], ch[l + 1]
        std = math.sqrt(2.0 / (cin * 5)) if l < 5 else 0.1 * math.sqrt(1.0 / (cin * 5))
        out.append(rng.standard_normal(cout * 5 * cin) * std)
        out.append(np.zeros(cout))
    p = np.concatenate(out).astype(np.float32)
    assert p.size == jfnk.net_param_count()
    return p


def generate(seeds, ncols: int = 50, steps: int = 20, nmin: int = 512, nmax: int = 8192,
             dt: float = 1e-5, log=print) -> List[Episode]:
    """Solve one episode per seed and keep every state."""
    import torch
    eps = []
    t0 = time.time()
    for s in seeds:
        packed = W.pack(W.config2(seed=s, ncols=ncols, nmin=nmin, nmax=nmax, dt=dt))
        prob, ne, phi, _, _ = jfnk.device_problem(packed)
        solver = jfnk.Solver(jfnk.config_for(packed))
        states = [(ne.clone(), phi.clone())]
        pne = pph = None
        for _ in range(steps):
            cur = states[-1]
            solver.step(prob, ne, phi, pne, pph)
            states.append((ne.clone(), phi.clone()))
            pne, pph = cur
        solver.close()
        eps.append(Episode(prob, states, packed.ncols, packed.total))
    torch.cuda.synchronize()
    log(f"generated {len(eps)} episodes x {steps} steps ({sum(e.cells for e in eps) * steps / 1e6:.1f} M "
        f"cell-steps) in {time.time() - t0:.1f} s")
    return eps


def train(net: "jfnk.Net", data: List[Episode], epochs: int = 8, lr: float = 2e-3, lr_min: float = 2e-5,
          seed: int = 0, log=print) -> list:
    """Adam over shuffled (episode, step) examples, cosine learning-rate decay."""
    rng = np.random.default_rng(seed)
    examples = [(i, k) for i, e in enumerate(data) for k in range(len(e.states) - 1)]
    total = epochs * len(examples)
    it = 0
    hist = []
    t0 = time.time()
    for ep in range(epochs):
        order = rng.permutation(len(examples))
        losses = []
        for j, idx in enumerate(order):
            i, k = examples[idx]
            e = data[i]
            rate = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * it / max(total - 1, 1)))
            prev = e.states[k - 1] if k > 0 else (None, None)
            want = j % 50 == 0
            loss = net.train_step(e.prob, e.states[k][0], e.states[k][1], prev[0], prev[1],
                                  e.states[k + 1][0], e.states[k + 1][1], rate, want_loss=want)
            if want:
                losses.append(loss)
            it += 1
        hist.append(float(np.mean(losses)))
        log(f"epoch {ep}: sampled loss {hist[-1]:.4e} ({time.time() - t0:.1f} s)")
    return hist


def make_net(data: List[Episode]) -> "jfnk.Net":
    return jfnk.Net(jfnk.net_default_config(max_cols=max(e.ncols for e in data),
                                            max_total_cells=max(e.cells for e in data),
                                            out_scale_ne=OUT_SCALE_NE, out_scale_phi=OUT_SCALE_PHI))


def load(path: str) -> "jfnk.Net":
    z = np.load(path, allow_pickle=False)
    net = jfnk.Net(jfnk.net_default_config(out_scale_ne=float(z["out_scale"][0]),
                                           out_scale_phi=float(z["out_scale"][1])))
    net.set_params(z["params"])
    return net


def save(net: "jfnk.Net", path: str):
    np.savez(path, params=net.get_params(),
             out_scale=np.array([net.config.out_scale_ne, net.config.out_scale_phi], np.float32))


def main(argv: Optional[list] = None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--seeds", type=int, default=100, help="training batches (seeds 1000, 1001, ...)")
    ap.add_argument("--ncols", type=int, default=50)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    seeds = list(W.training_seeds())[:a.seeds]
    data = generate(seeds, ncols=a.ncols, steps=a.steps)
    net = make_net(data)
    net.set_params(init_params(0))
    train(net, data, epochs=a.epochs, lr=a.lr)
    if a.out:
        save(net, a.out)


if __name__ == "__main__":
    main()
