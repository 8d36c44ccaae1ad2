"""Throughput of the batched JFNK electron/potential step on one MI355X.

Workload: 1024 independent flame columns of U{512..8192} cells, applied
voltage U[-1000, 1000] V, ion peak log-U[1e15, 1e17] m^-3, flame position
U[0.5, 1.5] cm (seed 2026), dt = 1e-5 s, marched in episodes of 20 steps
from n_e = n_ion (each episode restarts from the initial state).  One bench
step = one jfnk_step over the whole batch (1024 column-steps).

Prints one JSON line: whole-job column-steps/s of the batched solver at
||S_F^-1 F||_inf < 1e-10, with the plain (host-driven, one column at a time)
solver and the CPU oracle measured beside it, and the roofline of the solve
kernel from HIP events and the algorithmic byte model (solve_bytes_per_cell,
gather_bytes_per_cell).
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "column-steps/s at ||F||<1e-10, plain vs batched+learned JFNK, 1 MI355X"
EPISODE = 20
HBM_PEAK_GBS = 8000.0


def gather_bytes_per_cell(has_prev):
    """Algorithmic HBM bytes per cell of the gather launch: 7 caller arrays
    (mu, D, n_e, phi, source, loss, q) in; f, q and X^n out; X^{n-1} in and
    the extrapolation out when it is supplied; the 3 stored face/loss
    coefficients read for the factor-reuse test.  The coefficients equal to
    the stored ones are not written again: the workload's mu, D and loss do
    not change in time, so in the timed steps (after the warm-up) none is."""
    return 88.0 + (32.0 if has_prev else 0.0) + 24.0


WRITEBACK_BYTES_PER_CELL = 32.0               # X^{n+1} from the workspace to the caller's arrays


def solve_bytes_per_cell(has_prev, fb, counts):
    """Algorithmic HBM bytes per cell of one column-step inside the solve
    launch, from the phases the step executed (jfnk_stats.phase_counts:
    factorisations, preconditioner applies, residual evaluations, J.v
    products, CGS passes, direction assemblies, extra vector reads, learned
    candidates evaluated); each
    phase reads its operands from HBM and writes its results once (fb = bytes
    per stored preconditioner value).  The Arnoldi dot sweeps, Gram-Schmidt
    passes and direction assemblies also read a number of basis vectors that
    grows with the Krylov index: those are the extra vector reads, 16 bytes
    per cell each."""
    setup = 72.0                               # F(X^n): X + 5 coefficients -> F
    if has_prev:
        setup += 32.0                          # same sweep: the extrapolation in, its residual out
    per_phase = (40.0 + 20.0 * fb,             # factor: X + 3 coefficients -> 20 factor values
                 32.0 + 20.0 * fb,             # apply: v + 20 factor values -> z
                 104.0,                        # trial: X + direction + 5 coefficients -> X_t, F_t
                 120.0,                        # J.v: X, z, F, 5 coefficients, 2 basis vectors -> w
                 32.0,                         # CGS pass: w in and out (basis vectors: extra reads)
                 16.0,                         # direction: dX out (summed vectors: extra reads)
                 16.0,                         # one extra FP64 vector pair read
                 72.0)                         # learned candidate: X_l + 5 coefficients -> F_l
    return setup + sum(c * b for c, b in zip(counts, per_phase))


def measure_batched(J, prob, ne, phi, ne0, phi0, ns, args, prec, guess, net=None, stream=None, chord=None):
    """Warm-up then timed episodes of the batched solver; per-step records."""
    import torch
    kw = {} if chord is None else dict(chord_tol=chord)
    cfg = J.config_for_dims(len(ns), int(ns.sum()), int(ns.max()), prec_precision=prec, guess=guess,
                            schedule=J.SCHED_BATCHED, threads_override=args.threads, **kw)
    solver = J.Solver(cfg)
    if net is not None:
        solver.set_model(net)
    tuned = None
    if args.threads == 0 and not args.no_autotune:
        # workgroup size per column for this layout, timed over one whole
        # episode from the start state (its first steps alone favour small
        # workgroups: many columns at once, while the later steps are bound
        # by the columns that still iterate)
        ne.copy_(ne0)
        phi.copy_(phi0)
        tuned = solver.autotune(prob, ne, phi, steps=EPISODE, stream=stream)
    fb = 4.0 if prec == J.PREC_FP32 else 8.0
    # the caller's time loop alternates two states: a step reads X^n from one
    # and X^{n-1} from the other, and writes X^{n+1} over X^{n-1} (no copies)
    state = {"e": 0, "cur": (ne, phi), "other": (torch.empty_like(ne), torch.empty_like(phi))}
    stats = J.Stats(len(ns))   # filled by every step; records copy what they keep

    def report(rc, st, record):
        has_prev = state["queued"].pop(0)
        if record is not None:
            ms, _ = solver.last_timing()
            kms = solver.last_kernel_times()
            record.append(dict(rc=rc, ms=ms, kms=kms, has_prev=has_prev, newton=st.newton_iters.copy(),
                               gmres=st.gmres_iters.copy(), bt=st.backtracks.copy(),
                               res=st.res_scaled.copy(), status=st.status.copy(),
                               guess=st.guess_used.copy(), chords=st.chord_steps.copy(),
                               counts=st.phase_counts.copy()))

    # Steps are queued with jfnk_step_async: the host prepares step k+1 while
    # step k runs, and each call reports the step before it.
    state["queued"] = []

    def one_step(record):
        e = state["e"]
        cur_n, cur_p = state["cur"]
        oth_n, oth_p = state["other"]
        if e == 0:
            cur_n.copy_(ne0)
            cur_p.copy_(phi0)
        has_prev = e > 0
        state["queued"].append(has_prev)
        rc, st = solver.step_async(prob, cur_n, cur_p, oth_n if has_prev else None,
                                   oth_p if has_prev else None, stream=stream, prev_stats=stats,
                                   ne_out=oth_n, phi_out=oth_p)
        state["cur"], state["other"] = state["other"], state["cur"]
        state["e"] = (e + 1) % EPISODE
        if rc is not None:
            report(rc, st, record)

    def finish(record):
        rc, st = solver.step_finish(stats=stats)
        report(rc, st, record)

    for _ in range(args.warmup):
        one_step(None)
    if args.warmup > 0:
        finish(None)
    state["e"] = 0
    torch.cuda.synchronize()
    rec = []
    # Python's cyclic collector stays out of the timed loop (a pass over the
    # heap left by the network's training can take milliseconds)
    gc.collect()
    gc.disable()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(rec)
    finish(rec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gc.enable()
    solver.close()
    for r in rec:   # outside the timed region
        r["conv"] = int(np.sum(r["status"] == 0))
        r["res"] = float(r["res"].max())
        r["bytes"] = float(np.sum(ns * np.array([
            solve_bytes_per_cell(r["has_prev"], fb, r["counts"][i]) for i in range(len(ns))])))
        r["gbytes"] = float(np.sum(ns)) * gather_bytes_per_cell(r["has_prev"])
        r["wbytes"] = float(np.sum(ns)) * WRITEBACK_BYTES_PER_CELL
    converged = sum(r["conv"] for r in rec)
    kern_ms = sum(r["kms"][1] for r in rec)
    kern_bytes = sum(r["bytes"] for r in rec)
    g_ms = sum(r["kms"][0] for r in rec)
    w_ms = sum(r["kms"][2] for r in rec)
    step_ms = sum(r["ms"] for r in rec)
    newton = np.concatenate([r["newton"] for r in rec])
    gmres = np.concatenate([r["gmres"] for r in rec])
    used = np.concatenate([r["guess"] for r in rec])
    chords = np.concatenate([r["chords"] for r in rec])
    return dict(
        value=converged / wall, wall=wall, ms_per_step=1e3 * wall / args.steps,
        converged=converged, total=len(ns) * args.steps, max_res=max(r["res"] for r in rec),
        kernel_ms_avg=kern_ms / len(rec), achieved_gbs=kern_bytes / (kern_ms * 1e-3) / 1e9,
        bytes_per_launch=kern_bytes / len(rec),
        launches={
            "k_gather": dict(ms_avg=g_ms / len(rec), bytes_per_launch=sum(r["gbytes"] for r in rec) / len(rec),
                             achieved_gbs=sum(r["gbytes"] for r in rec) / (g_ms * 1e-3) / 1e9),
            "k_solve": dict(ms_avg=kern_ms / len(rec), bytes_per_launch=kern_bytes / len(rec),
                            achieved_gbs=kern_bytes / (kern_ms * 1e-3) / 1e9),
            "k_scatter": dict(ms_avg=w_ms / len(rec), bytes_per_launch=sum(r["wbytes"] for r in rec) / len(rec),
                              achieved_gbs=sum(r["wbytes"] for r in rec) / (w_ms * 1e-3) / 1e9),
            "step_ms_avg": step_ms / len(rec),
        },
        newton_mean=float(newton.mean()), newton_max=int(newton.max()),
        gmres_per_newton=float(gmres.sum() / max(newton.sum(), 1)),
        chord_mean=float(chords.mean()),
        autotune=None if tuned is None else dict(chosen=tuned[0], ms_per_episode=tuned[1]),
        guess_used={"prev": int(np.sum(used == 0)), "extrap": int(np.sum(used == 1)),
                    "learned": int(np.sum(used == 2))},
        # column-steps whose learned candidate was evaluated (network inference
        # and one residual), from jfnk_stats.phase_counts[:, 7]
        learned_evaluated=int(sum(int(np.sum(r["counts"][:, 7])) for r in rec)),
    )


def train_guess_net(J, args):
    """Train the learned-guess network on solver-generated episodes of the
    training seeds (disjoint from the benchmark batch's seed)."""
    import torch
    from paper_1904_08510_amd import train_guess as TG
    from paper_1904_08510_amd import workloads as W
    t0 = time.perf_counter()
    data = TG.generate(list(W.training_seeds())[:args.train_seeds], ncols=args.train_cols,
                       steps=EPISODE, log=lambda *a: None)
    t1 = time.perf_counter()
    net = TG.make_net(data)
    net.set_params(TG.init_params(0))
    hist = TG.train(net, data, epochs=args.train_epochs, log=lambda *a: None)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = dict(episodes=len(data), columns_per_episode=args.train_cols, steps=EPISODE,
                column_steps=len(data) * args.train_cols * EPISODE, epochs=args.train_epochs,
                data_s=t1 - t0, train_s=t2 - t1, loss_per_epoch=hist)
    del data
    torch.cuda.empty_cache()
    return net, info


def run_gpu(args):
    import torch
    from paper_1904_08510_amd import jfnk as J
    from paper_1904_08510_amd import workloads as W

    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.calib_copy:
        # one device-to-device copy of known size, to calibrate HBM counters
        from paper_1904_08510_amd.profiling import CALIB_BYTES
        src = torch.empty(CALIB_BYTES // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    net, train_info = (None, None)
    if args.guess == "learned":
        net, train_info = train_guess_net(J, args)
    cols = W.config2(seed=2026, ncols=args.ncols)
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed, dev)
    ne0, phi0 = ne.clone(), phi.clone()
    ns = np.diff(packed.col_offset)
    stream = torch.cuda.current_stream()
    prec = J.PREC_FP32 if args.prec == "fp32" else J.PREC_FP64
    guess = J.GUESS_LEARNED if args.guess == "learned" else J.GUESS_EXTRAP
    out = measure_batched(J, prob, ne, phi, ne0, phi0, ns, args, prec, guess, net, stream)
    out["cells"] = int(packed.col_offset[-1])
    out["train"] = train_info
    if not args.skip_ablations:
        abl = {}
        for name, pr, gs, ch in (("batched_fp32_extrap", J.PREC_FP32, J.GUESS_EXTRAP, None),
                                 ("batched_fp64_extrap", J.PREC_FP64, J.GUESS_EXTRAP, None),
                                 ("batched_fp32_extrap_no_chord", J.PREC_FP32, J.GUESS_EXTRAP, 0.0)):
            if pr == prec and gs == guess and ch is None:
                continue
            r = measure_batched(J, prob, ne, phi, ne0, phi0, ns, args, pr, gs, None, stream, ch)
            abl[name] = dict(value=r["value"], ms_per_step=r["ms_per_step"], converged=r["converged"],
                             max_res=r["max_res"], kernel_ms_avg=r["kernel_ms_avg"],
                             newton_mean=r["newton_mean"], chord_mean=r["chord_mean"],
                             threads=None if r["autotune"] is None else r["autotune"]["chosen"])
        out["ablations"] = abl
    if net is not None:
        net.close()

    # plain schedule on a bounded sample of the same batch (one column per call)
    if not args.skip_plain:
        idx = list(range(0, args.ncols, max(1, args.ncols // args.plain_cols)))[: args.plain_cols]
        sub = W.pack([cols[i] for i in idx])
        sprob, sne, sphi, _, _ = J.device_problem(sub, dev)
        pn, pp = torch.empty_like(sne), torch.empty_like(sphi)
        psolver = J.Solver(J.config_for(sub, prec_precision=J.PREC_FP64, guess=J.GUESS_EXTRAP,
                                        schedule=J.SCHED_PLAIN))
        torch.cuda.synchronize()
        tp = time.perf_counter()
        conv_p = 0
        for e in range(args.plain_steps):
            cn, cp = sne.clone(), sphi.clone()
            rc, st = psolver.step(sprob, sne, sphi, pn if e else None, pp if e else None, stream=stream)
            conv_p += int(np.sum(st.status == 0))
            pn.copy_(cn)
            pp.copy_(cp)
        torch.cuda.synchronize()
        tplain = time.perf_counter() - tp
        out["plain"] = dict(value=conv_p / tplain, columns=len(idx), steps=args.plain_steps,
                            sample=f"{len(idx)} columns (every {args.ncols // len(idx)}th) x "
                                   f"episode steps 0..{args.plain_steps - 1}, FP64 factors, extrapolated guess")
        psolver.close()
    return out


def _cpu_column_episode(args):
    """Oracle timed mode over the first `steps` steps of a column's episode."""
    ci, steps = args
    from oracle import oracle as O
    from paper_1904_08510_amd import workloads as W
    col = W.config2(seed=2026)[ci]
    t0 = time.process_time()
    ne, phi = col.ne.copy(), col.phi.copy()
    pne = pphi = None
    for k in range(steps):
        oc = O.OracleColumn(col, ne, phi)
        g_n, g_p = ne, phi
        if pne is not None:
            e_n, e_p = 2 * ne - pne, 2 * phi - pphi
            if O.scaled_residual_inf(oc, e_n, e_p) <= O.scaled_residual_inf(oc, ne, phi):
                g_n, g_p = e_n, e_p
        r = O.newton(oc, g_n, g_p, tol=1e-10)
        pne, pphi = ne, phi
        ne, phi = r.ne, r.phi
    return time.process_time() - t0


def run_cpu(args):
    import multiprocessing as mp
    ncores = min(len(os.sched_getaffinity(0)), 16)
    idx = list(range(0, 1024, 1024 // args.cpu_cols))[: args.cpu_cols]
    tasks = [(i, args.cpu_steps) for i in idx]
    from oracle import oracle as O
    O.lib()
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(ncores) as pool:
        cpu_times = pool.map(_cpu_column_episode, tasks, chunksize=1)
    wall = time.perf_counter() - t0
    n = len(tasks) * args.cpu_steps
    return dict(value=n / wall, unit="column-steps/s", cores=ncores, kind="oracle",
                sample=f"{len(tasks)} columns (every {1024 // len(tasks)}th of the batch) x episode steps "
                       f"0..{args.cpu_steps - 1}, timed mode (1e-10), one process per core; "
                       f"{sum(cpu_times):.1f} CPU-s",
                single_core_value=n / sum(cpu_times))


def measured_traffic():
    """HBM bytes per solve launch from the committed FETCH_SIZE/WRITE_SIZE
    counter runs, if they were taken with the current kernel sources."""
    from paper_1904_08510_amd.profiling import source_hash
    path = os.path.join(ROOT, "profiles", "k_solve_c2_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != source_hash():
        return None
    return rec["traffic_bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--ncols", type=int, default=1024)
    ap.add_argument("--prec", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--threads", type=int, default=0, help="workgroup size per column (0: autotuned)")
    ap.add_argument("--guess", choices=["learned", "extrap"], default="learned")
    ap.add_argument("--train-seeds", type=int, default=100)
    ap.add_argument("--train-cols", type=int, default=50)
    ap.add_argument("--train-epochs", type=int, default=4)
    ap.add_argument("--skip-ablations", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--plain-cols", type=int, default=16)
    ap.add_argument("--plain-steps", type=int, default=EPISODE)
    ap.add_argument("--cpu-cols", type=int, default=1024)
    ap.add_argument("--cpu-steps", type=int, default=EPISODE)
    ap.add_argument("--calib-copy", action="store_true",
                    help="one 256 MiB device copy first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the columns are independent and this build runs "
              f"on a single MI355X (asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)
    # the CPU leg forks its worker processes before this process touches the GPU
    cpu = None if args.skip_cpu else run_cpu(args)
    g = run_gpu(args)
    traffic = measured_traffic()
    line = {
        "metric": METRIC,
        "value": g["value"],
        "unit": "column-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": g["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.ncols} flame columns x U{{512..8192}} cells (seed 2026), V~U[-1000,1000], "
                        f"ion peak logU[1e15,1e17], dt=1e-5 s, 20-step episodes; batched, "
                        f"{args.prec.upper()} preconditioner factors, "
                        + ("learned guess (BF16 conv net) with extrapolated fallback" if args.guess == "learned"
                           else "extrapolated guess"),
            "columns": args.ncols,
            "cells": g["cells"],
            "episode_steps": EPISODE,
            "prec": args.prec,
            "guess": args.guess,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": g["achieved_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": g["achieved_gbs"] / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "k_solve",
            "kernel_ms_avg": g["kernel_ms_avg"],
            "bytes_per_launch": g["bytes_per_launch"],
        },
        "launches": g["launches"],
        "cpu_baseline": cpu,
        "plain": g.get("plain"),
        "ablations": g.get("ablations"),
        "learned": None if g.get("train") is None else dict(g["train"], guess_used=g["guess_used"],
                                                               evaluated=g["learned_evaluated"]),
        "speedup_vs_plain": (g["value"] / g["plain"]["value"]) if g.get("plain") else None,
        "solver": {
            "converged": g["converged"], "column_steps": g["total"], "max_res": g["max_res"],
            "newton_mean": g["newton_mean"], "newton_max": g["newton_max"],
            "gmres_per_newton": g["gmres_per_newton"], "guess_used": g["guess_used"],
            "chord_steps_mean": g["chord_mean"], "autotune": g["autotune"],
        },
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
