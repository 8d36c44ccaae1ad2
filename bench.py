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
_T0 = time.perf_counter()


def note(msg):
    """A progress line on stderr (the JSON result is the only stdout line)."""
    print(f"bench.py [{time.perf_counter() - _T0:6.1f} s] {msg}", file=sys.stderr, flush=True)


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
    setup, per_phase = solve_phase_bytes(has_prev, fb)
    return setup + sum(c * b for c, b in zip(counts, per_phase))


PHASE_NAMES = ("factor", "apply", "trial", "jv", "cgs", "direction", "vector_reads", "learned")


def solve_phase_bytes(has_prev, fb):
    """(set-up bytes per cell, bytes per cell of one execution of each phase
    in PHASE_NAMES order) for solve_bytes_per_cell."""
    setup = 72.0                               # F(X^n): X + 5 coefficients -> F
    if has_prev:
        setup += 32.0                          # same sweep: the extrapolation in, its residual out
    per_phase = (40.0 + 16.0 * fb,             # factor: X + 3 coefficients -> 16 factor values
                 32.0 + 16.0 * fb,             # apply: v + 16 factor values -> z
                 104.0,                        # trial: X + direction + 5 coefficients -> X_t, F_t
                 120.0,                        # J.v: X, z, F, 5 coefficients, 2 basis vectors -> w
                 32.0,                         # CGS pass: w in and out (basis vectors: extra reads)
                 16.0,                         # direction: dX out (summed vectors: extra reads)
                 16.0,                         # one extra FP64 vector pair read
                 72.0)                         # learned candidate: X_l + 5 coefficients -> F_l
    return setup, per_phase


def pick_parity_sample(rec, ns, episode=EPISODE, nextra=2, seed=99):
    """Columns whose every step the oracle re-checks: the shortest, the
    longest, the two that iterated latest in the timed episodes, and nextra
    more drawn at random."""
    last = np.zeros(len(ns), int)
    for k, r in enumerate(rec[:episode]):
        last[(r["newton"] + r["chords"]) > 0] = k
    late = [int(c) for c in np.argsort(-last * 100000 - ns)[:2]]
    rng = np.random.default_rng(seed)
    extra = [int(c) for c in rng.choice(len(ns), nextra, replace=False)]
    return sorted(set([int(np.argmin(ns)), int(np.argmax(ns))] + late + extra)), last


def measure_batched(J, prob, ne, phi, ne0, phi0, ns, args, prec, guess, net=None, stream=None, chord=None,
                    parity=False, episode=EPISODE):
    """Warm-up then timed episodes of the batched solver; per-step records.
    With parity, one more (untimed) episode is run exactly like the timed
    ones and the states of sampled columns are kept after every step."""
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
        tuned = solver.autotune(prob, ne, phi, steps=episode, stream=stream)
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
        state["e"] = (e + 1) % episode
        if state.get("snap") is not None:
            # X^{k+1} of the sampled columns, queued on the stream before the
            # next step can overwrite the buffer it was written to
            sl = state["snap_slices"]
            state["snap"].append((torch.cat([oth_n[x] for x in sl]).clone(),
                                  torch.cat([oth_p[x] for x in sl]).clone()))
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
    par = None
    if parity:
        sample, last = pick_parity_sample(rec, ns, episode, nextra=2 if len(ns) > 256 else 0)
        off = np.concatenate([[0], np.cumsum(ns)])
        state["snap_slices"] = [slice(int(off[c]), int(off[c + 1])) for c in sample]
        state["e"] = 0
        n0 = torch.cat([ne0[x] for x in state["snap_slices"]]).clone()
        p0 = torch.cat([phi0[x] for x in state["snap_slices"]]).clone()
        state["snap"] = [(n0, p0)]
        prec_rec = []
        for _ in range(episode):
            one_step(prec_rec)
        finish(prec_rec)
        torch.cuda.synchronize()
        par = dict(columns=sample, cells=[int(ns[c]) for c in sample], last_newton_step=[int(last[c]) for c in sample],
                   states=[(a.cpu().numpy(), b.cpu().numpy()) for a, b in state["snap"]],
                   converged=all(int(np.sum(r["status"] != 0)) == 0 for r in prec_rec))
        state["snap"] = None
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
    # the solve's algorithmic bytes per launch split by phase
    by_phase = dict.fromkeys(("setup",) + PHASE_NAMES, 0.0)
    for r in rec:
        setup, per_phase = solve_phase_bytes(r["has_prev"], fb)
        by_phase["setup"] += setup * float(np.sum(ns))
        for k, name in enumerate(PHASE_NAMES):
            by_phase[name] += per_phase[k] * float(np.sum(ns * r["counts"][:, k]))
    by_phase = {k: v / len(rec) for k, v in by_phase.items()}
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
        bytes_per_launch=kern_bytes / len(rec), bytes_by_phase=by_phase,
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
        per_step=[dict(newton_mean=float(r["newton"].mean()), newton_max=int(r["newton"].max()),
                       gmres_mean=float(r["gmres"].mean()), gmres_max=int(r["gmres"].max()),
                       chords_mean=float(r["chords"].mean()), solve_ms=float(r["kms"][1]))
                  for r in rec[:episode]],
        parity=par,
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
        note("learned guess trained")
    cols = W.config2(seed=2026, ncols=args.ncols)
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed, dev)
    ne0, phi0 = ne.clone(), phi.clone()
    ns = np.diff(packed.col_offset)
    stream = torch.cuda.current_stream()
    prec = J.PREC_FP32 if args.prec == "fp32" else J.PREC_FP64
    guess = J.GUESS_LEARNED if args.guess == "learned" else J.GUESS_EXTRAP
    out = measure_batched(J, prob, ne, phi, ne0, phi0, ns, args, prec, guess, net, stream,
                          parity=not args.skip_parity)
    out["cells"] = int(packed.col_offset[-1])
    note(f"headline leg: {out['value']:.3e} column-steps/s")
    out["train"] = train_info
    parities = {}
    if out["parity"] is not None:
        parities[f"headline_{args.prec}"] = (cols, out.pop("parity"), EPISODE)
    if not args.skip_ablations:
        abl = {}
        for name, pr, gs, ch in (("batched_fp32_extrap", J.PREC_FP32, J.GUESS_EXTRAP, None),
                                 ("batched_fp64_extrap", J.PREC_FP64, J.GUESS_EXTRAP, None),
                                 ("batched_fp32_extrap_no_chord", J.PREC_FP32, J.GUESS_EXTRAP, 0.0)):
            if pr == prec and gs == guess and ch is None:
                continue
            want = pr == J.PREC_FP64 and not args.skip_parity and args.prec == "fp32"
            r = measure_batched(J, prob, ne, phi, ne0, phi0, ns, args, pr, gs, None, stream, ch, parity=want)
            note(f"ablation {name}: {r['value']:.3e} column-steps/s")
            abl[name] = dict(value=r["value"], ms_per_step=r["ms_per_step"], converged=r["converged"],
                             max_res=r["max_res"], kernel_ms_avg=r["kernel_ms_avg"],
                             newton_mean=r["newton_mean"], chord_mean=r["chord_mean"],
                             threads=None if r["autotune"] is None else r["autotune"]["chosen"])
            if r["parity"] is not None:
                parities[name] = (cols, r["parity"], EPISODE)
        out["ablations"] = abl
    del prob, ne, phi, ne0, phi0
    if not args.skip_stiff:
        out["stiff"] = run_stiff(J, args, net, stream, parities)
        note(f"stiff leg: {out['stiff']['value']:.3e} column-steps/s")
    if not args.skip_table:
        out["table"] = run_table(J, args, stream, parities)
        note(f"table-transport leg: {out['table']['value']:.3e} column-steps/s")
    if not args.skip_precond:
        out["preconditioners"] = run_precond(J, args, stream)
        note("preconditioner leg: " + ", ".join(f"{k} {v['value']:.3e}" for k, v in out["preconditioners"].items()
                                                if isinstance(v, dict)))
    if not args.skip_misdc:
        out["misdc"] = run_misdc(J, args, stream)
        note(f"MISDC leg: {out['misdc']['value']:.3e} column-steps/s")
        torch.cuda.empty_cache()
    out["parities"] = parities
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
        note(f"plain leg: {out['plain']['value']:.3e} column-steps/s")
    return out


STIFF_EPISODE = 5


def run_stiff(J, args, net, stream, parities):
    """The stiff batch (256 columns x 65536 cells, 5-10 kV, dt = 1e-4 s):
    batched with FP32 factors and the learned guess (extrapolated fallback)
    against the plain schedule with FP64 factors on a sample of its columns.
    Newton and GMRES counts per step; the oracle re-checks sampled columns."""
    import torch
    from paper_1904_08510_amd import workloads as W
    cols = W.config4()
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed, "cuda:0")
    ne0, phi0 = ne.clone(), phi.clone()
    ns = np.diff(packed.col_offset)
    sargs = argparse.Namespace(**vars(args))
    sargs.warmup = STIFF_EPISODE
    sargs.steps = STIFF_EPISODE * args.stiff_episodes
    guess = J.GUESS_LEARNED if net is not None else J.GUESS_EXTRAP
    r = measure_batched(J, prob, ne, phi, ne0, phi0, ns, sargs, J.PREC_FP32, guess, net, stream,
                        parity=not args.skip_parity, episode=STIFF_EPISODE)
    if r["parity"] is not None:
        par = r["parity"]
        keep = par["columns"][: args.stiff_parity_cols]
        ix = [par["columns"].index(c) for c in keep]
        offs = np.concatenate([[0], np.cumsum(par["cells"])])
        sel = np.concatenate([np.arange(offs[i], offs[i + 1]) for i in ix])
        par = dict(columns=keep, cells=[par["cells"][i] for i in ix],
                   last_newton_step=[par["last_newton_step"][i] for i in ix],
                   states=[(a[sel], b[sel]) for a, b in par["states"]], converged=par["converged"])
        parities["stiff_fp32"] = (cols, par, STIFF_EPISODE)
    out = dict(value=r["value"], ms_per_step=r["ms_per_step"], converged=r["converged"], total=r["total"],
               max_res=r["max_res"], kernel_ms_avg=r["kernel_ms_avg"], achieved_gbs=r["achieved_gbs"],
               newton_mean=r["newton_mean"], gmres_per_newton=r["gmres_per_newton"],
               per_step=r["per_step"], guess_used=r["guess_used"], learned_evaluated=r["learned_evaluated"],
               threads=None if r["autotune"] is None else r["autotune"]["chosen"],
               workload=f"256 columns x 65536 cells, V~U[5,10] kV, ion peak 1e17, dt=1e-4 s, "
                        f"{STIFF_EPISODE}-step episodes (seed 4321); batched, FP32 factors, "
                        + ("learned guess with extrapolated fallback" if net is not None else "extrapolated guess"))
    del prob, ne, phi, ne0, phi0
    torch.cuda.empty_cache()
    # plain schedule, FP64 factors, on a sample of the columns
    idx = list(range(0, len(cols), len(cols) // args.stiff_plain_cols))[: args.stiff_plain_cols]
    sub = W.pack([cols[i] for i in idx])
    sprob, sne, sphi, _, _ = J.device_problem(sub, "cuda:0")
    pn, pp = torch.empty_like(sne), torch.empty_like(sphi)
    psolver = J.Solver(J.config_for(sub, prec_precision=J.PREC_FP64, guess=J.GUESS_EXTRAP,
                                    schedule=J.SCHED_PLAIN))
    torch.cuda.synchronize()
    tp = time.perf_counter()
    conv = 0
    newton, gmres = [], []
    for e in range(STIFF_EPISODE):
        cn, cp = sne.clone(), sphi.clone()
        rc, st = psolver.step(sprob, sne, sphi, pn if e else None, pp if e else None, stream=stream)
        conv += int(np.sum(st.status == 0))
        newton.append(float(st.newton_iters.mean()))
        gmres.append(float(st.gmres_iters.mean()))
        pn.copy_(cn)
        pp.copy_(cp)
    torch.cuda.synchronize()
    tplain = time.perf_counter() - tp
    psolver.close()
    out["plain"] = dict(value=conv / tplain, columns=len(idx), steps=STIFF_EPISODE,
                        newton_mean_per_step=newton, gmres_mean_per_step=gmres,
                        sample=f"{len(idx)} columns (every {len(cols) // len(idx)}th) x episode steps "
                               f"0..{STIFF_EPISODE - 1}, FP64 factors, extrapolated guess")
    out["speedup_vs_plain"] = out["value"] / out["plain"]["value"]
    return out


TABLE_DT = 1e-6


def run_table(J, args, stream, parities):
    """The headline batch with field-dependent electron transport from the
    synthetic table (Section 2.2): batched, FP32 factors, extrapolated guess,
    one warm-up and one timed 20-step episode; sampled columns go to the
    oracle afterwards."""
    import torch
    from paper_1904_08510_amd import workloads as W
    tab = W.synthetic_transport_table()
    # dt = 1e-6 s: at the headline's 1e-5 s the oracle's own Newton fails on a
    # few long high-voltage columns with this table's steep mobility drop
    cols = [W.with_transport_table(c, tab) for c in W.config2(seed=2026, ncols=args.ncols, dt=TABLE_DT)]
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed, "cuda:0")
    ne0, phi0 = ne.clone(), phi.clone()
    ns = np.diff(packed.col_offset)
    targs = argparse.Namespace(**vars(args))
    targs.warmup, targs.steps = EPISODE, EPISODE
    r = measure_batched(J, prob, ne, phi, ne0, phi0, ns, targs, J.PREC_FP32, J.GUESS_EXTRAP, None, stream,
                        parity=not args.skip_parity)
    if r["parity"] is not None:
        parities["table_fp32"] = (cols, r["parity"], EPISODE)
    del prob, ne, phi, ne0, phi0
    torch.cuda.empty_cache()
    return dict(value=r["value"], ms_per_step=r["ms_per_step"], converged=r["converged"], total=r["total"],
                max_res=r["max_res"], kernel_ms_avg=r["kernel_ms_avg"], newton_mean=r["newton_mean"],
                gmres_per_newton=r["gmres_per_newton"],
                threads=None if r["autotune"] is None else r["autotune"]["chosen"],
                workload=f"the {args.ncols}-column batch (seed 2026) with mu and D per face from the synthetic "
                         f"17 x 41 table in (c, log10 |E|/N), dt = {TABLE_DT:g} s; batched, FP32 factors, "
                         f"extrapolated guess, one timed 20-step episode after one warm-up episode")


PRECOND_VOLTS = (10.0, 50.0, 100.0, 500.0, 1000.0)


def run_precond(J, args, stream):
    """The paper's preconditioner study as throughput (Section 4.2): 256
    columns of 512 cells over 1 cm at dV = 10 ... 1000 V, each with the
    constant-CFL step dt = 0.5 h / (0.371 + 4e-3 dV / L), one step from the
    start state (pure Algorithm 2 iterations, FP64), with the exact block
    factorisation, the approximate Schur complement with exact tridiagonal
    blocks, and the same with multigrid V-cycles to gamma_MG = 1e-4."""
    import torch
    from paper_1904_08510_amd import workloads as W
    n, length, ncols = 512, 0.01, 256
    cols = []
    for i in range(ncols):
        dv = PRECOND_VOLTS[i % len(PRECOND_VOLTS)]
        dt = 0.5 * (length / n) / (0.371 + 4e-3 * dv / length)
        cols.append(W.flame_column(n, dv, length=length, x_f=0.005, dt=dt))
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed, "cuda:0")
    ne0, phi0 = ne.clone(), phi.clone()
    out = {}
    for name, kind, kw in (("block", J.PRECK_BLOCK, {}),
                           ("approx_schur", J.PRECK_SCHUR, dict(max_restarts=20)),
                           ("approx_schur_mg", J.PRECK_SCHUR_MG, dict(max_restarts=20, mg_tol=1e-4, mg_blocks=3))):
        solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64, prec_kind=kind, chord_tol=0.0,
                                       threads_override=64, **kw))
        times = []
        for rep in range(2):
            ne.copy_(ne0)
            phi.copy_(phi0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st = solver.step(prob, ne, phi, stream=stream, raw=True)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        conv = int(np.sum(st.status == 0))
        newton = int(st.newton_iters.sum())
        out[name] = dict(value=conv / min(times), converged=conv, total=ncols, ms_per_step=1e3 * min(times),
                         newton_per_column=newton / ncols,
                         gmres_per_newton=float(st.gmres_iters.sum()) / max(newton, 1),
                         v_cycles_per_column=float(st.mg_cycles.sum()) / ncols)
        solver.close()
    out["workload"] = (f"{ncols} columns x {n} cells over 1 cm, dV cycling through {PRECOND_VOLTS} V, "
                       f"dt at constant CFL 0.5 (0.5 h / (0.371 + 4e-3 dV / L)), one step from the start "
                       f"state, FP64, no simplified-Newton steps, workgroup 64")
    del prob, ne, phi, ne0, phi0
    torch.cuda.empty_cache()
    return out


MISDC_CFL = 0.5
MISDC_DT_CAP = 1e-6


def run_misdc(J, args, stream):
    """MISDC steps (k_max = 4 SDC iterations, each a batched JFNK solve) of
    the AC-forced batch: 1000 V at Table 4's frequencies, every column at its
    own phase, each step at ion-drift CFL 0.5 (Section 4.1).  The warm-up
    steps are backward-Euler predictor steps (k_max = 1) that relax the
    electrons from the columns' initial n_e = n_i.  Timed over whole MISDC
    steps; the last timed step's start and result on sampled columns go to
    the oracle afterwards."""
    import torch
    from paper_1904_08510_amd import workloads as W
    cols, ions, t0 = W.config_ac(ncols=args.misdc_cols, n=args.misdc_cells)
    for c in cols:
        c.dt = MISDC_DT_CAP
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed, "cuda:0")
    prob.kloss = None
    di = J.device_ions(np.concatenate([i.mu_i for i in ions]), np.concatenate([i.k_rec for i in ions]), packed.q,
                       np.array([i.ac_amp for i in ions]), np.array([i.ac_freq for i in ions]))
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP32, guess=J.GUESS_EXTRAP))
    # workgroup size for this layout, timed on backward-Euler steps of the batch
    tuned = solver.autotune(prob, ne, phi, steps=3, stream=stream)
    t = t0.copy()
    dt = np.zeros(len(cols))
    k_max = 4
    st = J.Stats(len(cols))
    for _ in range(args.misdc_warmup):
        solver.misdc_step(prob, di, t, 1, ne, phi, stream=stream, stats=st, cfl=MISDC_CFL, dt_out=dt)
        t += dt
    steps = args.misdc_steps
    sample = list(range(0, len(cols), max(1, len(cols) // 2)))[:2]
    off = packed.col_offset
    newton = gmres = conv = 0
    dts = []
    t_snap = 0.0
    torch.cuda.synchronize()
    tic = time.perf_counter()
    for k in range(steps):
        if k == steps - 1:
            # start of the last step on the sampled columns (this copy is not timed)
            t_snap = time.perf_counter()
            snap = [(ne[off[c]:off[c + 1]].cpu().numpy().copy(), phi[off[c]:off[c + 1]].cpu().numpy().copy(),
                     di.n_ion[off[c]:off[c + 1]].cpu().numpy().copy(), float(t[c])) for c in sample]
            t_snap = time.perf_counter() - t_snap
        rc, _ = solver.misdc_step(prob, di, t, k_max, ne, phi, stream=stream, stats=st, cfl=MISDC_CFL, dt_out=dt)
        t += dt
        dts.append(dt.copy())
        newton += int(st.newton_iters.sum())
        gmres += int(st.gmres_iters.sum())
        conv += int(np.sum(st.status == 0))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - tic - t_snap
    got = [(ne[off[c]:off[c + 1]].cpu().numpy(), phi[off[c]:off[c + 1]].cpu().numpy(),
            di.n_ion[off[c]:off[c + 1]].cpu().numpy(), float(dts[-1][c])) for c in sample]
    solver.close()
    total = len(cols) * steps
    dts = np.array(dts)
    return dict(value=conv / elapsed, unit="column-steps/s", converged=conv, total=total,
                ms_per_step=1e3 * elapsed / steps, k_max=k_max,
                newton_per_sdc_iteration=newton / (total * k_max), gmres_per_newton=gmres / max(newton, 1),
                dt_s=dict(min=float(dts.min()), median=float(np.median(dts)), max=float(dts.max())),
                threads=tuned[0], autotune_ms=tuned[1],
                workload=f"{len(cols)} columns x {args.misdc_cells} cells, right electrode 1000 V sin(2 pi f t), "
                         f"f cycling through Table 4 (1k..100k Hz), random phase, ion peak logU[1e15,1e17], "
                         f"dt at ion-drift CFL {MISDC_CFL} (cap {MISDC_DT_CAP:g} s), k_max=4, backward-Euler "
                         f"electrons (eq:nls), FP32 factors, extrapolated predictor guess (seed 77); "
                         f"{args.misdc_warmup} backward-Euler warm-up steps",
                parity_sample=dict(columns=sample, start=snap, got=got, cols=[cols[c] for c in sample],
                                   ions=[ions[c] for c in sample]))


def misdc_oracle_parity(rec):
    """Relative L2 differences of the sampled columns' last timed MISDC step
    against the oracle's step from the same start, at the oracle's own CFL
    step (checked against the step the GPU took)."""
    from oracle import misdc as M
    t0 = time.perf_counter()
    out = []
    for c, col, ion, (ne, phi, ni, t), (gn, gp, gi, gdt) in zip(rec["columns"], rec["cols"], rec["ions"],
                                                                rec["start"], rec["got"]):
        oi = M.Ions(ion.mu_i, ion.k_rec, ion.ac_amp, ion.ac_freq)
        dt = M.cfl_dt(col, oi, t, phi, MISDC_CFL)
        r = M.misdc_step(col, oi, t, ne, phi, ni, k_max=4, dt=dt)
        out.append(dict(column=int(c), cells=int(col.n), dt_rel_diff=abs(gdt - dt) / dt,
                        rel_l2_ne=float(np.linalg.norm(gn - r.ne) / np.linalg.norm(r.ne)),
                        rel_l2_phi=float(np.linalg.norm(gp - r.phi) / max(np.linalg.norm(r.phi), 1e-300)),
                        rel_l2_ni=float(np.linalg.norm(gi - r.ni) / np.linalg.norm(r.ni))))
    return dict(steps=1, columns=out,
                worst=max(max(x["rel_l2_ne"], x["rel_l2_phi"], x["rel_l2_ni"], x["dt_rel_diff"]) for x in out),
                oracle_s=time.perf_counter() - t0)


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


def cpu_model():
    """The host CPU's model name (lscpu's "Model name"), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def run_cpu(args):
    import multiprocessing as mp
    # one process per core, up to the CPU share a one-GPU job has on the
    # measuring machine (16 cores), whatever more the affinity mask shows
    affinity = len(os.sched_getaffinity(0))
    ncores = min(affinity, args.cpu_procs)
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
                single_core_value=n / sum(cpu_times),
                host=dict(cpu_model=cpu_model(), affinity_cores=affinity, os_cpu_count=os.cpu_count(),
                          processes=ncores),
                # the oracle's timed mode stops on the scaled residual alone
                # (||S_F^-1 F||_inf <= 1e-10); the GPU legs stop when that holds
                # and their error estimate ||S_X^-1 P^-1 S_F^-1 F||_inf <= 1e-10
                stop="oracle: residual only; GPU: residual and error estimate")


def oracle_parity(cols, par, episode=EPISODE):
    """Relative L2 errors of sampled GPU results against the oracle's
    reference root of the same step from the same X^n (the GPU's), for every
    step of a replayed episode.  Returns the worst per sampled column."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    states = par["states"]
    out = []
    for j, (c, n) in enumerate(zip(par["columns"], par["cells"])):
        o = int(sum(par["cells"][:j]))
        en_max = ep_max = 0.0
        for k in range(episode):
            xn = (states[k][0][o:o + n], states[k][1][o:o + n])
            got = (states[k + 1][0][o:o + n], states[k + 1][1][o:o + n])
            oc = O.OracleColumn(cols[c], xn[0], xn[1])
            g = xn
            if k > 0:
                xp = (states[k - 1][0][o:o + n], states[k - 1][1][o:o + n])
                e = (2 * xn[0] - xp[0], 2 * xn[1] - xp[1])
                if O.scaled_residual_inf(oc, *e) <= O.scaled_residual_inf(oc, *g):
                    g = e
            r = O.newton(oc, g[0].copy(), g[1].copy(), reference=True)
            en_max = max(en_max, float(np.linalg.norm(got[0] - r.ne) / np.linalg.norm(r.ne)))
            ep_max = max(ep_max, float(np.linalg.norm(got[1] - r.phi) / max(np.linalg.norm(r.phi), 1e-300)))
        out.append(dict(column=int(c), cells=int(n), last_newton_step=par["last_newton_step"][j],
                        rel_l2_ne=en_max, rel_l2_phi=ep_max))
    return dict(steps=episode, columns=out, worst=max(max(x["rel_l2_ne"], x["rel_l2_phi"]) for x in out),
                oracle_s=time.perf_counter() - t0)


def measured_traffic():
    """HBM bytes per solve launch from the committed counter run (the L2's
    DRAM-sector counters, 32 B each), if it was taken with the current
    sources of the step kernels."""
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
    ap.add_argument("--cpu-procs", type=int, default=16,
                    help="largest CPU-leg process pool (the CPU share of a one-GPU job)")
    ap.add_argument("--skip-parity", action="store_true")
    ap.add_argument("--skip-stiff", action="store_true")
    ap.add_argument("--stiff-episodes", type=int, default=2)
    ap.add_argument("--stiff-plain-cols", type=int, default=4)
    ap.add_argument("--stiff-parity-cols", type=int, default=2)
    ap.add_argument("--skip-misdc", action="store_true")
    ap.add_argument("--skip-table", action="store_true")
    ap.add_argument("--skip-precond", action="store_true")
    ap.add_argument("--misdc-only", action="store_true",
                    help="run only the MISDC leg and print its record (for profiling its kernels)")
    ap.add_argument("--misdc-cols", type=int, default=1024)
    ap.add_argument("--misdc-cells", type=int, default=1024)
    ap.add_argument("--misdc-steps", type=int, default=10)
    ap.add_argument("--misdc-warmup", type=int, default=3)
    ap.add_argument("--calib-copy", action="store_true",
                    help="one 256 MiB device copy first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the columns are independent and this build runs "
              f"on a single MI355X (asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)
    if args.misdc_only:
        import torch
        from paper_1904_08510_amd import jfnk as J
        torch.cuda.set_device(0)
        rec = run_misdc(J, args, torch.cuda.current_stream())
        rec.pop("parity_sample")
        print(json.dumps({"misdc": rec}), flush=True)
        return
    # the CPU leg forks its worker processes before this process touches the GPU
    cpu = None if args.skip_cpu else run_cpu(args)
    if cpu is not None:
        note(f"CPU oracle leg: {cpu['value']:.3e} column-steps/s on {cpu['cores']} processes")
    g = run_gpu(args)
    traffic = measured_traffic()
    # the oracle's roots of sampled steps of the timed configurations (CPU,
    # after the GPU legs, on the states those legs produced)
    if cpu is not None and g["parities"]:
        cpu["parity"] = {name: oracle_parity(cols, par, ep) for name, (cols, par, ep) in g["parities"].items()}
    if cpu is not None and g["parities"]:
        note("oracle parity of the sampled GPU steps done")
    misdc = g.get("misdc")
    if misdc is not None:
        rec = misdc.pop("parity_sample")
        if cpu is not None and not args.skip_parity:
            cpu.setdefault("parity", {})["misdc_fp32"] = misdc_oracle_parity(rec)
    # the headline carries the learned guess only if the network was evaluated
    learned_label = args.guess == "learned" and g["learned_evaluated"] > 0
    if args.guess == "learned" and not learned_label:
        print("bench.py: the learned candidate was never evaluated in the timed steps; the line is "
              "labelled as the extrapolated guess", file=sys.stderr)
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
                        + ("learned guess (BF16 conv net) with extrapolated fallback" if learned_label
                           else "extrapolated guess"),
            "columns": args.ncols,
            "cells": g["cells"],
            "episode_steps": EPISODE,
            "prec": args.prec,
            "guess": "learned" if learned_label else "extrap",
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
            "bytes_by_phase": g["bytes_by_phase"],
        },
        "launches": g["launches"],
        "cpu_baseline": cpu,
        "plain": g.get("plain"),
        "ablations": g.get("ablations"),
        "learned": None if g.get("train") is None else dict(g["train"], guess_used=g["guess_used"],
                                                               evaluated=g["learned_evaluated"]),
        "speedup_vs_plain": (g["value"] / g["plain"]["value"]) if g.get("plain") else None,
        "stiff": g.get("stiff"),
        "misdc": misdc,
        "table": g.get("table"),
        "preconditioners": g.get("preconditioners"),
        "solver": {
            "converged": g["converged"], "column_steps": g["total"], "max_res": g["max_res"],
            "newton_mean": g["newton_mean"], "newton_max": g["newton_max"],
            "gmres_per_newton": g["gmres_per_newton"], "guess_used": g["guess_used"],
            "chord_steps_mean": g["chord_mean"], "autotune": g["autotune"],
            "per_step": g["per_step"],
        },
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
