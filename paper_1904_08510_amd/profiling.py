"""Summaries of rocprofv3 output for the solve kernel.

    python -m paper_1904_08510_amd.profiling stats <dir>            # --kernel-trace --stats run
    python -m paper_1904_08510_amd.profiling pmc <fetch_dir> <write_dir> <out.json>
    python -m paper_1904_08510_amd.profiling dram <dir> <out.json>  # one --pmc run of DRAM_COUNTERS
    python -m paper_1904_08510_amd.profiling phase-run [n]          # the per-phase workload (GPU)
    python -m paper_1904_08510_amd.profiling phase-traffic <dir> [n]  # its DRAM counters per phase
    python -m paper_1904_08510_amd.profiling batch-run [rounds] [T] # the same exports on the 1024-column batch (GPU)
    python -m paper_1904_08510_amd.profiling batch-phases <dir>     # its kernel trace: time and GB/s per launch
    python -m paper_1904_08510_amd.profiling net-run [k]            # learned-guess inference over the batch, k times (GPU)
    python -m paper_1904_08510_amd.profiling sq <dir> <kernel>      # mean per dispatch of each counter of a --pmc run
    python -m paper_1904_08510_amd.profiling copy-bw                # a plain device copy's bandwidth (GPU)

`dram` reads HBM bytes directly from the L2's DRAM-sector counters of gfx950
(TCC_EA0_RDREQ_DRAM_32B and TCC_EA0_WRREQ_WRITE_DRAM_32B count 32-byte
sectors, a 64-byte request as 2 and a 128-byte one as 4), with the
calibration copy as a check rather than a scale, and records the 128-byte
read requests two ways (TCC_BUBBLE, which the FETCH_SIZE expression prices
at 128 bytes, and TCC_EA0_RDREQ_128B).

`phase-run` runs the single-phase exports (residual, J.v, block solve) twice
on one column of n cells (default 2^22, which streams through HBM: no cache
holds its fields), each phase its own launch; `phase-traffic` reads a
DRAM-counter run of it and prints the HBM bytes per cell of every phase.

`batch-run` runs the same exports on the 1024-column batch (uneven
512..8192-cell flame columns, FP32 factors, workgroup of T = 256 unless
given), every phase
one launch over all columns; `batch-phases` reads a kernel-trace run of it
and prints each launch's average duration, the trace's register fields (on
gfx950 half the compiler's VGPR + AGPR count) and achieved bandwidth by its
algorithmic bytes (PHASE_BYTES per cell of the batch).  The residual
and J.v launches are kernels holding that phase alone.

`stats` prints the per-kernel time table of a kernel-trace run.  `pmc`
combines a FETCH_SIZE run and a WRITE_SIZE run (counters in KiB per
dispatch) into HBM bytes per launch of each launch of a batched step (the
gather, the solve, the write-back), each counter scaled by what it reads for
the calibration copy (a device-to-device copy of known size that bench.py
--calib-copy performs), and records the hash of the kernel sources the
counters were taken with.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOLVE_KERNEL = "k_solve"
STEP_KERNELS = ("k_gather", "k_solve", "k_scatter")
COPY_KERNEL = "copyBuffer"
CALIB_BYTES = 256 * 1024 * 1024   # bench.py --calib-copy: one copy of this many bytes


# the sources the step kernels (gather, solve, write-back) are compiled from
STEP_SOURCES = ("jfnk_types.h", "jfnk_column.h", "jfnk_solver.h", "jfnk_lib.hip")


def source_hash() -> str:
    """Hash of the step kernels' sources: counters taken with other sources
    no longer describe the kernels."""
    h = hashlib.sha256()
    for path in [os.path.join(HERE, "csrc", f) for f in STEP_SOURCES]:
        with open(path, "rb") as fh:
            h.update(os.path.basename(path).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[-1]


def stats(d: str) -> str:
    rows = list(csv.DictReader(open(_find(d, "kernel_stats.csv"))))
    out = ["kernel | calls | total ms | avg ms | min ms | max ms | pct"]
    for r in rows:
        name = r["Name"]
        m = re.search(r"(k_\w+<[^>]*>|__amd_\w+|\w+::\w+<[^(]{0,40})", name)
        short = m.group(1) if m else name[:60]
        out.append(f"{short} | {r['Calls']} | {float(r['TotalDurationNs'])/1e6:.3f} | "
                   f"{float(r['AverageNs'])/1e6:.4f} | {float(r['MinNs'])/1e6:.4f} | "
                   f"{float(r['MaxNs'])/1e6:.4f} | {float(r['Percentage']):.2f}")
    return "\n".join(out)


def _counter_per_dispatch(d: str, counter: str):
    rows = list(csv.DictReader(open(_find(d, "counter_collection.csv"))))
    per = {k: [] for k in STEP_KERNELS}
    copy = []
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        name = r.get("Kernel_Name", "")
        v = float(r["Counter_Value"])
        for k in STEP_KERNELS:
            if k in name:
                per[k].append(v)
                break
        else:
            if COPY_KERNEL in name:
                copy.append(v)
    return per, copy


def pmc(fetch_dir: str, write_dir: str, out_path: str) -> dict:
    fs, fc = _counter_per_dispatch(fetch_dir, "FETCH_SIZE")
    ws, wc = _counter_per_dispatch(write_dir, "WRITE_SIZE")
    if not fs[SOLVE_KERNEL] or not ws[SOLVE_KERNEL] or not fc or not wc:
        raise RuntimeError("missing solve or calibration-copy dispatches in the counter runs")
    # the calibration copy is the largest copy dispatch (it reads and writes CALIB_BYTES)
    f_scale = CALIB_BYTES / (max(fc) * 1024.0)
    w_scale = CALIB_BYTES / (max(wc) * 1024.0)
    kernels = {}
    for k in STEP_KERNELS:
        if not fs[k] or not ws[k]:
            continue
        fetch = sum(fs[k]) / len(fs[k]) * 1024.0 * f_scale
        write = sum(ws[k]) / len(ws[k]) * 1024.0 * w_scale
        kernels[k] = dict(dispatches=len(fs[k]), fetch_kib_per_dispatch=sum(fs[k]) / len(fs[k]),
                          write_kib_per_dispatch=sum(ws[k]) / len(ws[k]), fetch_bytes=fetch,
                          write_bytes=write, traffic_bytes_per_launch=fetch + write)
    res = dict(source_hash=source_hash(), kernel=SOLVE_KERNEL, copy_fetch_kib=max(fc), copy_write_kib=max(wc),
               fetch_scale=f_scale, write_scale=w_scale, kernels=kernels,
               traffic_bytes_per_launch=kernels[SOLVE_KERNEL]["traffic_bytes_per_launch"])
    with open(out_path, "w") as fh:
        json.dump(res, fh, indent=1)
    return res


DRAM_COUNTERS = ("TCC_EA0_RDREQ_DRAM_32B_sum", "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum", "TCC_BUBBLE_sum",
                 "TCC_EA0_RDREQ_128B_sum")


def dram(d: str, out_path: str) -> dict:
    per = {c: _counter_per_dispatch(d, c) for c in DRAM_COUNTERS}
    rd, rdc = per["TCC_EA0_RDREQ_DRAM_32B_sum"]
    wr, wrc = per["TCC_EA0_WRREQ_WRITE_DRAM_32B_sum"]
    if not rd[SOLVE_KERNEL] or not wr[SOLVE_KERNEL]:
        raise RuntimeError("no solve dispatches in the counter run")

    def mean(v):
        return sum(v) / len(v) if v else 0.0

    kernels = {}
    for k in STEP_KERNELS:
        if not rd[k]:
            continue
        r, w = 32.0 * mean(rd[k]), 32.0 * mean(wr[k])
        kernels[k] = dict(dispatches=len(rd[k]), read_bytes=r, write_bytes=w, traffic_bytes_per_launch=r + w,
                          bubble_per_dispatch=mean(per["TCC_BUBBLE_sum"][0][k]),
                          rdreq_128b_per_dispatch=mean(per["TCC_EA0_RDREQ_128B_sum"][0][k]))
    copy = None
    if rdc and wrc:
        i = max(range(len(rdc)), key=lambda j: rdc[j])
        copy = dict(read_over_bytes=32.0 * rdc[i] / CALIB_BYTES, write_over_bytes=32.0 * wrc[i] / CALIB_BYTES,
                    bubble=per["TCC_BUBBLE_sum"][1][i] if per["TCC_BUBBLE_sum"][1] else None,
                    rdreq_128b=per["TCC_EA0_RDREQ_128B_sum"][1][i] if per["TCC_EA0_RDREQ_128B_sum"][1] else None)
    res = dict(source_hash=source_hash(), kernel=SOLVE_KERNEL, method="DRAM sector counters x 32 B", copy_check=copy,
               kernels=kernels, traffic_bytes_per_launch=kernels[SOLVE_KERNEL]["traffic_bytes_per_launch"])
    with open(out_path, "w") as fh:
        json.dump(res, fh, indent=1)
    return res


# the launches of each single-phase export, in order (one column)
PHASE_EXPORTS = (
    ("residual", ("set-up", "load X", "residual", "store F")),
    ("J.v", ("set-up", "load X", "residual", "load v", "direction copy", "direction norm", "J.v", "store w")),
    ("block solve", ("set-up", "load X", "factorisation", "load r", "apply", "store z")),
)
PHASE_ROUNDS = 2


def phase_run(n: int = 1 << 22) -> None:
    """Single-phase exports on one flame column of n cells (FP32 factors,
    workgroup of 256), PHASE_ROUNDS times each."""
    import torch
    from . import jfnk as J, workloads as W
    packed = W.pack([W.flame_column(n, 500.0)])
    prob, ne, phi, _, _ = J.device_problem(packed)
    cfg = J.config_for(packed, prec_precision=J.PREC_FP32, schedule=J.SCHED_BATCHED, threads_override=256)
    s = J.Solver(cfg)
    g = torch.Generator(device="cuda").manual_seed(1)
    r_ne = torch.randn(ne.shape, device="cuda", dtype=torch.float64, generator=g)
    r_phi = torch.randn(phi.shape, device="cuda", dtype=torch.float64, generator=g)
    for k in range(PHASE_ROUNDS):
        for name, call in (("residual", lambda: s.eval_residual(prob, ne, phi, ne, phi)),
                           ("J.v", lambda: s.eval_jv(prob, ne, phi, ne, phi, r_ne, r_phi)),
                           ("block solve", lambda: s.block_solve(prob, ne, phi, ne, phi, r_ne, r_phi))):
            call()
            torch.cuda.synchronize()
            print(f"phase-run: round {k} {name} done", flush=True)
    s.close()


# algorithmic bytes per cell of the launches that stream the column
# (FP32 factor values: 16 of 4 bytes)
PHASE_BYTES = {
    "residual": 72.0,          # X + 5 coefficients -> F
    "J.v": 104.0,              # X, z, F, 5 coefficients -> w
    "factorisation": 104.0,    # X + 3 coefficients -> 16 factor values
    "apply": 96.0,             # r + 16 factor values -> z
}
BATCH_ROUNDS = 3


def batch_run(rounds: int = BATCH_ROUNDS, threads: int = 256) -> None:
    """Single-phase exports over the 1024-column batch from its start state,
    rounds times each (FP32 factors, workgroups of the given size)."""
    import torch
    from . import jfnk as J, workloads as W
    packed = W.pack(W.config2())
    prob, ne, phi, _, _ = J.device_problem(packed)
    cfg = J.config_for(packed, prec_precision=J.PREC_FP32, schedule=J.SCHED_BATCHED, threads_override=threads)
    s = J.Solver(cfg)
    g = torch.Generator(device="cuda").manual_seed(1)
    r_ne = torch.randn(ne.shape, device="cuda", dtype=torch.float64, generator=g)
    r_phi = torch.randn(phi.shape, device="cuda", dtype=torch.float64, generator=g)
    for k in range(rounds):
        for name, call in (("residual", lambda: s.eval_residual(prob, ne, phi, ne, phi)),
                           ("J.v", lambda: s.eval_jv(prob, ne, phi, ne, phi, r_ne, r_phi)),
                           ("block solve", lambda: s.block_solve(prob, ne, phi, ne, phi, r_ne, r_phi))):
            call()
            torch.cuda.synchronize()
            print(f"batch-run: round {k} {name} done ({packed.ncols} columns, {packed.total} cells)", flush=True)
    s.close()


def batch_phases(d: str, rounds: int = BATCH_ROUNDS, cells: int | None = None) -> str:
    """Per launch of a kernel-trace run of batch_run: average duration over
    the rounds, registers, and GB/s by the algorithmic bytes."""
    if cells is None:
        from . import workloads as W
        cells = W.pack(W.config2()).total
    rows = [r for r in csv.DictReader(open(_find(d, "kernel_trace.csv"))) if "k_phase" in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    labels = [(e, p) for e, ps in PHASE_EXPORTS for p in ps]
    if len(rows) != rounds * len(labels):
        raise RuntimeError(f"{len(rows)} single-phase launches, expected {rounds * len(labels)}")
    out = [f"{cells} cells; export | launch | avg ms | trace VGPR_Count + Accum_VGPR_Count | GB/s (algorithmic) | of 8 TB/s",
           "---|---|---|---|---|---"]
    for i, (e, p) in enumerate(labels):
        rs = [rows[k * len(labels) + i] for k in range(rounds)]
        ms = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rs) / rounds / 1e6
        regs = f"{rs[0]['VGPR_Count']} + {rs[0]['Accum_VGPR_Count']}"
        b = PHASE_BYTES.get(p)
        bw = f"{b * cells / (ms * 1e-3) / 1e9:.0f} | {b * cells / (ms * 1e-3) / 8e12 * 100:.1f} %" if b else "— | —"
        out.append(f"{e} | {p} | {ms:.4f} | {regs} | {bw}")
    return "\n".join(out)


def net_run(k: int = 20) -> None:
    """The learned guess's inference over all 4.4 M cells of the 1024-column
    batch, k times after 3 untimed calls, with small random weights (the
    kernel's work does not depend on their values)."""
    import time
    import numpy as np
    import torch
    from . import jfnk as J, workloads as W
    packed = W.pack(W.config2())
    prob, ne, phi, _, _ = J.device_problem(packed)
    net = J.Net(J.net_default_config(max_cols=packed.ncols, max_total_cells=packed.total))
    rng = np.random.default_rng(0)
    net.set_params((rng.standard_normal(net.get_params().size) * 0.05).astype(np.float32))
    prev_n, prev_p = ne * 0.99, phi * 0.99
    for _ in range(3):
        net.predict(prob, ne, phi, prev_n, prev_p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(k):
        net.predict(prob, ne, phi, prev_n, prev_p)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / k
    print(f"net-run: full-batch inference {dt * 1e3:.3f} ms per call ({packed.total} cells, {k} calls)", flush=True)
    net.close()


def copy_bw(mib: int = 1024, k: int = 20) -> str:
    """Bytes read plus written per second of torch's device-to-device copy of
    mib MiB, k copies timed with events after 3 untimed ones: what a plain
    streaming kernel reaches on this GPU, beside the 8 TB/s peak."""
    import torch
    src = torch.ones(mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(k):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / k
    gbs = 2 * src.numel() * 8 / (ms * 1e-3) / 1e9
    return f"copy-bw: {mib} MiB device copy {ms:.4f} ms, {gbs:.0f} GB/s read + write ({gbs / 8000 * 100:.1f} % of 8 TB/s)"


def sq(d: str, kernel: str) -> str:
    """Mean per dispatch of every counter of a --pmc run, over the
    dispatches whose kernel name contains `kernel` (each counter summed over
    its hardware instances)."""
    tot, disp = {}, {}
    for r in csv.DictReader(open(_find(d, "counter_collection.csv"))):
        if kernel not in r.get("Kernel_Name", ""):
            continue
        c = r["Counter_Name"]
        tot[c] = tot.get(c, 0.0) + float(r["Counter_Value"])
        disp.setdefault(c, set()).add(r["Dispatch_Id"])
    return "\n".join(f"{c} | {len(disp[c])} | {tot[c] / len(disp[c]):.6g}" for c in sorted(tot))


def phase_traffic(d: str, n: int = 1 << 22) -> str:
    """Table of HBM bytes per cell (read, write) of every single-phase launch
    of a DRAM-counter run of phase_run, averaged over the rounds."""
    rows = list(csv.DictReader(open(_find(d, "counter_collection.csv"))))
    disp = {}
    for r in rows:
        if "k_phase" not in r.get("Kernel_Name", ""):
            continue
        e = disp.setdefault(int(r["Dispatch_Id"]), {})
        e[r["Counter_Name"]] = float(r["Counter_Value"])
    order = [disp[k] for k in sorted(disp)]
    labels = [(e, p) for e, ps in PHASE_EXPORTS for p in ps]
    if len(order) != PHASE_ROUNDS * len(labels):
        raise RuntimeError(f"{len(order)} single-phase launches, expected {PHASE_ROUNDS * len(labels)}")
    out = ["export | launch | read B/cell | write B/cell", "---|---|---|---"]
    for i, (e, p) in enumerate(labels):
        rd = sum(32.0 * order[k * len(labels) + i]["TCC_EA0_RDREQ_DRAM_32B_sum"] for k in range(PHASE_ROUNDS))
        wr = sum(32.0 * order[k * len(labels) + i]["TCC_EA0_WRREQ_WRITE_DRAM_32B_sum"] for k in range(PHASE_ROUNDS))
        out.append(f"{e} | {p} | {rd / PHASE_ROUNDS / n:.1f} | {wr / PHASE_ROUNDS / n:.1f}")
    return "\n".join(out)


if __name__ == "__main__":
    if len(sys.argv) == 1:
        print(source_hash())
    elif sys.argv[1] == "stats":
        print(stats(sys.argv[2]))
    elif sys.argv[1] == "pmc":
        print(json.dumps(pmc(sys.argv[2], sys.argv[3], sys.argv[4]), indent=1))
    elif sys.argv[1] == "dram":
        print(json.dumps(dram(sys.argv[2], sys.argv[3]), indent=1))
    elif sys.argv[1] == "phase-run":
        phase_run(*(int(a) for a in sys.argv[2:3]))
    elif sys.argv[1] == "phase-traffic":
        print(phase_traffic(sys.argv[2], *(int(a) for a in sys.argv[3:4])))
    elif sys.argv[1] == "batch-run":
        batch_run(*(int(a) for a in sys.argv[2:4]))
    elif sys.argv[1] == "batch-phases":
        print(batch_phases(sys.argv[2]))
    elif sys.argv[1] == "net-run":
        net_run(*(int(a) for a in sys.argv[2:3]))
    elif sys.argv[1] == "sq":
        print(sq(sys.argv[2], sys.argv[3]))
    elif sys.argv[1] == "copy-bw":
        print(copy_bw(), flush=True)
    else:
        raise SystemExit(__doc__)
