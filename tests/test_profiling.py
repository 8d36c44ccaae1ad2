"""Host-side checks of the rocprofv3 summaries (no GPU): HBM bytes per launch
from the L2's DRAM-sector counters (32 B per sector) and the per-phase table of
the single-phase launches, from synthetic counter files."""
import csv
import json
import os

from paper_1904_08510_amd import profiling as P

RD, WR = "TCC_EA0_RDREQ_DRAM_32B_sum", "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum"


def write_counters(d, rows):
    """rows: (dispatch id, kernel name, counter name, value)."""
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for di, k, c, v in rows:
            w.writerow(dict(Dispatch_Id=di, Kernel_Name=k, Counter_Name=c, Counter_Value=v))


def test_dram_bytes_per_launch(tmp_path):
    solve = "void (anonymous namespace)::k_solve<256, float, false>(SolveArgs)"
    launches = [("void (anonymous namespace)::k_gather<256, false>(SolveArgs)", 100, 50),
                (solve, 1000, 400), (solve, 2000, 600),
                ("__amd_rocclr_copyBuffer", P.CALIB_BYTES // 32, P.CALIB_BYTES // 32)]
    rows = []
    for di, (k, rd, wr) in enumerate(launches):
        rows += [(di, k, RD, rd), (di, k, WR, wr), (di, k, "TCC_BUBBLE_sum", 0), (di, k, "TCC_EA0_RDREQ_128B_sum", 7)]
    d = str(tmp_path / "prof")
    write_counters(d, rows)
    res = P.dram(d, str(tmp_path / "out.json"))
    s = res["kernels"]["k_solve"]
    assert s["dispatches"] == 2
    assert s["read_bytes"] == 32 * 1500 and s["write_bytes"] == 32 * 500
    assert res["traffic_bytes_per_launch"] == 32 * 2000
    assert res["kernels"]["k_gather"]["traffic_bytes_per_launch"] == 32 * 150
    assert res["copy_check"]["read_over_bytes"] == 1.0 and res["copy_check"]["write_over_bytes"] == 1.0
    assert json.load(open(tmp_path / "out.json"))["source_hash"] == P.source_hash()


def test_phase_table(tmp_path):
    labels = [(e, p) for e, ps in P.PHASE_EXPORTS for p in ps]
    n = 1000
    kname = "void (anonymous namespace)::k_phase<256, float, false>(PhaseArgs)"
    rows, di = [], 0
    for r in range(P.PHASE_ROUNDS):
        for i in range(len(labels)):
            rows += [(di, kname, RD, (i + 1 + r) * n), (di, kname, WR, n // 2)]
            di += 1
            # a copy between the launches is not a phase
            rows += [(di, "__amd_rocclr_copyBuffer", RD, 5), (di, "__amd_rocclr_copyBuffer", WR, 5)]
            di += 1
    d = str(tmp_path / "prof")
    write_counters(d, rows)
    table = P.phase_traffic(d, n).splitlines()
    assert len(table) == 2 + len(labels)
    for i, (e, p) in enumerate(labels):
        # read: 32 B x the mean over the rounds of (i + 1 + r) n sectors, per cell
        rd = 32.0 * sum(i + 1 + r for r in range(P.PHASE_ROUNDS)) / P.PHASE_ROUNDS
        assert table[2 + i] == f"{e} | {p} | {rd:.1f} | {16.0:.1f}"


def test_batch_phase_table(tmp_path):
    labels = [(e, p) for e, ps in P.PHASE_EXPORTS for p in ps]
    cells = 10 ** 6
    d = str(tmp_path / "prof")
    os.makedirs(d)
    fields = ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp", "VGPR_Count", "Accum_VGPR_Count"]
    with open(os.path.join(d, "run_kernel_trace.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        di, t = 0, 0
        for r in range(P.BATCH_ROUNDS):
            for i in range(len(labels)):
                # launch i lasts (i + 1) * 10 us plus r us; a copy in between is not a phase
                w.writerow(dict(Dispatch_Id=di, Kernel_Name="k_phase<256, float, false, -1>(PhaseArgs)",
                                Start_Timestamp=t, End_Timestamp=t + (i + 1) * 10000 + r * 1000,
                                VGPR_Count=100 + i, Accum_VGPR_Count=0))
                w.writerow(dict(Dispatch_Id=di + 1, Kernel_Name="__amd_rocclr_copyBuffer", Start_Timestamp=t,
                                End_Timestamp=t + 5, VGPR_Count=8, Accum_VGPR_Count=0))
                di, t = di + 2, t + 10 ** 6
    table = P.batch_phases(d, cells=cells).splitlines()
    assert len(table) == 2 + len(labels)
    for i, (e, p) in enumerate(labels):
        ms = ((i + 1) * 10000 + 1000 * sum(range(P.BATCH_ROUNDS)) / P.BATCH_ROUNDS) / 1e6
        cols = [c.strip() for c in table[2 + i].split("|")]
        assert cols[:4] == [e, p, f"{ms:.4f}", f"{100 + i} + 0"]
        if p in P.PHASE_BYTES:
            gbs = P.PHASE_BYTES[p] * cells / (ms * 1e-3) / 1e9
            assert cols[4] == f"{gbs:.0f}"
        else:
            assert cols[4] == "—"


def test_sq_means_per_dispatch(tmp_path):
    # two dispatches of the kernel, each counter reported by two hardware
    # instances; another kernel's dispatch is left out
    rows = []
    for di in (1, 2):
        for inst in (0, 1):
            rows += [(di, "k_fused<0>(FusedArgs)", "SQ_WAVES", 10 * di + inst),
                     (di, "k_fused<0>(FusedArgs)", "SQ_INSTS_MFMA", 100)]
    rows += [(3, "k_solve<256, float, false>", "SQ_WAVES", 7)]
    d = str(tmp_path / "prof")
    write_counters(d, rows)
    table = P.sq(d, "k_fused").splitlines()
    # instances summed per dispatch, then the mean over dispatches
    assert table == ["SQ_INSTS_MFMA | 2 | 200", "SQ_WAVES | 2 | 31"]
