"""The autotuner's persisted results (jfnk_autotune_save / _load,
jfnk_schedule_threads): a layout tuned and saved by one context is taken by
another of the same device, precision and preconditioner kind without
tuning, and a step at the loaded workgroup size equals a step at that size
given explicitly."""
import numpy as np
import pytest

from paper_1904_08510_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def J():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_08510_amd import jfnk
    jfnk.lib()
    return jfnk


def layout_hash(col_offset):
    """64-bit FNV-1a over the column offsets' bytes (int64, little endian)."""
    h = 1469598103934665603
    for b in np.ascontiguousarray(col_offset, dtype="<i8").tobytes():
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def step_copy(solver, prob, ne, phi):
    n, p = ne.clone(), phi.clone()
    rc, st = solver.step(prob, n, p)
    assert rc == 0, st.status
    return n, p


def test_tuned_layout_round_trip(J, tmp_path):
    packed = W.pack(W.config2(seed=2300, ncols=24, nmin=400, nmax=3000))
    prob, ne, phi, _, _ = J.device_problem(packed)
    cfg = J.config_for(packed, prec_precision=J.PREC_FP32)
    a = J.Solver(cfg)
    default = a.schedule_threads(prob)
    chosen, times = a.autotune(prob, ne, phi, steps=2)
    assert chosen in times and a.schedule_threads(prob) == chosen
    path = tmp_path / "tune.txt"
    a.autotune_save(str(path))
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    f = lines[0].split()
    assert f[:2] == ["jfnk-autotune", "v1"]
    # prec, kind, table, ncols, total, layout hash, workgroup size
    assert f[3:8] == [str(J.PREC_FP32), "0", "0", "24", str(packed.total)]
    assert int(f[8], 16) == layout_hash(packed.col_offset) and int(f[9]) == chosen
    b = J.Solver(cfg)
    assert b.schedule_threads(prob) == default
    assert b.autotune_load(str(path)) == 1
    assert b.schedule_threads(prob) == chosen
    # another precision keeps nothing; another layout is not matched
    assert J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64)).autotune_load(str(path)) == 0
    other = W.pack(W.config2(seed=2301, ncols=24, nmin=400, nmax=3000))
    oprob, _, _, _, _ = J.device_problem(other)
    fresh = J.Solver(J.config_for(other, prec_precision=J.PREC_FP32))
    assert b.schedule_threads(oprob) == fresh.schedule_threads(oprob)
    # a size other than the rule's, written by hand (with a malformed line and
    # an earlier entry for the same key before it: the last line wins)
    pick = 128 if default != 128 else 256
    assert (packed.col_offset[1:] - packed.col_offset[:-1]).max() <= 64 * pick
    key = f"{f[2]} {J.PREC_FP32} 0 0 24 {packed.total} {layout_hash(packed.col_offset):016x}"
    hand = tmp_path / "hand.txt"
    hand.write_text(f"jfnk-autotune v1 {key} {default} 1 1 1 1\nnot a line\n"
                    f"jfnk-autotune v1 {key} {pick} 1 1 1 1\n")
    c = J.Solver(cfg)
    assert c.autotune_load(str(hand)) == 2
    assert c.schedule_threads(prob) == pick
    got = step_copy(c, prob, ne, phi)
    ref = step_copy(J.Solver(J.config_for(packed, prec_precision=J.PREC_FP32, threads_override=pick)), prob, ne, phi)
    assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    # a file that cannot be opened is an error
    with pytest.raises(J.JfnkError):
        c.autotune_load(str(tmp_path / "missing.txt"))
