"""The allocation-free step (jfnk_step_noalloc, workspace in the library's
static device array) against jfnk_step on a fresh context: two calls in a
row, the second with a smaller input (and X^{n-1}), the same iterates bit
for bit."""
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


def _case(J, packed, prec, with_prev):
    """(problem, X^n, X^{n-1} or None) on the device: X^n is the start state,
    or the state after one step of jfnk_step when X^{n-1} is wanted."""
    prob, ne, phi, _, _ = J.device_problem(packed)
    if not with_prev:
        return prob, (ne, phi), None
    x0 = (ne.clone(), phi.clone())
    s = J.Solver(J.config_for(packed, prec_precision=prec))
    rc, _ = s.step(prob, ne, phi)
    assert rc == J.JFNK_OK
    s.close()
    return prob, (ne, phi), x0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_step_matches_jfnk_step(J, prec):
    p = J.PREC_FP64 if prec == "fp64" else J.PREC_FP32
    big = W.pack(W.config2(seed=31, ncols=12, nmin=300, nmax=3000))
    small = W.pack(W.config2(seed=32, ncols=3, nmin=100, nmax=700))
    for packed, with_prev in ((big, False), (small, True)):
        print(f"noalloc [{prec}]: {packed.ncols} columns, {packed.total} cells, X^(n-1) {with_prev}", flush=True)
        prob, x, xp = _case(J, packed, p, with_prev)
        cfg = J.config_for(packed, prec_precision=p, guess=J.GUESS_EXTRAP)
        ref = J.Solver(cfg)
        rn, rp = x[0].clone(), x[1].clone()
        rc_ref, st_ref = ref.step(prob, rn, rp, xp[0] if xp else None, xp[1] if xp else None)
        ref.close()
        gn, gp = torch.empty_like(x[0]), torch.empty_like(x[1])
        xin = (x[0].clone(), x[1].clone())
        rc, st, msg = J.step_noalloc(cfg, prob, x[0], x[1], xp[0] if xp else None, xp[1] if xp else None,
                                     ne_out=gn, phi_out=gp)
        torch.cuda.synchronize()
        assert rc == rc_ref == J.JFNK_OK, (rc, msg)
        # out of place: X^n untouched
        assert torch.equal(x[0], xin[0]) and torch.equal(x[1], xin[1])
        assert torch.equal(gn, rn) and torch.equal(gp, rp)
        for name in ("status", "newton_iters", "gmres_iters", "backtracks", "guess_used", "chord_steps",
                     "res_scaled"):
            assert np.array_equal(getattr(st, name), getattr(st_ref, name)), name
        assert np.array_equal(st.phase_counts, st_ref.phase_counts)
        if with_prev:
            assert np.any(st.guess_used == J.GUESS_EXTRAP) or np.any(st.guess_used == J.GUESS_PREV)


def test_noalloc_capacity_and_learned_guess_rejected(J):
    """Problems beyond the static array and the learned guess are refused
    before any launch; outputs stay untouched."""
    cols = [W.flame_column(60000, 100.0)]
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    before = ne.clone()
    cfg = J.config_for(packed)
    rc, _, msg = J.step_noalloc(cfg, prob, ne, phi)
    assert rc == J.JFNK_ECAPACITY and "capacity" in msg
    assert torch.equal(ne, before)
    small = W.pack([W.flame_column(100, 10.0)])
    sprob, sne, sphi, _, _ = J.device_problem(small)
    rc, _, msg = J.step_noalloc(J.config_for(small, guess=J.GUESS_LEARNED), sprob, sne, sphi)
    assert rc == J.JFNK_EINVAL and "learned" in msg
