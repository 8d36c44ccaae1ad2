"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every comparison runs the same seeded inputs through libjfnk (device) and the
oracle (host) and compares element by element.
"""
import numpy as np
import pytest

from paper_1904_08510_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def J():
    _need_gpu()
    from paper_1904_08510_amd import jfnk
    jfnk.lib()
    return jfnk


def ragged_batch(seed=7):
    """Uneven columns covering tiny, ragged (not a multiple of the
    workgroup) and multi-chunk sizes, both wall conditions."""
    rng = np.random.default_rng(seed)
    sizes = [3, 5, 64, 65, 127, 300, 1000, 1500, 2049]
    cols = []
    for i, n in enumerate(sizes):
        c = W.flame_column(n, float(rng.uniform(-900, 900)), a_ion=float(10 ** rng.uniform(15, 16.5)),
                           x_f=float(rng.uniform(0.006, 0.014)))
        if i % 3 == 1:
            c.bc_right = W.BC_ZERO_FLUX
        if i % 4 == 2:
            c.ne_left = 1e12
        cols.append(c)
    return cols


def oracle_scaled_jacobian(orc, col, ne, phi):
    oc = orc.OracleColumn(col)
    s = orc.scalings(oc)
    Jd = orc.jacobian_dense(oc, ne, phi)
    n = col.n
    sf = np.tile([1 / s[0], 1 / s[1]], n)
    sx = np.tile([s[2], s[3]], n)
    return (Jd * sf[:, None]) * sx[None, :], s


def test_residual_matches_oracle(J, orc):
    cols = ragged_batch()
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    rng = np.random.default_rng(1)
    xn = packed.ne * rng.uniform(0.5, 1.5, packed.total) + 1e10
    xp = packed.phi + rng.uniform(-5, 5, packed.total)
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64))
    fe, fp, scal = solver.eval_residual(prob, ne, phi, torch.from_numpy(xn).cuda(),
                                        torch.from_numpy(xp).cuda())
    fe, fp = fe.cpu().numpy(), fp.cpu().numpy()
    for i, col in enumerate(cols):
        sl = slice(packed.col_offset[i], packed.col_offset[i + 1])
        oc = orc.OracleColumn(col)
        s = orc.scalings(oc)
        np.testing.assert_allclose(scal[i], s, rtol=1e-14, atol=0)
        ofe, ofp = orc.residual(oc, xn[sl], xp[sl])
        assert np.max(np.abs(fe[sl] - ofe)) / s[0] < 1e-13, i
        assert np.max(np.abs(fp[sl] - ofp)) / s[1] < 1e-13, i


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_block_solve_backward_error(J, orc, prec):
    cols = ragged_batch(seed=3)
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    rng = np.random.default_rng(2)
    xn = packed.ne * rng.uniform(0.7, 1.3, packed.total)
    xp = packed.phi + rng.uniform(-2, 2, packed.total)
    r = rng.standard_normal((2, packed.total))
    p = J.PREC_FP64 if prec == "fp64" else J.PREC_FP32
    solver = J.Solver(J.config_for(packed, prec_precision=p))
    zn, zp = solver.block_solve(prob, ne, phi, torch.from_numpy(xn).cuda(), torch.from_numpy(xp).cuda(),
                                torch.from_numpy(r[0].copy()).cuda(), torch.from_numpy(r[1].copy()).cuda())
    zn, zp = zn.cpu().numpy(), zp.cpu().numpy()
    worst_be = worst_fe = 0.0
    for i, col in enumerate(cols):
        sl = slice(packed.col_offset[i], packed.col_offset[i + 1])
        Js, _ = oracle_scaled_jacobian(orc, col, xn[sl], xp[sl])
        z = np.empty(2 * col.n)
        z[0::2], z[1::2] = zn[sl], zp[sl]
        b = np.empty(2 * col.n)
        b[0::2], b[1::2] = r[0][sl], r[1][sl]
        be = np.linalg.norm(Js @ z - b) / (np.linalg.norm(Js, np.inf) * np.linalg.norm(z) + np.linalg.norm(b))
        zt = orc.dense_solve(Js, b) if col.n <= 300 else np.linalg.solve(Js, b)
        fe = np.linalg.norm(z - zt) / np.linalg.norm(zt)
        worst_be, worst_fe = max(worst_be, be), max(worst_fe, fe)
        # The solve is unpivoted block elimination (chunk recursions, then PCR on
        # the interface system), backward stable only up to its growth factor:
        # on the 127-cell column (64 chunks of two rows, nearly all of the
        # elimination in the PCR) it reaches 3e-12 ... 1.7e-11 over seeds 3, 5
        # and 11, the other columns <= 5e-12.  The residual is taken with the
        # oracle's Jacobian, whose entries the GPU forms in another rounding
        # order (Bernoulli pairs, face-coefficient ratios).
        if prec == "fp64":
            assert be < 5e-11 and fe < 1e-7, (i, col.n, be, fe)
        else:
            assert be < 1e-6 and fe < 1e-4, (i, col.n, be, fe)
    print(f"block solve [{prec}]: worst backward error {worst_be:.2e}, forward error {worst_fe:.2e}", flush=True)


def test_jv_matches_analytic_jacobian(J, orc):
    cols = ragged_batch(seed=4)
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    rng = np.random.default_rng(5)
    xn = packed.ne * rng.uniform(0.7, 1.3, packed.total) + 1e12
    xp = packed.phi + rng.uniform(-2, 2, packed.total)
    v = rng.standard_normal((2, packed.total))
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64))
    wn, wp = solver.eval_jv(prob, ne, phi, torch.from_numpy(xn).cuda(), torch.from_numpy(xp).cuda(),
                            torch.from_numpy(v[0].copy()).cuda(), torch.from_numpy(v[1].copy()).cuda())
    wn, wp = wn.cpu().numpy(), wp.cpu().numpy()
    for i, col in enumerate(cols):
        sl = slice(packed.col_offset[i], packed.col_offset[i + 1])
        Js, _ = oracle_scaled_jacobian(orc, col, xn[sl], xp[sl])
        vv = np.empty(2 * col.n)
        vv[0::2], vv[1::2] = v[0][sl], v[1][sl]
        ref = Js @ vv
        got = np.empty(2 * col.n)
        got[0::2], got[1::2] = wn[sl], wp[sl]
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err < 1e-4, (i, col.n, err)


def _check_roots(orc, cols, packed, got_n, got_p, tol):
    worst = 0.0
    for i, col in enumerate(cols):
        sl = slice(packed.col_offset[i], packed.col_offset[i + 1])
        r = orc.newton(orc.OracleColumn(col), reference=True)
        assert r.status == orc.CONVERGED
        en = np.linalg.norm(got_n[sl] - r.ne) / np.linalg.norm(r.ne)
        ep = np.linalg.norm(got_p[sl] - r.phi) / max(np.linalg.norm(r.phi), 1e-300)
        worst = max(worst, en, ep)
        assert en <= tol and ep <= tol, (i, col.n, en, ep)
        # the GPU answer itself satisfies the stopping test in the oracle's arithmetic
        assert orc.scaled_residual_inf(orc.OracleColumn(col), got_n[sl], got_p[sl]) < 2e-10
    return worst


@pytest.mark.parametrize("sched", ["batched", "plain"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_step_matches_oracle_root(J, orc, sched, prec):
    cols = ragged_batch(seed=11)
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    cfg = J.config_for(packed, prec_precision=J.PREC_FP64 if prec == "fp64" else J.PREC_FP32,
                       schedule=J.SCHED_BATCHED if sched == "batched" else J.SCHED_PLAIN)
    solver = J.Solver(cfg)
    rc, st = solver.step(prob, ne, phi)
    assert rc == J.JFNK_OK, (st.status, st.res_scaled)
    assert np.all(st.res_scaled <= 1e-10)
    tol = 1e-9 if prec == "fp64" else 1e-5
    _check_roots(orc, cols, packed, ne.cpu().numpy(), phi.cpu().numpy(), tol)


def test_plain_and_batched_agree(J):
    cols = ragged_batch(seed=12)
    packed = W.pack(cols)
    out = {}
    for sched in (J.SCHED_PLAIN, J.SCHED_BATCHED):
        prob, ne, phi, _, _ = J.device_problem(packed)
        solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64, schedule=sched))
        rc, st = solver.step(prob, ne, phi)
        assert rc == J.JFNK_OK
        out[sched] = (ne.cpu().numpy(), phi.cpu().numpy(), st.newton_iters.copy(), st.gmres_iters.copy())
    a, b = out[J.SCHED_PLAIN], out[J.SCHED_BATCHED]
    # same iterations; the host and device scalar arithmetic (sqrt, hypot)
    # may differ in the last bit, so the roots agree to rounding level
    np.testing.assert_allclose(a[0], b[0], rtol=1e-11, atol=1e-11 * np.abs(a[0]).max())
    np.testing.assert_allclose(a[1], b[1], rtol=1e-11, atol=1e-11 * np.abs(a[1]).max())
    assert np.array_equal(a[2], b[2])


@pytest.mark.parametrize("threads", [64, 256])
def test_batched_steps_are_reproducible(J, threads):
    """The solve launch has no data race between the threads of a column:
    the same steps from the same state give bit-identical states and
    iteration counts (every reduction runs in a fixed order)."""
    packed = W.pack(W.config2(seed=2300, ncols=24, nmin=400, nmax=3000))
    runs = []
    for rep in range(2):
        prob, ne, phi, _, _ = J.device_problem(packed)
        solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP32, threads_override=threads))
        pne = pph = None
        counts = []
        for k in range(6):
            cur = (ne.clone(), phi.clone())
            rc, st = solver.step(prob, ne, phi, pne, pph)
            assert rc == J.JFNK_OK, st.status
            counts.append(np.stack([st.newton_iters, st.gmres_iters, st.chord_steps, st.phase_counts[:, 0]]))
            pne, pph = cur
        solver.close()
        runs.append((ne.cpu().numpy(), phi.cpu().numpy(), np.array(counts)))
    for x, y in zip(runs[0], runs[1]):
        assert np.array_equal(x, y)


def test_batched_step_launch_times(J):
    """A batched step is three launches (gather, solve, write-back), each
    timed on the step's stream; the plain schedule reports none of them."""
    cols = ragged_batch(seed=13)
    packed = W.pack(cols)
    for sched in (J.SCHED_BATCHED, J.SCHED_PLAIN):
        prob, ne, phi, _, _ = J.device_problem(packed)
        solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64, schedule=sched))
        rc, st = solver.step(prob, ne, phi)
        assert rc == J.JFNK_OK
        ms, launches = solver.last_timing()
        kt = solver.last_kernel_times()
        if sched == J.SCHED_BATCHED:
            assert launches == 3
            assert all(x > 0.0 for x in kt), kt
            # the three launches lie inside the span the step timing covers
            assert sum(kt) <= ms * 1.001 + 1e-3, (kt, ms)
        else:
            assert launches == -1
            assert kt == (-1.0, -1.0, -1.0)
        solver.close()


def test_config0_single_column(J, orc):
    cols = W.config0()
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64, schedule=J.SCHED_PLAIN))
    rc, st = solver.step(prob, ne, phi)
    assert rc == J.JFNK_OK
    _check_roots(orc, cols, packed, ne.cpu().numpy(), phi.cpu().numpy(), 1e-9)


def test_config1_march_with_extrapolation(J, orc):
    """The 4096-cell column at 1000 V marched 10 steps with the extrapolated
    guess, each step compared with the oracle's root from the same X^n."""
    col = W.config1()[0]
    packed = W.pack([col])
    prob, ne, phi, _, _ = J.device_problem(packed)
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64, guess=J.GUESS_EXTRAP))
    ne_prev = phi_prev = None
    for k in range(10):
        xn_n, xn_p = ne.cpu().numpy().copy(), phi.cpu().numpy().copy()
        old_n, old_p = ne.clone(), phi.clone()
        rc, st = solver.step(prob, ne, phi, ne_prev, phi_prev)
        assert rc == J.JFNK_OK
        if k == 1:
            # right after the initial transient X^n beats the extrapolation
            assert st.guess_used[0] == J.GUESS_PREV
        r = orc.newton(orc.OracleColumn(col, xn_n, xn_p), reference=True)
        got_n, got_p = ne.cpu().numpy(), phi.cpu().numpy()
        assert np.linalg.norm(got_n - r.ne) / np.linalg.norm(r.ne) < 1e-9
        assert np.linalg.norm(got_p - r.phi) / np.linalg.norm(r.phi) < 1e-9
        ne_prev, phi_prev = old_n, old_p


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stiff_batch_sampled_columns(J, orc, prec):
    """The stiff batch (256 columns x 65536 cells, 5-10 kV, dt = 1e-4 s, dt
    over the dielectric relaxation time ~1e6) marched 5 steps in one batch;
    sampled columns are compared, step by step, with the oracle's root from
    the same X^n (the GPU's) and the final states must be roots in the
    oracle's arithmetic."""
    cols = W.config4()
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    p = J.PREC_FP64 if prec == "fp64" else J.PREC_FP32
    solver = J.Solver(J.config_for(packed, prec_precision=p, guess=J.GUESS_EXTRAP))
    sample = [0, 97, 170, 255]
    tol = 1e-9 if prec == "fp64" else 1e-5
    pne = pph = None
    for k in range(5):
        off = packed.col_offset
        xn = {c: (ne[off[c]:off[c + 1]].cpu().numpy(), phi[off[c]:off[c + 1]].cpu().numpy()) for c in sample}
        xp = None if pne is None else {c: (pne[off[c]:off[c + 1]].cpu().numpy(), pph[off[c]:off[c + 1]].cpu().numpy())
                                       for c in sample}
        cur = (ne.clone(), phi.clone())
        rc, st = solver.step(prob, ne, phi, pne, pph)
        assert rc == J.JFNK_OK, (k, np.bincount(st.status))
        assert st.res_scaled.max() <= 1e-10
        for c in sample:
            oc = orc.OracleColumn(cols[c], *xn[c])
            g = xn[c]
            if xp is not None:
                e = (2 * xn[c][0] - xp[c][0], 2 * xn[c][1] - xp[c][1])
                if orc.scaled_residual_inf(oc, *e) <= orc.scaled_residual_inf(oc, *g):
                    g = e
            r = orc.newton(oc, g[0].copy(), g[1].copy(), reference=True)
            got_n = ne[off[c]:off[c + 1]].cpu().numpy()
            got_p = phi[off[c]:off[c + 1]].cpu().numpy()
            en = np.linalg.norm(got_n - r.ne) / np.linalg.norm(r.ne)
            ep = np.linalg.norm(got_p - r.phi) / np.linalg.norm(r.phi)
            assert en < tol and ep < tol, (k, c, en, ep)
            assert orc.scaled_residual_inf(oc, got_n, got_p) <= 2e-10, (k, c)
        pne, pph = cur


def test_advection_velocity(J, orc):
    """Face velocities enter the Scharfetter-Gummel Peclet number."""
    col = W.flame_column(333, 150.0)
    uf = np.linspace(-40.0, 60.0, col.n + 1)
    col.uface = uf
    packed = W.pack([col])
    prob, ne, phi, _, _ = J.device_problem(packed)
    prob.uface = torch.from_numpy(uf.copy()).cuda()
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64))
    rc, st = solver.step(prob, ne, phi)
    assert rc == J.JFNK_OK
    r = orc.newton(orc.OracleColumn(col), reference=True)
    assert np.linalg.norm(ne.cpu().numpy() - r.ne) / np.linalg.norm(r.ne) < 1e-9
    assert np.linalg.norm(phi.cpu().numpy() - r.phi) / np.linalg.norm(r.phi) < 1e-9


def test_invalid_arguments_leave_outputs_untouched(J):
    cols = [W.flame_column(100, 50.0)]
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    solver = J.Solver(J.config_for(packed))
    before = ne.clone()
    prob.dt = np.array([-1.0])
    rc, _ = solver.step(prob, ne, phi, raw=True)
    assert rc == J.JFNK_EINVAL
    assert torch.equal(ne, before)
    prob.dt = np.array([1e-5])
    big = W.pack([W.flame_column(200, 50.0)])
    prob2, ne2, phi2, _, _ = J.device_problem(big)
    rc, _ = solver.step(prob2, ne2, phi2, raw=True)
    assert rc == J.JFNK_ECAPACITY


def test_empty_batch_and_short_columns_are_rejected(J):
    """An empty batch (ncols = 0) and a column of fewer than 3 cells (the
    smallest grid with an interior cell) are invalid arguments: the call
    returns JFNK_EINVAL and leaves the state untouched; the same context
    then steps a valid batch."""
    packed = W.pack([W.flame_column(50, 20.0), W.flame_column(40, -20.0)])
    prob, ne, phi, _, _ = J.device_problem(packed)
    solver = J.Solver(J.config_for(packed))
    before = (ne.clone(), phi.clone())
    prob.ncols = 0
    rc, _ = solver.step(prob, ne, phi, raw=True)
    assert rc == J.JFNK_EINVAL
    assert torch.equal(ne, before[0]) and torch.equal(phi, before[1])
    prob.ncols = 2
    prob.col_offset = np.array([0, 2, 90], dtype=packed.col_offset.dtype)    # a 2-cell column
    rc, _ = solver.step(prob, ne, phi, raw=True)
    assert rc == J.JFNK_EINVAL
    assert torch.equal(ne, before[0]) and torch.equal(phi, before[1])
    prob.col_offset = packed.col_offset.copy()
    rc, st = solver.step(prob, ne, phi)
    assert rc == J.JFNK_OK and np.all(st.res_scaled <= 1e-10)


@pytest.mark.parametrize("sched", ["batched", "plain"])
def test_bad_input_columns_are_isolated(J, sched):
    """Per-cell inputs outside the problem's domain (a non-finite source, a
    negative mobility, a zero diffusivity, a negative loss rate, a non-finite
    start state) are found on the device: the column is not iterated, keeps
    X^n and reports JFNK_COL_BAD_INPUT; the other columns are solved as if
    alone."""
    base = [W.flame_column(200, 100.0), W.flame_column(300, -200.0), W.flame_column(150, 40.0),
            W.flame_column(260, 500.0), W.flame_column(90, -60.0), W.flame_column(333, 250.0)]
    packed = W.pack(base)
    o = packed.col_offset
    packed.src[o[1] + 17] = np.nan
    packed.mu[o[2] + 149] = -0.1          # the last cell: its wall face too
    packed.diff[o[3]] = 0.0               # the first cell
    packed.kloss[o[4] + 40] = -1.0
    packed.ne[o[5] + 100] = np.inf
    prob, ne, phi, _, _ = J.device_problem(packed)
    ne0, phi0 = ne.clone(), phi.clone()
    cfg = J.config_for(packed, prec_precision=J.PREC_FP64,
                       schedule=J.SCHED_BATCHED if sched == "batched" else J.SCHED_PLAIN)
    solver = J.Solver(cfg)
    rc, st = solver.step(prob, ne, phi)
    assert rc == J.JFNK_NOT_CONVERGED
    assert list(st.status) == [J.COL_CONVERGED] + [J.COL_BAD_INPUT] * 5, st.status
    assert np.all(st.newton_iters[1:] == 0)
    for c in range(1, 6):
        sl = slice(o[c], o[c + 1])
        assert torch.equal(ne[sl], ne0[sl]) and torch.equal(phi[sl], phi0[sl])
    # column 0 equals the same column solved alone in the same schedule (the
    # plain schedule's Givens rotations run on the host, so across schedules
    # the roots agree to rounding level only: test_plain_and_batched_agree)
    alone = W.pack(base[:1])
    p1, n1, f1, _, _ = J.device_problem(alone)
    s1 = J.Solver(J.config_for(alone, prec_precision=J.PREC_FP64,
                               schedule=J.SCHED_BATCHED if sched == "batched" else J.SCHED_PLAIN))
    s1.step(p1, n1, f1)
    assert torch.equal(ne[o[0]:o[1]], n1) and torch.equal(phi[o[0]:o[1]], f1)
    # the flag clears once the input is repaired (same context, same layout)
    packed.src[o[1] + 17] = 0.0
    prob.src = torch.from_numpy(packed.src.copy()).cuda()
    rc, st = solver.step(prob, ne, phi)
    assert st.status[1] == J.COL_CONVERGED


def test_newton_cap_flags_columns(J):
    cols = [W.flame_column(400, 700.0)]
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    solver = J.Solver(J.config_for(packed, max_newton=1))
    rc, st = solver.step(prob, ne, phi)
    assert rc == J.JFNK_NOT_CONVERGED
    assert st.status[0] == J.COL_MAX_NEWTON and st.newton_iters[0] == 1


def test_autotune_keeps_state_and_roots(J):
    """The tuner times workgroup sizes on copies (the caller's state is not
    touched) and the tuned schedule reaches the same roots."""
    cols = ragged_batch(seed=21)
    packed = W.pack(cols)
    res = {}
    for tune in (False, True):
        prob, ne, phi, _, _ = J.device_problem(packed)
        solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64))
        if tune:
            before = (ne.clone(), phi.clone())
            T, times = solver.autotune(prob, ne, phi, steps=2)
            assert T in times and times[T] == min(times.values()) and T in (64, 128, 256, 512)
            assert torch.equal(ne, before[0]) and torch.equal(phi, before[1])
        pne = pph = None
        for _ in range(3):
            cur = (ne.clone(), phi.clone())
            rc, _ = solver.step(prob, ne, phi, pne, pph)
            assert rc == J.JFNK_OK
            pne, pph = cur
        res[tune] = (ne.cpu().numpy(), phi.cpu().numpy())
    for a, b in zip(res[False], res[True]):
        assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(a)


def test_factor_reuse_follows_coefficient_changes(J):
    """A context that keeps its factors between steps gives the roots a fresh
    context gives, also when the mobility and diffusivity change between two
    steps (the stale factors must then be replaced)."""
    cols = ragged_batch(seed=23)
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    kept = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64))
    pne = pph = None
    for k in range(5):
        if k == 3:
            prob.mu.mul_(1.3)
            prob.diff.mul_(1.3)
        before = (ne.clone(), phi.clone())
        fresh = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64))
        fn, fp = ne.clone(), phi.clone()
        rc, _ = fresh.step(prob, fn, fp, pne, pph)
        assert rc == J.JFNK_OK
        fresh.close()
        rc, _ = kept.step(prob, ne, phi, pne, pph)
        assert rc == J.JFNK_OK
        for a, b in ((fn, ne), (fp, phi)):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(a), k
        pne, pph = before


def test_schur_preconditioner_apply(J, orc):
    """The approximate-Schur preconditioner (eq:prec_recast with S~ = L +
    I_e dt D_r) against its definition composed from the oracle's scaled
    Jacobian blocks with dense solves."""
    cols = [c for c in ragged_batch(seed=5) if c.n <= 1000]
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    rng = np.random.default_rng(8)
    xn = packed.ne * rng.uniform(0.8, 1.2, packed.total)
    xp = packed.phi + rng.uniform(-1, 1, packed.total)
    r = rng.standard_normal((2, packed.total))
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64, prec_kind=J.PRECK_SCHUR))
    zn, zp = solver.block_solve(prob, ne, phi, torch.from_numpy(xn).cuda(), torch.from_numpy(xp).cuda(),
                                torch.from_numpy(r[0].copy()).cuda(), torch.from_numpy(r[1].copy()).cuda())
    zn, zp = zn.cpu().numpy(), zp.cpu().numpy()
    for i, col in enumerate(cols):
        sl = slice(packed.col_offset[i], packed.col_offset[i + 1])
        Js, s = oracle_scaled_jacobian(orc, col, xn[sl], xp[sl])
        Jnn, Jnp = Js[0::2, 0::2], Js[0::2, 1::2]
        Jpn, Jpp = Js[1::2, 0::2], Js[1::2, 1::2]
        # (dt D_f - I)^-1 ~ -I in unscaled units, i.e. -(s_Fn / s_Xn) I here
        St = Jpp + (s[0] / s[2]) * (Jpn @ Jnp)
        ze1 = np.linalg.solve(Jnn, r[0][sl])
        zphi = np.linalg.solve(St, r[1][sl] - Jpn @ ze1)
        ze = ze1 - np.linalg.solve(Jnn, Jnp @ zphi)
        ref = np.concatenate([ze, zphi])
        got = np.concatenate([zn[sl], zp[sl]])
        # three chained solves: forward error up to ~cond(S~) x 1e-16 (|z| reaches 1e5 here)
        assert np.linalg.norm(got - ref) <= 1e-7 * np.linalg.norm(ref), (i, col.n)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_schur_preconditioner_reaches_the_same_roots(J, prec):
    """JFNK with the paper's approximate-Schur preconditioner converges to the
    roots the exact block preconditioner gives, with more GMRES iterations.
    S~ replaces (dt D_f - I)^-1 by -I, which the paper states is good for small
    time steps: dt = 1e-8 s here (dt D / h^2 <= ~3); at the workloads' 1e-5 s
    (dt D / h^2 up to ~1e5) the approximation is poor and Newton stalls."""
    cols = W.config2(seed=2200, ncols=12, nmin=512, nmax=2048, dt=1e-8)
    packed = W.pack(cols)
    p = J.PREC_FP64 if prec == "fp64" else J.PREC_FP32
    out = {}
    for kind in (J.PRECK_BLOCK, J.PRECK_SCHUR):
        prob, ne, phi, _, _ = J.device_problem(packed)
        solver = J.Solver(J.config_for(packed, prec_precision=p, prec_kind=kind))
        pne = pph = None
        gm = 0
        for _ in range(3):
            cur = (ne.clone(), phi.clone())
            rc, st = solver.step(prob, ne, phi, pne, pph)
            assert rc == J.JFNK_OK, np.bincount(st.status)
            gm += int(st.gmres_iters.sum())
            pne, pph = cur
        out[kind] = (ne.cpu().numpy(), phi.cpu().numpy(), gm)
    (a0, a1, ga), (b0, b1, gb) = out[J.PRECK_BLOCK], out[J.PRECK_SCHUR]
    tol = 1e-9 if prec == "fp64" else 1e-5
    assert np.linalg.norm(a0 - b0) <= tol * np.linalg.norm(a0)
    assert np.linalg.norm(a1 - b1) <= tol * np.linalg.norm(a1)
    print(f"GMRES iterations over 3 steps, {prec}: block {ga}, approximate Schur {gb}")


def test_unpreconditioned_gmres(J):
    """Without a preconditioner (P = I, the baseline of the paper's comparison
    of iteration counts in Section 3.2) the apply is the identity, and JFNK
    reaches the roots of the preconditioned runs with many more GMRES
    iterations.  Short columns and dt = 1e-8 s keep the scaled Jacobian's
    condition number within reach of restarted GMRES(30)."""
    cols = W.config2(seed=2400, ncols=6, nmin=40, nmax=96, dt=1e-8)
    packed = W.pack(cols)
    rng = np.random.default_rng(31)
    prob, ne, phi, _, _ = J.device_problem(packed)
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64, prec_kind=J.PRECK_NONE))
    xn = torch.from_numpy(packed.ne * rng.uniform(0.8, 1.2, packed.total)).cuda()
    xp = torch.from_numpy(packed.phi + rng.uniform(-1, 1, packed.total)).cuda()
    r = rng.standard_normal((2, packed.total))
    zn, zp = solver.block_solve(prob, ne, phi, xn, xp, torch.from_numpy(r[0].copy()).cuda(),
                                torch.from_numpy(r[1].copy()).cuda())
    assert np.array_equal(zn.cpu().numpy(), r[0]) and np.array_equal(zp.cpu().numpy(), r[1])
    solver.close()
    out = {}
    for kind in (J.PRECK_BLOCK, J.PRECK_SCHUR, J.PRECK_NONE):
        prob, ne, phi, _, _ = J.device_problem(packed)
        solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64, prec_kind=kind, max_restarts=60))
        pne = pph = None
        gm = nw = 0
        for _ in range(3):
            cur = (ne.clone(), phi.clone())
            rc, st = solver.step(prob, ne, phi, pne, pph)
            assert rc == J.JFNK_OK, (kind, np.bincount(st.status))
            gm += int(st.gmres_iters.sum())
            nw += int(st.newton_iters.sum())
            pne, pph = cur
        solver.close()
        out[kind] = (ne.cpu().numpy(), phi.cpu().numpy(), gm, nw)
    a = out[J.PRECK_BLOCK]
    for kind in (J.PRECK_SCHUR, J.PRECK_NONE):
        b = out[kind]
        assert np.linalg.norm(a[0] - b[0]) <= 1e-8 * np.linalg.norm(a[0]), kind
        assert np.linalg.norm(a[1] - b[1]) <= 1e-8 * np.linalg.norm(a[1]), kind
    print("GMRES iterations / Newton iterations over 3 steps: block %d/%d, approximate Schur %d/%d, none %d/%d"
          % (out[0][2], out[0][3], out[1][2], out[1][3], out[2][2], out[2][3]))
    assert out[J.PRECK_NONE][2] > out[J.PRECK_SCHUR][2] >= out[J.PRECK_BLOCK][2]


@pytest.mark.parametrize("kind", ["schur", "none"])
def test_plain_schedule_other_preconditioners(J, kind):
    """The host-driven schedule runs the same phase code with the approximate
    Schur and the identity preconditioners: same iterations and roots as the
    batched launch."""
    cols = W.config2(seed=2401, ncols=4, nmin=40, nmax=96, dt=1e-8)
    packed = W.pack(cols)
    k = J.PRECK_SCHUR if kind == "schur" else J.PRECK_NONE
    out = {}
    for sched in (J.SCHED_PLAIN, J.SCHED_BATCHED):
        prob, ne, phi, _, _ = J.device_problem(packed)
        solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64, schedule=sched, prec_kind=k,
                                       max_restarts=60))
        rc, st = solver.step(prob, ne, phi)
        assert rc == J.JFNK_OK, np.bincount(st.status)
        solver.close()
        out[sched] = (ne.cpu().numpy(), phi.cpu().numpy(), st.newton_iters.copy(), st.gmres_iters.copy())
    a, b = out[J.SCHED_PLAIN], out[J.SCHED_BATCHED]
    assert np.array_equal(a[2], b[2])
    # host and device scalar arithmetic (sqrt, hypot) may differ in the last
    # bit.  Unpreconditioned GMRES runs hundreds of iterations and stops on the
    # residual alone, so its two roots agree only to the accuracy that
    # criterion fixes (relative 1e-9 here); with a preconditioner the error
    # estimate pins them to rounding level.
    tol = 1e-10 if kind == "schur" else 1e-8
    for x, y in ((a[0], b[0]), (a[1], b[1])):
        assert np.linalg.norm(x - y) <= tol * np.linalg.norm(x), (kind, np.linalg.norm(x - y) / np.linalg.norm(x))


def test_problem_struct_follows_reassigned_fields(J):
    """The binding caches the C argument struct of a problem: in-place updates
    of its arrays reach the library through the cached pointers, and a
    reassigned field rebuilds it."""
    packed = W.pack(W.config2(seed=2600, ncols=3, nmin=100, nmax=200))
    prob, ne, phi, _, _ = J.device_problem(packed)
    p1 = prob.cstruct()
    assert prob.cstruct() is p1
    assert p1.mu == prob.mu.data_ptr()
    dt_ptr = prob.dt.ctypes.data
    prob.dt *= 0.5                       # in place: same array, same struct
    assert prob.cstruct() is p1 and prob.dt.ctypes.data == dt_ptr
    prob.mu = prob.mu * 1.3              # a new tensor
    p2 = prob.cstruct()
    assert p2 is not p1 and p2.mu == prob.mu.data_ptr()
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64))
    rc, _ = solver.step(prob, ne, phi)
    assert rc == J.JFNK_OK
    solver.close()


@pytest.mark.parametrize("asynchronous", [False, True])
def test_out_of_place_steps_alternate_two_states(J, asynchronous):
    """With ne_out/phi_out a step leaves X^n in place and writes X^{n+1}
    elsewhere; written over X^{n-1}, it lets a caller alternate two states
    without copies.  The states equal those of in-place steps bit for bit."""
    packed = W.pack(W.config2(seed=2700, ncols=16, nmin=300, nmax=2000))
    n = packed.ncols
    prob, ne, phi, _, _ = J.device_problem(packed)
    ne0, phi0 = ne.clone(), phi.clone()
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP32))
    pn = pp = None
    ref = []
    for k in range(6):
        cur = (ne.clone(), phi.clone())
        rc, _ = solver.step(prob, ne, phi, pn, pp)
        assert rc == J.JFNK_OK
        ref.append((ne.cpu().numpy(), phi.cpu().numpy()))
        pn, pp = cur
    solver.close()
    a = (ne0.clone(), phi0.clone())
    b = (torch.empty_like(ne0), torch.empty_like(phi0))
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP32))
    got = []
    for k in range(6):
        prev = b if k else (None, None)
        if asynchronous:
            solver.step_async(prob, a[0], a[1], prev[0], prev[1], ne_out=b[0], phi_out=b[1],
                              prev_stats=J.Stats(n))
        else:
            rc, _ = solver.step(prob, a[0], a[1], prev[0], prev[1], ne_out=b[0], phi_out=b[1])
            assert rc == J.JFNK_OK
        got.append((b[0].clone(), b[1].clone()))      # in stream order after the step
        a, b = b, a
    if asynchronous:
        rc, _ = solver.step_finish(stats=J.Stats(n))
        assert rc == J.JFNK_OK
    torch.cuda.synchronize()
    solver.close()
    for (rn, rp), (gn, gp) in zip(ref, got):
        assert np.array_equal(rn, gn.cpu().numpy()) and np.array_equal(rp, gp.cpu().numpy())
    # both outputs or neither
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP32))
    rc, _ = solver.step(prob, a[0], a[1], ne_out=b[0], raw=True)
    assert rc == J.JFNK_EINVAL
    solver.close()


def test_degenerate_columns(J):
    """Degenerate inputs: a column with no charge, source or loss starts at
    its exact root (n = 0, phi linear between the electrodes) and must stay
    there without a Newton iteration; a 3-cell column and a column with both
    electrodes at 0 V converge beside it."""
    empty = W.flame_column(700, 250.0, a_ion=0.0, src_peak=0.0, krec=0.0)
    tiny = W.flame_column(3, 10.0)
    grounded = W.flame_column(900, 0.0, a_ion=5e15)
    cols = [empty, tiny, grounded]
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64))
    rc, st = solver.step(prob, ne, phi)
    assert rc == J.JFNK_OK, st.status
    assert st.newton_iters[0] == 0 and st.chord_steps[0] == 0
    got_n = ne.cpu().numpy()[:700]
    got_p = phi.cpu().numpy()[:700]
    assert np.all(got_n == 0.0)
    np.testing.assert_allclose(got_p, empty.phi, rtol=0, atol=1e-12 * 250.0)
    assert np.all(st.res_scaled <= 1e-10)


def test_mirror_symmetry_of_a_symmetric_column(J):
    """A column whose coefficients are mirror symmetric (ion and source peaks
    at the centre, uniform 1000 K gas) with both electrodes grounded has a
    mirror-symmetric root; so has the GPU's (4096 cells, 3 steps)."""
    col = W.flame_column(4096, 0.0, a_ion=3e16, x_f=0.01)
    col.temp = np.full(col.n, 1000.0)
    col.mu = 0.4 * col.temp / 300.0
    col.diff = col.mu * W.K_BOLTZMANN * col.temp / W.E_CHARGE
    packed = W.pack([col])
    prob, ne, phi, _, _ = J.device_problem(packed)
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64))
    pne = pph = None
    for _ in range(3):
        cur = (ne.clone(), phi.clone())
        rc, _ = solver.step(prob, ne, phi, pne, pph)
        assert rc == J.JFNK_OK
        pne, pph = cur
    n = ne.cpu().numpy()
    p = phi.cpu().numpy()
    assert np.linalg.norm(n - n[::-1]) <= 1e-9 * np.linalg.norm(n)
    assert np.linalg.norm(p - p[::-1]) <= 1e-9 * np.linalg.norm(p)


def test_zero_flux_walls_conserve_electrons(J):
    """With zero-flux walls, no source and no loss the electron count is
    conserved by every step (flux telescoping), for uneven columns of up to
    8192 cells."""
    rng = np.random.default_rng(31)
    cols = []
    for n in (777, 2048, 8192):
        c = W.flame_column(n, float(rng.uniform(-500, 500)), a_ion=float(10 ** rng.uniform(15, 16.5)),
                           src_peak=0.0, krec=0.0)
        c.bc_left = c.bc_right = W.BC_ZERO_FLUX
        cols.append(c)
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64))
    before = ne.cpu().numpy().copy()
    for _ in range(3):
        rc, _ = solver.step(prob, ne, phi)
        assert rc == J.JFNK_OK
    after = ne.cpu().numpy()
    for i in range(len(cols)):
        sl = slice(packed.col_offset[i], packed.col_offset[i + 1])
        assert abs(after[sl].sum() - before[sl].sum()) <= 1e-9 * before[sl].sum(), i
