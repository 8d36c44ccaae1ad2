"""GPU parity of the MISDC step (Algorithm 1 with the provisional charged
species of Section 3.1 and the electron/Poisson system eq:nls; electrons and
potential implicit, one ion species explicit) against the oracle's
(oracle.misdc): every step of several columns against the oracle's step from
the same start and at the same constant-CFL time step, in both factor
precisions and both schedules, in both readings of the electrons' time
discretisation, with per-cell and table transport, DC and AC electrodes; the
orders in time on the GPU; conservation in closed columns at sizes past the
oracle's; bad ion data isolated to its column; argument errors.  Start
states are relaxed by the oracle's own backward-Euler steps (the flame
columns' initial n_e = n_i with a linear potential is far from the
electrons' quasi-equilibrium)."""
import math

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


@pytest.fixture(scope="module")
def M():
    from oracle import misdc
    return misdc


def misdc_batch(seed=3, sizes=(5, 64, 127, 300, 1000), table=None, ac=True):
    """Columns of the MISDC workload: random voltages (DC, or AC through a
    polarity change), ion peaks, one zero-flux wall."""
    rng = np.random.default_rng(seed)
    cols, ions = [], []
    for i, n in enumerate(sizes):
        volts = float(rng.uniform(-400, 400))
        amp, freq = (float(rng.uniform(200, 600)), float(rng.uniform(2e4, 1e5))) if (i % 2 and ac) else (0.0, 0.0)
        c, ion = W.misdc_column(n, volts, ac_amp=amp, ac_freq=freq, a_ion=float(10 ** rng.uniform(15, 16)),
                                x_f=float(rng.uniform(0.008, 0.012)))
        if i % 3 == 2:
            c.bc_right = W.BC_ZERO_FLUX
        if table is not None:
            c = W.with_transport_table(c, table)
        cols.append(c)
        ions.append(ion)
    return cols, ions


def with_flow(cols, seed=9):
    rng = np.random.default_rng(seed)
    for c in cols:
        c.uface = rng.uniform(-2.0, 2.0) + np.linspace(-1.0, 1.0, c.n + 1)
    return cols


def oracle_ions(M, ion):
    return M.Ions(ion.mu_i, ion.k_rec, ion.ac_amp, ion.ac_freq)


def relax(M, cols, ions, steps=3, cfl=0.5):
    """The oracle's backward-Euler MISDC steps (k_max = 1) at the CFL step
    from each column's initial state: (columns with that state, start times)."""
    t = np.zeros(len(cols))
    out = []
    for i, (c, ion) in enumerate(zip(cols, ions)):
        ne, phi, ni, t[i] = M.march(c, oracle_ions(M, ion), steps, k_max=1, cfl=cfl)
        c = c.copy()
        c.ne, c.phi, c.q = ne, phi, ni
        out.append(c)
    return out, t


def device_ions(J, packed, ions):
    mu = np.concatenate([i.mu_i for i in ions])
    kr = np.concatenate([i.k_rec for i in ions])
    return J.device_ions(mu, kr, packed.q, np.array([i.ac_amp for i in ions]),
                         np.array([i.ac_freq for i in ions]))


def run_parity(J, M, cols, ions, t0, *, steps, k_max, prec, sched, tol, electron_sdc=False, cfl=0.5):
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    prob.kloss = None
    di = device_ions(J, packed, ions)
    cfg = J.config_for(packed, prec_precision=J.PREC_FP64 if prec == "fp64" else J.PREC_FP32,
                       schedule=J.SCHED_BATCHED if sched == "batched" else J.SCHED_PLAIN)
    solver = J.Solver(cfg)
    off = packed.col_offset
    t = np.array(t0, dtype=np.float64)
    dt = np.zeros(len(cols))
    worst = 0.0
    newton = 0
    for k in range(steps):
        start = [a.cpu().numpy().copy() for a in (ne, phi, di.n_ion)]
        print(f"misdc parity [{prec}, {sched}, electron_sdc={electron_sdc}]: step {k}", flush=True)
        rc, st = solver.misdc_step(prob, di, t, k_max, ne, phi, electron_sdc=electron_sdc, cfl=cfl, dt_out=dt)
        assert rc == J.JFNK_OK, (k, st.status)
        newton += int(st.newton_iters.sum())
        got = [a.cpu().numpy() for a in (ne, phi, di.n_ion)]
        for i, col in enumerate(cols):
            sl = slice(off[i], off[i + 1])
            oi = oracle_ions(M, ions[i])
            dref = M.cfl_dt(col, oi, t[i], start[1][sl], cfl) if cfl > 0 else col.dt
            assert dt[i] == pytest.approx(dref, rel=1e-14, abs=0), (k, i, dt[i], dref)
            r = M.misdc_step(col, oi, t[i], start[0][sl], start[1][sl], start[2][sl], k_max=k_max, dt=dref,
                             electron_sdc=electron_sdc)
            for name, g, ref in (("ne", got[0][sl], r.ne), ("phi", got[1][sl], r.phi), ("ni", got[2][sl], r.ni)):
                e = np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-300)
                worst = max(worst, e)
                assert e <= tol, (k, i, col.n, name, e)
        t += dt
    return worst, newton


@pytest.mark.parametrize("sched", ["batched", "plain"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_misdc_steps_match_oracle(J, M, prec, sched):
    """Three MISDC steps (k_max = 4, CFL 0.5) of five relaxed columns, each
    against the oracle's step from the same (n_e, phi, n_i), time and step."""
    cols, ions = misdc_batch()
    cols, t0 = relax(M, cols, ions)
    worst, newton = run_parity(J, M, cols, ions, t0, steps=3, k_max=4, prec=prec, sched=sched, tol=1e-9)
    print(f"MISDC [{prec}, {sched}]: worst rel L2 {worst:.1e} over 3 steps, {newton} Newton iterations", flush=True)


def test_misdc_electron_sdc_matches_oracle(J, M):
    """The electrons' SDC-corrected reading (trapezoidal fixed point), DC
    columns, against the oracle's."""
    cols, ions = misdc_batch(seed=4, ac=False)
    cols, t0 = relax(M, cols, ions)
    worst, newton = run_parity(J, M, cols, ions, t0, steps=3, k_max=4, prec="fp64", sched="batched", tol=1e-9,
                               electron_sdc=True)
    print(f"MISDC, electron SDC: worst rel L2 {worst:.1e}, {newton} Newton iterations", flush=True)


def test_misdc_with_table_transport_and_flow(J, M):
    """Field-dependent electron transport from the table and a flow through
    the faces (the electrons' Peclet numbers and the ions' drift both see
    it), in both readings."""
    for esdc in (False, True):
        cols, ions = misdc_batch(seed=5, sizes=(9, 200, 513), table=W.synthetic_transport_table(), ac=not esdc)
        cols, t0 = relax(M, with_flow(cols), ions)
        worst, _ = run_parity(J, M, cols, ions, t0, steps=2, k_max=3, prec="fp64", sched="batched", tol=1e-9,
                              electron_sdc=esdc)
        print(f"MISDC, table transport and flow, electron_sdc={esdc}: worst rel L2 {worst:.1e}", flush=True)


def test_misdc_ac_run_through_polarity_switch(J, M):
    """An AC electrode (Section 4.5) swept through a change of sign, the
    state carried on the GPU at the CFL step: every step against the
    oracle's from the GPU's start, the time advancing with each step."""
    n = 256
    col, ion = W.misdc_column(n, 0.0, ac_amp=500.0, ac_freq=5e4, a_ion=3e15)
    col.dt = 0.5 / ion.ac_freq / 24                  # cap: at least 24 steps over the half period
    oi = oracle_ions(M, ion)
    t_start = 0.3 / ion.ac_freq
    (col,), (t,) = relax(M, [col], [ion])
    t += t_start
    packed = W.pack([col])
    prob, ne, phi, _, _ = J.device_problem(packed)
    prob.kloss = None
    di = device_ions(J, packed, [ion])
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64))
    dt = np.zeros(1)
    worst = 0.0
    signs = set()
    steps = 0
    while t < t_start + 0.5 / ion.ac_freq and steps < 200:
        start = [a.cpu().numpy().copy() for a in (ne, phi, di.n_ion)]
        rc, st = solver.misdc_step(prob, di, t, 4, ne, phi, cfl=0.5, dt_out=dt)
        assert rc == J.JFNK_OK, (steps, st.status)
        dref = M.cfl_dt(col, oi, t, start[1], 0.5)
        assert dt[0] == pytest.approx(dref, rel=1e-14, abs=0)
        r = M.misdc_step(col, oi, t, *start, k_max=4, dt=dref)
        for g, ref in ((ne, r.ne), (phi, r.phi), (di.n_ion, r.ni)):
            e = np.linalg.norm(g.cpu().numpy() - ref) / np.linalg.norm(ref)
            worst = max(worst, e)
            assert e <= 1e-9, (steps, e)
        t += dt[0]
        steps += 1
        signs.add(math.copysign(1.0, M.phi_right_at(col, oi, t)))
    assert signs == {1.0, -1.0} and steps >= 24
    print(f"AC run, {steps} steps through the polarity change: worst rel L2 {worst:.1e}", flush=True)


def _gpu_orders(J, M, col, ions, start, t_end, k_max, electron_sdc):
    res = []
    for m in (4, 8, 16, 32, 64):
        c = col.copy()
        c.dt = t_end / m
        c.ne, c.phi, c.q = start[0].copy(), start[1].copy(), start[2].copy()
        packed = W.pack([c])
        prob, ne, phi, _, _ = J.device_problem(packed)
        prob.kloss = None
        di = J.device_ions(ions.mu_i, ions.k_rec, start[2])
        # differences of the finest steps are ~1e-9 of the fields: the
        # solves stop two decades below them
        solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64, tol_f=1e-12, tol_x=1e-12))
        for s in range(m):
            rc, _ = solver.misdc_step(prob, di, s * c.dt, k_max, ne, phi, electron_sdc=electron_sdc)
            assert rc == J.JFNK_OK
        res.append([a.cpu().numpy() for a in (ne, phi, di.n_ion)])
    out = []
    for fld in range(3):
        e = [np.linalg.norm(res[i][fld] - res[i + 1][fld]) for i in range(4)]
        out.append([math.log2(e[i] / e[i + 1]) for i in range(3)])
    return out


def test_misdc_orders_in_time_on_gpu(J, M):
    """Self-convergence in dt of the GPU's MISDC steps, 64 cells at 10 V
    with the ions held in place (mobility 0), from a relaxed state (the
    oracle's, as input).  Backward-Euler electrons (eq:nls): ions second
    order, electrons near it, the potential first order with k_max = 4;
    every field first order with the predictor alone.  Electrons' SDC
    correction: every field second order."""
    n = 64
    col, _ = W.misdc_column(n, 10.0, a_ion=1e15)
    frozen = M.Ions(np.zeros(n), np.full(n, 1e-12))
    c0 = col.copy()
    c0.dt = 2e-6
    start = M.march(c0, frozen, 30, k_max=2)[:3]
    ne_o, phi_o, ni_o = _gpu_orders(J, M, col, frozen, start, 4e-6, 4, False)
    print(f"backward-Euler electrons, k_max 4: orders ne {np.round(ne_o, 3)} phi {np.round(phi_o, 3)} "
          f"ni {np.round(ni_o, 3)}", flush=True)
    assert all(o > 1.8 for o in ne_o) and all(1.9 <= o <= 2.1 for o in ni_o) and all(0.9 <= o <= 1.1 for o in phi_o)
    for fld, orders in enumerate(_gpu_orders(J, M, col, frozen, start, 4e-6, 1, False)):
        assert all(0.9 <= o <= 1.1 for o in orders), (fld, orders)
    for fld, orders in enumerate(_gpu_orders(J, M, col, frozen, start, 4e-6, 4, True)):
        print(f"electron SDC, k_max 4, field {fld}: orders {np.round(orders, 3)}", flush=True)
        assert all(1.9 <= o <= 2.1 for o in orders), (fld, orders)


def test_misdc_closed_columns_conserve_particles_at_size(J):
    """Zero-flux electron walls, ions away from the electrodes, no
    chemistry: electrons and ions are conserved by every step, at column
    lengths up to 8192 cells (no oracle needed: a property of the flux
    form)."""
    cols, ions = [], []
    for n in (1024, 4096, 8192):
        c, ion = W.misdc_column(n, 50.0, a_ion=1e15)
        c.bc_left = c.bc_right = W.BC_ZERO_FLUX
        c.src = np.zeros(n)
        x = W.cell_centres(n, c.length)
        bump = 1e15 * np.exp(-((x - 0.01) / 0.001) ** 2)
        c.ne, c.q = bump.copy(), bump.copy()
        ion.k_rec = np.zeros(n)
        cols.append(c)
        ions.append(ion)
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    prob.kloss = None
    di = device_ions(J, packed, ions)
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP32))
    off = packed.col_offset
    n0 = [float(ne[off[i]:off[i + 1]].sum()) for i in range(len(cols))]
    i0 = [float(di.n_ion[off[i]:off[i + 1]].sum()) for i in range(len(cols))]
    for k in range(5):
        rc, _ = solver.misdc_step(prob, di, 0.0, 4, ne, phi)
        assert rc == J.JFNK_OK
    for i in range(len(cols)):
        ne_sum = float(ne[off[i]:off[i + 1]].sum())
        ni_sum = float(di.n_ion[off[i]:off[i + 1]].sum())
        assert abs(ne_sum - n0[i]) <= 1e-10 * n0[i], (i, ne_sum, n0[i])
        assert abs(ni_sum - i0[i]) <= 1e-12 * i0[i], (i, ni_sum, i0[i])


def test_misdc_bad_ion_data_is_isolated(J, M):
    """A negative ion mobility in one cell flags its column (bad input; its
    state is the start of the step) and leaves the others as the oracle's."""
    cols, ions = misdc_batch(seed=8, sizes=(64, 100, 77))
    ions[1].mu_i = ions[1].mu_i.copy()
    ions[1].mu_i[40] = -1e-3
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    prob.kloss = None
    di = device_ions(J, packed, ions)
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64))
    start = [a.cpu().numpy().copy() for a in (ne, phi, di.n_ion)]
    rc, st = solver.misdc_step(prob, di, 0.0, 3, ne, phi)
    assert rc == J.JFNK_NOT_CONVERGED
    assert list(st.status) == [J.COL_CONVERGED, J.COL_BAD_INPUT, J.COL_CONVERGED]
    off = packed.col_offset
    sl = slice(off[1], off[2])
    assert np.array_equal(ne.cpu().numpy()[sl], start[0][sl])
    assert np.array_equal(phi.cpu().numpy()[sl], start[1][sl])
    assert np.array_equal(di.n_ion.cpu().numpy()[sl], start[2][sl])
    for i in (0, 2):
        sl = slice(off[i], off[i + 1])
        r = M.misdc_step(cols[i], oracle_ions(M, ions[i]), 0.0, start[0][sl], start[1][sl], start[2][sl], k_max=3)
        assert np.linalg.norm(ne.cpu().numpy()[sl] - r.ne) <= 1e-9 * np.linalg.norm(r.ne)


def test_misdc_argument_errors(J):
    cols, ions = misdc_batch(seed=2, sizes=(32, 40))
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    di = device_ions(J, packed, ions)
    solver = J.Solver(J.config_for(packed))
    before = ne.clone()
    rc, _ = solver.misdc_step(prob, di, 0.0, 4, ne, phi, raw=True)     # k_loss given
    assert rc == J.JFNK_EINVAL and "k_loss" in solver.last_error()
    prob.kloss = None
    for k_max in (0, 65):
        rc, _ = solver.misdc_step(prob, di, 0.0, k_max, ne, phi, raw=True)
        assert rc == J.JFNK_EINVAL
    di.ac_freq = None                  # amplitude without frequency
    rc, _ = solver.misdc_step(prob, di, 0.0, 4, ne, phi, raw=True)
    assert rc == J.JFNK_EINVAL
    di.ac_freq = np.array([1e4, np.inf])
    rc, _ = solver.misdc_step(prob, di, 0.0, 4, ne, phi, raw=True)
    assert rc == J.JFNK_EINVAL
    di.ac_freq = np.array([1e4, 1e4])
    for cfl in (-0.5, float("nan"), float("inf")):
        rc, _ = solver.misdc_step(prob, di, 0.0, 4, ne, phi, raw=True, cfl=cfl)
        assert rc == J.JFNK_EINVAL and "cfl" in solver.last_error()
    assert torch.equal(ne, before)


def test_misdc_benchmark_configuration_matches_oracle(J, M):
    """The MISDC leg as the benchmark runs it: the AC batch (1024 columns x
    1024 cells, Table 4's frequencies at 1000 V, each column at its own phase),
    dt capped at 1e-6 s and set by ion-drift CFL 0.5, FP32 factors, the
    workgroup size autotuned, three backward-Euler steps (k_max = 1) and then
    k_max = 4 steps.  Sampled columns (the first, the last, one per forcing
    frequency) are checked against the oracle at every step from the GPU's
    start, the CFL step included."""
    cols, ions, t0 = W.config_ac()
    for c in cols:
        c.dt = 1e-6
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    prob.kloss = None
    di = device_ions(J, packed, ions)
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP32, guess=J.GUESS_EXTRAP))
    tuned = solver.autotune(prob, ne, phi, steps=3)
    sample = sorted({0, len(cols) - 1} | set(range(1, 8)))
    off = packed.col_offset
    t = t0.copy()
    dt = np.zeros(len(cols))
    worst = 0.0
    for k, k_max in enumerate((1, 1, 1, 4, 4)):
        start = [(ne[off[c]:off[c + 1]].cpu().numpy().copy(), phi[off[c]:off[c + 1]].cpu().numpy().copy(),
                  di.n_ion[off[c]:off[c + 1]].cpu().numpy().copy()) for c in sample]
        rc, st = solver.misdc_step(prob, di, t, k_max, ne, phi, cfl=0.5, dt_out=dt)
        assert rc == J.JFNK_OK, (k, np.flatnonzero(st.status))
        for (c, s0) in zip(sample, start):
            oi = oracle_ions(M, ions[c])
            dref = M.cfl_dt(cols[c], oi, t[c], s0[1], 0.5)
            assert dt[c] == pytest.approx(dref, rel=1e-14, abs=0), (k, c)
            r = M.misdc_step(cols[c], oi, t[c], *s0, k_max=k_max, dt=dref)
            sl = slice(off[c], off[c + 1])
            for g, ref in ((ne, r.ne), (phi, r.phi), (di.n_ion, r.ni)):
                e = np.linalg.norm(g[sl].cpu().numpy() - ref) / np.linalg.norm(ref)
                worst = max(worst, e)
                assert e <= 1e-9, (k, c, e)
        t += dt
        print(f"benchmark MISDC configuration, step {k} (k_max {k_max}): worst rel L2 so far {worst:.1e}",
              flush=True)
    print(f"benchmark MISDC configuration (T = {tuned[0]}): {len(sample)} columns x 5 steps, worst rel L2 "
          f"{worst:.1e}", flush=True)


def test_misdc_with_a_learned_guess_keeps_the_oracle_roots(J, M):
    """A network attached for the predictor's guess (untrained weights: its
    candidate is evaluated and, if it loses, dropped): every MISDC step still
    ends at the oracle's result, and later SDC iterations are unaffected (they
    start from X^(k))."""
    from paper_1904_08510_amd import train_guess as TG
    cols, ions = misdc_batch(seed=12, sizes=(64, 300, 777))
    cols, t0 = relax(M, cols, ions)
    packed = W.pack(cols)
    net = J.Net(J.net_default_config(max_cols=packed.ncols, max_total_cells=packed.total))
    net.set_params(TG.init_params(3))
    prob, ne, phi, _, _ = J.device_problem(packed)
    prob.kloss = None
    di = device_ions(J, packed, ions)
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64, guess=J.GUESS_LEARNED))
    solver.set_model(net)
    off = packed.col_offset
    t = np.array(t0)
    dt = np.zeros(len(cols))
    evaluated = 0
    for k in range(3):
        start = [a.cpu().numpy().copy() for a in (ne, phi, di.n_ion)]
        pn = None if k == 0 else torch.from_numpy(prev[0]).cuda()
        pp = None if k == 0 else torch.from_numpy(prev[1]).cuda()
        rc, st = solver.misdc_step(prob, di, t, 4, ne, phi, pn, pp, cfl=0.5, dt_out=dt)
        assert rc == J.JFNK_OK, (k, st.status)
        evaluated += int(st.phase_counts[:, 7].sum())
        for i, col in enumerate(cols):
            sl = slice(off[i], off[i + 1])
            dref = M.cfl_dt(col, oracle_ions(M, ions[i]), t[i], start[1][sl], 0.5)
            r = M.misdc_step(col, oracle_ions(M, ions[i]), t[i], start[0][sl], start[1][sl], start[2][sl],
                             k_max=4, dt=dref)
            for g, ref in ((ne, r.ne), (phi, r.phi), (di.n_ion, r.ni)):
                e = np.linalg.norm(g[sl].cpu().numpy() - ref) / np.linalg.norm(ref)
                assert e <= 1e-9, (k, i, e)
        prev = start
        t += dt
    net.close()
    print(f"MISDC with a learned guess: candidate evaluated for {evaluated} predictor solves", flush=True)
    assert evaluated > 0
