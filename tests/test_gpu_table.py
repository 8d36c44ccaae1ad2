"""GPU parity of field-dependent electron transport (Section 2.2: mobility
and diffusivity from a table in the progress variable and |E|/N) against the
oracle: residual and scalings element by element, J.v against the oracle's
Jacobian, and the roots of batched and host-driven steps in both factor
precisions.  The synthetic table stands in for the paper's BOLSIG+ tables."""
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


TAB = W.synthetic_transport_table()


def table_batch(seed=7, sizes=(3, 5, 64, 65, 127, 300, 1000, 2049)):
    rng = np.random.default_rng(seed)
    cols = []
    for i, n in enumerate(sizes):
        c = W.flame_column(n, float(rng.uniform(-1000, 1000)), a_ion=float(10 ** rng.uniform(15, 16.5)),
                           x_f=float(rng.uniform(0.006, 0.014)))
        if i % 3 == 1:
            c.bc_right = W.BC_ZERO_FLUX
        if i % 4 == 2:
            c.ne_left = 1e12
        cols.append(W.with_transport_table(c, TAB))
    return cols


def test_table_residual_and_scalings_match_oracle(J, orc):
    cols = table_batch()
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    prob.mu = prob.diff = None          # not read with a table
    rng = np.random.default_rng(1)
    xn = packed.ne * rng.uniform(0.5, 1.5, packed.total) + 1e10
    xp = packed.phi + rng.uniform(-5, 5, packed.total)
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64))
    fe, fp, scal = solver.eval_residual(prob, ne, phi, torch.from_numpy(xn).cuda(), torch.from_numpy(xp).cuda())
    fe, fp = fe.cpu().numpy(), fp.cpu().numpy()
    worst = 0.0
    for i, col in enumerate(cols):
        sl = slice(packed.col_offset[i], packed.col_offset[i + 1])
        oc = orc.OracleColumn(col)
        s = orc.scalings(oc)
        assert np.allclose(scal[i], s, rtol=1e-13, atol=0), (i, scal[i], s)
        re, rp = orc.residual(oc, xn[sl], xp[sl])
        e = max(np.max(np.abs(fe[sl] - re)) / s[0], np.max(np.abs(fp[sl] - rp)) / s[1])
        worst = max(worst, e)
        assert e < 1e-12, (i, col.n, e)
    print(f"table transport: worst residual difference {worst:.1e} of S_F", flush=True)


def test_table_jv_matches_oracle_jacobian(J, orc):
    """The finite-difference J.v sees the field dependence of the table
    coefficients: it matches the oracle's Jacobian (central differences of
    its own residual).  Bilinear interpolation makes the residual only
    piecewise smooth in phi (kinks where a face's log10(|E|/N) crosses a
    table knot), so the one-sided difference of the GPU and the oracle's
    central one agree to ~1e-3 rather than to the ~1e-6 of smooth transport;
    leaving the field dependence out would be an O(0.1) error here."""
    cols = table_batch(seed=4, sizes=(9, 64, 200))
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
        oc = orc.OracleColumn(col)
        s = orc.scalings(oc)
        Jd = orc.jacobian_dense(oc, xn[sl], xp[sl])
        sf = np.tile([1 / s[0], 1 / s[1]], col.n)
        sx = np.tile([s[2], s[3]], col.n)
        Js = (Jd * sf[:, None]) * sx[None, :]
        vv = np.empty(2 * col.n)
        vv[0::2], vv[1::2] = v[0][sl], v[1][sl]
        ref = Js @ vv
        got = np.empty(2 * col.n)
        got[0::2], got[1::2] = wn[sl], wp[sl]
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"table J.v, {col.n} cells: rel difference {err:.1e}", flush=True)
        assert err < 3e-3, (i, col.n, err)


@pytest.mark.parametrize("sched", ["batched", "plain"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_table_steps_match_oracle_roots(J, orc, sched, prec):
    """Three steps of every column with table transport, each against the
    oracle's root from the same X^n."""
    cols = table_batch(seed=11)
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    cfg = J.config_for(packed, prec_precision=J.PREC_FP64 if prec == "fp64" else J.PREC_FP32,
                       schedule=J.SCHED_BATCHED if sched == "batched" else J.SCHED_PLAIN, guess=J.GUESS_PREV)
    solver = J.Solver(cfg)
    tol = 1e-9 if prec == "fp64" else 1e-5
    worst = 0.0
    newton = gmres = 0
    for k in range(3):
        xn = ne.cpu().numpy().copy(), phi.cpu().numpy().copy()
        rc, st = solver.step(prob, ne, phi)
        assert rc == J.JFNK_OK, (k, st.status)
        newton += int(st.newton_iters.sum())
        gmres += int(st.gmres_iters.sum())
        got = ne.cpu().numpy(), phi.cpu().numpy()
        for i, col in enumerate(cols):
            sl = slice(packed.col_offset[i], packed.col_offset[i + 1])
            oc = orc.OracleColumn(col, xn[0][sl], xn[1][sl])
            r = orc.newton(oc, reference=True)
            assert r.status == orc.CONVERGED, (k, i)
            en = np.linalg.norm(got[0][sl] - r.ne) / np.linalg.norm(r.ne)
            ep = np.linalg.norm(got[1][sl] - r.phi) / max(np.linalg.norm(r.phi), 1e-300)
            worst = max(worst, en, ep)
            assert en <= tol and ep <= tol, (k, i, col.n, en, ep)
            assert orc.scaled_residual_inf(oc, got[0][sl], got[1][sl]) < 2e-10, (k, i)
    print(f"table transport [{sched}, {prec}]: worst rel L2 {worst:.1e}; Newton {newton}, GMRES {gmres} "
          f"over 3 steps", flush=True)


def test_table_preconditioner_inverts_the_full_jacobian(J, orc):
    """With table transport the preconditioner's Jacobian includes the
    coefficients' dependence on the face field: its solve inverts the
    oracle's Jacobian (central differences of the oracle's residual) up to
    the difference error at table knots, where holding the coefficients at
    the iterate's field would leave an O(0.1) error."""
    cols = table_batch(seed=4, sizes=(9, 64, 200, 1000))
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    rng = np.random.default_rng(6)
    # smooth states in a strong field: every face's potential difference is far
    # above the oracle's difference step (1e-6 of the column's potential scale),
    # so its central differences stay inside one table cell almost everywhere
    xn = packed.ne * rng.uniform(0.9, 1.1, packed.total) + 1e12
    xp = packed.phi * rng.uniform(0.99, 1.01, packed.total)
    r = rng.standard_normal((2, packed.total))
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64))
    zn, zp = solver.block_solve(prob, ne, phi, torch.from_numpy(xn).cuda(), torch.from_numpy(xp).cuda(),
                                torch.from_numpy(r[0].copy()).cuda(), torch.from_numpy(r[1].copy()).cuda())
    zn, zp = zn.cpu().numpy(), zp.cpu().numpy()
    worst = 0.0
    for i, col in enumerate(cols):
        sl = slice(packed.col_offset[i], packed.col_offset[i + 1])
        oc = orc.OracleColumn(col)
        s = orc.scalings(oc)
        Jd = orc.jacobian_dense(oc, xn[sl], xp[sl])
        sf = np.tile([1 / s[0], 1 / s[1]], col.n)
        sx = np.tile([s[2], s[3]], col.n)
        Js = (Jd * sf[:, None]) * sx[None, :]
        z = np.empty(2 * col.n)
        z[0::2], z[1::2] = zn[sl], zp[sl]
        b = np.empty(2 * col.n)
        b[0::2], b[1::2] = r[0][sl], r[1][sl]
        res = np.linalg.norm(Js @ z - b)
        be = res / (np.linalg.norm(Js, np.inf) * np.linalg.norm(z) + np.linalg.norm(b))
        worst = max(worst, be)
        print(f"table preconditioner, {col.n} cells: backward error {be:.1e} "
              f"(||J z - r|| / ||r|| = {res / np.linalg.norm(b):.1e})", flush=True)
        # the differences still cross a table knot at an occasional face (the
        # interpolant's kink), and the phi block's condition number grows as
        # n^2: the backward error, not the residual, measures the Jacobian
        assert be < 1e-6, (i, col.n, be)
    print(f"table preconditioner: worst relative residual {worst:.1e}", flush=True)


def test_table_headline_batch_converges_and_matches_oracle(J, orc):
    """The headline batch with table transport (1024 columns, 512 ... 8192
    cells, up to 1000 V) at dt = 1e-6 s, the batched step with FP32 factors:
    every column converges on every step, and sampled columns (among them
    long high-voltage ones) match the oracle's roots.  (At the headline's
    1e-5 s the oracle's own Newton fails on a few long high-voltage columns
    with this table's steep mobility drop.)"""
    tab = W.synthetic_transport_table()
    cols = [W.with_transport_table(c, tab) for c in W.config2(seed=2026, ncols=1024, dt=1e-6)]
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP32, guess=J.GUESS_EXTRAP))
    sample = [48, 258, 690, 798, int(np.argmin(np.diff(packed.col_offset)))]
    off = packed.col_offset
    pn = pp = None
    newton = gmres = 0
    worst = 0.0
    for k in range(6):
        cur = (ne.clone(), phi.clone())
        rc, st = solver.step(prob, ne, phi, pn, pp)
        assert rc == J.JFNK_OK, (k, np.flatnonzero(st.status))
        newton += int(st.newton_iters.sum())
        gmres += int(st.gmres_iters.sum())
        for c in sample:
            sl = slice(off[c], off[c + 1])
            xn = (cur[0][sl].cpu().numpy(), cur[1][sl].cpu().numpy())
            oc = orc.OracleColumn(cols[c], xn[0], xn[1])
            g = xn
            if pn is not None:
                e = (2 * xn[0] - pn[sl].cpu().numpy(), 2 * xn[1] - pp[sl].cpu().numpy())
                if orc.scaled_residual_inf(oc, *e) <= orc.scaled_residual_inf(oc, *g):
                    g = e
            ref = orc.newton(oc, g[0].copy(), g[1].copy(), reference=True)
            assert ref.status == orc.CONVERGED, (k, c)
            for a, bref in ((ne[sl].cpu().numpy(), ref.ne), (phi[sl].cpu().numpy(), ref.phi)):
                e = np.linalg.norm(a - bref) / np.linalg.norm(bref)
                worst = max(worst, e)
                assert e <= 1e-9, (k, c, e)
        pn, pp = cur
        print(f"table headline batch, step {k}: Newton {st.newton_iters.mean():.2f} per column, GMRES per Newton "
              f"{st.gmres_iters.sum() / max(st.newton_iters.sum(), 1):.2f}", flush=True)
    print(f"table headline batch: 6 steps, all columns converged, worst rel L2 {worst:.1e} on {len(sample)} "
          f"columns; GMRES per Newton {gmres / max(newton, 1):.2f}", flush=True)
