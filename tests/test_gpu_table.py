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
