"""The paper's own preconditioner at the paper's own setting (Section 3.2,
eq:prec_recast; Section 4.2, fig:Precond_tests and fig:MG_tests).

Setting of the paper's study: a 1 cm column of 512 cells (19.5 um), applied
voltages 0, 10, 50, 100, 500 and 1000 V, and a time step from a constant
charged-species convective CFL number, so that it shrinks as the voltage
grows.  The CFL number, the ion mobility and the gas velocity are readings
(0.5; 4e-3 m^2/(V s), the H3O+ value of Table 3; 0.371 m/s, the inlet speed
of Table 2): dt = 0.5 h / (0.371 + 4e-3 dV / L).  The synthetic flame column
of the workloads stands in for the paper's flame, its flame centre at 5 mm.

Compared: the approximate-Schur preconditioner with exact tridiagonal block
solves (the paper's 1D baseline), the same with multigrid V-cycles to
gamma_MG (the paper's solver), no preconditioner, and the exact block
preconditioner of this library.  Roots are checked against the oracle.
"""
import numpy as np
import pytest

from paper_1904_08510_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

VOLTS = [0.0, 10.0, 50.0, 100.0, 500.0, 1000.0]
NONE_CAP = 100            # restarts of GMRES(30) for the unpreconditioned system: 3030 iterations


@pytest.fixture(scope="module")
def J():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_08510_amd import jfnk
    jfnk.lib()
    return jfnk


def dt_cfl(n, dv, length=0.01):
    return 0.5 * (length / n) / (0.371 + 4e-3 * abs(dv) / length)


def paper_column(n, dv, dt=None):
    return W.flame_column(n, dv, length=0.01, x_f=0.005, dt=dt_cfl(n, dv) if dt is None else dt)


def one_step(J, col, kind, **kw):
    packed = W.pack([col])
    prob, ne, phi, _, _ = J.device_problem(packed)
    cfg = J.config_for(packed, prec_precision=J.PREC_FP64, prec_kind=kind, chord_tol=0.0, **kw)
    s = J.Solver(cfg)
    rc, st = s.step(prob, ne, phi, raw=True)
    s.close()
    torch.cuda.synchronize()
    return dict(rc=rc, status=int(st.status[0]), newton=int(st.newton_iters[0]), gmres=int(st.gmres_iters[0]),
                mg=int(st.mg_cycles[0]), ne=ne.cpu().numpy(), phi=phi.cpu().numpy())


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_multigrid_apply_matches_the_definition(J, orc):
    """With a tight V-cycle tolerance the multigrid block solves give the
    approximate-Schur apply of eq:prec_recast (its definition composed from
    the oracle's scaled Jacobian blocks with dense solves)."""
    cols = [paper_column(n, dv) for n, dv in ((5, 30.0), (37, 200.0), (300, 100.0), (777, 700.0))]
    packed = W.pack(cols)
    prob, ne, phi, _, _ = J.device_problem(packed)
    rng = np.random.default_rng(8)
    xn = packed.ne * rng.uniform(0.8, 1.2, packed.total)
    xp = packed.phi + rng.uniform(-1, 1, packed.total)
    r = rng.standard_normal((2, packed.total))
    for transfer in (1, 3):
        solver = J.Solver(J.config_for(packed, prec_precision=J.PREC_FP64, prec_kind=J.PRECK_SCHUR_MG,
                                       mg_tol=1e-13, mg_blocks=3, mg_transfer=transfer))
        zn, zp = solver.block_solve(prob, ne, phi, torch.from_numpy(xn).cuda(), torch.from_numpy(xp).cuda(),
                                    torch.from_numpy(r[0].copy()).cuda(), torch.from_numpy(r[1].copy()).cuda())
        solver.close()
        _check_against_definition(orc, cols, packed, xn, xp, r, zn.cpu().numpy(), zp.cpu().numpy(), transfer)


def _check_against_definition(orc, cols, packed, xn, xp, r, zn, zp, transfer):
    for i, col in enumerate(cols):
        sl = slice(packed.col_offset[i], packed.col_offset[i + 1])
        oc = orc.OracleColumn(col)
        s = orc.scalings(oc)
        Jd = orc.jacobian_dense(oc, xn[sl], xp[sl])
        sf = np.tile([1 / s[0], 1 / s[1]], col.n)
        sx = np.tile([s[2], s[3]], col.n)
        Js = (Jd * sf[:, None]) * sx[None, :]
        Jnn, Jnp = Js[0::2, 0::2], Js[0::2, 1::2]
        Jpn, Jpp = Js[1::2, 0::2], Js[1::2, 1::2]
        St = Jpp + (s[0] / s[2]) * (Jpn @ Jnp)
        ze1 = np.linalg.solve(Jnn, r[0][sl])
        zphi = np.linalg.solve(St, r[1][sl] - Jpn @ ze1)
        ze = ze1 - np.linalg.solve(Jnn, Jnp @ zphi)
        ref = np.concatenate([ze, zphi])
        got = np.concatenate([zn[sl], zp[sl]])
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"multigrid apply (transfer {transfer}), {col.n} cells: rel error {err:.1e}", flush=True)
        assert err <= 1e-7, (col.n, err)


def test_preconditioner_comparison_at_the_papers_setting(J, orc):
    """fig:Precond_tests: GMRES iterations per Newton iteration with the
    approximate-Schur preconditioner against none, 512 cells, 0-1000 V."""
    rows = []
    for dv in VOLTS:
        col = paper_column(512, dv)
        cap = 4 if dv == 0.0 else 20     # 0 V: GMRES runs to its restart cap in every Newton iteration
        sch = one_step(J, col, J.PRECK_SCHUR, max_restarts=20, max_newton=cap)
        mg = one_step(J, col, J.PRECK_SCHUR_MG, max_restarts=20, max_newton=cap, mg_tol=1e-4, mg_blocks=3)
        non = one_step(J, col, J.PRECK_NONE, max_restarts=NONE_CAP, max_newton=1)
        blk = one_step(J, col, J.PRECK_BLOCK)
        ref = orc.newton(orc.OracleColumn(col), reference=True)
        errs = {}
        for name, r in (("schur", sch), ("schur+mg", mg), ("block", blk)):
            if r["status"] == 0:
                errs[name] = max(rel(r["ne"], ref.ne), rel(r["phi"], ref.phi))
        rows.append((dv, col.dt, sch, mg, non, blk, errs))
        per = lambda r: r["gmres"] / max(r["newton"], 1)
        print(f"dV {dv:6.0f} V dt {col.dt:.2e} s | approx. Schur: status {sch['status']} Newton {sch['newton']} "
              f"GMRES/Newton {per(sch):7.1f} | + multigrid 1e-4: status {mg['status']} GMRES/Newton {per(mg):7.1f} "
              f"V-cycles {mg['mg']} | none: first Newton system {non['gmres']} GMRES "
              f"({'converged' if non['gmres'] < 30 * (NONE_CAP + 1) else 'cap'}) | block: GMRES/Newton "
              f"{per(blk):.1f} | rel L2 vs oracle {', '.join(f'{k} {v:.1e}' for k, v in errs.items())}", flush=True)
    for dv, dt, sch, mg, non, blk, errs in rows:
        assert blk["status"] == 0 and errs["block"] < 1e-9
        if dv == 0.0:
            continue   # dt D/h^2 ~ 1e5 at the CFL step of 0 V: S~ is far from S (reported, not asserted)
        assert sch["status"] == 0 and errs["schur"] < 1e-9, dv
        assert mg["status"] == 0 and errs["schur+mg"] < 1e-9, dv
        # preconditioned GMRES needs >= 20x fewer iterations per Newton system
        assert non["gmres"] >= 20 * sch["gmres"] / sch["newton"], dv
    per = [r[2]["gmres"] / r[2]["newton"] for r in rows[1:]]
    # the approximation S~ improves as the CFL time step shrinks with the voltage
    assert all(b <= a for a, b in zip(per, per[1:])), per


def test_preconditioner_size_dependence(J):
    """Size dependence at 100 V, 128 ... 2048 cells: at a constant CFL number
    (dt proportional to h) and at the fixed time step of the 512-cell grid."""
    out = {}
    for mode in ("cfl", "fixed"):
        for n in (128, 256, 512, 1024, 2048):
            col = paper_column(n, 100.0, dt=None if mode == "cfl" else dt_cfl(512, 100.0))
            sch = one_step(J, col, J.PRECK_SCHUR, max_restarts=20)
            non = one_step(J, col, J.PRECK_NONE, max_restarts=NONE_CAP, max_newton=1)
            out[(mode, n)] = (sch, non)
            print(f"{mode:5s} n {n:5d} dt {col.dt:.2e} | approx. Schur: status {sch['status']} Newton {sch['newton']} "
                  f"GMRES/Newton {sch['gmres'] / max(sch['newton'], 1):7.1f} | none: first Newton system "
                  f"{non['gmres']} GMRES", flush=True)
    for key, (sch, non) in out.items():
        assert sch["status"] == 0, key
    per = [out[("cfl", n)][0]["gmres"] / out[("cfl", n)][0]["newton"] for n in (128, 256, 512, 1024, 2048)]
    # at a constant CFL number the preconditioned count does not grow with the grid
    assert per[-1] <= per[0], per


TOLS = (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-8)


def test_multigrid_tolerance_study(J, orc):
    """fig:MG_tests: one block solved by V-cycles to gamma_MG, the other
    exactly; GMRES iterations and V-cycles of one step (512 cells, 100 V).
    S~ with the textbook linear interpolation; the electron block with the
    matrix-dependent one (one V-cycle is then an exact solve in 1D) and, to
    show why, with the linear one, whose V-cycles diverge there."""
    col = paper_column(512, 100.0)
    ref = orc.newton(orc.OracleColumn(col), reference=True)
    res = {}
    cases = ((2, 0, "S~, linear P"), (1, 1, "electron block, matrix-dependent P"),
             (1, 0, "electron block, linear P"))
    for blocks, transfer, name in cases:
        for tol in TOLS:
            kw = dict(max_restarts=20, max_newton=20, mg_tol=tol, mg_blocks=blocks, mg_transfer=transfer)
            if transfer == 0 and blocks == 1:
                kw.update(max_newton=1, max_restarts=0)     # reported only: the V-cycles diverge
            r = one_step(J, col, J.PRECK_SCHUR_MG, **kw)
            res[(blocks, transfer, tol)] = r
            err = max(rel(r["ne"], ref.ne), rel(r["phi"], ref.phi)) if r["status"] == 0 else float("nan")
            print(f"multigrid on {name:36s} gamma_MG {tol:.0e}: status {r['status']} Newton {r['newton']} "
                  f"GMRES {r['gmres']} V-cycles {r['mg']} rel L2 {err:.1e}", flush=True)
            if r["status"] == 0:
                assert err < 1e-9
    phi_blk = [res[(2, 0, t)] for t in TOLS]
    assert all(r["status"] == 0 for r in phi_blk)
    # S~: GMRES barely depends on gamma_MG; the V-cycles grow as it tightens
    assert max(r["gmres"] for r in phi_blk[1:]) <= 2 * min(r["gmres"] for r in phi_blk)
    assert phi_blk[-1]["mg"] > phi_blk[0]["mg"]
    # electron block, matrix-dependent P: one V-cycle per solve whatever gamma_MG
    e_md = [res[(1, 1, t)] for t in TOLS]
    assert all(r["status"] == 0 for r in e_md)
    assert len(set(r["gmres"] for r in e_md)) == 1
