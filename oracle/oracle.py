"""ctypes wrapper of the CPU oracle (oracle/jfnk_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark.  The product library never imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

KL, KU = 2, 3
BAND_W = 2 * KL + KU + 1
CONVERGED, MAX_ITERS, NONFINITE, SINGULAR = 0, 1, 2, 3

_dp = C.POINTER(C.c_double)


class _Table(C.Structure):
    _fields_ = [("nc", C.c_int), ("nx", C.c_int), ("c_min", C.c_double), ("c_max", C.c_double),
                ("x_min", C.c_double), ("x_max", C.c_double), ("mu", _dp), ("diff", _dp)]


class _Column(C.Structure):
    _fields_ = [("n", C.c_int), ("length", C.c_double), ("dt", C.c_double),
                ("phi_left", C.c_double), ("phi_right", C.c_double),
                ("eps_over_e", C.c_double), ("bc_left", C.c_int), ("bc_right", C.c_int),
                ("ne_left", C.c_double), ("ne_right", C.c_double),
                ("mu", _dp), ("diff", _dp), ("src", _dp), ("kloss", _dp), ("q", _dp),
                ("uface", _dp), ("ne_old", _dp), ("phi_old", _dp), ("table", C.POINTER(_Table)),
                ("prog", _dp), ("gas_n", _dp)]


class _Opts(C.Structure):
    _fields_ = [("max_iters", C.c_int), ("tol", C.c_double), ("reference_mode", C.c_int),
                ("floor_tol", C.c_double), ("ls_theta", C.c_double),
                ("lambda_min", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("backtracks", C.c_int), ("status", C.c_int),
                ("res_scaled", C.c_double), ("scal", C.c_double * 4)]


def lib():
    global _LIB
    if _LIB is None:
        # JFNK_ORACLE_LIB: another build of the same source (the sanitizer run)
        path = os.environ.get("JFNK_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b  # noqa: F401  (package-relative when imported as oracle.oracle)
            _b.build()
        L = C.CDLL(path)
        L.orc_bernoulli.restype = C.c_double
        L.orc_bernoulli.argtypes = [C.c_double]
        L.orc_bernoulli_deriv.restype = C.c_double
        L.orc_bernoulli_deriv.argtypes = [C.c_double]
        for name in ("orc_source_term",):
            getattr(L, name).argtypes = [C.POINTER(_Column), _dp]
        L.orc_face_fluxes.argtypes = [C.POINTER(_Column), _dp, _dp, _dp]
        L.orc_residual.argtypes = [C.POINTER(_Column), _dp, _dp, _dp, _dp, _dp]
        L.orc_scalings.argtypes = [C.POINTER(_Column), _dp]
        L.orc_jacobian_dense.argtypes = [C.POINTER(_Column), _dp, _dp, _dp]
        L.orc_jacobian_band.argtypes = [C.POINTER(_Column), _dp, _dp, _dp]
        L.orc_band_solve.restype = C.c_int
        L.orc_band_solve.argtypes = [C.c_int, _dp, _dp]
        L.orc_dense_solve.restype = C.c_int
        L.orc_dense_solve.argtypes = [C.c_int, _dp, _dp]
        L.orc_table_lookup.argtypes = [C.POINTER(_Table), C.c_double, C.c_double, _dp, _dp]
        L.orc_table_lookup.restype = None
        L.orc_face_coeffs.argtypes = [C.POINTER(_Column), _dp, _dp, _dp]
        L.orc_face_coeffs.restype = None
        L.orc_newton.restype = C.c_int
        L.orc_newton.argtypes = [C.POINTER(_Column), C.POINTER(_Opts), _dp, _dp,
                                 C.POINTER(_Stats)]
        _LIB = L
    return _LIB


def _p(a: Optional[np.ndarray]):
    if a is None:
        return C.cast(None, _dp)
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


class OracleColumn:
    """Holds a column's arrays alive and the C struct that points at them."""

    def __init__(self, col, ne_old=None, phi_old=None):
        self.col = col
        self._keep = []

        def arr(x):
            if x is None:
                return None
            a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
            self._keep.append(a)
            return a

        self.mu = arr(col.mu)
        self.diff = arr(col.diff)
        self.src = arr(col.src)
        self.kloss = arr(col.kloss)
        self.q = arr(col.q)
        self.uface = arr(getattr(col, "uface", None))
        self.ne_old = arr(col.ne if ne_old is None else ne_old)
        self.phi_old = arr(col.phi if phi_old is None else phi_old)
        tab = getattr(col, "table", None)
        self.table = None if tab is None else table_struct(tab, self._keep)
        self.prog = arr(getattr(col, "prog", None))
        self.gas_n = arr(getattr(col, "gas_n", None))
        self.s = _Column(col.n, col.length, col.dt, col.phi_left, col.phi_right,
                         col.eps_over_e, col.bc_left, col.bc_right, col.ne_left,
                         col.ne_right, _p(self.mu), _p(self.diff), _p(self.src),
                         _p(self.kloss), _p(self.q), _p(self.uface), _p(self.ne_old),
                         _p(self.phi_old),
                         C.pointer(self.table) if self.table is not None else C.cast(None, C.POINTER(_Table)),
                         _p(self.prog), _p(self.gas_n))

    @property
    def n(self):
        return self.col.n


def table_struct(tab, keep) -> _Table:
    """The C struct of a transport table (arrays kept alive in keep)."""
    mu = np.ascontiguousarray(tab.mu, dtype=np.float64)
    d = np.ascontiguousarray(tab.diff, dtype=np.float64)
    keep += [mu, d]
    return _Table(mu.shape[0], mu.shape[1], tab.c_min, tab.c_max, tab.x_min, tab.x_max, _p(mu), _p(d))


def table_lookup(tab, c: float, en_td: float):
    """(mu, D) of the table at progress variable c and reduced field en_td (Td)."""
    keep = []
    t = table_struct(tab, keep)
    mu, d = C.c_double(), C.c_double()
    lib().orc_table_lookup(C.byref(t), float(c), float(en_td), C.byref(mu), C.byref(d))
    return mu.value, d.value


def face_coeffs(oc: OracleColumn, phi):
    """(mu_f, D_f) of every face (n + 1) in state phi."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    mu = np.empty(oc.n + 1)
    d = np.empty(oc.n + 1)
    lib().orc_face_coeffs(C.byref(oc.s), _p(phi), _p(mu), _p(d))
    return mu, d


def bernoulli(x: float) -> float:
    return lib().orc_bernoulli(float(x))


def bernoulli_deriv(x: float) -> float:
    return lib().orc_bernoulli_deriv(float(x))


def source_term(oc: OracleColumn) -> np.ndarray:
    f = np.empty(oc.n)
    lib().orc_source_term(C.byref(oc.s), _p(f))
    return f


def face_fluxes(oc: OracleColumn, ne, phi) -> np.ndarray:
    ne = np.ascontiguousarray(ne, dtype=np.float64)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    g = np.empty(oc.n + 1)
    lib().orc_face_fluxes(C.byref(oc.s), _p(ne), _p(phi), _p(g))
    return g


def residual(oc: OracleColumn, ne, phi, f=None):
    """(F_e, F_phi) at (ne, phi); f defaults to n^n + dt s."""
    if f is None:
        f = source_term(oc)
    ne = np.ascontiguousarray(ne, dtype=np.float64)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    fe = np.empty(oc.n)
    fp = np.empty(oc.n)
    lib().orc_residual(C.byref(oc.s), _p(f), _p(ne), _p(phi), _p(fe), _p(fp))
    return fe, fp


def scalings(oc: OracleColumn) -> np.ndarray:
    s = np.empty(4)
    lib().orc_scalings(C.byref(oc.s), _p(s))
    return s


def jacobian_dense(oc: OracleColumn, ne, phi) -> np.ndarray:
    ne = np.ascontiguousarray(ne, dtype=np.float64)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    a = np.empty((2 * oc.n, 2 * oc.n))
    lib().orc_jacobian_dense(C.byref(oc.s), _p(ne), _p(phi), _p(a))
    return a


def jacobian_band(oc: OracleColumn, ne, phi) -> np.ndarray:
    ne = np.ascontiguousarray(ne, dtype=np.float64)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    ab = np.empty((2 * oc.n, BAND_W))
    lib().orc_jacobian_band(C.byref(oc.s), _p(ne), _p(phi), _p(ab))
    return ab


def band_solve(ab: np.ndarray, b: np.ndarray) -> np.ndarray:
    ab = np.ascontiguousarray(ab, dtype=np.float64).copy()
    x = np.ascontiguousarray(b, dtype=np.float64).copy()
    info = lib().orc_band_solve(int(x.shape[0]), _p(ab), _p(x))
    if info:
        raise np.linalg.LinAlgError(f"zero pivot {info}")
    return x


def dense_solve(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64).copy()
    x = np.ascontiguousarray(b, dtype=np.float64).copy()
    info = lib().orc_dense_solve(int(x.shape[0]), _p(a), _p(x))
    if info:
        raise np.linalg.LinAlgError(f"zero pivot {info}")
    return x


def band_to_dense(ab: np.ndarray) -> np.ndarray:
    n = ab.shape[0]
    a = np.zeros((n, n))
    for i in range(n):
        for d in range(-KL, KL + KU + 1):
            j = i + d
            if 0 <= j < n:
                a[i, j] = ab[i, d + KL]
    return a


@dataclass
class NewtonResult:
    ne: np.ndarray
    phi: np.ndarray
    iters: int
    backtracks: int
    status: int
    res_scaled: float
    scal: np.ndarray


def newton(oc: OracleColumn, ne0=None, phi0=None, *, tol=1e-10, reference=False,
           max_iters=100, floor_tol=1e-15, ls_theta=0.25,
           lambda_min=2.0 ** -10) -> NewtonResult:
    """Root of the backward-Euler system from the guess (ne0, phi0) (default X^n)."""
    ne = np.array(oc.ne_old if ne0 is None else ne0, dtype=np.float64, copy=True)
    phi = np.array(oc.phi_old if phi0 is None else phi0, dtype=np.float64, copy=True)
    o = _Opts(max_iters, tol, 1 if reference else 0, floor_tol, ls_theta, lambda_min)
    st = _Stats()
    lib().orc_newton(C.byref(oc.s), C.byref(o), _p(ne), _p(phi), C.byref(st))
    return NewtonResult(ne, phi, st.iters, st.backtracks, st.status, st.res_scaled,
                        np.array(list(st.scal)))


def scaled_residual_inf(oc: OracleColumn, ne, phi) -> float:
    """||S_F^-1 F(X)||_inf with the scalings of the column's X^n."""
    fe, fp = residual(oc, ne, phi)
    s = scalings(oc)
    return float(max(np.max(np.abs(fe)) / s[0], np.max(np.abs(fp)) / s[1]))


def march(col, steps: int, *, reference=True, tol=1e-10, guess="prev", on_step=None):
    """Advance a column ``steps`` backward-Euler steps with the oracle.

    Returns the list of (ne, phi) after each step.  ``guess`` is "prev"
    (X^n) or "extrap" (the better of X^n and 2 X^n - X^{n-1} by scaled
    residual, ties to the extrapolation)."""
    ne, phi = col.ne.copy(), col.phi.copy()
    pne, pphi = None, None
    out = []
    for k in range(steps):
        oc = OracleColumn(col, ne, phi)
        g0, g1 = ne, phi
        if guess == "extrap" and pne is not None:
            # the extrapolation if its scaled residual is not larger than X^n's
            e0, e1 = 2 * ne - pne, 2 * phi - pphi
            if scaled_residual_inf(oc, e0, e1) <= scaled_residual_inf(oc, ne, phi):
                g0, g1 = e0, e1
        r = newton(oc, g0, g1, tol=tol, reference=reference)
        if on_step is not None:
            on_step(k, r)
        pne, pphi = ne, phi
        ne, phi = r.ne, r.phi
        out.append((ne.copy(), phi.copy()))
    return out
