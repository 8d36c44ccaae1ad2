"""Seeded synthetic inputs for the implicit electron / electric-potential step.

This module holds no solver arithmetic (no residual, Jacobian, Newton or
Krylov step).  It only builds the coefficient profiles and the start state of
the test columns, so that the CPU oracle and the GPU library are fed the same
arrays.  The profiles stand in for the paper's 1D burner-stabilised methane/air
flame (Section 4.1, Table 2), whose chemistry, transport data and initial
solution are not available:

  gas temperature   T(x) = 300 + 1700 (1 + tanh((x - x_f)/5e-4)) / 2      [K]
  net ion density   q(x) = A_ion exp(-(x - x_f)^2 / (2 sigma^2))          [m^-3]
  ionisation        s(x) = 1e21 exp(-(x - x_f)^2 / (2 sigma^2))           [m^-3 s^-1]
  recombination     k(x) = 1e-13 q(x)                                      [s^-1]
  electron mobility mu(x) = 0.4 T / 300                                    [m^2 V^-1 s^-1]
  diffusivity       D = mu k_B T / e   (Einstein relation, Section 2.1)    [m^2 s^-1]

with sigma = 1 mm on a 2 cm column.  The constant mobility 0.4 m^2/(V s) is
the value the paper quotes for thermal electrons (Section 2.2); the linear
temperature factor is a choice of these workloads.  The start state is
n_e = q with a linear potential between the electrodes.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# SI 2019 exact values and CODATA 2018 vacuum permittivity.
E_CHARGE = 1.602176634e-19      # C
K_BOLTZMANN = 1.380649e-23      # J/K
EPS0 = 8.8541878128e-12         # F/m
EPS_OVER_E = EPS0 / E_CHARGE    # (V m)^-1, relative permittivity 1

BC_DIRICHLET = 0
BC_ZERO_FLUX = 1


@dataclass
class Column:
    """One 1D column: per-cell coefficient arrays plus per-column scalars.

    Cell i has centre (i + 1/2) * length / n.  ``ne``/``phi`` hold the state
    X^n at the start of the step; ``ne_prev``/``phi_prev`` optionally X^{n-1}.
    """
    n: int
    length: float
    dt: float
    phi_left: float
    phi_right: float
    mu: np.ndarray
    diff: np.ndarray
    src: np.ndarray
    kloss: np.ndarray
    q: np.ndarray
    temp: np.ndarray
    ne: np.ndarray
    phi: np.ndarray
    eps_over_e: float = EPS_OVER_E
    bc_left: int = BC_DIRICHLET
    bc_right: int = BC_DIRICHLET
    ne_left: float = 0.0
    ne_right: float = 0.0
    ne_prev: Optional[np.ndarray] = None
    phi_prev: Optional[np.ndarray] = None
    # field-dependent electron transport (see TransportTable): with a table,
    # mu and D of every face come from it and mu, diff above are not used
    table: Optional["TransportTable"] = None
    prog: Optional[np.ndarray] = None      # progress variable per cell
    gas_n: Optional[np.ndarray] = None     # background gas number density, m^-3
    uface: Optional[np.ndarray] = None     # flow velocity at the n + 1 faces, m/s (None: 0)
    meta: dict = field(default_factory=dict)

    def copy(self) -> "Column":
        c = Column(**{k: (v.copy() if isinstance(v, np.ndarray) else v)
                      for k, v in self.__dict__.items() if k != "meta"})
        c.meta = dict(self.meta)
        return c


@dataclass
class TransportTable:
    """Electron mobility and diffusivity tabulated against the progress
    variable c (nc points on [c_min, c_max]) and x = log10(|E|/N / 1 Td)
    (nx points on [x_min, x_max]); arrays [nc, nx] (the shape of the paper's
    BOLSIG+ tables, Section 2.2, whose data are not available here)."""
    c_min: float
    c_max: float
    x_min: float
    x_max: float
    mu: np.ndarray
    diff: np.ndarray

    @property
    def nc(self) -> int:
        return int(self.mu.shape[0])

    @property
    def nx(self) -> int:
        return int(self.mu.shape[1])


T_IN, T_MAX, PRESSURE = 300.0, 2000.0, 101325.0


def synthetic_transport_table(nc: int = 17, nx: int = 41) -> TransportTable:
    """A smooth stand-in for the paper's non-thermal electron transport
    tables: at low reduced field the thermal values of the workloads
    (mu = 0.4 T/300, D = mu k_B T/e at T = T_in + c (T_max - T_in)); above
    ~3 Td the electrons heat up: mobility falls by up to 60 % and the
    electron temperature in D = mu k_B T_e / e rises by up to 2e4 K, with a
    logistic switch in log10(|E|/N) centred at 0.5."""
    c = np.linspace(0.0, 1.0, nc)
    x = np.linspace(-2.0, 3.0, nx)
    temp = T_IN + c[:, None] * (T_MAX - T_IN)
    w = 1.0 / (1.0 + np.exp(-3.0 * (x[None, :] - 0.5)))
    mu = 0.4 * temp / 300.0 * (1.0 - 0.6 * w)
    te = temp + 2e4 * w
    diff = mu * K_BOLTZMANN * te / E_CHARGE
    return TransportTable(0.0, 1.0, -2.0, 3.0, np.ascontiguousarray(mu), np.ascontiguousarray(diff))


def with_transport_table(col: "Column", table: TransportTable) -> "Column":
    """The column with table transport: progress variable from its gas
    temperature, c = (T - T_in)/(T_max - T_in) (Section 2.2), and the ideal-gas
    number density N = p / (k_B T) at atmospheric pressure."""
    c = col.copy()
    c.table = table
    c.prog = np.clip((col.temp - T_IN) / (T_MAX - T_IN), 0.0, 1.0)
    c.gas_n = PRESSURE / (K_BOLTZMANN * col.temp)
    return c


def cell_centres(n: int, length: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) * (length / n)


def flame_column(n: int, volts: float, *, a_ion: float = 1e16, x_f: float = 0.01,
                 length: float = 0.02, sigma: float = 1e-3, dt: float = 1e-5,
                 src_peak: float = 1e21, krec: float = 1e-13) -> Column:
    """Synthetic flame column of ``n`` cells with ``volts`` across it."""
    x = cell_centres(n, length)
    g = np.exp(-((x - x_f) ** 2) / (2.0 * sigma * sigma))
    temp = 300.0 + 1700.0 * 0.5 * (1.0 + np.tanh((x - x_f) / 5e-4))
    mu = 0.4 * temp / 300.0
    diff = mu * K_BOLTZMANN * temp / E_CHARGE
    q = a_ion * g
    src = src_peak * g
    kloss = krec * q
    ne = q.copy()
    phi = 0.0 + (volts - 0.0) * x / length
    return Column(n=n, length=length, dt=dt, phi_left=0.0, phi_right=float(volts),
                  mu=mu, diff=diff, src=src, kloss=kloss, q=q, temp=temp,
                  ne=ne, phi=phi,
                  meta=dict(volts=float(volts), a_ion=float(a_ion), x_f=float(x_f)))


# ---------------------------------------------------------------------------
# The five workloads, index 0..4: a single column, a single-column march, the
# 1024-column batch, the learned guess's training batches and the stiff batch.
# ---------------------------------------------------------------------------

def config0() -> List[Column]:
    """1 column x 256 cells, 100 V, one step of dt = 1e-5 s."""
    return [flame_column(256, 100.0, dt=1e-5)]


def config1(n: int = 4096) -> List[Column]:
    """1 column x 4096 cells, 1000 V, dt = 1e-5 s (50 steps in the workload)."""
    return [flame_column(n, 1000.0, dt=1e-5)]


def config2(seed: int = 2026, ncols: int = 1024, nmin: int = 512, nmax: int = 8192,
            dt: float = 1e-5) -> List[Column]:
    """Batch of uneven columns: cells U{nmin..nmax}, V ~ U[-1000, 1000],
    ion peak log-uniform in [1e15, 1e17] m^-3, flame position U[0.5, 1.5] cm."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(nmin, nmax + 1, size=ncols)
    vs = rng.uniform(-1000.0, 1000.0, size=ncols)
    amps = 10.0 ** rng.uniform(15.0, 17.0, size=ncols)
    xfs = rng.uniform(0.005, 0.015, size=ncols)
    return [flame_column(int(n), float(v), a_ion=float(a), x_f=float(xf), dt=dt)
            for n, v, a, xf in zip(ns, vs, amps, xfs)]


def config4(seed: int = 4321, ncols: int = 256, n: int = 65536,
            dt: float = 1e-4) -> List[Column]:
    """Stiff batch: 65536-cell columns, V ~ U[5, 10] kV, ion peak 1e17 m^-3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    vs = rng.uniform(5000.0, 10000.0, size=ncols)
    xfs = rng.uniform(0.005, 0.015, size=ncols)
    return [flame_column(n, float(v), a_ion=1e17, x_f=float(xf), dt=dt)
            for v, xf in zip(vs, xfs)]


# ---------------------------------------------------------------------------
# Time steps of the charged species (MISDC): one positive ion species
# drifting in the field (mobility of H3O+, Table 3) and the ionisation /
# recombination chemistry of the flame columns, electrodes at phi = 0 and
# phi_right(t) = V + A sin(2 pi f t).
# ---------------------------------------------------------------------------
ION_MOBILITY = 4e-3        # m^2/(V s), H3O+ (Table 3)


@dataclass
class IonData:
    mu_i: np.ndarray           # per cell, m^2/(V s)
    k_rec: np.ndarray          # per cell, m^3/s
    ac_amp: float = 0.0        # V
    ac_freq: float = 0.0       # Hz


def misdc_column(n: int, volts: float, *, ac_amp: float = 0.0, ac_freq: float = 0.0, cfl: float = 0.5,
                 length: float = 0.02, x_f: float = 0.01, a_ion: float = 1e16, krec: float = 1e-13):
    """A flame column for the MISDC step and its ion data.  n_i starts as
    the column's ion charge q and n_e = n_i with a linear potential (no space
    charge); dt is cfl times the ion drift CFL limit at the largest
    electrode voltage |V| + |A| (uniform field estimate)."""
    col = flame_column(n, volts, a_ion=a_ion, x_f=x_f, length=length, krec=krec)
    h = length / n
    vmax = ION_MOBILITY * (abs(volts) + abs(ac_amp)) / length
    col.dt = cfl * h / max(vmax, 1e-30)
    col.kloss = np.zeros(n)
    ions = IonData(np.full(n, ION_MOBILITY), np.full(n, krec), ac_amp, ac_freq)
    return col, ions


AC_FREQS = (1e3, 2.5e3, 5e3, 1e4, 2.5e4, 5e4, 1e5)     # Hz, the forcing frequencies of Table 4


def config_ac(seed: int = 77, ncols: int = 1024, n: int = 1024, amp: float = 1000.0, cfl: float = 0.5):
    """AC-forced batch for the MISDC step (Section 4.5): right electrode
    A sin(2 pi f t) with A = 1000 V and f cycling through Table 4's seven
    frequencies, each column at its own phase (start time uniform over its
    period), ion peak log-uniform in [1e15, 1e17] m^-3, flame position
    U[0.8, 1.2] cm, one dt for every column (cfl times the ion drift limit
    at 1000 V).  Returns (columns, ion data, start times)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    peaks = 10.0 ** rng.uniform(15.0, 17.0, size=ncols)
    xfs = rng.uniform(0.008, 0.012, size=ncols)
    phase = rng.uniform(0.0, 1.0, size=ncols)
    cols, ions, t0 = [], [], np.empty(ncols)
    for i in range(ncols):
        f = AC_FREQS[i % len(AC_FREQS)]
        c, ion = misdc_column(n, 0.0, ac_amp=amp, ac_freq=f, cfl=cfl, a_ion=float(peaks[i]), x_f=float(xfs[i]))
        cols.append(c)
        ions.append(ion)
        t0[i] = phase[i] / f
    return cols, ions, t0


def training_seeds() -> range:
    """Seeds of the learned-guess training batches (disjoint from 2026)."""
    return range(1000, 1100)


# ---------------------------------------------------------------------------
# Packing: columns back to back in one flat array per field.
# ---------------------------------------------------------------------------

@dataclass
class Packed:
    ncols: int
    col_offset: np.ndarray      # int64 [ncols + 1]
    length: np.ndarray          # float64 [ncols]
    dt: np.ndarray
    phi_left: np.ndarray
    phi_right: np.ndarray
    eps_over_e: np.ndarray
    ne_left: np.ndarray
    ne_right: np.ndarray
    bc_left: np.ndarray         # int32 [ncols]
    bc_right: np.ndarray
    mu: np.ndarray              # float64 [total]
    diff: np.ndarray
    src: np.ndarray
    kloss: np.ndarray
    q: np.ndarray
    temp: np.ndarray
    ne: np.ndarray
    phi: np.ndarray
    ne_prev: Optional[np.ndarray]
    phi_prev: Optional[np.ndarray]
    table: Optional[TransportTable] = None
    prog: Optional[np.ndarray] = None
    gas_n: Optional[np.ndarray] = None
    uface: Optional[np.ndarray] = None          # [total + ncols]: column c's faces from col_offset[c] + c

    @property
    def total(self) -> int:
        return int(self.col_offset[-1])


def pack(cols: List[Column]) -> Packed:
    ns = np.array([c.n for c in cols], dtype=np.int64)
    off = np.zeros(len(cols) + 1, dtype=np.int64)
    off[1:] = np.cumsum(ns)

    def cat(name):
        return np.ascontiguousarray(np.concatenate([getattr(c, name) for c in cols]))

    def per(name, dtype=np.float64):
        return np.array([getattr(c, name) for c in cols], dtype=dtype)

    has_prev = all(c.ne_prev is not None for c in cols)
    tabs = {id(c.table) for c in cols}
    if len(tabs) != 1:
        raise ValueError("the columns of a batch share one transport table (or none)")
    table = cols[0].table
    nu = sum(c.uface is not None for c in cols)
    if nu not in (0, len(cols)):
        raise ValueError("face velocities for every column of a batch or for none")
    return Packed(
        ncols=len(cols), col_offset=off,
        length=per("length"), dt=per("dt"), phi_left=per("phi_left"),
        phi_right=per("phi_right"), eps_over_e=per("eps_over_e"),
        ne_left=per("ne_left"), ne_right=per("ne_right"),
        bc_left=per("bc_left", np.int32), bc_right=per("bc_right", np.int32),
        mu=cat("mu"), diff=cat("diff"), src=cat("src"), kloss=cat("kloss"),
        q=cat("q"), temp=cat("temp"), ne=cat("ne"), phi=cat("phi"),
        ne_prev=cat("ne_prev") if has_prev else None,
        phi_prev=cat("phi_prev") if has_prev else None,
        table=table,
        prog=cat("prog") if table is not None else None,
        gas_n=cat("gas_n") if table is not None else None,
        uface=cat("uface") if nu else None,
    )


def unpack_field(p: Packed, arr: np.ndarray) -> List[np.ndarray]:
    return [arr[p.col_offset[i]:p.col_offset[i + 1]] for i in range(p.ncols)]
