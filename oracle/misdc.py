"""Oracle of the MISDC time step around the electron/potential solve.

TEST INFRASTRUCTURE ONLY: imported by the tests (never by the product
library).  Plain numpy plus the oracle's Newton root (oracle.newton), one
column at a time, written from the paper's Algorithm 1 (algo:misdc), the
update of the provisional charged species of Section 3.1 and the
electron/Poisson system eq:nls of Section 3.2, restricted to the charged
species:

  state         n_e, phi (implicit, JFNK in the product) and one positive
                ion species n_i (explicit advection in the drift velocity)
  operators     R(n_e, n_i)    chemistry: ionisation S - recombination
                               k_r n_e n_i, the same for both species
                A(n_i; v, F)   ion advection -div(n_i v): second-order
                               Godunov fluxes (MUSCL, monotonised-central
                               limiter, face values extrapolated to the half
                               step with the forcing F = R - n_i div v of the
                               upwind cell), v = u + mu_i E (ions drift down
                               the potential gradient), electrodes absorbing
  SDC iteration k = 0 .. k_max - 1 (predictor: X^(0) = X^n):
    I_R^(k)    = (R^n + R^(k)) / 2      integral of the chemistry over the
                                        step, per unit time, from the last
                                        evaluation (trapezoidal)
    v^(k)      = (v(phi^n, t^n) + v(phi^(k), t^n+1)) / 2
    n_i~       = n_i^n + dt [A(n_i^n; v^(k), R^n) + I_R^(k)]
    X^(k+1)    = root of eq:nls, the backward-Euler electron/Poisson system,
                 with f_e = n_e^n + dt I_R^(k), no implicit loss, ion charge
                 n_i~ and the electrode potentials at t^n+1
    n_i^(k+1)  = n_i~
  At the fixed point the ions follow the time-centred Godunov update with
  trapezoidal chemistry and the electrons backward Euler in their transport
  (L-stable: the electrons relax on time scales far below dt, Section 4.1)
  with trapezoidal chemistry; the potential is then first order in time.
  electron_sdc: the electrons' transport gets the SDC correction the other
  species' diffusion gets in Section 3.1, f_e = n_e^n + dt [(T_e^n -
  T_e^(k)) / 2 + I_R^(k)] with T_e = -div Gamma: the fixed point is then the
  trapezoidal rule for the electrons (second order, A- but not L-stable:
  modes with dt |lambda| >> 1 contract by 1/2 per iteration and flip sign
  from step to step instead of decaying).

Time step: the column's dt, or a constant ion-drift CFL number (cfl_dt).
Electrode potentials: phi_left = 0 and phi_right(t) = V + A sin(2 pi f t)
(DC when A = 0; AC forcing of Section 4.5, Table 4).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import oracle as O


@dataclass
class Ions:
    """Ion and chemistry data of a column (per cell)."""
    mu_i: np.ndarray            # ion mobility, m^2/(V s)
    k_rec: np.ndarray           # recombination coefficient, m^3/s
    ac_amp: float = 0.0         # right-electrode AC amplitude, V
    ac_freq: float = 0.0        # Hz


def phi_right_at(col, ions: Ions, t: float) -> float:
    return col.phi_right + ions.ac_amp * math.sin(2.0 * math.pi * ions.ac_freq * t)


def _at_time(col, ions, t):
    c = col.copy()
    c.phi_right = phi_right_at(col, ions, t)
    c.kloss = np.zeros(col.n)
    return c


def electron_transport(col, ions, t, ne, phi) -> np.ndarray:
    """T_e = -(Gamma_{i+1/2} - Gamma_{i-1/2}) / h with the potentials at t
    (the electron transport of eq:nls; used to state the fixed point)."""
    c = _at_time(col, ions, t)
    gam = O.face_fluxes(O.OracleColumn(c), ne, phi)
    return -(gam[1:] - gam[:-1]) / (col.length / col.n)


def reaction(col, ions: Ions, ne, ni) -> np.ndarray:
    """R = ionisation - recombination (per species)."""
    return col.src - ions.k_rec * ne * ni


def ion_face_velocity(col, ions, t, phi) -> np.ndarray:
    """Ion drift velocity at the n + 1 faces: v = u + mu_i,f (phi_a - phi_b) / h_f
    (h/2 and the electrode potential at the walls; u: the column's face
    velocities, when it has them)."""
    n, h = col.n, col.length / col.n
    pr = phi_right_at(col, ions, t)
    v = np.empty(n + 1)
    muf = 0.5 * (ions.mu_i[:-1] + ions.mu_i[1:])
    v[1:-1] = muf * (phi[:-1] - phi[1:]) / h
    v[0] = ions.mu_i[0] * (col.phi_left - phi[0]) / (0.5 * h)
    v[-1] = ions.mu_i[-1] * (phi[-1] - pr) / (0.5 * h)
    u = getattr(col, "uface", None)
    return v if u is None else u + v


def cfl_dt(col, ions, t, phi, cfl: float) -> float:
    """Time step at a constant ion-drift CFL number (Section 4.1: the
    explicit advection of the charged species limits the step):
    min(col.dt, cfl h / max_f |v_f|) with the face velocities of the state
    (phi at t); col.dt when no face moves."""
    vmax = float(np.max(np.abs(ion_face_velocity(col, ions, t, phi))))
    h = col.length / col.n
    return col.dt if vmax == 0.0 else min(col.dt, cfl * h / vmax)


def mc_slopes(ni) -> np.ndarray:
    """Monotonised-central limited slopes; zero in the first and last cells."""
    s = np.zeros_like(ni)
    a = 2.0 * (ni[1:-1] - ni[:-2])
    b = 0.5 * (ni[2:] - ni[:-2])
    c = 2.0 * (ni[2:] - ni[1:-1])
    same = (np.sign(a) == np.sign(b)) & (np.sign(b) == np.sign(c)) & (a != 0.0)
    s[1:-1] = np.where(same, np.sign(b) * np.minimum(np.minimum(np.abs(a), np.abs(b)), np.abs(c)), 0.0)
    return s


def ion_advection(col, ni, v, dt, rate) -> np.ndarray:
    """A = -(Phi_{i+1/2} - Phi_{i-1/2}) / h, Phi = v n_face with the upwind
    cell's value extrapolated in space to the face and in time to the half
    step (second-order Godunov with forcing): from cell a (v >= 0)
    n_a + (1 - v dt/h) sigma_a / 2 + (dt/2) (rate_a - n_a div_a v), from cell
    b (v < 0) n_b - (1 + v dt/h) sigma_b / 2 + (dt/2) (rate_b - n_b div_b v),
    div_i v = (v_{i+1/2} - v_{i-1/2}) / h; electrodes absorb: a wall face
    carries ions out of the column only (first-order value there)."""
    n, h = col.n, col.length / col.n
    sg = mc_slopes(ni)
    src = 0.5 * dt * (rate - ni * (v[1:] - v[:-1]) / h)
    flux = np.zeros(n + 1)
    for f in range(n + 1):
        vf = v[f]
        if f == 0:
            flux[f] = vf * ni[0] if vf < 0.0 else 0.0
        elif f == n:
            flux[f] = vf * ni[n - 1] if vf > 0.0 else 0.0
        elif vf >= 0.0:
            flux[f] = vf * (ni[f - 1] + 0.5 * (1.0 - vf * dt / h) * sg[f - 1] + src[f - 1])
        else:
            flux[f] = vf * (ni[f] - 0.5 * (1.0 + vf * dt / h) * sg[f] + src[f])
    return -(flux[1:] - flux[:-1]) / h


@dataclass
class StepResult:
    ne: np.ndarray
    phi: np.ndarray
    ni: np.ndarray
    newton: int
    iterates: list


def misdc_step(col, ions: Ions, t: float, ne, phi, ni, k_max: int = 4, keep_iterates: bool = False,
               tol_floor: float = 1e-15, dt: Optional[float] = None, electron_sdc: bool = False) -> StepResult:
    """One MISDC step t -> t + dt of one column (dt: col.dt unless given)."""
    if dt is not None:
        col = col.copy()
        col.dt = dt
    dt = col.dt
    Rn = reaction(col, ions, ne, ni)
    Tn = electron_transport(col, ions, t, ne, phi) if electron_sdc else None
    vn = ion_face_velocity(col, ions, t, phi)
    k_ne, k_phi, k_ni = ne.copy(), phi.copy(), ni.copy()
    newton = 0
    its = []
    for k in range(k_max):
        Rk = reaction(col, ions, k_ne, k_ni)
        i_r = 0.5 * (Rn + Rk)
        vk = ion_face_velocity(col, ions, t + dt, k_phi)
        v = 0.5 * (vn + vk)
        ni_t = ni + dt * (ion_advection(col, ni, v, dt, Rn) + i_r)
        c = _at_time(col, ions, t + dt)
        c.src = i_r
        if electron_sdc:
            c.src = 0.5 * (Tn - electron_transport(col, ions, t + dt, k_ne, k_phi)) + i_r
        c.q = ni_t
        oc = O.OracleColumn(c, ne, phi)           # f_e = n_e^n + dt src
        r = O.newton(oc, k_ne.copy(), k_phi.copy(), reference=True, floor_tol=tol_floor)
        if r.status != O.CONVERGED:
            raise RuntimeError(f"oracle Newton did not converge in SDC iteration {k}")
        newton += r.iters
        k_ne, k_phi, k_ni = r.ne, r.phi, ni_t
        if keep_iterates:
            its.append((k_ne.copy(), k_phi.copy(), k_ni.copy()))
    return StepResult(k_ne, k_phi, k_ni, newton, its)


def march(col, ions: Ions, steps: int, t0: float = 0.0, k_max: int = 4, ne=None, phi=None, ni=None,
          cfl: Optional[float] = None, electron_sdc: bool = False):
    """steps MISDC steps from (ne, phi, ni) (default: the column's start
    state with n_i = its ion charge), each of col.dt or, with cfl, of
    cfl_dt at the step's start; returns the final state and time."""
    ne = col.ne.copy() if ne is None else ne.copy()
    phi = col.phi.copy() if phi is None else phi.copy()
    ni = col.q.copy() if ni is None else ni.copy()
    t = t0
    for _ in range(steps):
        dt = col.dt if cfl is None else cfl_dt(col, ions, t, phi, cfl)
        r = misdc_step(col, ions, t, ne, phi, ni, k_max=k_max, dt=dt, electron_sdc=electron_sdc)
        ne, phi, ni = r.ne, r.phi, r.ni
        t += dt
    return ne, phi, ni, t
