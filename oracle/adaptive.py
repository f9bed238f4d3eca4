"""Adaptive-step integration of the low-rank equation of motion -- oracle.

Test infrastructure only (see the package header).  Plain FP64 numpy.

The paper integrates eq. "nosse" with an adaptive-timestep ODE solver (main
text, "Computational performance") without naming it.  Reading used here:
the explicit Runge-Kutta pair of Dormand and Prince of orders 5 and 4
(J. R. Dormand, P. J. Prince, J. Comput. Appl. Math. 6 (1980) 19), advancing
with the fifth-order solution, with

  error     e = dt sum_j (b_j - bhat_j) k_j   (difference of the two solutions)
  norm      err = sqrt( mean_i |e_i|^2 / sc_i^2 ),
            sc_i = atol + rtol max(|y_i|, |ynew_i|)   over the N M complex entries
  accept    err <= 1
  control   dt <- dt min(5, max(0.2, 0.9 err^(-1/5)))   (no growth after a rejection)
  outputs   the step is shortened to land on each requested output time,
            the proposal for the next step is kept

and the last stage evaluated at the new solution reused as the first stage
of the next step (first same as last).
"""
from __future__ import annotations

import numpy as np

from . import lowrank

# Butcher tableau of the Dormand-Prince 5(4) pair
C = np.array([0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0])
A = [
    [],
    [1.0 / 5.0],
    [3.0 / 40.0, 9.0 / 40.0],
    [44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0],
    [19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0],
    [9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0],
    [35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0],
]
B5 = np.array([35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0, 0.0])
B4 = np.array([5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0, -92097.0 / 339200.0, 187.0 / 2100.0,
               1.0 / 40.0])

FAC, FAC_MIN, FAC_MAX = 0.9, 0.2, 5.0


class StepUnderflow(ArithmeticError):
    """The step size fell below the resolution of the time axis."""


def dp_step(fun, t, dt, y, k1):
    """One Dormand-Prince step from (t, y) with k1 = f(t, y): returns
    (ynew, error vector, k7 = f(t + dt, ynew))."""
    k = [k1]
    for s in range(1, 7):
        ys = y + dt * sum(A[s][j] * k[j] for j in range(s) if A[s][j] != 0.0)
        k.append(fun(t + C[s] * dt, ys))
    ynew = y + dt * sum(B5[j] * k[j] for j in range(6) if B5[j] != 0.0)
    err = dt * sum((B5[j] - B4[j]) * k[j] for j in range(7))
    return ynew, err, k[6]


def error_norm(e, y, ynew, rtol, atol):
    sc = atol + rtol * np.maximum(np.abs(y), np.abs(ynew))
    return float(np.sqrt(np.mean((np.abs(e) / sc) ** 2)))


def integrate_ode(fun, t0, y0, t_out, dt0, rtol, atol, max_steps=10 ** 6):
    """Adaptive integration of y' = fun(t, y) through the increasing output
    times t_out (all > t0).  Returns (list of y at t_out, accepted, rejected)."""
    t = float(t0)
    y = np.array(y0, dtype=np.complex128, copy=True)
    k1 = fun(t, y)
    dt = float(dt0)
    out, acc, rej = [], 0, 0
    for t_end in t_out:
        while t < t_end:
            if acc + rej >= max_steps:
                raise StepUnderflow("step budget exhausted")
            h = min(dt, t_end - t)
            last = h >= t_end - t
            if h <= 1e-14 * max(1.0, abs(t)):
                raise StepUnderflow(f"step {h} at t = {t}")
            ynew, e, k7 = dp_step(fun, t, h, y, k1)
            err = error_norm(e, y, ynew, rtol, atol)
            if err <= 1.0:
                t = t_end if last else t + h
                y, k1 = ynew, k7
                acc += 1
                fac = FAC_MAX if err == 0.0 else min(FAC_MAX, max(FAC_MIN, FAC * err ** -0.2))
                if not (last and h < dt):  # a step shortened to an output time keeps the proposal
                    dt = h * fac
            else:
                rej += 1
                dt = h * min(1.0, max(FAC_MIN, FAC * err ** -0.2)) if np.isfinite(err) else h * FAC_MIN
        out.append(y.copy())
    return out, acc, rej


def integrate(model, pulse, t0, grid, nsteps, B0, rtol, atol, obs_stride=0, dt0=None):
    """Adaptive integration of the low-rank equation of motion from B(t0) = B0
    over the duration nsteps * grid, with observables recorded at t0 and every
    obs_stride * grid (as the fixed-step integrator records every obs_stride
    steps of dt = grid).  Returns (B at the end, obs, accepted, rejected)."""
    fun = lambda t, X: lowrank.rhs(model, pulse, t, X)  # noqa: E731
    stride = obs_stride if obs_stride > 0 else nsteps
    n_out = nsteps // stride
    t_out = [t0 + (k + 1) * stride * grid for k in range(n_out)]
    if nsteps % stride:
        t_out.append(t0 + nsteps * grid)
    ys, acc, rej = integrate_ode(fun, t0, B0, t_out, grid if dt0 is None else dt0, rtol, atol)
    rec = []
    if obs_stride > 0:
        rec.append(lowrank.observables(model, np.asarray(B0), pulse=pulse, t=t0))
        rec += [lowrank.observables(model, y, pulse=pulse, t=tk) for y, tk in zip(ys[:n_out], t_out)]
    obs = np.array(rec) if rec else np.zeros((0, 6 + model.d_q))
    return ys[-1], obs, acc, rej
