"""Drive coefficient d(t) multiplying (f + f^) -- oracle side.

The paper drives the filter with a smooth-edged square envelope and its
stepwise generalisation (supplement S2.C, eq. "square_pulse"); the workloads
here use a lab-frame carrier cos(w_d t) with a cosine-ramped flat-top window,
and a two-level variant with per-level amplitude, phase and detuning (the
paper finds a two-step optimum, main text "Fidelity optimization").

The smoothed stepwise envelope of S2.C is the complex Omega(t) =
sum_{j=1}^{n} (h_{j+1} - h_j) f(t, j T / n, sigma) of logistic steps f, with the
drive off before the first and after the last step (h_1 = h_{n+1} = 0); on the
carrier it drives (f + f^) with d(t) = Re[Omega(t) e^{-i w_d t}].

Window conventions (ramp length t_r, duration T):
  r(x)   = 0 for x < 0,  1/2 (1 - cos(pi x / t_r)) for 0 <= x < t_r,  1 otherwise
  w(t)   = r(t) r(T - t)
  c(t)   = 0 for t <= T/2 - t_r/2, 1 for t >= T/2 + t_r/2,
           1/2 (1 - cos(pi (t - T/2 + t_r/2) / t_r)) in between
  w_1(t) = r(t) (1 - c(t)),   w_2(t) = r(T - t) c(t)
"""
import math

FLATTOP = 0
PIECEWISE6 = 1
STEPWISE = 2


def ramp(x: float, t_r: float) -> float:
    if x < 0.0:
        return 0.0
    if x >= t_r:
        return 1.0
    return 0.5 * (1.0 - math.cos(math.pi * x / t_r))


def crossfade(t: float, T: float, t_r: float) -> float:
    a = 0.5 * T - 0.5 * t_r
    if t <= a:
        return 0.0
    if t >= a + t_r:
        return 1.0
    return 0.5 * (1.0 - math.cos(math.pi * (t - a) / t_r))


def window(t: float, T: float, t_r: float) -> float:
    return ramp(t, t_r) * ramp(T - t, t_r)


def logistic(t: float, t0: float, sigma: float) -> float:
    """f(t, t0, sigma) = 1 / (1 + exp(-(t - t0) / sigma)) (supplement S2.C)."""
    return 1.0 / (1.0 + math.exp(-(t - t0) / sigma))


def stepwise_envelope(pulse, t: float) -> complex:
    """Omega(t) = sum_{j=1}^{n} (h_{j+1} - h_j) f(t, j T / n, sigma) with h_1 = h_{n+1} = 0
    (the drive is off at the start and the end) and h_2 .. h_n = pulse.h."""
    hs = [0j] + [complex(x) for x in pulse.h] + [0j]  # hs[k] = h_{k+1}
    n = len(hs) - 1
    om = 0j
    for j in range(1, n + 1):
        om += (hs[j] - hs[j - 1]) * logistic(t, j * pulse.T / n, pulse.sigma)
    return om


def drive(pulse, t: float) -> float:
    """d(t) for the pulse description (see paper_2508_18114_amd.inputs.PulseParams)."""
    if pulse.kind == FLATTOP:
        return pulse.amp * window(t, pulse.T, pulse.t_ramp) * math.cos(pulse.w_d * t)
    if pulse.kind == PIECEWISE6:
        A1, phi1, D1, A2, phi2, D2 = pulse.p
        c = crossfade(t, pulse.T, pulse.t_ramp)
        w1 = ramp(t, pulse.t_ramp) * (1.0 - c)
        w2 = ramp(pulse.T - t, pulse.t_ramp) * c
        return (A1 * w1 * math.cos((pulse.w_d + D1) * t + phi1)
                + A2 * w2 * math.cos((pulse.w_d + D2) * t + phi2))
    if pulse.kind == STEPWISE:
        # the complex envelope on the carrier: Re[Omega(t) e^{-i w_d t}]
        om = stepwise_envelope(pulse, t)
        return om.real * math.cos(pulse.w_d * t) + om.imag * math.sin(pulse.w_d * t)
    raise ValueError("unknown pulse kind")
