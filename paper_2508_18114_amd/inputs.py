"""Seeded synthetic inputs for the low-rank readout integrator.

This module holds the parameter containers, the named workload presets and the
seeded draws (initial-state padding, pulse parameters, batch shapes, serving
arrivals).  It contains none of the integrator's arithmetic: the equation of
motion, the Gram solve, the Runge-Kutta scheme, the observables and the loss
live on their own in the HIP library and, independently, in the CPU oracle.
Both consume the arrays produced here as plain data.

Units: angular frequencies and rates in rad/ns, times in ns.  A frequency
quoted as X GHz enters as 2*pi*X rad/ns; the transmon decay rate gamma_1 is
already a rate (1/ns) and is used as is.

Model (transmon as a Duffing oscillator, bare resonator and filter modes,
lab-frame drive on the filter) -- the readout model of the paper's main text
(Hamiltonian eq. "hamiltonianpurcell", master equation eq. "hamiltonian"),
with the charge-basis transmon replaced by a Duffing oscillator and the
normal-mode basis by bare modes:

    H(t) = w_q n_q + alpha/2 n_q(n_q-1) + w_r n_r + w_f n_f
           + g (b+b^)(a+a^) + G (a+a^)(f+f^) + d(t) (f+f^)
    L_1 = sqrt(kappa_f) f,  L_2 = sqrt(gamma_1) b

Basis index (Kronecker order transmon x resonator x filter):
    n = (i_q * d_r + i_r) * d_f + i_f,  N = d_q * d_r * d_f.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

TWO_PI = 2.0 * math.pi

PULSE_FLATTOP = 0
PULSE_PIECEWISE6 = 1
PULSE_STEPWISE = 2   # smoothed stepwise complex envelope (supplement S2.C)
MODEL_DUFFING, MODEL_TRANSMON, MODEL_NORMAL = 0, 1, 2
MAX_DQ = 8
PULSE_MAX_HEIGHTS = 63
FRAME_LAB = 0        # B and <a>, <f> in the lab frame
FRAME_DRIVE = 1      # frame rotating at the drive carrier w_d (counter-rotating terms kept)

FP64 = 0
FP32 = 1
BF16X3 = 2


def ghz(x: float) -> float:
    """Angular frequency (rad/ns) of a frequency given in GHz."""
    return TWO_PI * x


@dataclasses.dataclass
class ModelParams:
    """kind MODEL_DUFFING: the benchmark's Duffing transmon and couplings
    g (b+b^)(a+a^), G (a+a^)(f+f^), drive d(t) (f+f^).
    kind MODEL_TRANSMON: the paper's Hamiltonian in the bare resonator/filter
    basis with the transmon in its eigenbasis: levels E_t (d_q values, rad/ns),
    charge operator n_t (d_q x d_q, row-major, real symmetric); couplings
    i g n_t (a^ - a) and -G (a^ - a)(f^ - f) (G plays J), drive d(t) i (f^ - f);
    w_q and alpha unused.  Jumps in both: sqrt(kappa_f) f, sqrt(gamma_1) b with
    b the ladder sum_q sqrt(q) |q-1><q|.
    kind MODEL_NORMAL: the paper's Hamiltonian in its normal-mode basis
    (supplement S2.D): transmon levels E_t and charge operator n_t as for
    MODEL_TRANSMON (d_q levels), the lower normal mode c_l in the resonator
    slot (d_r levels, frequency w_r = w_l) and the upper mode c_u in the filter
    slot (d_f levels, w_f = w_u); couplings i g n_t [mu_l (c_l^ - c_l) + mu_u
    (c_u^ - c_u)], drive d(t) i [nu_l (c_l^ - c_l) + nu_u (c_u^ - c_u)], jumps
    sqrt(kappa_f) f with f = s_21 c_u^ + s_22 c_l^ + s_23 c_l + s_24 c_u and
    sqrt(gamma_1) b; mu_u = s_14 - s_11, mu_l = s_13 - s_12, nu_u = s_24 - s_21,
    nu_l = s_23 - s_22 from the 8 entries of S; w_q, alpha and G unused."""
    d_q: int
    d_r: int
    d_f: int
    w_q: float
    alpha: float
    w_r: float
    w_f: float
    g: float
    G: float
    kappa_f: float
    gamma_1: float
    kind: int = 0
    E_t: tuple = ()
    n_t: tuple = ()
    S: tuple = ()      # kind MODEL_NORMAL: a and f through (c_u^, c_l^, c_l, c_u), s_11 .. s_14, s_21 .. s_24

    @property
    def N(self) -> int:
        return self.d_q * self.d_r * self.d_f

    def replace(self, **kw) -> "ModelParams":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class PulseParams:
    """Drive d(t) on (f + f^).

    kind PULSE_FLATTOP:     d(t) = amp * w(t) * cos(w_d t)
    kind PULSE_PIECEWISE6:  d(t) = sum_s A_s w_s(t) cos((w_d + Delta_s) t + phi_s)
                            p = (A_1, phi_1, Delta_1, A_2, phi_2, Delta_2)
    w(t) is a flat-top window on [0, T] with cosine ramps of length t_ramp;
    w_1, w_2 split it at T/2 with a cosine cross-fade of length t_ramp.
    kind PULSE_STEPWISE:    d(t) = Re[ Omega(t) e^{-i w_d t} ],
                            Omega(t) = sum_{j=1}^{n} (h_{j+1} - h_j) f(t, j T / n, sigma)
                            with f the logistic function, h_1 = h_{n+1} = 0 and the
                            n - 1 complex heights h_2 .. h_n given in `h`.
    frame FRAME_LAB or FRAME_DRIVE: the frame the state is integrated in.
    """
    kind: int
    w_d: float
    amp: float
    t_ramp: float
    T: float
    p: tuple = (0.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    frame: int = FRAME_LAB
    sigma: float = 0.5       # logistic steepness of PULSE_STEPWISE (ns)
    h: tuple = ()            # PULSE_STEPWISE heights h_2 .. h_n (complex, rad/ns)

    def replace(self, **kw) -> "PulseParams":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# Model presets
# --------------------------------------------------------------------------

def readout_model(d_q: int, d_r: int, d_f: int) -> ModelParams:
    """Transmon-resonator-filter readout model at the given truncations."""
    return ModelParams(
        d_q=d_q, d_r=d_r, d_f=d_f,
        w_q=ghz(5.0), alpha=ghz(-0.25), w_r=ghz(7.0), w_f=ghz(7.0),
        g=ghz(0.15), G=ghz(0.05),
        kappa_f=ghz(0.02), gamma_1=1e-5,
    )


T_RAMP = 2.5          # ns, the ramp time used for the paper's square pulse
W_DRIVE = ghz(7.0)    # drive carrier


def flattop_pulse(amp_ghz: float, T: float, t_ramp: float = T_RAMP,
                  w_d: float = W_DRIVE) -> PulseParams:
    return PulseParams(kind=PULSE_FLATTOP, w_d=w_d, amp=ghz(amp_ghz),
                       t_ramp=t_ramp, T=T)


# --------------------------------------------------------------------------
# Seeded draws
# --------------------------------------------------------------------------

def stepwise_pulse(heights, T: float, sigma: float = 0.5, w_d: float = W_DRIVE) -> PulseParams:
    """Smoothed stepwise pulse with complex heights h_2 .. h_n (rad/ns)."""
    return PulseParams(kind=PULSE_STEPWISE, w_d=w_d, amp=0.0, t_ramp=0.0, T=T, sigma=sigma,
                       h=tuple(complex(x) for x in heights))


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def basis_index(model: ModelParams, i_q: int, i_r: int, i_f: int) -> int:
    return (i_q * model.d_r + i_r) * model.d_f + i_f


def initial_state(model: ModelParams, M: int, which: str, seed: int,
                  scale: float = 1e-6) -> np.ndarray:
    """Rank-padded initial factor B0 (N x M complex128).

    Column 0 is the pure state |q, r=0, f=0> with q = 0 ('g') or 1 ('e')
    (initial states of supplement S2.A).  Columns 1..M-1 are seeded iid complex
    Gaussian vectors with the psi component removed, orthonormalised (numpy QR)
    and multiplied by `scale`, which makes B0^ B0 non-singular (the padding
    recipe of supplement S1.A; the padded weight is scale**2 per column).
    """
    N = model.N
    if not (1 <= M <= N):
        raise ValueError("need 1 <= M <= N")
    q = {"g": 0, "e": 1}[which]
    n0 = basis_index(model, q, 0, 0)
    B = np.zeros((N, M), dtype=np.complex128)
    B[n0, 0] = 1.0
    if M > 1:
        r = rng(seed)
        Z = r.standard_normal((N, M - 1)) + 1j * r.standard_normal((N, M - 1))
        Z[n0, :] = 0.0
        Q, _ = np.linalg.qr(Z)
        B[:, 1:] = scale * Q
    return B


def draw_amplitudes_ghz(seed: int, n: int, lo: float = 0.02, hi: float = 0.1) -> np.ndarray:
    return rng(seed).uniform(lo, hi, size=n)


def draw_piecewise6(r: np.random.Generator, T: float, t_ramp: float = T_RAMP,
                    w_d: float = W_DRIVE) -> PulseParams:
    """Two-level amplitude/phase/detuning pulse drawn from seeded uniform ranges:
    A_s/2pi in [0.02, 0.1] GHz, phi_s in [0, 2pi), Delta_s/2pi in [-0.02, 0.02] GHz."""
    A1, A2 = r.uniform(0.02, 0.1, size=2)
    p1, p2 = r.uniform(0.0, TWO_PI, size=2)
    D1, D2 = r.uniform(-0.02, 0.02, size=2)
    return PulseParams(kind=PULSE_PIECEWISE6, w_d=w_d, amp=0.0, t_ramp=t_ramp, T=T,
                       p=(ghz(A1), p1, ghz(D1), ghz(A2), p2, ghz(D2)))


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Trajectory:
    model: ModelParams
    M: int
    pulse: PulseParams
    which: str          # 'g' or 'e'
    seed: int           # padding seed
    dt: float
    nsteps: int
    precision: int = FP64
    pad_scale: float = 1e-6  # norm of each padding column of B0

    def B0(self, scale: float = None) -> np.ndarray:
        return initial_state(self.model, self.M, self.which, self.seed,
                             self.pad_scale if scale is None else scale)


def config_small() -> List[Trajectory]:
    """Plain FP64 single-trajectory case: dims (4, 10, 5), N = 200, M = 4,
    flat-top drive 0.05 GHz, RK4 dt = 1e-3 ns, T = 10 ns; g and e."""
    m = readout_model(4, 10, 5)
    p = flattop_pulse(0.05, 10.0)
    return [Trajectory(m, 4, p, w, seed=1, dt=1e-3, nsteps=10_000) for w in ("g", "e")]


def config_paper_size() -> List[Trajectory]:
    """Paper-size case: dims (8, 50, 5), N = 2000, M = 20, T = 40 ns,
    dt = 5e-4 ns (8e4 RK4 steps), seeded amplitude in [0.02, 0.1] GHz; g and e."""
    m = readout_model(8, 50, 5)
    amp = float(draw_amplitudes_ghz(2, 1)[0])
    p = flattop_pulse(amp, 40.0)
    return [Trajectory(m, 20, p, w, seed=2, dt=5e-4, nsteps=80_000) for w in ("g", "e")]


# the paper's padding weight p_j = 1e-5 (supplement S1.A, initial condition):
# padding columns of norm sqrt(1e-5)
PAPER_PAD_SCALE = 1e-5 ** 0.5


def config_paper_size_paper_padding() -> List[Trajectory]:
    """config_paper_size with the paper's padding weight p_j = 1e-5 instead of
    the 1e-6 column scale (the reduced-precision modes need padding above their
    rounding noise)."""
    return [dataclasses.replace(t, pad_scale=PAPER_PAD_SCALE) for t in config_paper_size()]


def config_small_paper_padding() -> List[Trajectory]:
    """config_small with the paper's padding weight p_j = 1e-5."""
    return [dataclasses.replace(t, pad_scale=PAPER_PAD_SCALE) for t in config_small()]


def config_batched(n_pulses: int = 256, seed: int = 4, dt: float = 5e-4) -> List[Trajectory]:
    """Batched case: n_pulses piecewise pulses x {g, e}.  d_r in {25, 38, 50, 75}
    (N in {1000, 1520, 2000, 3000} at d_q = 8, d_f = 5), M uniform in [8, 32],
    T uniform in [20, 60] ns, nsteps = round(T / dt)."""
    r = rng(seed)
    out = []
    for k in range(n_pulses):
        d_r = int(r.choice([25, 38, 50, 75]))
        M = int(r.integers(8, 33))
        T = float(r.uniform(20.0, 60.0))
        nsteps = int(round(T / dt))
        T = nsteps * dt
        p = draw_piecewise6(r, T)
        m = readout_model(8, d_r, 5)
        for w in ("g", "e"):
            out.append(Trajectory(m, M, p, w, seed=seed * 100003 + k, dt=dt, nsteps=nsteps))
    return out


def batch_uniform(n_pulses: int, d_r: int = 50, M: int = 20, T: float = 40.0,
                  dt: float = 5e-4, seed: int = 4) -> List[Trajectory]:
    """n_pulses piecewise pulses x {g, e} all at one shape (default N = 2000, M = 20)."""
    r = rng(seed)
    nsteps = int(round(T / dt))
    m = readout_model(8, d_r, 5)
    out = []
    for k in range(n_pulses):
        p = draw_piecewise6(r, nsteps * dt)
        for w in ("g", "e"):
            out.append(Trajectory(m, M, p, w, seed=seed * 100003 + k, dt=dt, nsteps=nsteps))
    return out


def serving_request_shapes(seed: int, n: int, dt: float = 5e-4) -> List[dict]:
    """Per-request shapes for the serving form: d_r uniform in [13, 75]
    (N = 40 d_r in [520, 3000]), M in [4, 32], T in [10, 60] ns, precision in
    {FP32, FP64}."""
    r = rng(seed)
    out = []
    for _ in range(n):
        d_r = int(r.integers(13, 76))
        M = int(r.integers(4, 33))
        T = float(r.uniform(10.0, 60.0))
        prec = int(r.choice([FP32, FP64]))
        out.append(dict(d_r=d_r, M=M, nsteps=int(round(T / dt)), precision=prec))
    return out


def poisson_arrivals(seed: int, n: int, rate_per_s: float) -> np.ndarray:
    """Open-loop Poisson arrival times (s) of n requests at the given rate."""
    return np.cumsum(rng(seed).exponential(1.0 / rate_per_s, size=n))
