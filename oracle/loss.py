"""Readout figures of merit -- oracle.

Test infrastructure only (see the package header).  Supplement S3.A-B:

  SNR(tau)      = sqrt( 2 eta kappa int_0^tau |beta_e(t) - beta_g(t)|^2 dt )   eq. "SNR"
  eps_sep(tau)  = 1/2 erfc( SNR / 2 )                                        eq. "separation_error"
  eps_decay     = tau gamma / 2,   eps_a = eps_sep + eps_decay                eq. "assignment_error"
  T(tau)        = 1/tau sum_{j=g,e} sum_{k>=2} int_0^tau P_k^(j)(t) dt         eq. "transmon_ionization"
  Lambda(tau)   = log10( eps_a + T )                                         eq. "loss_function"

beta = tr(rho f) (filter field), kappa = kappa_f, eta = 0.6; transmon levels
are 0-based, so the ionisation sum runs over k = 2 .. d_q-1.  Integrals use
the composite trapezoid rule on the observation grid.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special

ETA = 0.6
COL_RE_F, COL_IM_F = 2, 3
COL_PQ = 6


def trapezoid(y, h):
    y = np.asarray(y, dtype=np.float64)
    if y.shape[0] < 2:
        return 0.0
    return h * (0.5 * y[0] + np.sum(y[1:-1], axis=0) + 0.5 * y[-1])


def readout_loss(obs_g, obs_e, h, kappa_f, gamma_1, eta=ETA):
    """Figures of merit from two observation series sampled every h ns."""
    beta_g = obs_g[:, COL_RE_F] + 1j * obs_g[:, COL_IM_F]
    beta_e = obs_e[:, COL_RE_F] + 1j * obs_e[:, COL_IM_F]
    tau = h * (obs_g.shape[0] - 1)
    integ = trapezoid(np.abs(beta_e - beta_g) ** 2, h)
    snr = math.sqrt(2.0 * eta * kappa_f * integ)
    eps_sep = 0.5 * float(scipy.special.erfc(snr / 2.0))
    eps_decay = tau * gamma_1 / 2.0
    ion = 0.0
    for obs in (obs_g, obs_e):
        ion += float(np.sum(trapezoid(obs[:, COL_PQ + 2:], h))) if obs.shape[1] > COL_PQ + 2 else 0.0
    ion /= tau
    eps_a = eps_sep + eps_decay
    return dict(snr=snr, eps_sep=eps_sep, eps_decay=eps_decay, eps_a=eps_a,
                ionisation=ion, loss=math.log10(eps_a + ion))
