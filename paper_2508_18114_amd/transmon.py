"""Transmon eigenbasis tables for the paper's Hamiltonian (model kind 1).

Supplement S2.A: the transmon 4 E_c n^2 - E_j cos(phi) is written in its own
eigenbasis, keeping the lowest N_t levels.  `eigenbasis` diagonalises it in
the charge basis |n>, n = -n_cut..n_cut (cos(phi) links n and n +- 1 with
weight 1/2) and returns the levels, shifted so the ground level is 0, and the
charge operator n_t in that basis (real symmetric, zero diagonal at zero
offset charge).  `paper_model` fills a ModelParams of kind MODEL_TRANSMON with
the parameters of supplement S2.B: E_c / 2 pi = 315 MHz, E_j / E_c = 51,
g / 2 pi = 150 MHz, J / 2 pi = 30 MHz, w_r / 2 pi = 7.2 GHz, w_f / 2 pi =
7.21 GHz, kappa / 2 pi = 30 MHz (filter), gamma / 2 pi = 8 kHz (transmon).
"""
from __future__ import annotations

import numpy as np

from . import inputs as I

PAPER_EC_GHZ = 0.315
PAPER_EJ_OVER_EC = 51.0
PAPER_W_DRIVE = I.ghz(7.18)


def eigenbasis(E_c: float, E_j: float, n_levels: int, n_cut: int = 40):
    charges = np.arange(-n_cut, n_cut + 1, dtype=np.float64)
    h = np.diag(4.0 * E_c * charges ** 2) - 0.5 * E_j * (np.eye(2 * n_cut + 1, k=1) + np.eye(2 * n_cut + 1, k=-1))
    levels, vec = np.linalg.eigh(h)
    vec = vec[:, :n_levels]
    for k in range(n_levels):  # a fixed sign per eigenvector: its largest component positive
        if vec[np.argmax(np.abs(vec[:, k])), k] < 0:
            vec[:, k] = -vec[:, k]
    n_t = vec.T @ (charges[:, None] * vec)
    n_t = 0.5 * (n_t + n_t.T)
    return levels[:n_levels] - levels[0], n_t


def paper_model(d_q: int, d_r: int, d_f: int) -> I.ModelParams:
    E_c = I.ghz(PAPER_EC_GHZ)
    levels, n_t = eigenbasis(E_c, PAPER_EJ_OVER_EC * E_c, d_q)
    return I.ModelParams(d_q=d_q, d_r=d_r, d_f=d_f, w_q=0.0, alpha=0.0, w_r=I.ghz(7.2), w_f=I.ghz(7.21),
                         g=I.ghz(0.15), G=I.ghz(0.03), kappa_f=I.ghz(0.03), gamma_1=I.ghz(8e-6),
                         kind=I.MODEL_TRANSMON, E_t=tuple(levels), n_t=tuple(n_t.ravel()))
