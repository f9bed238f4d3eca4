"""Transmon eigenbasis tables and normal modes for the paper's Hamiltonian (model kinds 1 and 2).

Supplement S2.A: the transmon 4 E_c n^2 - E_j cos(phi) is written in its own
eigenbasis, keeping the lowest N_t levels.  `eigenbasis` diagonalises it in
the charge basis |n>, n = -n_cut..n_cut (cos(phi) links n and n +- 1 with
weight 1/2) and returns the levels, shifted so the ground level is 0, and the
charge operator n_t in that basis (real symmetric, zero diagonal at zero
offset charge).  `paper_model` fills a ModelParams of kind MODEL_TRANSMON with
the parameters of supplement S2.B: E_c / 2 pi = 315 MHz, E_j / E_c = 51,
g / 2 pi = 150 MHz, J / 2 pi = 30 MHz, w_r / 2 pi = 7.2 GHz, w_f / 2 pi =
7.21 GHz, kappa / 2 pi = 30 MHz (filter), gamma / 2 pi = 8 kHz (transmon).

Supplement S2.D: `normal_modes` finds the normal modes c_l, c_u of the
resonator-filter pair w_r a^a + w_f f^f - J (a^ - a)(f^ - f) and the rows of S
that give a and f in terms of (c_u^, c_l^, c_l, c_u); `paper_model_normal`
fills a ModelParams of kind MODEL_NORMAL (the paper's truncation basis).
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


def normal_modes(w_r: float, w_f: float, J: float):
    """(w_l, w_u, S2) for the resonator-filter pair: the normal-mode frequencies w_l < w_u and the rows
    S2 = [s_1j; s_2j] of S = (U^T)^-1, with a = s_11 c_u^ + s_12 c_l^ + s_13 c_l + s_14 c_u and f likewise.
    A normal mode c = x . (a, f, a^, f^) with [H, c] = -w c has x an eigenvector of the matrix below with
    eigenvalue w; the modes are normalised to x_1^2 + x_2^2 - x_3^2 - x_4^2 = 1 ([c, c^] = 1) and the
    columns of U run over -w_u, -w_l, w_l, w_u, the negative ones being the creation operators (the
    coefficients of c with the (a, f) and (a^, f^) halves exchanged)."""
    om = np.array([[w_r, J, 0.0, J], [J, w_f, J, 0.0], [0.0, -J, -w_r, -J], [-J, 0.0, -J, -w_f]])
    vals, vecs = np.linalg.eig(om)
    idx = np.argsort(vals.real)
    vals, vecs = vals.real[idx], vecs.real[:, idx]
    metric = np.array([1.0, 1.0, -1.0, -1.0])
    cols = {}
    for k in (2, 3):
        x = vecs[:, k] / np.sqrt(np.sum(metric * vecs[:, k] ** 2))
        cols[k] = -x if x[np.argmax(np.abs(x))] < 0 else x
    U = np.column_stack([np.roll(cols[3], 2), np.roll(cols[2], 2), cols[2], cols[3]])
    S = np.linalg.inv(U.T)
    return vals[2], vals[3], S[:2].copy()


def paper_model_normal(d_q: int, d_l: int, d_u: int) -> I.ModelParams:
    """The paper's Hamiltonian of supplement S2.B in its normal-mode basis (S2.D): d_q transmon levels,
    d_l levels of the lower normal mode (resonator slot), d_u of the upper one (filter slot)."""
    E_c = I.ghz(PAPER_EC_GHZ)
    levels, n_t = eigenbasis(E_c, PAPER_EJ_OVER_EC * E_c, d_q)
    w_l, w_u, S2 = normal_modes(I.ghz(7.2), I.ghz(7.21), I.ghz(0.03))
    return I.ModelParams(d_q=d_q, d_r=d_l, d_f=d_u, w_q=0.0, alpha=0.0, w_r=w_l, w_f=w_u,
                         g=I.ghz(0.15), G=0.0, kappa_f=I.ghz(0.03), gamma_1=I.ghz(8e-6),
                         kind=I.MODEL_NORMAL, E_t=tuple(levels), n_t=tuple(n_t.ravel()),
                         S=tuple(S2.ravel()))
