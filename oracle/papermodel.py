"""The paper's own mode basis -- oracle (no device path yet).

Test infrastructure only (see the package header).  Plain FP64 numpy.

Supplement S2.A: the transmon Hamiltonian 4 E_c n^2 - E_j cos(phi) is
diagonalised in the charge basis |n>, n = -n_cut..n_cut, where cos(phi) couples
n and n +- 1 with weight 1/2 (canonical pair [phi, n] = i); the lowest N_t
eigenstates give the levels omega_j and the charge operator n_t in that basis.

Supplement S2.D: the resonator-filter Hamiltonian
    H_rf = w_r a^a + w_f f^f - J (a^ - a)(f^ - f)
has normal modes c_i = alpha a + beta f + gamma a^ + delta f^ with
[H_rf, c_i] = -w_i c_i.  Matching the coefficients of a, f, a^, f^ gives the
eigenproblem of the 4 x 4 matrix Omega below (its eigenvalues come in pairs
+-w_l, +-w_u); each eigenvector is normalised to |alpha|^2 + |beta|^2 -
|gamma|^2 - |delta|^2 = 1 (bosonic commutator) for the positive frequencies.
S = inv(U^T) expresses (a, f, a^, f^) through (c_u^, c_l^, c_l, c_u) and gives
the couplings mu_u = s14 - s11, mu_l = s13 - s12 (of a^ - a) and nu_u = s24 -
s21, nu_l = s23 - s22 (of f^ - f).
"""
from __future__ import annotations

import numpy as np


def transmon_levels(E_c: float, E_j: float, n_levels: int, n_cut: int = 40):
    """Lowest n_levels eigenvalues (ascending) and the charge operator n_t in
    their eigenbasis (real symmetric, n_levels x n_levels)."""
    n = np.arange(-n_cut, n_cut + 1, dtype=np.float64)
    H = np.diag(4.0 * E_c * n ** 2)
    off = -0.5 * E_j * np.ones(2 * n_cut)
    H += np.diag(off, 1) + np.diag(off, -1)
    w, V = np.linalg.eigh(H)
    V = V[:, :n_levels]
    # fix each eigenvector's sign (largest component positive) so n_t is reproducible
    V = V * np.sign(V[np.argmax(np.abs(V), axis=0), np.arange(n_levels)])
    nt = V.T @ np.diag(n) @ V
    return w[:n_levels], nt


def omega_matrix(w_r: float, w_f: float, J: float) -> np.ndarray:
    """The 4 x 4 matrix of the normal-mode condition in the basis (a, f, a^, f^)."""
    return np.array([[w_r, J, 0.0, J],
                     [J, w_f, J, 0.0],
                     [0.0, -J, -w_r, -J],
                     [-J, 0.0, -J, -w_f]])


def normal_modes(w_r: float, w_f: float, J: float):
    """(w_l, w_u, U, S): normal-mode frequencies w_l < w_u, the eigenvector
    matrix U with columns ordered by frequency -w_u, -w_l, w_l, w_u (each
    normalised to the bosonic norm +-1), and S = inv(U^T)."""
    Om = omega_matrix(w_r, w_f, J)
    ev, vecs = np.linalg.eig(Om)  # Omega acts on the coefficient vector (alpha, beta, gamma, delta)
    order = np.argsort(ev.real)
    ev, vecs = ev.real[order], vecs[:, order].real
    g = np.diag([1.0, 1.0, -1.0, -1.0])
    U = np.empty((4, 4))
    for k in (2, 3):  # w_l, w_u: bosonic norm +1, largest component positive (s_ij real)
        v = vecs[:, k] / np.sqrt(vecs[:, k] @ g @ vecs[:, k])
        U[:, k] = v if v[np.argmax(np.abs(v))] > 0 else -v
    # c^ has the coefficients of c with (a, f) and (a^, f^) exchanged: the
    # -w columns follow from the +w ones
    swap = lambda v: np.array([v[2], v[3], v[0], v[1]])  # noqa: E731
    U[:, 1], U[:, 0] = swap(U[:, 2]), swap(U[:, 3])
    S = np.linalg.inv(U.T)
    return ev[2], ev[3], U, S


def couplings(S: np.ndarray):
    """mu_u, mu_l (a^ - a) and nu_u, nu_l (f^ - f) from S (1-based s_ij of S2.D)."""
    s = lambda i, j: S[i - 1, j - 1]  # noqa: E731
    return (s(1, 4) - s(1, 1), s(1, 3) - s(1, 2), s(2, 4) - s(2, 1), s(2, 3) - s(2, 2))


def bosonic_norms(U: np.ndarray) -> np.ndarray:
    g = np.diag([1.0, 1.0, -1.0, -1.0])
    return np.array([U[:, k] @ g @ U[:, k] for k in range(4)])
