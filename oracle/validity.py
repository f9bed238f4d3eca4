"""Validity control quantities of the low-rank approximation -- oracle.

Test infrastructure only (see the package header).  Supplement S1.B: the
low-rank density matrix rho = m m^ (eq. "lowrank_diagonal") carries weights
p_1 >= ... >= p_M, the nonzero eigenvalues of rho; the paper follows the
ratio p_M / p_1 in time as the proxy of the truncation error, and the purity
tr(rho^2) = sum_j p_j^2, which the approximation overestimates and which
approaches the exact value as M grows.  For the full solution the same
ratio is taken between the M-th and the first eigenvalue of rho.

The nonzero eigenvalues of B B^ are those of the M x M matrix B^ B; this
module takes them from the latter with a library Hermitian eigensolver.
"""
from __future__ import annotations

import numpy as np


def spectrum(B):
    """p_1 >= ... >= p_M: the eigenvalues of B^ B (= the nonzero eigenvalues of rho = B B^)."""
    B = np.asarray(B, dtype=np.complex128)
    G = B.conj().T @ B
    return np.sort(np.linalg.eigvalsh(G))[::-1]


def control_ratio(p):
    """p_M / p_1 from a descending spectrum."""
    return float(p[-1] / p[0])


def purity(p):
    """tr(rho^2) = sum_j p_j^2 from the spectrum of the low-rank rho."""
    return float(np.sum(np.asarray(p) ** 2))


def dense_top(rho, M):
    """The M largest eigenvalues of a full density matrix, descending."""
    return np.sort(np.linalg.eigvalsh(np.asarray(rho, dtype=np.complex128)))[::-1][:M]
