"""Brute-force dense operators and the full Lindblad master equation -- oracle.

Test infrastructure only (see the package header).  Every operator is built
as an explicit N x N matrix from single-mode d x d matrices with numpy.kron in
the order transmon (x) resonator (x) filter, independently of the slicing
code in ``lowrank``.  The master equation is the one of supplement S1.A
(eq. "master_equation", dissipator eq. "lindblad_dissipator"):

    d rho/dt = -i [H, rho] + sum_k ( L_k rho L_k^ - 1/2 {L_k^ L_k, rho} ).
"""
from __future__ import annotations

import numpy as np

from . import pulses


def annihilation(d):
    """<n-1| b |n> = sqrt(n)."""
    return np.diag(np.sqrt(np.arange(1, d, dtype=np.float64)), 1).astype(np.complex128)


def _embed(model, op, mode):
    Iq = np.eye(model.d_q)
    Ir = np.eye(model.d_r)
    If = np.eye(model.d_f)
    mats = [Iq, Ir, If]
    mats[mode] = op
    return np.kron(mats[0], np.kron(mats[1], mats[2]))


def operators(model):
    """Dense b, a, f (annihilation) on the full space."""
    b = _embed(model, annihilation(model.d_q), 0)
    a = _embed(model, annihilation(model.d_r), 1)
    f = _embed(model, annihilation(model.d_f), 2)
    return b, a, f


def _normal_constants(model):
    S = np.asarray(model.S, dtype=np.float64).reshape(2, 4)
    return S, S[0, 2] - S[0, 1], S[0, 3] - S[0, 0], S[1, 2] - S[1, 1], S[1, 3] - S[1, 0]


def hamiltonian(model, d_t):
    """Dense H(t) for the drive coefficient d_t (kind 1: the paper's
    Hamiltonian with the transmon in its eigenbasis, see lowrank.apply_heff;
    kind 2: the same in the normal-mode basis, modes c_l and c_u in the
    resonator and filter slots)."""
    b, a, f = operators(model)
    if getattr(model, "kind", 0) == 2:
        cl, cu = a, f
        _, mu_l, mu_u, nu_l, nu_u = _normal_constants(model)
        Ht = _embed(model, np.diag(np.asarray(model.E_t, dtype=np.float64)).astype(np.complex128), 0)
        Nt = _embed(model, np.asarray(model.n_t, dtype=np.float64).reshape(model.d_q, model.d_q).astype(np.complex128), 0)
        Xl = cl.conj().T - cl
        Xu = cu.conj().T - cu
        H = Ht + model.w_r * cl.conj().T @ cl + model.w_f * cu.conj().T @ cu
        return H + 1j * model.g * Nt @ (mu_l * Xl + mu_u * Xu) + 1j * d_t * (nu_l * Xl + nu_u * Xu)
    if getattr(model, "kind", 0) == 1:
        Ht = _embed(model, np.diag(np.asarray(model.E_t, dtype=np.float64)).astype(np.complex128), 0)
        Nt = _embed(model, np.asarray(model.n_t, dtype=np.float64).reshape(model.d_q, model.d_q).astype(np.complex128), 0)
        Xa = a.conj().T - a
        Xf = f.conj().T - f
        H = Ht + model.w_r * a.conj().T @ a + model.w_f * f.conj().T @ f
        H = H + 1j * model.g * Nt @ Xa - model.G * Xa @ Xf + d_t * 1j * Xf
        return H
    nq = b.conj().T @ b
    Nn = nq.shape[0]
    I = np.eye(Nn)
    H = (model.w_q * nq + 0.5 * model.alpha * nq @ (nq - I)
         + model.w_r * a.conj().T @ a + model.w_f * f.conj().T @ f)
    H = H + model.g * (b + b.conj().T) @ (a + a.conj().T)
    H = H + model.G * (a + a.conj().T) @ (f + f.conj().T)
    H = H + d_t * (f + f.conj().T)
    return H


def hamiltonian_drive_frame(model, d_t, w_d, t):
    """Dense H'(t) in the frame rotating at w_d: U H U^ - w_d (n_q + n_r + n_f)
    with U = exp(i w_d t (n_q + n_r + n_f)), built from the phased ladder
    operators b e^{-i w_d t}, a e^{-i w_d t}, f e^{-i w_d t} (all terms kept)."""
    if getattr(model, "kind", 0) in (1, 2):  # U H U^ - w_d n, n = q + n_r + n_f, from the lab-frame matrix
        n = np.array([q + r + f for q in range(model.d_q) for r in range(model.d_r) for f in range(model.d_f)],
                     dtype=np.float64)
        u = np.exp(1j * w_d * t * n)
        return (u[:, None] * hamiltonian(model, d_t) * np.conj(u)[None, :]) - w_d * np.diag(n)
    b, a, f = operators(model)
    ph = np.exp(-1j * w_d * t)
    bt, at, ft = b * ph, a * ph, f * ph
    nq = b.conj().T @ b
    Nn = nq.shape[0]
    I = np.eye(Nn)
    H = ((model.w_q - w_d) * nq + 0.5 * model.alpha * nq @ (nq - I)
         + (model.w_r - w_d) * a.conj().T @ a + (model.w_f - w_d) * f.conj().T @ f)
    H = H + model.g * (bt + bt.conj().T) @ (at + at.conj().T)
    H = H + model.G * (at + at.conj().T) @ (ft + ft.conj().T)
    H = H + d_t * (ft + ft.conj().T)
    return H


def frame_hamiltonian(model, pulse, t):
    """H(t) of the pulse's frame (lab, or rotating at w_d)."""
    d_t = pulses.drive(pulse, t) if pulse is not None else 0.0
    if pulse is not None and getattr(pulse, "frame", 0) == 1:
        return hamiltonian_drive_frame(model, d_t, pulse.w_d, t)
    return hamiltonian(model, d_t)


def filter_operator(model, pulse=None, t=0.0):
    """Kind 2: the filter's annihilation operator f = s_21 c_u^ + s_22 c_l^ + s_23 c_l + s_24 c_u in the
    normal-mode basis, turned into the frame of the pulse as U f U^ (U = exp(i w_d t n), n = q + n_r +
    n_f) in the drive frame."""
    b, a, f = operators(model)
    S = _normal_constants(model)[0]
    fn = S[1, 0] * f.conj().T + S[1, 1] * a.conj().T + S[1, 2] * a + S[1, 3] * f
    if pulse is not None and getattr(pulse, "frame", 0) == 1:
        n = np.array([q + r + k for q in range(model.d_q) for r in range(model.d_r) for k in range(model.d_f)],
                     dtype=np.float64)
        u = np.exp(1j * pulse.w_d * t * n)
        fn = u[:, None] * fn * np.conj(u)[None, :]
    return fn


def jump_operators(model, pulse=None, t=0.0):
    """sqrt(kappa_f) f and sqrt(gamma_1) b.  kind 2: f in the normal-mode basis and the frame of the
    pulse (filter_operator); for kinds 0 and 1 the frame rotation of f is a global phase, which leaves
    the dissipator unchanged."""
    b, a, f = operators(model)
    if getattr(model, "kind", 0) == 2:
        return [np.sqrt(model.kappa_f) * filter_operator(model, pulse, t), np.sqrt(model.gamma_1) * b]
    return [np.sqrt(model.kappa_f) * f, np.sqrt(model.gamma_1) * b]


def lindbladian(model, pulse, t, rho):
    """Right-hand side of the master equation on a dense rho."""
    H = frame_hamiltonian(model, pulse, t)
    out = -1j * (H @ rho - rho @ H)
    for L in jump_operators(model, pulse, t):
        LdL = L.conj().T @ L
        out = out + L @ rho @ L.conj().T - 0.5 * (LdL @ rho + rho @ LdL)
    return out


def lowrank_rhs_pinv(model, pulse, t, B):
    """Literal low-rank right-hand side with dense matrices and numpy's pinv:
    -i H B + 1/2 sum_k [ L_k B (pinv(B) L_k B)^ - L_k^ L_k B ]."""
    H = frame_hamiltonian(model, pulse, t)
    Bp = np.linalg.pinv(B)
    out = -1j * (H @ B)
    for L in jump_operators(model, pulse, t):
        LB = L @ B
        out = out + 0.5 * (LB @ (Bp @ LB).conj().T - L.conj().T @ L @ B)
    return out


def observables(model, rho, pulse=None, t=0.0):
    """Same record as lowrank.observables, computed from a dense rho (kind 2: <f> = e1 tr(U f U^ rho)
    with the filter operator of filter_operator, e1 = e^{i w_d t} in the drive frame, 1 in the lab
    frame)."""
    b, a, f = operators(model)
    ea = np.trace(a @ rho)
    ef = np.trace(f @ rho)
    if getattr(model, "kind", 0) == 2:
        e1 = np.exp(1j * pulse.w_d * t) if pulse is not None and getattr(pulse, "frame", 0) == 1 else 1.0
        ef = e1 * np.trace(filter_operator(model, pulse, t) @ rho)
    tr = np.trace(rho).real
    tr2 = np.trace(rho @ rho).real
    Pq = []
    for k in range(model.d_q):
        Pk = np.zeros((model.d_q, model.d_q))
        Pk[k, k] = 1.0
        Pq.append(np.trace(_embed(model, Pk, 0) @ rho).real)
    return np.concatenate([[ea.real, ea.imag, ef.real, ef.imag, tr, tr2], Pq])


def integrate(model, pulse, t0, dt, nsteps, rho0, obs_stride=0):
    """Classic RK4 on the dense rho with the same stage times as the low-rank path."""
    rho = np.array(rho0, dtype=np.complex128, copy=True)
    fun = lambda t, X: lindbladian(model, pulse, t, X)  # noqa: E731
    rec = [observables(model, rho, pulse, t0)] if obs_stride > 0 else []
    for n in range(nsteps):
        t = t0 + n * dt
        k1 = fun(t, rho)
        k2 = fun(t + 0.5 * dt, rho + (0.5 * dt) * k1)
        k3 = fun(t + 0.5 * dt, rho + (0.5 * dt) * k2)
        k4 = fun(t + dt, rho + dt * k3)
        rho = rho + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        if obs_stride > 0 and (n + 1) % obs_stride == 0:
            rec.append(observables(model, rho, pulse, t0 + (n + 1) * dt))
    return rho, (np.array(rec) if rec else np.zeros((0, 6 + model.d_q)))
