"""Low-rank Lindblad equation of motion, classic RK4 and observables -- oracle.

Test infrastructure only (see the package header).  Plain FP64 numpy.

Notation (supplement S1.A): the density matrix is rho = m m^ (eq.
"lowrank_diagonal") with m = B an N x M matrix whose columns are
sqrt(p_j) psi_j.  Its equation of motion (eq. "nosse") is

    dB/dt = -i H B + O[B],
    O[B]  = 1/2 sum_k [ L_k B (B^+ L_k B)^  -  L_k^ L_k B ],
    B^+   = (B^ B)^-1 B^        (Moore-Penrose inverse of the tall factor)

where the factor 1/2 multiplies both terms (the reading for which
O B^ + B O^ reproduces the dissipator of eq. "lindblad_dissipator").

The operators act mode-wise on the state tensor T[i_q, i_r, i_f, j] (B
reshaped, basis index n = (i_q d_r + i_r) d_f + i_f).  The anti-Hermitian
part -1/2 sum_k L_k^ L_k is diagonal for L_1 = sqrt(kappa_f) f and
L_2 = sqrt(gamma_1) b and is folded into H_eff = H - i/2 (kappa_f n_f + gamma_1 n_q),
so that  dB/dt = -i H_eff B + 1/2 sum_k Y_k X_k^  with

    Y_k = L_k B,   G = B^ B,   C_k = B^ Y_k,   X_k = G^-1 C_k  (= B^+ L_k B).

G^-1 C_k is evaluated through the Cholesky factor G = R R^ and two triangular
solves; a non-positive pivot raises GramNotPD.

Summation order.  The row sums of the Gram and cross products (G, C_k) and of
the observables are mathematically fixed but their rounding depends on the
order in which the N rows are added.  `sum_order` selects it: "matmul" (the
library product, the reference order), "reversed" (the rows taken in reverse
basis order) or "blocked" (sums over consecutive blocks of `_BLOCK` rows,
then the block sums in order).  Runs that differ only in this order measure
the oracle's own rounding floor at a given workload.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import pulses


class GramNotPD(ArithmeticError):
    """B^ B is not Hermitian positive definite (Cholesky pivot <= 0)."""


# ---------------------------------------------------------------- operators

def _as_tensor(model, B):
    return B.reshape(model.d_q, model.d_r, model.d_f, B.shape[1])


def lower(T, axis):
    """Annihilation operator along `axis`: (b T)[n] = sqrt(n+1) T[n+1]."""
    d = T.shape[axis]
    out = np.zeros_like(T)
    shape = [1] * T.ndim
    shape[axis] = d - 1
    coef = np.sqrt(np.arange(1, d, dtype=np.float64)).reshape(shape)
    dst = [slice(None)] * T.ndim
    src = [slice(None)] * T.ndim
    dst[axis] = slice(0, d - 1)
    src[axis] = slice(1, d)
    out[tuple(dst)] = coef * T[tuple(src)]
    return out


def raise_(T, axis):
    """Creation operator along `axis`: (b^ T)[n] = sqrt(n) T[n-1]."""
    d = T.shape[axis]
    out = np.zeros_like(T)
    shape = [1] * T.ndim
    shape[axis] = d - 1
    coef = np.sqrt(np.arange(1, d, dtype=np.float64)).reshape(shape)
    dst = [slice(None)] * T.ndim
    src = [slice(None)] * T.ndim
    dst[axis] = slice(1, d)
    src[axis] = slice(0, d - 1)
    out[tuple(dst)] = coef * T[tuple(src)]
    return out


def quadrature(T, axis):
    """(b + b^) along `axis`."""
    return lower(T, axis) + raise_(T, axis)


def iquadrature(T, axis):
    """i (b^ - b) along `axis` (Hermitian)."""
    return 1j * (raise_(T, axis) - lower(T, axis))


def diag_heff(model):
    """Diagonal of H_eff on the (d_q, d_r, d_f) grid (complex).  Transmon
    levels: Duffing w_q q + alpha/2 q (q - 1), or the given eigenvalues E_t."""
    q = np.arange(model.d_q, dtype=np.float64)[:, None, None]
    r = np.arange(model.d_r, dtype=np.float64)[None, :, None]
    f = np.arange(model.d_f, dtype=np.float64)[None, None, :]
    if getattr(model, "kind", 0) in (1, 2):
        hq = np.asarray(model.E_t, dtype=np.float64)[:, None, None]
    else:
        hq = model.w_q * q + 0.5 * model.alpha * q * (q - 1.0)
    h = hq + model.w_r * r + model.w_f * f
    if getattr(model, "kind", 0) == 2:  # -1/2 L_1^ L_1 is not diagonal there (applied in apply_heff)
        return h - 0.5j * (model.gamma_1 * q)
    return h - 0.5j * (model.kappa_f * f + model.gamma_1 * q)


# ---------------------------------------------------------------- normal-mode basis (kind 2)

def normal_mode_constants(model):
    """(S rows, mu_l, mu_u, nu_l, nu_u): a = S[0] . (c_u^, c_l^, c_l, c_u), f = S[1] . (same), and the
    coefficients of a^ - a = mu_u (c_u^ - c_u) + mu_l (c_l^ - c_l), f^ - f likewise with nu (S2.D)."""
    S = np.asarray(model.S, dtype=np.float64).reshape(2, 4)
    return S, S[0, 2] - S[0, 1], S[0, 3] - S[0, 0], S[1, 2] - S[1, 1], S[1, 3] - S[1, 0]


def _frame_phase(pulse, t):
    """e^{i w_d t} in the frame rotating at the drive carrier, 1 in the lab frame."""
    if pulse is not None and getattr(pulse, "frame", 0) == 1:
        return np.exp(1j * pulse.w_d * t)
    return 1.0 + 0.0j


def _filter_jump(model, T, e1, adjoint=False):
    """sqrt(kappa_f) f T for kind 2, f = s_21 c_u^ + s_22 c_l^ + s_23 c_l + s_24 c_u (modes: l = axis 1,
    u = axis 2); in the drive frame each creation term carries e1 = e^{i w_d t} and each annihilation
    term its conjugate.  adjoint: the Hermitian adjoint f^ instead."""
    S = normal_mode_constants(model)[0]
    s21, s22, s23, s24 = S[1]
    c = np.conj(e1)
    if adjoint:  # f^ = s_21 c_u + s_22 c_l + s_23 c_l^ + s_24 c_u^ (phases conjugated)
        out = s21 * c * lower(T, 2) + s22 * c * lower(T, 1) + s23 * e1 * raise_(T, 1) + s24 * e1 * raise_(T, 2)
    else:
        out = s21 * e1 * raise_(T, 2) + s22 * e1 * raise_(T, 1) + s23 * c * lower(T, 1) + s24 * c * lower(T, 2)
    return np.sqrt(model.kappa_f) * out


def _apply_heff_normal(model, d_t, B, pulse=None, t=0.0):
    """H_eff B for kind 2 in the lab frame or, when pulse.frame is the drive frame, in the frame
    U = exp(i w_d t (q + n_l + n_u)): levels E_q - w_d q, mode frequencies w - w_d, and every term
    that changes the excitation count by D carries e^{i w_d t D} (nothing dropped)."""
    T = _as_tensor(model, B)
    dq = model.d_q
    rot = pulse is not None and getattr(pulse, "frame", 0) == 1
    w_d = pulse.w_d if rot else 0.0
    e1 = _frame_phase(pulse, t)
    _, mu_l, mu_u, nu_l, nu_u = normal_mode_constants(model)
    m2 = model.replace(E_t=tuple(np.asarray(model.E_t) - w_d * np.arange(dq)), w_r=model.w_r - w_d,
                       w_f=model.w_f - w_d)
    Z = diag_heff(m2)[..., None] * T
    nt = np.asarray(model.n_t, dtype=np.float64).reshape(dq, dq)
    qd = np.arange(dq)[:, None] - np.arange(dq)[None, :]          # q' - q (row q', column q)
    up = nt * (e1 ** (qd + 1) if rot else 1.0)                     # n_t x (raising of a mode)
    dn = nt * (e1 ** (qd - 1) if rot else 1.0)                     # n_t x (lowering)
    for mu, ax in ((mu_l, 1), (mu_u, 2)):
        Z = Z + 1j * model.g * mu * (np.einsum("qp,prfj->qrfj", up, raise_(T, ax))
                                     - np.einsum("qp,prfj->qrfj", dn, lower(T, ax)))
    for nu, ax in ((nu_l, 1), (nu_u, 2)):
        Z = Z + d_t * 1j * nu * (e1 * raise_(T, ax) - np.conj(e1) * lower(T, ax))
    # -1/2 L_1^ L_1 B with the filter jump of this frame
    Z = Z - 0.5j * _filter_jump(model, _filter_jump(model, T, e1), e1, adjoint=True)
    return Z.reshape(B.shape)


def apply_heff(model, d_t, B):
    """Z = H_eff(t) B, with d_t the drive coefficient d(t).

    kind 1 (the paper's Hamiltonian, eq. "hamiltonianpurcell", transmon in its
    eigenbasis, bare resonator and filter): i g n_t (a^ - a) - J (a^ - a)(f^ - f)
    + d(t) i (f^ - f), J held in model.G; the drive quadrature i (f^ - f) takes
    d(t) in place of the paper's Omega_d(t) sin(w_d t)."""
    if getattr(model, "kind", 0) == 2:
        return _apply_heff_normal(model, d_t, B)
    T = _as_tensor(model, B)
    Z = diag_heff(model)[..., None] * T
    if getattr(model, "kind", 0) == 1:
        nt = np.asarray(model.n_t, dtype=np.float64).reshape(model.d_q, model.d_q)
        Z = Z + model.g * np.einsum("qp,prfj->qrfj", nt, iquadrature(T, 1))
        Z = Z - model.G * (raise_(raise_(T, 2) - lower(T, 2), 1) - lower(raise_(T, 2) - lower(T, 2), 1))
        Z = Z + d_t * iquadrature(T, 2)
        return Z.reshape(B.shape)
    Z = Z + model.g * quadrature(quadrature(T, 0), 1)
    Z = Z + model.G * quadrature(quadrature(T, 1), 2)
    Z = Z + d_t * quadrature(T, 2)
    return Z.reshape(B.shape)


def apply_heff_drive_frame(model, d_t, w_d, t, B):
    """Z = H'_eff(t) B in the frame rotating at the drive carrier w_d.

    The state is B' = U B with U = exp(i w_d t (n_q + n_r + n_f)); every
    ladder operator picks up a phase, c -> c e^{-i w_d t}, c^ -> c^ e^{i w_d t},
    and the frame change subtracts w_d from each mode frequency:

      H' = (w_q - w_d) n_q + alpha/2 n_q (n_q - 1) + (w_r - w_d) n_r + (w_f - w_d) n_f
           + g  [ b^ a + b a^ + b^ a^ e^{2 i w_d t} + b a e^{-2 i w_d t} ]
           + G  [ a^ f + a f^ + a^ f^ e^{2 i w_d t} + a f e^{-2 i w_d t} ]
           + d(t) [ f^ e^{i w_d t} + f e^{-i w_d t} ]

    with no term dropped (the paper's rotated Hamiltonian, supplement S2.E,
    eq. "hamiltonian_rotated", keeps the counter-rotating terms).  The jump operators only gain a phase,
    which leaves the dissipator unchanged, so H_eff = H' - i/2 (kappa_f n_f +
    gamma_1 n_q) as in the lab frame."""
    if getattr(model, "kind", 0) == 1:
        return _apply_heff_drive_frame_transmon(model, d_t, w_d, t, B)
    if getattr(model, "kind", 0) == 2:
        from types import SimpleNamespace
        return _apply_heff_normal(model, d_t, B, SimpleNamespace(frame=1, w_d=w_d), t)
    T = _as_tensor(model, B)
    m2 = model.replace(w_q=model.w_q - w_d, w_r=model.w_r - w_d, w_f=model.w_f - w_d)
    e1 = np.exp(1j * w_d * t)
    e2 = np.exp(2j * w_d * t)
    Z = diag_heff(m2)[..., None] * T
    Z = Z + model.g * (raise_(lower(T, 1), 0) + lower(raise_(T, 1), 0)
                       + e2 * raise_(raise_(T, 1), 0) + np.conj(e2) * lower(lower(T, 1), 0))
    Z = Z + model.G * (raise_(lower(T, 2), 1) + lower(raise_(T, 2), 1)
                       + e2 * raise_(raise_(T, 2), 1) + np.conj(e2) * lower(lower(T, 2), 1))
    Z = Z + d_t * (e1 * raise_(T, 2) + np.conj(e1) * lower(T, 2))
    return Z.reshape(B.shape)


def _apply_heff_drive_frame_transmon(model, d_t, w_d, t, B):
    """Kind 1 in the frame U = exp(i w_d t (q + n_r + n_f)), q the transmon
    level index: every term X that changes the excitation count by D becomes
    e^{i w_d t D} X, and the diagonal loses w_d (q + r + f).  The levels are
    E_q - w_d q; i g n_t[q'][q] a^ gains e^{i w_d t (q' - q + 1)} and the a part
    e^{i w_d t (q' - q - 1)}; -J (a^ - a)(f^ - f) has D = 2 (a^ f^), 0, 0, -2
    (a f); the drive i (f^ - f) has D = +1, -1.  Nothing is dropped."""
    T = _as_tensor(model, B)
    dq = model.d_q
    m2 = model.replace(E_t=tuple(np.asarray(model.E_t) - w_d * np.arange(dq)), w_r=model.w_r - w_d,
                       w_f=model.w_f - w_d)
    Z = diag_heff(m2)[..., None] * T
    nt = np.asarray(model.n_t, dtype=np.float64).reshape(dq, dq)
    qd = np.arange(dq)[:, None] - np.arange(dq)[None, :]          # q' - q (row q', column q)
    up = nt * np.exp(1j * w_d * t * (qd + 1))
    dn = nt * np.exp(1j * w_d * t * (qd - 1))
    Z = Z + 1j * model.g * (np.einsum("qp,prfj->qrfj", up, raise_(T, 1))
                            - np.einsum("qp,prfj->qrfj", dn, lower(T, 1)))
    e1 = np.exp(1j * w_d * t)
    e2 = e1 * e1
    Z = Z - model.G * (e2 * raise_(raise_(T, 2), 1) - raise_(lower(T, 2), 1)
                       - lower(raise_(T, 2), 1) + np.conj(e2) * lower(lower(T, 2), 1))
    Z = Z + d_t * 1j * (e1 * raise_(T, 2) - np.conj(e1) * lower(T, 2))
    return Z.reshape(B.shape)


def apply_jumps(model, B, pulse=None, t=0.0):
    """[Y_1, Y_2] = [sqrt(kappa_f) f B, sqrt(gamma_1) b B].  kind 2: f is the filter operator in the
    normal-mode basis, in the frame of the pulse (its terms phased in the drive frame; a phase common
    to a whole jump operator, as for kinds 0 and 1, leaves the dissipator unchanged and is dropped)."""
    T = _as_tensor(model, B)
    if getattr(model, "kind", 0) == 2:
        Y1 = _filter_jump(model, T, _frame_phase(pulse, t))
    else:
        Y1 = np.sqrt(model.kappa_f) * lower(T, 2)
    Y2 = np.sqrt(model.gamma_1) * lower(T, 0)
    return [Y1.reshape(B.shape), Y2.reshape(B.shape)]


# ---------------------------------------------------------------- row sums

SUM_ORDERS = ("matmul", "reversed", "blocked")
_BLOCK = 40


def inner(X, Y, sum_order="matmul"):
    """X^ Y = sum over rows n of conj(X[n, :])^T Y[n, :], rows added in the
    given order (see the module header)."""
    if sum_order == "matmul":
        return X.conj().T @ Y
    if sum_order == "reversed":
        return X[::-1].conj().T @ Y[::-1]
    if sum_order == "blocked":
        acc = np.zeros((X.shape[1], Y.shape[1]), dtype=np.complex128)
        for b in range(0, X.shape[0], _BLOCK):
            acc = acc + X[b:b + _BLOCK].conj().T @ Y[b:b + _BLOCK]
        return acc
    raise ValueError(f"unknown sum_order {sum_order!r}")


def total(x, sum_order="matmul"):
    """Sum of all entries of x (flattened in C order), in the given order."""
    if sum_order == "matmul":
        return np.sum(x)
    v = np.ravel(x)
    if sum_order == "reversed":
        return np.sum(v[::-1])
    if sum_order == "blocked":
        blk = _BLOCK * 64
        acc = 0.0
        for b in range(0, v.size, blk):
            acc = acc + np.sum(v[b:b + blk])
        return acc
    raise ValueError(f"unknown sum_order {sum_order!r}")


# ---------------------------------------------------------------- RHS

def gram_solve(G, C_list):
    """X_k = G^-1 C_k through the Cholesky factor of G (lower R, G = R R^)."""
    try:
        R = np.linalg.cholesky(G)
    except np.linalg.LinAlgError as exc:
        raise GramNotPD(str(exc)) from None
    if not np.all(np.isfinite(R)) or np.any(np.real(np.diag(R)) <= 0.0):
        raise GramNotPD("non-positive pivot")
    out = []
    for C in C_list:
        Y = scipy.linalg.solve_triangular(R, C, lower=True)
        out.append(scipy.linalg.solve_triangular(R.conj().T, Y, lower=False))
    return out


def rhs(model, pulse, t, B, sum_order="matmul"):
    """dB/dt at time t (equation of motion of supplement S1.A)."""
    d_t = pulses.drive(pulse, t) if pulse is not None else 0.0
    if pulse is not None and getattr(pulse, "frame", 0) == 1:
        Z = apply_heff_drive_frame(model, d_t, pulse.w_d, t, B)
    else:
        Z = apply_heff(model, d_t, B)
    Y = apply_jumps(model, B, pulse, t)
    G = inner(B, B, sum_order)
    C = [inner(B, Yk, sum_order) for Yk in Y]
    X = gram_solve(G, C)
    dB = -1j * Z
    for Yk, Xk in zip(Y, X):
        dB = dB + 0.5 * (Yk @ Xk.conj().T)
    return dB


# ---------------------------------------------------------------- observables

OBS_HEADER = ("re_a", "im_a", "re_f", "im_f", "tr_rho", "tr_rho2")


def observables(model, B, sum_order="matmul", pulse=None, t=0.0):
    """[Re<a>, Im<a>, Re<f>, Im<f>, tr rho, tr rho^2, P_q(0..d_q-1)].

    <O> = tr(O rho) = sum_j b_j^ O b_j (unnormalised); tr rho^2 = ||B^ B||_F^2
    (since tr (B B^)^2 = tr (B^ B)^2); P_q(k) = tr(|k><k|_q rho).  The two fields
    are those of the lowering operators of the resonator and filter slots, in
    the frame of the state (in the drive frame e^{i w_d t} times the lab-frame
    field).  Kind 2 (normal-mode basis): <a> is the lower mode's <c_l>, and <f>
    is the filter field that the readout separation takes (S2.D: f = s_21 c_u^ +
    s_22 c_l^ + s_23 c_l + s_24 c_u), e^{i w_d t} <f>_lab in the drive frame,
    which is s_23 <c_l> + s_24 <c_u> + e^{2 i w_d t} (s_21 <c_u>* + s_22 <c_l>*)
    in terms of the drive-frame mode fields (pulse, t: the frame and the time of
    the record).
    """
    T = _as_tensor(model, B)
    a = total(T.conj() * lower(T, 1), sum_order)
    f = total(T.conj() * lower(T, 2), sum_order)
    if getattr(model, "kind", 0) == 2:
        s21, s22, s23, s24 = normal_mode_constants(model)[0][1]
        e2 = _frame_phase(pulse, t) ** 2
        f = s23 * a + s24 * f + e2 * (s21 * np.conj(f) + s22 * np.conj(a))
    tr = total(np.abs(T) ** 2, sum_order)
    G = inner(B, B, sum_order)
    tr2 = np.sum(np.abs(G) ** 2)
    if sum_order == "matmul":
        Pq = np.sum(np.abs(T) ** 2, axis=(1, 2, 3))
    else:
        Pq = np.array([total(np.abs(T[q]) ** 2, sum_order) for q in range(model.d_q)])
    return np.concatenate([[a.real, a.imag, f.real, f.imag, tr, tr2], Pq])


# ---------------------------------------------------------------- RK4

def rk4_step(fun, t, dt, B):
    k1 = fun(t, B)
    k2 = fun(t + 0.5 * dt, B + (0.5 * dt) * k1)
    k3 = fun(t + 0.5 * dt, B + (0.5 * dt) * k2)
    k4 = fun(t + dt, B + dt * k3)
    return B + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def integrate(model, pulse, t0, dt, nsteps, B0, obs_stride=0, sum_order="matmul"):
    """Classic fixed-step RK4 from B(t0) = B0 over nsteps steps of dt.

    Step n runs from t_n = t0 + n dt.  Observables are recorded at step 0 and
    after every obs_stride-th step; returns (B(t0 + nsteps dt), obs) with obs
    of shape (nsteps // obs_stride + 1, 6 + d_q) (empty if obs_stride == 0).
    """
    B = np.array(B0, dtype=np.complex128, copy=True)
    fun = lambda t, X: rhs(model, pulse, t, X, sum_order)  # noqa: E731
    rec = []
    if obs_stride > 0:
        rec.append(observables(model, B, sum_order, pulse, t0))
    for n in range(nsteps):
        B = rk4_step(fun, t0 + n * dt, dt, B)
        if obs_stride > 0 and (n + 1) % obs_stride == 0:
            rec.append(observables(model, B, sum_order, pulse, t0 + (n + 1) * dt))
    obs = np.array(rec) if rec else np.zeros((0, 6 + model.d_q))
    return B, obs
