"""Host logic of the pulse optimiser (supplement S3.C): the SPSA gradient
estimate and its update rule, and the projection onto the drive bound.  The
device half (loss batches of stepwise pulses) is in the GPU parity tests."""
import itertools

import numpy as np

from paper_2508_18114_amd import inputs as I
from paper_2508_18114_amd import serve


def _quadratic(n, seed):
    r = np.random.default_rng(seed)
    Q = r.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    b = r.standard_normal(n)
    return A, b, (lambda x: 0.5 * x @ A @ x + b @ x), (lambda x: A @ x + b)


def test_spsa_estimate_is_unbiased_on_quadratics():
    """For a quadratic loss the central difference along delta is exactly g . delta, so the mean of
    the estimate over all 2^n sign vectors is the gradient itself (the cross terms cancel in pairs)."""
    n = 5
    A, b, L, grad = _quadratic(n, 3)
    theta = np.random.default_rng(4).standard_normal(n)
    ck = 0.3
    acc = np.zeros(n)
    for signs in itertools.product((-1.0, 1.0), repeat=n):
        d = np.array(signs)
        acc += serve.spsa_gradient(L(theta + ck * d), L(theta - ck * d), ck, d)
    np.testing.assert_allclose(acc / 2 ** n, grad(theta), rtol=1e-12, atol=1e-12)


def test_spsa_estimate_of_a_linear_loss_along_one_axis():
    """A loss that depends on one coordinate only: the estimate's component on that coordinate is
    exact for every sign vector, the others are +-3 with the sign of d_2 d_i."""
    n = 4
    ck = 0.1
    for signs in itertools.product((-1.0, 1.0), repeat=n):
        d = np.array(signs)
        x0 = np.array([0.5, -1.0, 2.0, 0.0])
        L = lambda x: 3.0 * x[2] - 1.0
        g = serve.spsa_gradient(L(x0 + ck * d), L(x0 - ck * d), ck, d)
        assert abs(g[2] - 3.0) <= 1e-13
        np.testing.assert_allclose(g, 3.0 * d[2] / d, rtol=1e-13)


def test_spsa_converges_on_a_quadratic():
    n = 6
    A, b, L, grad = _quadratic(n, 5)
    xstar = np.linalg.solve(A, -b)
    opt = serve.SPSA(np.zeros(n), seed=6, a=0.05, c=0.1)
    for _ in range(4000):
        xp, xm = opt.ask()
        np.testing.assert_allclose(xp + xm, 2 * opt.theta, atol=1e-15)  # symmetric probes
        opt.tell(L(xp), L(xm))
    assert np.linalg.norm(opt.theta - xstar) <= 1e-2 * np.linalg.norm(xstar)
    assert L(opt.theta) < L(np.zeros(n))


def test_spsa_gain_sequences():
    opt = serve.SPSA(np.zeros(2), seed=0, a=0.2, c=0.05, A=10.0, alpha=0.602, gamma=0.101)
    for k in range(3):
        ak, ck = opt.gains()
        assert ak == 0.2 / (k + 11) ** 0.602 and ck == 0.05 / (k + 1) ** 0.101
        opt.ask()
        opt.tell(1.0, 1.0)  # equal losses: no move
        np.testing.assert_array_equal(opt.theta, np.zeros(2))


def test_project_heights_holds_the_drive_bound():
    bound = I.ghz(0.4)
    h = np.array([0.1 + 0.2j, 3.0 + 0.0j, -2.0 + 2.0j, 0.0j])
    theta = np.empty(8)
    theta[0::2], theta[1::2] = h.real, h.imag
    out = serve.heights_from(serve.project_heights(theta))
    assert np.all(np.abs(out) < bound)
    assert out[0] == h[0] and out[3] == 0.0          # inside: unchanged
    np.testing.assert_allclose(np.angle(out[1:3]), np.angle(h[1:3]))  # outside: radial scaling
    np.testing.assert_allclose(np.abs(out[1:3]), bound, rtol=1e-8)


def test_autotune_signature_and_candidates():
    """Host logic of the schedule autotuner: the signature is the multiset of shapes, and every candidate
    maps to the library's flags."""
    from paper_2508_18114_amd import autotune, lr
    m1, m2 = I.readout_model(8, 50, 5), I.readout_model(8, 25, 5)
    items = [dict(model=m1, M=20), dict(model=m2, M=8, precision=1), dict(model=m1, M=20)]
    assert autotune.signature(items) == "8x25x5:M8:p1*1;8x50x5:M20:p0*2"
    assert autotune.signature(list(reversed(items))) == autotune.signature(items)
    cands = autotune.candidates(3)
    assert [c["schedule"] for c in cands] == ["spread"] * 3 + ["packed"]
    assert autotune.flags_of(cands[1]) == lr.LR_BATCH_SPREAD_LAYERS(2) == 2 << 8
    assert autotune.flags_of(cands[-1]) == lr.LR_BATCH_PACKED


def test_square_start_is_the_papers_square_pulse_in_each_model():
    """Kinds 1 and 2 carry the drive on i (f^ - f): the paper's real square amplitude is an imaginary
    height there, so d(t) = Re[Omega e^{-i w_d t}] = A sin(w_d t) (its sin carrier); the Duffing model's
    (f + f^) drive starts from real heights (cos carrier)."""
    from oracle import pulses as opulses
    from paper_2508_18114_amd import serve, transmon
    A = I.ghz(0.15)
    for model, imag in ((I.readout_model(3, 4, 3), False), (transmon.paper_model(4, 3, 3), True),
                        (transmon.paper_model_normal(4, 3, 3), True)):
        h = serve.heights_from(serve.square_start(model, 3))
        assert np.allclose(h, 1j * A if imag else A)
        p = I.stepwise_pulse(h, 40.0, sigma=0.5, w_d=transmon.PAPER_W_DRIVE)
        t = 20.0  # on the plateau, far from every step
        d = opulses.drive(p, t)
        expect = A * (np.sin(p.w_d * t) if imag else np.cos(p.w_d * t))
        assert abs(d - expect) < 1e-8 * A  # the outer steps, 10 ns = 20 sigma away, leave e^-20
