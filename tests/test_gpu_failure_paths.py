"""Failure handling on the device, driven from the host.

The on-chip integrator's group barriers are bounded waits.  lr_wait_limits /
lr_batch_wait_limits make every wait target a flag value that no workgroup
writes, with a small poll budget, so each wait expires after a few thousand
polls: every kernel still runs to its end (no fault, no hang), the trajectory
reports LR_ERR_TIMEOUT, and the same context or batch integrates normally once
the limits are back to their defaults.
"""
import numpy as np
import pytest

from paper_2508_18114_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_18114_amd import lr as _lr
    return _lr


def _case():
    m = I.readout_model(4, 10, 5).replace(kappa_f=0.5, gamma_1=0.05)
    p = I.flattop_pulse(0.05, 0.2, t_ramp=0.05)
    return m, p, I.initial_state(m, 4, "e", seed=21, scale=1e-3)


def test_context_wait_expiry_reports_timeout_and_recovers(lr):
    m, p, B0 = _case()
    ctx = lr.Context(m, 4)
    ctx.wait_limits(spins=2000, never=True)
    Bd = lr.to_device(B0)
    obs = ctx.new_obs(60, 20)
    ctx.integrate(p, 0.0, 1e-3, 60, Bd, 20, obs)
    rc, fs = ctx.status()
    print(f"[failure] context with expiring waits: {lr.lr_strerror(rc)} at step {fs}")
    assert rc == lr.LR_ERR_TIMEOUT and fs == 0
    # defaults again: the same context integrates normally, bitwise as a fresh one
    ctx.wait_limits()
    Bd = lr.to_device(B0)
    obs = ctx.new_obs(60, 20)
    ctx.integrate(p, 0.0, 1e-3, 60, Bd, 20, obs)
    assert ctx.status()[0] == lr.LR_OK
    fresh = lr.Context(m, 4)
    Bf = lr.to_device(B0)
    of = fresh.new_obs(60, 20)
    fresh.integrate(p, 0.0, 1e-3, 60, Bf, 20, of)
    assert fresh.status()[0] == lr.LR_OK
    assert np.array_equal(lr.from_device(Bd), lr.from_device(Bf))
    assert np.array_equal(obs.cpu().numpy(), of.cpu().numpy())
    ctx.close()
    fresh.close()


def test_batch_wait_expiry_stops_only_spread_trajectories(lr):
    """Expiring waits stop a spread batch with LR_ERR_TIMEOUT, while a packed batch under the same
    limits (its kernel has no group barriers) completes; with the defaults restored the spread batch
    completes and equals a fresh one bitwise."""
    import torch
    m, p, B0 = _case()

    def items():
        return [dict(model=m, M=4, pulse=p, dt=1e-3, nsteps=60, B=lr.to_device(B0))]

    its = items()
    b = lr.Batch(its, stream=torch.cuda.current_stream())
    b.wait_limits(spins=2000, never=True)
    b.run()
    rc, codes, steps = b.status()
    print(f"[failure] spread batch with expiring waits: codes {codes}, steps {steps}")
    assert codes == [lr.LR_ERR_TIMEOUT]
    pk = items()
    bp = lr.Batch(pk, packed=True)
    bp.wait_limits(spins=2000, never=True)
    bp.run()
    assert bp.status()[1] == [lr.LR_OK]
    # defaults again: the spread batch, rerun from fresh inputs, equals a fresh batch
    b.wait_limits()
    its[0]["B"].copy_(lr.to_device(B0))
    b.run()
    assert b.status()[0] == lr.LR_OK
    its2 = items()
    b2 = lr.Batch(its2)
    b2.run()
    assert b2.status()[0] == lr.LR_OK
    assert np.array_equal(lr.from_device(its[0]["B"]), lr.from_device(its2[0]["B"]))
    b.close()
    b2.close()
    bp.close()


def test_split_wait_expiry_reports_timeout_and_recovers(lr):
    """Layer-split packed trajectories (fixed-step and adaptive) have group barriers: with expiring waits
    every part's kernel ends and the trajectory reports LR_ERR_TIMEOUT; with the defaults restored the
    same batch completes and equals a fresh one bitwise."""
    import torch
    m, p, B0 = _case()

    def items():
        return [dict(model=m, M=4, pulse=p, dt=1e-3, nsteps=60, B=lr.to_device(B0))]

    for adaptive in (None, (1e-8, 1e-11)):
        its = items()
        b = lr.Batch(its, packed=True, parts=4, adaptive=adaptive, stream=torch.cuda.current_stream())
        b.wait_limits(spins=2000, never=True)
        b.run()
        rc, codes, steps = b.status()
        print(f"[failure] split batch (adaptive {adaptive}) with expiring waits: codes {codes}, steps {steps}")
        assert codes == [lr.LR_ERR_TIMEOUT]
        b.wait_limits()
        its[0]["B"].copy_(lr.to_device(B0))
        b.run()
        assert b.status()[0] == lr.LR_OK
        its2 = items()
        b2 = lr.Batch(its2, packed=True, parts=4, adaptive=adaptive)
        b2.run()
        assert b2.status()[0] == lr.LR_OK
        assert np.array_equal(lr.from_device(its[0]["B"]), lr.from_device(its2[0]["B"]))
        b.close()
        b2.close()
