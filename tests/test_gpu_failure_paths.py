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
    """A batch with a spread trajectory (FP32, which the packed kernel does not take) and a packed one:
    with expiring waits the spread trajectory reports LR_ERR_TIMEOUT and the packed one (no group
    barriers) is unaffected; with the defaults restored both complete."""
    import torch
    m, p, B0 = _case()

    def items():
        return [dict(model=m, M=4, pulse=p, dt=1e-3, nsteps=60, B=lr.to_device(B0), precision=1),
                dict(model=m, M=4, pulse=p, dt=1e-3, nsteps=60, B=lr.to_device(B0))]

    its = items()
    b = lr.Batch(its, packed=True, stream=torch.cuda.current_stream())
    b.wait_limits(spins=2000, never=True)
    b.run()
    rc, codes, steps = b.status()
    print(f"[failure] batch with expiring waits: codes {codes}, steps {steps}")
    assert codes == [lr.LR_ERR_TIMEOUT, lr.LR_OK]
    packed_B = lr.from_device(its[1]["B"])
    b.wait_limits()
    its2 = items()
    b2 = lr.Batch(its2, packed=True)
    b2.run()
    assert b2.status()[0] == lr.LR_OK
    assert np.array_equal(packed_B, lr.from_device(its2[1]["B"]))
    # the first batch, rerun from fresh inputs with the defaults, completes and equals the second
    for it, B in zip(its, (B0, B0)):
        it["B"].copy_(lr.to_device(B))
    b.run()
    assert b.status()[0] == lr.LR_OK
    for x, y in zip(its, its2):
        assert np.array_equal(lr.from_device(x["B"]), lr.from_device(y["B"]))
    b.close()
    b2.close()
