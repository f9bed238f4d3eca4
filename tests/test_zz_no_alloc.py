"""lr_integrate_noalloc (the integration for callers that cannot allocate) against lr_integrate.

Both run the same kernels, so the state and the records must agree bitwise; two calls in a row (the
second on a smaller problem) check that the fixed workspace is re-initialised by every call.
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


def _with_context(lr, tr, nsteps, stride):
    ctx = lr.Context(tr.model, tr.M)
    Bd = lr.to_device(tr.B0())
    obs = ctx.new_obs(nsteps, stride)
    ctx.integrate(tr.pulse, 0.0, tr.dt, nsteps, Bd, stride, obs)
    assert ctx.status()[0] == lr.LR_OK
    out = lr.from_device(Bd), obs.cpu().numpy()
    ctx.close()
    return out


def _noalloc(lr, model, M, pulse, dt, nsteps, B0, stride):
    import torch
    Bd = lr.to_device(B0)
    obs = torch.zeros((nsteps // stride + 1, 6 + model.d_q), dtype=torch.float64, device="cuda")
    st = torch.full((2,), 7, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    rc = lr.lr_integrate_noalloc(model, M, 0, pulse, 0.0, dt, nsteps, Bd.data_ptr(), stride, obs.data_ptr(),
                                 st.data_ptr(), stream.cuda_stream)
    assert rc == lr.LR_OK, lr.lr_strerror(rc)
    stream.synchronize()
    return lr.from_device(Bd), obs.cpu().numpy(), st.cpu().tolist()


def test_noalloc_equals_integrate_two_calls(lr):
    """Paper size (N = 2000, M = 20), then the small readout case (N = 200, M = 4): bitwise equal to
    lr_integrate on a bound context, device status {LR_OK, -1}."""
    cases = [(I.config_paper_size()[0], 300, 50), (I.config_small()[1], 500, 100)]
    for tr, n, stride in cases:
        B_ref, obs_ref = _with_context(lr, tr, n, stride)
        B, obs, st = _noalloc(lr, tr.model, tr.M, tr.pulse, tr.dt, n, tr.B0(), stride)
        print(f"[noalloc] dims {tr.model.d_q, tr.model.d_r, tr.model.d_f} M={tr.M} {n} steps: status {st}, "
              f"max |dB| vs lr_integrate {np.max(np.abs(B - B_ref)):.1e}")
        assert st == [lr.LR_OK, -1]
        assert np.array_equal(B, B_ref)
        assert np.array_equal(obs, obs_ref)


def test_noalloc_reports_device_errors_and_limits(lr):
    """A rank-deficient state stops with GRAM_NOT_PD at step 0 through the status output; a shape whose
    workspace exceeds the fixed array is refused on the host (LR_ERR_OOM, nothing enqueued)."""
    import torch
    m = I.readout_model(2, 3, 2)
    p = I.flattop_pulse(0.05, 1.0)
    B0 = I.initial_state(m, 3, "g", seed=3, scale=1e-3)
    B0[:, 1] = 0.0
    _, _, st = _noalloc(lr, m, 3, p, 1e-3, 5, B0, 5)
    assert st == [lr.LR_ERR_GRAM_NOT_PD, 0]
    big = I.readout_model(8, 300, 5)  # N = 12000, M = 32: about 46 MiB of workspace
    Bd = torch.zeros((32, big.N), dtype=torch.complex128, device="cuda")
    rc = lr.lr_integrate_noalloc(big, 32, 0, p, 0.0, 1e-3, 1, Bd.data_ptr(), 0, 0, 0,
                                 torch.cuda.current_stream().cuda_stream)
    assert rc == lr.LR_ERR_OOM
    assert lr.lr_integrate_noalloc(m, 3, 0, p, 0.0, -1.0, 1, Bd.data_ptr(), 0, 0, 0, 0) == lr.LR_ERR_ARG
