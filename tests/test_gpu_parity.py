"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Trajectory tolerances are 100 times the oracle's own rounding floor: the
largest difference between two oracle runs that differ only in the order of
the row sums of the Gram / cross products and observables (both equally
valid FP64 results), never looser than the FP64 parity contract's bounds
  <a>, <f>          |d|    <= 1e-8 * max(1, max|<a>|, max|<f>|)
  P_q               |d|    <= 1e-10
  tr rho, tr rho^2  |d|    <= 1e-10
  SNR               relative 1e-8
and never tighter than 100 ulps.  The floor of a cached full-length workload
is measured once (tests/golden/oracle_floor.py -> oracle_floor.json); for a
short run the test reruns the oracle in reversed row order itself.
Right-hand side:  |d dB| <= 1e-11 * max|dB| (normwise over the factor).
The measured errors are printed beside their bounds.
"""
import json
import os

import numpy as np
import pytest

from oracle import loss, lowrank
from oracle import pulses as opulses
from paper_2508_18114_amd import inputs as I

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def lr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_18114_amd import lr as _lr
    return _lr


def _rand_B(N, M, seed, scales=None):
    r = np.random.default_rng(seed)
    B = r.standard_normal((N, M)) + 1j * r.standard_normal((N, M))
    if scales is not None:
        B = B * np.asarray(scales)[None, :]
    return B


def _gpu_rhs(lr, model, M, pulse, t, B):
    import torch
    ctx = lr.Context(model, M)
    dB = torch.empty((M, model.N), dtype=torch.complex128, device="cuda")
    ctx.rhs(pulse, t, lr.to_device(B), dB)
    rc, _ = ctx.status()
    assert rc == lr.LR_OK, lr.lr_strerror(rc)
    return lr.from_device(dB)


def _gpu_integrate(lr, model, M, pulse, dt, nsteps, B0, stride, t0=0.0):
    ctx = lr.Context(model, M)
    Bd = lr.to_device(B0)
    obs = ctx.new_obs(nsteps, stride)
    ctx.integrate(pulse, t0, dt, nsteps, Bd, stride, obs)
    rc, fs = ctx.status()
    assert rc == lr.LR_OK, (lr.lr_strerror(rc), fs)
    return lr.from_device(Bd), obs.cpu().numpy()


# upper bounds of the FP64 parity contract (field relative to max(1, |field|); the others absolute)
BOUNDS = dict(field=1e-8, pop=1e-10, trace=1e-10, snr_rel=1e-8)
EPS = np.finfo(np.float64).eps


def _obs_errors(got, ref):
    fa = max(1.0, np.max(np.abs(ref[:, 0:4])))
    return dict(field=float(np.max(np.abs(got[:, 0:4] - ref[:, 0:4]))) / fa,
                trace=float(np.max(np.abs(got[:, 4:6] - ref[:, 4:6]))),
                pop=float(np.max(np.abs(got[:, 6:] - ref[:, 6:]))))


def floor_tol(floor):
    """100 x an oracle rounding floor, within [100 ulps, the contract's bounds]."""
    return {k: min(BOUNDS[k], 100.0 * max(float(floor.get(k, 0.0)), EPS)) for k in BOUNDS}


def _golden_tol(name):
    """Tolerances of a cached workload from its measured oracle floor."""
    path = os.path.join(HERE, "golden", "oracle_floor.json")
    floors = json.load(open(path)) if os.path.exists(path) else {}
    if name not in floors:
        pytest.skip(f"no oracle floor measured for {name} (tests/golden/oracle_floor.py)")
    return floor_tol(floors[name]["floor"])


def oracle_with_tol(model, pulse, t0, dt, nsteps, B0, stride):
    """Oracle run in the reference order and the tolerances from a second run in reversed row order."""
    B, ref = lowrank.integrate(model, pulse, t0, dt, nsteps, B0, obs_stride=stride)
    if stride <= 0:  # no records to compare
        return B, ref, dict(BOUNDS)
    _, alt = lowrank.integrate(model, pulse, t0, dt, nsteps, B0, obs_stride=stride, sum_order="reversed")
    return B, ref, floor_tol(_obs_errors(alt, ref))


def _assert_obs(got, ref, what, tol=None):
    """Records against reference records; tol: per-quantity bounds (default: the contract's)."""
    tol = BOUNDS if tol is None else tol
    assert got.shape == ref.shape, (got.shape, ref.shape)
    e = _obs_errors(got, ref)
    print(f"[parity] {what}: field err {e['field']:.3e} (tol {tol['field']:.1e}), populations err "
          f"{e['pop']:.3e} (tol {tol['pop']:.1e}), traces err {e['trace']:.3e} (tol {tol['trace']:.1e})")
    for k in ("field", "pop", "trace"):
        assert e[k] <= tol[k], (k, e[k], tol[k])


# ------------------------------------------------------------ right-hand side

@pytest.mark.parametrize("dims,M", [((3, 4, 3), 3), ((2, 5, 3), 1), ((2, 2, 2), 8), ((4, 10, 5), 4),
                                    ((8, 50, 5), 20), ((8, 75, 5), 32), ((8, 13, 5), 7)])
def test_rhs_matches_oracle(lr, dims, M):
    m = I.readout_model(*dims).replace(kappa_f=0.7, gamma_1=0.3)
    p = I.flattop_pulse(0.09, 6.0)
    B = _rand_B(m.N, M, 1, scales=np.logspace(0, -3, M))
    for t in (0.0, 1.3, 3.7):
        ref = lowrank.rhs(m, p, t, B)
        got = _gpu_rhs(lr, m, M, p, t, B)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"[parity] rhs dims={dims} M={M} t={t}: rel err {err:.3e}")
        assert err <= 1e-11


def test_rhs_padded_initial_state(lr):
    """The rank-padded B0 (columns of norm 1e-6) of the paper-size workload."""
    tr = I.config_paper_size()[1]
    B0 = tr.B0()
    for t in (0.0, 5.0, 20.0):
        ref = lowrank.rhs(tr.model, tr.pulse, t, B0)
        got = _gpu_rhs(lr, tr.model, tr.M, tr.pulse, t, B0)
        colref = np.linalg.norm(ref, axis=0)
        colerr = np.linalg.norm(got - ref, axis=0)
        err = np.max(colerr / np.maximum(colref, 1e-300))
        print(f"[parity] rhs padded B0 t={t}: max column rel err {err:.3e}")
        assert err <= 1e-9


def test_rhs_piecewise_pulse(lr):
    m = I.readout_model(3, 6, 4)
    p = I.draw_piecewise6(I.rng(3), 12.0)
    B = _rand_B(m.N, 5, 2)
    for t in (0.7, 5.9, 6.0, 6.3, 11.5):
        ref = lowrank.rhs(m, p, t, B)
        got = _gpu_rhs(lr, m, 5, p, t, B)
        assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))


# ------------------------------------------------------------ observables

def test_observables_match_oracle(lr):
    import torch
    for dims, M in [((4, 10, 5), 4), ((8, 50, 5), 20), ((3, 1, 2), 2)]:
        m = I.readout_model(*dims)
        B = _rand_B(m.N, M, 4)
        ctx = lr.Context(m, M)
        out = torch.zeros(lr.obs_len(m), dtype=torch.float64, device="cuda")
        ctx.observables(lr.to_device(B), out)
        assert ctx.status()[0] == lr.LR_OK
        ref = lowrank.observables(m, B)
        got = out.cpu().numpy()
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))


# ------------------------------------------------------------ integration

def test_integrate_short_ragged(lr):
    """Several tiles, ragged observation stride, piecewise drive, mixed column scales."""
    m = I.readout_model(3, 7, 4).replace(kappa_f=0.5, gamma_1=0.05)
    p = I.draw_piecewise6(I.rng(5), 0.6)
    B0 = _rand_B(m.N, 5, 6, scales=[1.0, 0.3, 0.1, 0.05, 0.01])
    B0 /= np.linalg.norm(B0)
    dt, n, stride = 1e-3, 203, 7
    Bo, ref, tol = oracle_with_tol(m, p, 0.0, dt, n, B0, stride)
    Bg, got = _gpu_integrate(lr, m, 5, p, dt, n, B0, stride)
    _assert_obs(got, ref, "short ragged", tol)
    assert np.max(np.abs(Bg - Bo)) <= 1e-10


def test_integrate_nonzero_t0(lr):
    m = I.readout_model(2, 5, 3)
    p = I.flattop_pulse(0.1, 3.0, t_ramp=1.0)
    B0 = I.initial_state(m, 3, "e", seed=7, scale=1e-3)
    Bo, ref, tol = oracle_with_tol(m, p, 0.8, 1e-3, 300, B0, 50)
    Bg, got = _gpu_integrate(lr, m, 3, p, 1e-3, 300, B0, 50, t0=0.8)
    _assert_obs(got, ref, "t0 = 0.8", tol)


def _golden(name):
    path = os.path.join(HERE, "golden", f"config_{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return np.load(path)


def _check_config(lr, name, trajs):
    gd = _golden(name)
    tol = _golden_tol(name)
    stride = int(gd["stride"])
    obs = {}
    for tr, key in zip(trajs, ("obs_g", "obs_e")):
        _, got = _gpu_integrate(lr, tr.model, tr.M, tr.pulse, tr.dt, tr.nsteps, tr.B0(), stride)
        _assert_obs(got, gd[key], f"{name} {tr.which}", tol)
        obs[key] = got
    tr = trajs[0]
    # figures of merit of the GPU series, computed on the device
    import torch
    fm = lr.readout_loss(torch.from_numpy(obs["obs_g"]).cuda(), torch.from_numpy(obs["obs_e"]).cuda(), tr.model.d_q,
                         stride * tr.dt, tr.model.kappa_f, tr.model.gamma_1)
    snr_ref = float(gd["snr"])
    d = abs(fm["snr"] - snr_ref)
    print(f"[parity] {name} SNR gpu {fm['snr']:.12e} oracle {snr_ref:.12e} (rel {d / snr_ref:.2e}, tol "
          f"{tol['snr_rel']:.1e}) eps_sep {fm['eps_sep']:.6e} loss {fm['loss']:.9f} vs {float(gd['loss']):.9f}")
    assert d <= tol["snr_rel"] * snr_ref
    # eps_sep = erfc(SNR / 2) / 2 has slope <= 1 / (2 sqrt(pi)) in SNR
    assert abs(fm["eps_sep"] - float(gd["eps_sep"])) <= 0.3 * d + 1e-15
    assert abs(fm["eps_decay"] - float(gd["eps_decay"])) <= 1e-15
    # T averages P_q(k >= 2) over time for g and e: |d T| <= 2 d_q max |d P_q|
    dT = 2 * tr.model.d_q * tol["pop"]
    assert abs(fm["ionisation"] - float(gd["ionisation"])) <= dT
    # Lambda = log10(eps_a + T): |d Lambda| <= (|d eps_sep| + |d T|) / (ln 10 (eps_a + T))
    assert abs(fm["loss"] - float(gd["loss"])) <= (0.3 * d + dT) / (np.log(10) * (fm["eps_a"] + fm["ionisation"])) + 1e-14


def test_readout_loss_matches_oracle_on_same_series(lr):
    """Device figures of merit (S3.A-B) on the cached oracle series equal the oracle's own, up to
    summation order."""
    import torch
    for name, trajs in (("small", I.config_small()), ("paper_size", I.config_paper_size())):
        gd = _golden(name)
        tr = trajs[0]
        h = int(gd["stride"]) * tr.dt
        ref = loss.readout_loss(gd["obs_g"], gd["obs_e"], h, tr.model.kappa_f, tr.model.gamma_1)
        got = lr.readout_loss(torch.from_numpy(gd["obs_g"]).cuda(), torch.from_numpy(gd["obs_e"]).cuda(),
                              tr.model.d_q, h, tr.model.kappa_f, tr.model.gamma_1)
        for k in lr.LOSS_KEYS:
            print(f"[parity] loss {name} {k}: gpu {got[k]:.15e} oracle {ref[k]:.15e}")
            assert abs(got[k] - ref[k]) <= 1e-12 * max(1.0, abs(ref[k])), k
    # argument checks
    o = torch.zeros((1, 6 + 4), dtype=torch.float64, device="cuda")
    with pytest.raises(lr.LrError):
        lr.readout_loss(o, o, 4, 0.1, 0.1, 1e-5)


def test_integrate_config_small(lr):
    """dims (4,10,5), M = 4, 1e4 RK4 steps of 1e-3 ns, g and e, against the cached oracle run."""
    _check_config(lr, "small", I.config_small())


def test_integrate_config_paper_size(lr):
    """dims (8,50,5) (N = 2000), M = 20, 8e4 RK4 steps of 5e-4 ns, g and e, against the cached oracle run."""
    _check_config(lr, "paper_size", I.config_paper_size())


# ------------------------------------------------------------ edge cases

def test_zero_steps_and_degenerate_shapes(lr):
    m = I.readout_model(2, 3, 2)
    B0 = _rand_B(m.N, 4, 8)
    p = I.flattop_pulse(0.05, 1.0)
    Bg, got = _gpu_integrate(lr, m, 4, p, 1e-3, 0, B0, 5)
    assert np.array_equal(Bg, B0)
    np.testing.assert_allclose(got[0], lowrank.observables(m, B0), rtol=1e-12)
    # M = N (full rank) and M = 1; a single resonator layer; stride > nsteps
    for dims, M in [((2, 3, 2), 12), ((2, 3, 2), 1), ((3, 1, 4), 3)]:
        mm = I.readout_model(*dims).replace(kappa_f=0.4, gamma_1=0.1)
        B0 = _rand_B(mm.N, M, 9)
        B0 /= np.linalg.norm(B0)
        Bo, ref, tol = oracle_with_tol(mm, p, 0.0, 1e-3, 40, B0, 50)
        Bg, got = _gpu_integrate(lr, mm, M, p, 1e-3, 40, B0, 50)
        _assert_obs(got, ref, f"dims {dims} M {M}", tol)
        assert np.max(np.abs(Bg - Bo)) <= 1e-12


def test_device_errors_are_reported(lr):
    m = I.readout_model(2, 3, 2)
    p = I.flattop_pulse(0.05, 1.0)
    B0 = _rand_B(m.N, 3, 10)
    B0[:, 1] = 0.0
    ctx = lr.Context(m, 3)
    Bd = lr.to_device(B0)
    ctx.integrate(p, 0.0, 1e-3, 5, Bd, 0, None)
    rc, fs = ctx.status()
    assert rc == lr.LR_ERR_GRAM_NOT_PD and fs == 0
    B1 = _rand_B(m.N, 3, 11)
    B1[4, 2] = np.nan
    ctx.integrate(p, 0.0, 1e-3, 5, lr.to_device(B1), 0, None)
    rc, fs = ctx.status()
    assert rc == lr.LR_ERR_NONFINITE and fs == 0
    # the context is usable again afterwards
    B2 = _rand_B(m.N, 3, 12)
    ctx.integrate(p, 0.0, 1e-3, 5, lr.to_device(B2), 0, None)
    assert ctx.status()[0] == lr.LR_OK
    # argument errors are synchronous
    bad = I.flattop_pulse(0.5, 1.0)   # 0.5 GHz > 0.4 GHz bound
    assert lr.lr_integrate(ctx.handle, bad, 0.0, 1e-3, 5, lr.to_device(B2).data_ptr(), 0, 0) == lr.LR_ERR_PULSE
    assert lr.lr_integrate(ctx.handle, p, 0.0, 0.0, 5, lr.to_device(B2).data_ptr(), 0, 0) == lr.LR_ERR_ARG


def test_deterministic_replay(lr):
    """Same inputs twice: bitwise-equal state and records (fixed reduction order)."""
    tr = I.config_small()[1]
    a = _gpu_integrate(lr, tr.model, tr.M, tr.pulse, tr.dt, 500, tr.B0(), 10)
    b = _gpu_integrate(lr, tr.model, tr.M, tr.pulse, tr.dt, 500, tr.B0(), 10)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ------------------------------------------------------------ batches

def _batch_items(lr, specs):
    items = []
    for (dims, M, which, nsteps, stride, pseed) in specs:
        m = I.readout_model(*dims).replace(kappa_f=0.5, gamma_1=0.02)
        p = I.draw_piecewise6(I.rng(pseed), nsteps * 1e-3)
        B0 = I.initial_state(m, M, which, seed=pseed, scale=1e-3)
        it = dict(model=m, M=M, pulse=p, dt=1e-3, nsteps=nsteps, B0=B0, B=lr.to_device(B0),
                  obs_stride=stride)
        if stride:
            import torch
            it["obs"] = torch.zeros((nsteps // stride + 1, 6 + dims[0]), dtype=torch.float64, device="cuda")
        items.append(it)
    return items


BATCH_SPECS = [((4, 10, 5), 4, "g", 120, 10, 1), ((3, 7, 4), 6, "e", 97, 0, 2), ((8, 13, 5), 20, "e", 60, 20, 3),
               ((2, 5, 3), 1, "g", 150, 25, 4), ((4, 10, 5), 4, "e", 120, 10, 5)]


def test_batch_equals_single_runs_bitwise(lr):
    """Trajectories of different shapes, lengths and strides in one batch give
    bitwise the states and records of the same trajectories run alone."""
    items = _batch_items(lr, BATCH_SPECS)
    b = lr.Batch(items)
    b.run()
    rc, codes, _ = b.status()
    assert rc == lr.LR_OK, codes
    for it in items:
        ctx = lr.Context(it["model"], it["M"])
        Bd = lr.to_device(it["B0"])
        obs = ctx.new_obs(it["nsteps"], it["obs_stride"]) if it["obs_stride"] else None
        ctx.integrate(it["pulse"], 0.0, it["dt"], it["nsteps"], Bd, it["obs_stride"], obs)
        assert ctx.status()[0] == lr.LR_OK
        assert np.array_equal(lr.from_device(Bd), lr.from_device(it["B"]))
        if obs is not None:
            assert np.array_equal(obs.cpu().numpy(), it["obs"].cpu().numpy())


def test_batch_matches_oracle(lr):
    items = _batch_items(lr, BATCH_SPECS[:3])
    b = lr.Batch(items)
    b.run()
    assert b.status()[0] == lr.LR_OK
    for it in items:
        Bo, ref, tol = oracle_with_tol(it["model"], it["pulse"], 0.0, it["dt"], it["nsteps"], it["B0"],
                                       it["obs_stride"])
        got_B = lr.from_device(it["B"])
        assert np.max(np.abs(got_B - Bo)) <= 1e-12
        if it["obs_stride"]:
            _assert_obs(it["obs"].cpu().numpy(), ref, f"batch dims {it['model'].d_q, it['model'].d_r}", tol)


@pytest.mark.parametrize("dims,M", [((8, 75, 5), 32), ((8, 38, 5), 24), ((8, 9, 6), 22)])
def test_spread_largest_shapes_match_oracle(lr, dims, M):
    """The spread schedule at the largest shape of the batched workload (N = 3000, M = 32: three
    register rows, two solve entries per thread) and at the other two variants (M = 24: two rows, two
    entries; 48-row layers at M = 22: three rows, one entry), integrated against the oracle."""
    m = I.readout_model(*dims).replace(kappa_f=0.5, gamma_1=0.02)
    nsteps, stride, dt = 40, 10, 5e-4
    p = I.draw_piecewise6(I.rng(17), nsteps * dt)
    B0 = I.initial_state(m, M, "e", seed=17, scale=1e-3)
    import torch
    it = dict(model=m, M=M, pulse=p, dt=dt, nsteps=nsteps, B=lr.to_device(B0), obs_stride=stride,
              obs=torch.zeros((nsteps // stride + 1, 6 + dims[0]), dtype=torch.float64, device="cuda"))
    print(f"[parity] spread dims={dims} M={M}", flush=True)
    b = lr.Batch([it])
    b.run()
    assert b.status()[0] == lr.LR_OK
    Bo, ref, tol = oracle_with_tol(m, p, 0.0, dt, nsteps, B0, stride)
    err = np.max(np.abs(lr.from_device(it["B"]) - Bo))
    print(f"[parity] spread dims={dims} M={M}: max |dB| {err:.3e} (tol 1e-12)")
    assert err <= 1e-12
    _assert_obs(it["obs"].cpu().numpy(), ref, f"spread dims {dims} M={M}", tol)


# ------------------------------------------------------------ dense comparison solve

def _dense_case(seed):
    model = I.readout_model(3, 4, 3)
    pulse = I.flattop_pulse(0.08, 2.0, t_ramp=0.5)
    r = np.random.default_rng(seed)
    N = model.N
    # mixed, full-rank rho0 = V V^ / tr with the excited state dominant
    V = 0.05 * (r.standard_normal((N, N)) + 1j * r.standard_normal((N, N)))
    V[I.basis_index(model, 1, 0, 0), 0] += 1.0
    rho0 = V @ V.conj().T
    rho0 = 0.5 * (rho0 + rho0.conj().T)
    return model, pulse, rho0 / np.trace(rho0).real


def test_dense_lindblad_matches_oracle(lr):
    """Dense full-Lindblad RK4 on the device vs the oracle's dense master equation (same stage times)."""
    import torch
    from oracle import dense
    model, pulse, rho0 = _dense_case(11)
    dt, nsteps, stride = 2e-3, 300, 100
    rho = torch.from_numpy(rho0.copy()).cuda()
    obs = torch.zeros((nsteps // stride + 1, 6 + model.d_q), dtype=torch.float64, device="cuda")
    lr.dense_integrate(model, pulse, 0.0, dt, nsteps, rho, stride, obs)
    torch.cuda.synchronize()
    ref_rho, ref_obs = dense.integrate(model, pulse, 0.0, dt, nsteps, rho0, obs_stride=stride)
    got = rho.cpu().numpy()
    err = np.max(np.abs(got - ref_rho))
    print(f"[parity] dense rho err {err:.3e}")
    assert err <= 1e-12
    assert np.array_equal(got, got.conj().T)  # exactly Hermitian
    e = _obs_errors(obs.cpu().numpy(), ref_obs)
    print(f"[parity] dense obs: field err {e['field']:.3e}, populations err {e['pop']:.3e}, traces err {e['trace']:.3e}")
    assert e["field"] <= 1e-12 and e["pop"] <= 1e-12 and e["trace"] <= 1e-12


def test_dense_lindblad_edge_cases(lr):
    import torch
    model, pulse, rho0 = _dense_case(12)
    rho = torch.from_numpy(rho0.copy()).cuda()
    lr.dense_integrate(model, pulse, 0.0, 1e-3, 0, rho)  # zero steps: unchanged
    torch.cuda.synchronize()
    assert np.array_equal(rho.cpu().numpy(), rho0)
    with pytest.raises(lr.LrError):
        lr.dense_integrate(model, pulse, 0.0, -1e-3, 5, rho)
    with pytest.raises(lr.LrError):
        lr.dense_integrate(model, pulse, 0.0, 1e-3, 5, rho, obs_stride=2, obs=None)


# ------------------------------------------------------------ reduced-precision modes

def _mixed_errors(lr, name, trajs, precision, packed=False):
    """Integrate g and e in one batch at the given precision (spread or packed schedule); errors of the
    record vs the FP64 oracle."""
    import torch
    gd = _golden(name)
    stride = int(gd["stride"])
    items = []
    for tr in trajs:
        nrec = tr.nsteps // stride + 1
        items.append(dict(model=tr.model, M=tr.M, pulse=tr.pulse, dt=tr.dt, nsteps=tr.nsteps,
                          B=lr.to_device(tr.B0()), obs_stride=stride, precision=precision,
                          obs=torch.zeros((nrec, 6 + tr.model.d_q), dtype=torch.float64, device="cuda")))
    b = lr.Batch(items, packed=packed)
    b.run()
    rc, codes, steps = b.status()
    assert rc == lr.LR_OK, (lr.lr_strerror(rc), codes, steps)
    tr = trajs[0]
    og, oe = items[0]["obs"], items[1]["obs"]
    fm = lr.readout_loss(og, oe, tr.model.d_q, stride * tr.dt, tr.model.kappa_f, tr.model.gamma_1)
    out = {}
    for key, it in (("g", items[0]), ("e", items[1])):
        got, ref = it["obs"].cpu().numpy(), gd["obs_" + key]
        out["field_" + key] = float(np.max(np.abs(got[:, 0:4] - ref[:, 0:4])))
        out["pop_" + key] = float(np.max(np.abs(got[:, 6:] - ref[:, 6:])))
        out["trace_" + key] = float(np.max(np.abs(got[:, 4] - ref[:, 4])))
    out["snr_rel"] = abs(fm["snr"] - float(gd["snr"])) / float(gd["snr"])
    out["eps_sep"] = abs(fm["eps_sep"] - float(gd["eps_sep"]))
    return out


def test_integrate_paper_padding_fp64(lr):
    """FP64 parity at the paper's padding weight p_j = 1e-5 (the reference for the reduced modes)."""
    _check_config(lr, "small_paper_padding", I.config_small_paper_padding())
    _check_config(lr, "paper_size_paper_padding", I.config_paper_size_paper_padding())


# sanity bounds of the reduced modes against the FP64 oracle at the paper's padding
# (measured: FP32 field 7e-6, populations 2e-6; BF16x3 field 1.5e-4, populations 2e-5)
MIXED_BOUNDS = {1: dict(field=1e-4, pop=2e-5, snr_rel=1e-3), 2: dict(field=1e-3, pop=2e-4, snr_rel=1e-2)}


@pytest.mark.parametrize("precision", [1, 2], ids=["fp32", "bf16x3"])
def test_reduced_precision_errors(lr, precision):
    """Reduced-precision operator/Gram arithmetic (FP64 solve and accumulation) at the paper's padding
    weight: max abs error of <a>, <f>, transmon populations and the g/e separation against the FP64
    oracle, reported and held to sanity bounds."""
    bnd = MIXED_BOUNDS[precision]
    for name, trajs in (("small_paper_padding", I.config_small_paper_padding()),
                        ("paper_size_paper_padding", I.config_paper_size_paper_padding())):
        e = _mixed_errors(lr, name, trajs, precision)
        print(f"[mixed] {name} precision {precision}: " + ", ".join(f"{k} {v:.3e}" for k, v in e.items()))
        for k, v in e.items():
            assert np.isfinite(v), k
        assert max(e["field_g"], e["field_e"]) <= bnd["field"]
        assert max(e["pop_g"], e["pop_e"]) <= bnd["pop"]
        assert e["snr_rel"] <= bnd["snr_rel"]


@pytest.mark.parametrize("precision", [1, 2], ids=["fp32", "bf16x3"])
def test_packed_reduced_precision_errors(lr, precision):
    """The packed schedule's reduced modes (Gram and cross products on the matrix cores: FP32 MFMA, or
    three BF16 part products with FP32 accumulation for C_k and FP64 for G; stencil, assembly, solve and
    RK4 in FP64) at the paper's padding weight, against the FP64 oracle: every observable's error reported
    and held to the bounds of the reduced modes.  The small workload runs whole (1e4 steps, with the
    figures of merit); the paper-size one for its first 6000 steps (one workgroup per trajectory is the
    throughput schedule, not the latency one)."""
    import torch
    bnd = MIXED_BOUNDS[precision]
    e = _mixed_errors(lr, "small_paper_padding", I.config_small_paper_padding(), precision, packed=True)
    print(f"[mixed packed] small_paper_padding precision {precision}: " +
          ", ".join(f"{k} {v:.3e}" for k, v in e.items()))
    for k, v in e.items():
        assert np.isfinite(v), k
    assert max(e["field_g"], e["field_e"]) <= bnd["field"]
    assert max(e["pop_g"], e["pop_e"]) <= bnd["pop"]
    assert e["snr_rel"] <= bnd["snr_rel"]
    trajs = I.config_paper_size_paper_padding()
    gd = _golden("paper_size_paper_padding")
    stride, n = int(gd["stride"]), 6000
    items = [dict(model=t.model, M=t.M, pulse=t.pulse, dt=t.dt, nsteps=n, B=lr.to_device(t.B0()), precision=precision,
                  obs_stride=stride, obs=torch.zeros((n // stride + 1, 6 + t.model.d_q), dtype=torch.float64,
                                                     device="cuda"))
             for t in trajs]
    rc, codes, _ = _run_packed(lr, items)
    assert rc == lr.LR_OK, codes
    for it, key in zip(items, ("obs_g", "obs_e")):
        err = _obs_errors(it["obs"].cpu().numpy(), gd[key][:n // stride + 1])
        print(f"[mixed packed] paper_size_paper_padding (3 ns) {key} precision {precision}: "
              + ", ".join(f"{k} {v:.3e}" for k, v in err.items()))
        assert err["field"] <= bnd["field"] and err["pop"] <= bnd["pop"], err


def test_reduced_precision_needs_padding_above_rounding(lr):
    """With the 1e-6 padding of the paper-size workload, FP32 products cannot resolve G (its smallest
    eigenvalues are 1e-12 of its largest): the integrator must either stop with GRAM_NOT_PD at a reported
    step, or -- if it runs through -- agree with the FP64 oracle run to the FP32 bounds.  What it may not
    do is finish with silently wrong records."""
    import torch
    trajs = I.config_paper_size()
    gd = _golden("paper_size")
    stride, n = int(gd["stride"]), 6000
    items = [dict(model=t.model, M=t.M, pulse=t.pulse, dt=t.dt, nsteps=n, B=lr.to_device(t.B0()), precision=1,
                  obs_stride=stride, obs=torch.zeros((n // stride + 1, 6 + t.model.d_q), dtype=torch.float64,
                                                     device="cuda"))
             for t in trajs]
    b = lr.Batch(items)
    b.run()
    rc, codes, steps = b.status()
    print(f"[mixed] padding 1e-6, FP32: codes {codes}, steps {steps}")
    bnd = MIXED_BOUNDS[1]
    for it, key, code, step in zip(items, ("obs_g", "obs_e"), codes, steps):
        if code == lr.LR_ERR_GRAM_NOT_PD:
            assert 0 <= step < n
        else:
            assert code == lr.LR_OK
            e = _obs_errors(it["obs"].cpu().numpy(), gd[key][:n // stride + 1])
            assert e["field"] <= bnd["field"] and e["pop"] <= bnd["pop"], e
    b.close()


# ------------------------------------------------------------ serving (continuous batching)

def _serving_reqs():
    from paper_2508_18114_amd import serve
    reqs = []
    shapes = [(13, 6, 1), (20, 8, 0), (13, 4, 0), (16, 12, 1)]  # d_r, M, precision
    for k, (d_r, M, prec) in enumerate(shapes):
        m = I.readout_model(8, d_r, 5)
        nsteps = 1400 + 200 * k
        pulse = serve.pulse_from(np.array([0.3 + 0.05 * k, 0.4, 0.01, 0.5, 1.0 + k, -0.02]), nsteps * 5e-4)
        reqs.append(serve.Request(rid=k, model=m, M=M, pulse=pulse, dt=5e-4, nsteps=nsteps, precision=prec,
                                  obs_stride=200, seed=77 + k, arrival=0.0))
    return reqs


def test_serving_result_alone_equals_mix(lr):
    """Spread-schedule serving: a request served alone, and in a mix with others that arrive later and
    run with a different tick length, gives bitwise the same state, observation series and loss; a
    continued run equals one call."""
    import copy
    import torch
    from paper_2508_18114_amd import serve
    reqs = _serving_reqs()
    alone = serve.Server(hbm_budget_bytes=1 << 34, chunk=1000, packed=False)
    st1 = alone.run([copy.deepcopy(reqs[0])])
    r_alone = alone.results[0]
    assert st1["errors"] == 0 and st1["requests"] == 1
    mixed = [copy.deepcopy(r) for r in reqs]
    for k, r in enumerate(mixed):
        r.arrival = 0.0 if k < 2 else 0.01 * k
    mix = serve.Server(hbm_budget_bytes=1 << 34, chunk=600, packed=False)
    st2 = mix.run(mixed)
    assert st2["errors"] == 0 and st2["requests"] == len(reqs)
    r_mix = mix.results[0]
    for key in ("B_g", "B_e", "obs_g", "obs_e"):
        assert torch.equal(r_alone[key], r_mix[key]), key
    assert r_alone["loss"] == r_mix["loss"]
    # the same trajectories integrated in one call
    r = reqs[0]
    nrec = r.nsteps // r.obs_stride + 1
    items = [dict(model=r.model, M=r.M, pulse=r.pulse, dt=r.dt, nsteps=r.nsteps, precision=r.precision,
                  B=lr.to_device(I.initial_state(r.model, r.M, w, r.seed, r.pad_scale)), obs_stride=r.obs_stride,
                  obs=torch.zeros((nrec, 6 + r.model.d_q), dtype=torch.float64, device="cuda")) for w in ("g", "e")]
    b = lr.Batch(items)
    b.run()
    assert b.status()[0] == lr.LR_OK
    assert torch.equal(items[0]["B"], r_alone["B_g"]) and torch.equal(items[1]["obs"], r_alone["obs_e"])
    print(f"[serving] alone {st1}, mix {st2}")


def test_serving_packed_alone_equals_mix(lr):
    """Packed serving (the default, asynchronous ticks on two streams): request 1 (FP64) alone and in
    the mix (FP32 requests in their own packed launches, concurrent on a forked stream) gives bitwise
    the same result, and agrees with the spread server to the FP64 tolerances."""
    import copy
    import torch
    from paper_2508_18114_amd import serve
    reqs = _serving_reqs()
    assert reqs[1].precision == I.FP64
    alone = serve.Server(hbm_budget_bytes=1 << 34, chunk=1000, packed=True)
    st1 = alone.run([copy.deepcopy(reqs[1])])
    assert st1["errors"] == 0
    mixed = [copy.deepcopy(r) for r in reqs]
    for k, r in enumerate(mixed):
        r.arrival = 0.0 if k < 2 else 0.01 * k
    mix = serve.Server(hbm_budget_bytes=1 << 34, chunk=600, packed=True)
    st2 = mix.run(mixed)
    assert st2["errors"] == 0 and st2["requests"] == len(reqs)
    for key in ("B_g", "B_e", "obs_g", "obs_e"):
        assert torch.equal(alone.results[1][key], mix.results[1][key]), key
    spread = serve.Server(hbm_budget_bytes=1 << 34, chunk=1000, packed=False)
    assert spread.run([copy.deepcopy(reqs[1])])["errors"] == 0
    for key in ("obs_g", "obs_e"):
        _assert_obs(mix.results[1][key].cpu().numpy(), spread.results[1][key].cpu().numpy(), f"packed serving {key}")
    print(f"[serving] packed alone {st1}, packed mix {st2}")


def test_serving_admission_by_footprint(lr):
    """With an HBM budget that holds one request at a time, requests are served one after another and all
    complete; a budget below one request's footprint never admits it."""
    import copy
    from paper_2508_18114_amd import serve
    reqs = [copy.deepcopy(r) for r in _serving_reqs()[:2]]
    need = max(serve.Server(1)._need(r)[0] for r in reqs)
    s = serve.Server(hbm_budget_bytes=need, chunk=800)
    st = s.run(reqs)
    assert st["requests"] == 2 and st["errors"] == 0
    a, b = s.results[0], s.results[1]
    assert b["admitted"] >= a["done"] - 1e-9  # the second waited for the first to retire


def test_serving_rejects_request_above_budget(lr):
    import copy
    from paper_2508_18114_amd import serve
    r = copy.deepcopy(_serving_reqs()[0])
    s = serve.Server(hbm_budget_bytes=1024, chunk=800)
    st = s.run([r])
    assert st["requests"] == 0 and "error" in s.results[0]


# ------------------------------------------------------------ validity spectrum (S1.B)

def _gpu_spectrum(lr, model, M, B):
    ctx = lr.Context(model, M)
    p = ctx.spectrum(lr.to_device(B)).cpu().numpy()
    rc, _ = ctx.status()
    assert rc == lr.LR_OK, lr.lr_strerror(rc)
    return p


@pytest.mark.parametrize("M", [1, 4, 20, 32])
def test_spectrum_matches_oracle(lr, M):
    """lr_spectrum against the eigenvalues of B^ B: |d p_j| <= 1e-13 p_1 (both FP64; G is
    formed in a different summation order and each eigensolver is backward stable), for a
    well-conditioned factor and one padded like the initial state (columns 2..M at 1e-6)."""
    from oracle import validity
    m = I.readout_model(4, 10, 5)
    for seed, scales in ((31, None), (32, [1.0] + [1e-6] * (M - 1))):
        B = _rand_B(m.N, M, seed, scales)
        got = _gpu_spectrum(lr, m, M, B)
        ref = validity.spectrum(B)
        err = float(np.max(np.abs(got - ref)))
        print(f"[spectrum] M={M} seed={seed}: max |dp| / p_1 = {err / ref[0]:.2e}, "
              f"p_M/p_1 {got[-1] / got[0]:.6e} (oracle {ref[-1] / ref[0]:.6e})")
        assert err <= 1e-13 * ref[0]
        assert np.all(np.diff(got) <= 0)


def test_spectrum_of_integrated_paper_size_state(lr):
    """The spectrum of a state the GPU integrated (N=2000, M=20, 400 steps) against the oracle
    spectrum of the same factor, and sum p_j = tr rho, sum p_j^2 = tr rho^2 of lr_observables."""
    import torch
    from oracle import validity
    tr = I.config_paper_size()[1]
    B, _ = _gpu_integrate(lr, tr.model, tr.M, tr.pulse, tr.dt, 400, tr.B0(), 0)
    got = _gpu_spectrum(lr, tr.model, tr.M, B)
    ref = validity.spectrum(B)
    assert float(np.max(np.abs(got - ref))) <= 1e-13 * ref[0]
    ctx = lr.Context(tr.model, tr.M)
    obs = torch.zeros((lr.obs_len(tr.model),), dtype=torch.float64, device="cuda")
    ctx.observables(lr.to_device(B), obs)
    o = obs.cpu().numpy()
    assert float(np.sum(got)) == pytest.approx(o[4], rel=1e-12)
    assert float(np.sum(got ** 2)) == pytest.approx(o[5], rel=1e-11)


def test_spectrum_nonfinite_input_ends(lr):
    """A non-finite factor ends the Jacobi loop at once; the output is not finite."""
    m = I.readout_model(4, 10, 5)
    B = _rand_B(m.N, 4, 33)
    B[7, 2] = np.nan
    got = _gpu_spectrum(lr, m, 4, B)
    assert not np.all(np.isfinite(got))


# ------------------------------------------------------------ drive frame (S2.E)

def test_rhs_drive_frame_matches_oracle(lr):
    """lr_rhs in the frame rotating at w_d (counter-rotating terms kept) vs the oracle."""
    m = I.readout_model(3, 5, 4).replace(kappa_f=0.7, gamma_1=0.3)
    p = I.flattop_pulse(0.09, 6.0).replace(frame=I.FRAME_DRIVE)
    B = _rand_B(m.N, 4, 51, scales=np.logspace(0, -3, 4))
    for t in (0.0, 1.3, 3.7):
        ref = lowrank.rhs(m, p, t, B)
        got = _gpu_rhs(lr, m, 4, p, t, B)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"[parity] rhs drive frame t={t}: rel err {err:.3e}")
        assert err <= 1e-11


@pytest.mark.parametrize("kind", ["flattop", "piecewise6"])
def test_integrate_drive_frame_matches_oracle(lr, kind):
    """Persistent RK4 in the drive frame vs the oracle: several tiles, ragged stride, a
    rank-padded start; the records hold the rotating-frame <a>', <f>'."""
    m = I.readout_model(3, 7, 4).replace(kappa_f=0.5, gamma_1=0.05)
    p = (I.flattop_pulse(0.08, 0.5, t_ramp=0.1) if kind == "flattop"
         else I.draw_piecewise6(I.rng(5), 0.6)).replace(frame=I.FRAME_DRIVE)
    B0 = I.initial_state(m, 4, "e", seed=52, scale=1e-3)
    dt, n, stride = 1e-3, 203, 7
    Bo, ref, tol = oracle_with_tol(m, p, 0.0, dt, n, B0, stride)
    Bg, got = _gpu_integrate(lr, m, 4, p, dt, n, B0, stride)
    _assert_obs(got, ref, f"drive frame {kind}", tol)
    assert np.max(np.abs(Bg - Bo)) <= 1e-10


def test_batch_drive_frame_equals_single_bitwise(lr):
    """A lab-frame and a drive-frame trajectory in one batch: each bitwise equal to its run alone."""
    m = I.readout_model(3, 6, 4)
    items = []
    for frame in (I.FRAME_LAB, I.FRAME_DRIVE):
        p = I.flattop_pulse(0.07, 0.4, t_ramp=0.1).replace(frame=frame)
        B0 = I.initial_state(m, 3, "g", seed=53, scale=1e-3)
        items.append(dict(model=m, M=3, pulse=p, dt=1e-3, nsteps=150, B=lr.to_device(B0), B0=B0,
                          obs_stride=10, obs=lr.Context(m, 3).new_obs(150, 10)))
    b = lr.Batch([{k: v for k, v in it.items() if k != "B0"} for it in items])
    b.run()
    rc, codes, _ = b.status()
    assert rc == lr.LR_OK, codes
    for it in items:
        Bg, got = _gpu_integrate(lr, m, 3, it["pulse"], 1e-3, 150, it["B0"], 10)
        assert np.array_equal(Bg, lr.from_device(it["B"]))
        assert np.array_equal(got, it["obs"].cpu().numpy())


def test_dense_lindblad_drive_frame_matches_oracle(lr):
    """Dense full-Lindblad RK4 in the drive frame vs the oracle's dense master equation."""
    import torch
    from oracle import dense
    model, pulse, rho0 = _dense_case(54)
    pulse = pulse.replace(frame=I.FRAME_DRIVE)
    dt, nsteps, stride = 2e-3, 300, 100
    rho = torch.from_numpy(rho0.copy()).cuda()
    obs = torch.zeros((nsteps // stride + 1, 6 + model.d_q), dtype=torch.float64, device="cuda")
    lr.dense_integrate(model, pulse, 0.0, dt, nsteps, rho, stride, obs)
    torch.cuda.synchronize()
    ref_rho, ref_obs = dense.integrate(model, pulse, 0.0, dt, nsteps, rho0, obs_stride=stride)
    err = np.max(np.abs(rho.cpu().numpy() - ref_rho))
    print(f"[parity] dense drive frame rho err {err:.3e}")
    assert err <= 1e-12
    e = _obs_errors(obs.cpu().numpy(), ref_obs)
    assert e["field"] <= 1e-12 and e["pop"] <= 1e-12 and e["trace"] <= 1e-12


def test_drive_frame_rejects_unknown_frame(lr):
    m = I.readout_model(2, 3, 2)
    p = I.flattop_pulse(0.05, 1.0).replace(frame=7)
    B = _rand_B(m.N, 2, 55)
    ctx = lr.Context(m, 2)
    with pytest.raises(lr.LrError):
        ctx.integrate(p, 0.0, 1e-3, 5, lr.to_device(B))


# ------------------------------------------------------------ smoothed stepwise pulse (S2.C)

def _stepwise(n, seed, T=0.6, sigma=0.02):
    r = np.random.default_rng(seed)
    h = I.ghz(0.15) * (r.uniform(0.2, 1.0, n) * np.exp(1j * r.uniform(0, 2 * np.pi, n)))
    return I.stepwise_pulse(h, T, sigma=sigma)


def test_rhs_stepwise_pulse(lr):
    m = I.readout_model(3, 6, 4)
    p = _stepwise(9, 61)
    B = _rand_B(m.N, 5, 62)
    for t in (0.0, 0.07, 0.31, 0.6, 0.75):
        ref = lowrank.rhs(m, p, t, B)
        got = _gpu_rhs(lr, m, 5, p, t, B)
        assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("nh,frame", [(1, 0), (20, 0), (63, 0), (20, 1)])
def test_integrate_stepwise_pulse(lr, nh, frame):
    """Persistent RK4 with the stepwise envelope (up to the 63-height maximum; each drive
    table refill evaluates one stage time per thread) against the oracle, lab and drive frame."""
    m = I.readout_model(3, 7, 4).replace(kappa_f=0.5, gamma_1=0.05)
    p = _stepwise(nh, 63 + nh).replace(frame=frame)
    B0 = I.initial_state(m, 4, "g", seed=64, scale=1e-3)
    dt, n, stride = 1e-3, 203, 7
    Bo, ref, tol = oracle_with_tol(m, p, 0.0, dt, n, B0, stride)
    Bg, got = _gpu_integrate(lr, m, 4, p, dt, n, B0, stride)
    _assert_obs(got, ref, f"stepwise nh={nh} frame={frame}", tol)
    assert np.max(np.abs(Bg - Bo)) <= 1e-10


def test_stepwise_pulse_rejections(lr):
    m = I.readout_model(2, 3, 2)
    B = lr.to_device(_rand_B(m.N, 2, 65))
    ctx = lr.Context(m, 2)
    bad = [I.stepwise_pulse([], 1.0), I.stepwise_pulse([0.1] * 64, 1.0), I.stepwise_pulse([0.1], 1.0, sigma=0.0),
           I.stepwise_pulse([I.ghz(0.41)], 1.0), I.stepwise_pulse([0.1], 0.0)]
    for p in bad:
        with pytest.raises(lr.LrError):
            ctx.integrate(p, 0.0, 1e-3, 3, B)


def test_pulse_loss_batch_matches_oracle(lr):
    """Loss of stepwise pulses (S3.A-C) from one device batch of g/e pairs, lab and drive frame,
    against the oracle's integration and figures of merit."""
    from paper_2508_18114_amd import serve
    m = I.readout_model(3, 7, 4).replace(kappa_f=0.5, gamma_1=0.05)
    M, dt, T, stride = 4, 1e-3, 0.4, 8
    n = int(round(T / dt))
    pulses = [_stepwise(5, 71, T=T).replace(frame=fr) for fr in (0, 1)] + [_stepwise(12, 72, T=T)]
    got = serve.pulse_loss_batch(m, M, pulses, dt, n, stride)
    for p, fm in zip(pulses, got):
        obs = {}
        for which in ("g", "e"):
            B0 = I.initial_state(m, M, which, 0, I.PAPER_PAD_SCALE)
            _, obs[which] = lowrank.integrate(m, p, 0.0, dt, n, B0, obs_stride=stride)
        ref = loss.readout_loss(obs["g"], obs["e"], stride * dt, m.kappa_f, m.gamma_1)
        print(f"[parity] pulse loss nh={len(p.h)} frame={p.frame}: gpu {fm['loss']:.15e} oracle {ref['loss']:.15e}")
        assert abs(fm["loss"] - ref["loss"]) <= 1e-8
        assert abs(fm["snr"] - ref["snr"]) <= 1e-8 * max(1.0, ref["snr"])


def test_spsa_optimize_runs_on_device(lr):
    """Three SPSA steps (S3.C) over a 4-height stepwise pulse: every probe loss is finite, the heights
    stay inside the drive bound and the iterate moves."""
    from paper_2508_18114_amd import serve
    m = I.readout_model(3, 7, 4).replace(kappa_f=0.5, gamma_1=0.05)
    theta, hist = serve.spsa_optimize(m, 4, T=0.3, nh=4, iters=3, dt=1e-3, obs_stride=10, seed=3)
    assert len(hist) == 3
    assert all(np.isfinite(h["loss_plus"]) and np.isfinite(h["loss_minus"]) for h in hist)
    assert np.all(np.abs(serve.heights_from(theta)) < I.ghz(0.4))
    assert np.any(serve.heights_from(theta) != I.ghz(0.15))  # (a 0.3 ns pulse moves the loss very little)


# ------------------------------------------------------------ packed batch schedule (one workgroup per trajectory)

def _run_packed(lr, items, packed=True, flags=0):
    b = lr.Batch(items, packed=packed, flags=flags)
    b.run()
    rc, codes, steps = b.status()
    b.close()
    return rc, codes, steps


def test_packed_config_small_matches_oracle(lr):
    """Configuration 1 (dims (4,10,5), M = 4, 1e4 RK4 steps, g and e) in the packed schedule against the
    cached oracle run, with the figures of merit."""
    import torch
    trajs = I.config_small()
    gd = _golden("small")
    stride = int(gd["stride"])
    items = [dict(model=t.model, M=t.M, pulse=t.pulse, dt=t.dt, nsteps=t.nsteps, B=lr.to_device(t.B0()),
                  obs_stride=stride,
                  obs=torch.zeros((t.nsteps // stride + 1, 6 + t.model.d_q), dtype=torch.float64, device="cuda"))
             for t in trajs]
    rc, codes, _ = _run_packed(lr, items)
    assert rc == lr.LR_OK, codes
    tol = _golden_tol("small")
    for it, key in zip(items, ("obs_g", "obs_e")):
        _assert_obs(it["obs"].cpu().numpy(), gd[key], f"packed small {key}", tol)
    t = trajs[0]
    fm = lr.readout_loss(items[0]["obs"], items[1]["obs"], t.model.d_q, stride * t.dt, t.model.kappa_f,
                         t.model.gamma_1)
    assert abs(fm["snr"] - float(gd["snr"])) <= tol["snr_rel"] * float(gd["snr"])
    assert abs(fm["loss"] - float(gd["loss"])) <= 1e-8


def test_packed_batch_matches_oracle(lr):
    """Mixed shapes (M = 1 .. 20, different lengths and strides) and a drive-frame stepwise pulse, all in
    one packed launch, against the oracle."""
    items = _batch_items(lr, BATCH_SPECS)
    m = I.readout_model(3, 7, 4).replace(kappa_f=0.5, gamma_1=0.05)
    p = _stepwise(20, 83).replace(frame=1)
    B0 = I.initial_state(m, 4, "e", seed=84, scale=1e-3)
    import torch
    items.append(dict(model=m, M=4, pulse=p, dt=1e-3, nsteps=203, B0=B0, B=lr.to_device(B0), obs_stride=7,
                      obs=torch.zeros((203 // 7 + 1, 6 + 3), dtype=torch.float64, device="cuda")))
    rc, codes, _ = _run_packed(lr, items)
    assert rc == lr.LR_OK, codes
    for it in items:
        Bo, ref, tol = oracle_with_tol(it["model"], it["pulse"], 0.0, it["dt"], it["nsteps"], it["B0"],
                                       it["obs_stride"])
        got_B = lr.from_device(it["B"])
        err = np.max(np.abs(got_B - Bo))
        print(f"[parity] packed dims {it['model'].d_q, it['model'].d_r, it['model'].d_f} M={it['M']}: |dB| {err:.3e}")
        assert err <= 1e-10
        if it["obs_stride"]:
            _assert_obs(it["obs"].cpu().numpy(), ref, f"packed dims {it['model'].d_q, it['model'].d_r}", tol)


def test_packed_result_does_not_depend_on_the_batch(lr):
    """A packed trajectory alone and among others: bitwise the same state and records."""
    alone = _batch_items(lr, BATCH_SPECS[2:3])
    assert _run_packed(lr, alone)[0] == lr.LR_OK
    mix = _batch_items(lr, BATCH_SPECS)
    assert _run_packed(lr, mix)[0] == lr.LR_OK
    assert np.array_equal(lr.from_device(alone[0]["B"]), lr.from_device(mix[2]["B"]))
    assert np.array_equal(alone[0]["obs"].cpu().numpy(), mix[2]["obs"].cpu().numpy())


@pytest.mark.parametrize("gram", ["mfma", "valu"])
def test_packed_paper_size_matches_oracle(lr, gram):
    """Paper size (N = 2000, M = 20), g and e in the packed schedule for the first 6000 steps (3 ns),
    against the cached oracle run's records over the same span, with the paper-size floor tolerances;
    Gram terms on the vector ALU (the default) and on the matrix cores (FP64 instruction)."""
    import torch
    trajs = I.config_paper_size()
    gd = _golden("paper_size")
    tol = _golden_tol("paper_size")
    stride, n = int(gd["stride"]), 6000
    items = [dict(model=t.model, M=t.M, pulse=t.pulse, dt=t.dt, nsteps=n, B=lr.to_device(t.B0()),
                  obs_stride=stride, obs=torch.zeros((n // stride + 1, 6 + t.model.d_q), dtype=torch.float64,
                                                     device="cuda"))
             for t in trajs]
    rc, codes, _ = _run_packed(lr, items, flags=lr.LR_BATCH_PACKED_MFMA64 if gram == "mfma" else 0)
    assert rc == lr.LR_OK, codes
    for it, key in zip(items, ("obs_g", "obs_e")):
        _assert_obs(it["obs"].cpu().numpy(), gd[key][:n // stride + 1], f"packed ({gram}) paper size {key} (3 ns)",
                    tol)


def test_packed_limits_and_fallback(lr):
    """The largest packed layer (d_q d_f M = 1536, three output tiles per wave on the matrix cores)
    against the oracle with both Gram forms; ranks 1 to 32 across the tile boundaries (one and two row
    tiles, ragged column tiles) against the oracle; FP32 and BF16x3 trajectories run packed (matrix-core
    Gram terms) and stay within the reduced-precision bounds of their FP64 result, and an adaptive batch
    refuses them."""
    import torch
    m = I.readout_model(8, 3, 6).replace(kappa_f=0.5, gamma_1=0.05)
    assert m.d_q * m.d_f * 32 == lr.LR_PACKED_MAX_LM
    p = I.flattop_pulse(0.05, 0.1, t_ramp=0.02)
    B0 = I.initial_state(m, 32, "g", seed=91, scale=1e-2)
    Bo, ref, tol = oracle_with_tol(m, p, 0.0, 1e-3, 40, B0, 10)
    for flags in (0, lr.LR_BATCH_PACKED_MFMA64):
        it = dict(model=m, M=32, pulse=p, dt=1e-3, nsteps=40, B=lr.to_device(B0), obs_stride=10,
                  obs=torch.zeros((5, 6 + 8), dtype=torch.float64, device="cuda"))
        assert _run_packed(lr, [it], flags=flags)[0] == lr.LR_OK
        _assert_obs(it["obs"].cpu().numpy(), ref, f"packed largest layer (flags {flags})", tol)
    ms = I.readout_model(3, 4, 3).replace(kappa_f=0.5, gamma_1=0.05)
    ranks = (1, 5, 16, 17, 21, 22, 27)
    items = [dict(model=ms, M=M, pulse=p, dt=1e-3, nsteps=30, B=lr.to_device(I.initial_state(ms, M, "e", 93 + M, 1e-2)),
                  obs_stride=10, obs=torch.zeros((4, 6 + 3), dtype=torch.float64, device="cuda")) for M in ranks]
    assert _run_packed(lr, items)[0] == lr.LR_OK
    for M, it in zip(ranks, items):
        _, refm, tolm = oracle_with_tol(ms, p, 0.0, 1e-3, 30, I.initial_state(ms, M, "e", 93 + M, 1e-2), 10)
        _assert_obs(it["obs"].cpu().numpy(), refm, f"packed matrix-core Gram M={M}", tolm)
    # FP32 and BF16x3 run packed, near their FP64 result
    mm = I.readout_model(4, 6, 5)
    res = {}
    for prec in (0, 1, 2):
        items = [dict(model=mm, M=6, pulse=p, dt=1e-3, nsteps=30, precision=prec,
                      B=lr.to_device(I.initial_state(mm, 6, "e", 92, scale=1e-2)))]
        assert _run_packed(lr, items)[0] == lr.LR_OK
        res[prec] = lr.from_device(items[0]["B"])
    for prec in (1, 2):
        err = np.max(np.abs(res[prec] - res[0])) / np.max(np.abs(res[0]))
        print(f"[packed] precision {prec}: max rel deviation of B from FP64 {err:.2e}")
        assert 0.0 < err < (1e-5 if prec == 1 else 1e-4)
    with pytest.raises(lr.LrError):
        lr.Batch([dict(model=mm, M=6, pulse=p, dt=1e-3, nsteps=3, precision=1,
                       B=lr.to_device(I.initial_state(mm, 6, "e", 92, scale=1e-2)))], adaptive=(1e-8, 1e-10))


def test_packed_device_errors(lr):
    """Rank-deficient and non-finite initial states stop their own trajectory at step 0 with the error
    code; a healthy trajectory in the same packed launch is unaffected."""
    m = I.readout_model(2, 3, 2)
    p = I.flattop_pulse(0.05, 1.0)
    B0 = _rand_B(m.N, 3, 10)
    B0[:, 1] = 0.0
    B1 = _rand_B(m.N, 3, 11)
    B1[4, 2] = np.nan
    B2 = _rand_B(m.N, 3, 12)
    items = [dict(model=m, M=3, pulse=p, dt=1e-3, nsteps=5, B=lr.to_device(B)) for B in (B0, B1, B2)]
    rc, codes, steps = _run_packed(lr, items)
    assert list(codes) == [lr.LR_ERR_GRAM_NOT_PD, lr.LR_ERR_NONFINITE, lr.LR_OK]
    assert list(steps[:2]) == [0, 0]
    alone = [dict(model=m, M=3, pulse=p, dt=1e-3, nsteps=5, B=lr.to_device(B2))]
    assert _run_packed(lr, alone)[0] == lr.LR_OK
    assert np.array_equal(lr.from_device(alone[0]["B"]), lr.from_device(items[2]["B"]))


# ------------------------------------------------------------ adaptive Dormand-Prince steps (packed schedule)

def _adaptive_case(lr, frame, seed=5):
    import torch
    m = I.readout_model(3, 5, 3).replace(kappa_f=0.5, gamma_1=0.05)
    h = I.ghz(0.15) * np.array([0.5, 1.0 + 0.3j, 0.8])
    p = I.stepwise_pulse(h, 2.0, sigma=0.1).replace(frame=frame)
    B0 = I.initial_state(m, 3, "e", seed=seed, scale=1e-2)
    it = dict(model=m, M=3, pulse=p, dt=0.05, nsteps=40, B0=B0, B=lr.to_device(B0), obs_stride=8,
              obs=torch.zeros((6, 6 + 3), dtype=torch.float64, device="cuda"))
    return it


def test_adaptive_matches_oracle(lr):
    """Dormand-Prince 5(4) with per-trajectory steps, drive and lab frame, against the oracle's adaptive
    integration at the same tolerances: observables to the tolerance scale, step counts nearly equal."""
    from oracle import adaptive
    rtol, atol = 1e-9, 1e-12
    for frame in (I.FRAME_DRIVE, I.FRAME_LAB):
        it = _adaptive_case(lr, frame)
        b = lr.Batch([it], adaptive=(rtol, atol))
        b.run()
        rc, codes, _ = b.status()
        assert rc == lr.LR_OK, codes
        acc, rej = b.adaptive_stats()
        Bo, ref, acc_o, rej_o = adaptive.integrate(it["model"], it["pulse"], 0.0, 0.05, 40, it["B0"], rtol, atol,
                                                   obs_stride=8)
        got = it["obs"].cpu().numpy()
        scale = max(1.0, np.max(np.abs(ref[:, 0:4])))
        ef = np.max(np.abs(got[:, 0:4] - ref[:, 0:4])) / scale
        ep = np.max(np.abs(got[:, 4:] - ref[:, 4:]))
        print(f"[parity] adaptive frame={frame}: steps gpu {acc[0]}+{rej[0]} rejected, oracle {acc_o}+{rej_o}; "
              f"field err {ef:.3e}, populations err {ep:.3e}")
        assert ef <= 1e-7 and ep <= 1e-7
        assert abs(acc[0] - acc_o) <= 3 and abs(rej[0] - rej_o) <= 3
        b.close()


def test_adaptive_result_does_not_depend_on_the_batch(lr):
    alone = [_adaptive_case(lr, I.FRAME_DRIVE)]
    b = lr.Batch(alone, adaptive=(1e-8, 1e-11))
    b.run()
    assert b.status()[0] == lr.LR_OK
    mix = [_adaptive_case(lr, I.FRAME_LAB, seed=6), _adaptive_case(lr, I.FRAME_DRIVE), _adaptive_case(lr, I.FRAME_DRIVE, 7)]
    bm = lr.Batch(mix, adaptive=(1e-8, 1e-11))
    bm.run()
    assert bm.status()[0] == lr.LR_OK
    assert np.array_equal(lr.from_device(alone[0]["B"]), lr.from_device(mix[1]["B"]))
    assert np.array_equal(alone[0]["obs"].cpu().numpy(), mix[1]["obs"].cpu().numpy())
    assert b.adaptive_stats()[0][0] == bm.adaptive_stats()[0][1]


def test_adaptive_paper_size_drive_frame(lr):
    """Paper size (N = 2000, M = 20), 2 ns of g and e in the drive frame, adaptive at rtol 1e-8, against
    the oracle's adaptive integration of the same problem (cached): the same accepted and rejected step
    counts (within 3) and records to 1e-9 (steps of 1e-8 relative local error)."""
    import torch
    gd = np.load(os.path.join(HERE, "golden", "adaptive_paper_size.npz"))
    trajs = I.config_paper_size()
    dt, n, stride = float(gd["dt"]), int(gd["nsteps"]), int(gd["stride"])
    items = [dict(model=t.model, M=t.M, pulse=t.pulse.replace(frame=I.FRAME_DRIVE), dt=dt, nsteps=n,
                  B=lr.to_device(t.B0()), obs_stride=stride,
                  obs=torch.zeros((n // stride + 1, 6 + t.model.d_q), dtype=torch.float64, device="cuda"))
             for t in trajs]
    b = lr.Batch(items, adaptive=(float(gd["rtol"]), float(gd["atol"])))
    b.run()
    rc, codes, _ = b.status()
    assert rc == lr.LR_OK, codes
    acc, rej = b.adaptive_stats()
    for k, (it, key) in enumerate(zip(items, ("g", "e"))):
        got, ref = it["obs"].cpu().numpy(), gd["obs_" + key]
        e = _obs_errors(got, ref)
        print(f"[adaptive] paper size 2 ns drive frame {key}: gpu {acc[k]} + {rej[k]} rejected, oracle "
              f"{int(gd['acc_' + key])} + {int(gd['rej_' + key])}; field err {e['field']:.3e}, populations err "
              f"{e['pop']:.3e}")
        assert abs(acc[k] - int(gd["acc_" + key])) <= 3 and abs(rej[k] - int(gd["rej_" + key])) <= 3
        assert e["field"] <= 1e-9 and e["pop"] <= 1e-9 and e["trace"] <= 1e-9
    b.close()


def test_adaptive_rejections(lr):
    it = _adaptive_case(lr, I.FRAME_DRIVE)
    for tol in ((0.0, 1e-12), (1e-8, -1.0), (float("nan"), 1e-12)):
        with pytest.raises(lr.LrError):
            lr.Batch([it], adaptive=tol)
    fp32 = dict(it, precision=1)
    with pytest.raises(lr.LrError):
        lr.Batch([fp32], adaptive=(1e-8, 1e-12))
    b = lr.Batch([_adaptive_case(lr, I.FRAME_DRIVE)], packed=True)
    with pytest.raises(lr.LrError):
        b.adaptive_stats()


@pytest.mark.parametrize("d_r,M", [(1, 1), (2, 3), (3, 8)])
def test_packed_and_adaptive_few_layers(lr, d_r, M):
    """Packed RK4 and adaptive steps with one to three resonator layers (the three-layer window at its
    edges) and rank 1, against the oracle."""
    import torch
    from oracle import adaptive
    m = I.readout_model(3, d_r, 4).replace(kappa_f=0.5, gamma_1=0.05)
    p = _stepwise(6, 90 + d_r, T=0.3).replace(frame=1)
    B0 = I.initial_state(m, M, "e", seed=91 + d_r, scale=1e-2)
    it = dict(model=m, M=M, pulse=p, dt=2e-3, nsteps=150, B=lr.to_device(B0), obs_stride=30,
              obs=torch.zeros((6, 6 + 3), dtype=torch.float64, device="cuda"))
    assert _run_packed(lr, [it])[0] == lr.LR_OK
    _, ref, tol = oracle_with_tol(m, p, 0.0, 2e-3, 150, B0, 30)
    _assert_obs(it["obs"].cpu().numpy(), ref, f"packed d_r={d_r} M={M}", tol)
    ia = dict(model=m, M=M, pulse=p, dt=0.05, nsteps=6, B=lr.to_device(B0), obs_stride=2,
              obs=torch.zeros((4, 6 + 3), dtype=torch.float64, device="cuda"))
    b = lr.Batch([ia], adaptive=(1e-9, 1e-12))
    b.run()
    assert b.status()[0] == lr.LR_OK
    acc, rej = b.adaptive_stats()
    _, refa, acc_o, rej_o = adaptive.integrate(m, p, 0.0, 0.05, 6, B0, 1e-9, 1e-12, obs_stride=2)
    _assert_obs(ia["obs"].cpu().numpy(), refa, f"adaptive d_r={d_r} M={M}")
    assert abs(acc[0] - acc_o) <= 3 and abs(rej[0] - rej_o) <= 3


# ------------------------------------------------------------ HIP graph capture of a packed batch

def test_graph_replays_equal_eager_run(lr):
    """A packed batch (several chunks and records) captured once and replayed three times, with eager
    work (state resets, another batch) between the replays: every replay bitwise equals the eager run;
    the same for an adaptive batch and for a batch of three kernel families (launch sequences forked
    onto streams of their own and joined back inside the capture)."""
    import torch
    for adaptive in (None, (1e-8, 1e-11), "families"):
        if adaptive == "families":
            # three kernel families (FP64, FP32, BF16x3: forked streams inside the capture), the FP64
            # one with a large-footprint member (M = 32 holds one workgroup per CU)
            items = _batch_items(lr, BATCH_SPECS[:3] + [((8, 4, 5), 32, "g", 40, 10, 6)])
            items[0]["precision"], items[1]["precision"] = 1, 2
            adaptive = None
        elif adaptive is None:
            items = _batch_items(lr, BATCH_SPECS[:3])
        else:
            items = [_adaptive_case(lr, I.FRAME_DRIVE), _adaptive_case(lr, I.FRAME_LAB, seed=8)]
        st = torch.cuda.Stream()  # a capturable stream (not the null stream)
        b = lr.Batch(items, stream=st, packed=True, adaptive=adaptive)
        b.run()
        assert b.status()[0] == lr.LR_OK
        ref = [(it["B"].clone(), it["obs"].clone() if it.get("obs") is not None else None) for it in items]
        b.graph(True)
        for rep in range(3):
            for it in items:
                it["B"].copy_(lr.to_device(it["B0"]))
                if it.get("obs") is not None:
                    it["obs"].zero_()
            other = _batch_items(lr, BATCH_SPECS[3:4])  # eager work between replays
            ob = lr.Batch(other)
            ob.run()
            assert ob.status()[0] == lr.LR_OK
            torch.cuda.synchronize()
            b.run()
            assert b.status()[0] == lr.LR_OK
            for it, (Br, Or) in zip(items, ref):
                assert torch.equal(it["B"], Br), (adaptive, rep)
                if Or is not None:
                    assert torch.equal(it["obs"], Or), (adaptive, rep)
        b.graph(False)
        b.close()


def test_graph_needs_packed_batch_on_a_stream(lr):
    import torch
    items = _batch_items(lr, BATCH_SPECS[:1])
    b = lr.Batch(items, stream=torch.cuda.Stream())
    with pytest.raises(lr.LrError):
        b.graph(True)
    b2 = lr.Batch(_batch_items(lr, BATCH_SPECS[:1]), packed=True)  # the null stream
    with pytest.raises(lr.LrError):
        b2.graph(True)


def test_spread_tile_height_and_autotuner(lr, tmp_path):
    """Tile heights 1..3 of the spread schedule agree to the FP64 tolerances (other summation orders);
    the autotuner picks a configuration that runs, its tuned batch equals bitwise a batch built with the
    picked flags, and the choice is cached on disk."""
    from paper_2508_18114_amd import autotune
    specs = [((4, 10, 5), 4, "g", 120, 10, 1), ((3, 7, 4), 6, "e", 120, 10, 2)]
    res = {}
    for k in (1, 2, 3):
        items = _batch_items(lr, specs)
        b = lr.Batch(items, flags=lr.LR_BATCH_SPREAD_LAYERS(k))
        b.run()
        assert b.status()[0] == lr.LR_OK
        res[k] = [it["obs"].cpu().numpy() for it in items]
    for k in (2, 3):
        for a, r in zip(res[k], res[1]):
            _assert_obs(a, r, f"spread tile height {k} vs 1")
    items = _batch_items(lr, specs)
    path = str(tmp_path / "tune.json")
    choice = autotune.tune(items, steps=10, cache_path=path)
    print(f"[autotune] {choice}")
    assert choice["schedule"] in ("spread", "packed") and max(v for v in choice["rates"].values() if v) > 0
    tb = autotune.tuned_batch(items, cache_path=path)
    tb.run()
    assert tb.status()[0] == lr.LR_OK
    ref = _batch_items(lr, specs)
    rb = lr.Batch(ref, flags=choice["flags"])
    rb.run()
    assert rb.status()[0] == lr.LR_OK
    for a, r in zip(items, ref):
        assert np.array_equal(lr.from_device(a["B"]), lr.from_device(r["B"]))
    import json
    assert autotune.signature(items) in json.load(open(path))


# ------------------------------------------------------------ the paper's Hamiltonian, transmon eigenbasis (kind 1)

def _tm_items(lr, model, M, pulse, dt, nsteps, stride, which="e", seed=101, scale=1e-2):
    import torch
    B0 = I.initial_state(model, M, which, seed=seed, scale=scale)
    return dict(model=model, M=M, pulse=pulse, dt=dt, nsteps=nsteps, B0=B0, B=lr.to_device(B0), obs_stride=stride,
                obs=torch.zeros((nsteps // stride + 1, 6 + model.d_q), dtype=torch.float64, device="cuda"))


def test_transmon_model_packed_matches_oracle(lr):
    """The paper's Hamiltonian (transmon eigenbasis tables, dense n_t coupling, -J (a^ - a)(f^ - f),
    drive on i (f^ - f)) in the packed kernel against the oracle: a small model with strong dissipation,
    and the paper's parameters at N_t = 6 with a stepwise drive."""
    from paper_2508_18114_amd import transmon
    small = transmon.paper_model(4, 6, 4).replace(kappa_f=0.5, gamma_1=0.05, g=0.9, G=0.4)
    paper = transmon.paper_model(6, 12, 5)
    cases = [(small, 4, _stepwise(8, 102, T=0.3).replace(w_d=transmon.PAPER_W_DRIVE), 1e-3, 240, 40),
             (paper, 8, I.stepwise_pulse(I.ghz(0.15) * np.array([1.0, 1.0j, 0.7]), 0.5, sigma=0.05,
                                         w_d=transmon.PAPER_W_DRIVE), 5e-4, 600, 100),
             # the frame rotating at the drive carrier, every term kept
             (small, 4, _stepwise(8, 103, T=0.3).replace(w_d=transmon.PAPER_W_DRIVE, frame=1), 1e-3, 240, 40),
             (paper, 8, I.stepwise_pulse(I.ghz(0.15) * np.array([1.0, 1.0j, 0.7]), 0.5, sigma=0.05,
                                         w_d=transmon.PAPER_W_DRIVE).replace(frame=1), 5e-4, 600, 100)]
    items = [_tm_items(lr, m, M, p, dt, n, s) for (m, M, p, dt, n, s) in cases]
    rc, codes, _ = _run_packed(lr, items)
    assert rc == lr.LR_OK, codes
    for it in items:
        Bo, ref, tol = oracle_with_tol(it["model"], it["pulse"], 0.0, it["dt"], it["nsteps"], it["B0"],
                                       it["obs_stride"])
        _assert_obs(it["obs"].cpu().numpy(), ref,
                    f"transmon model dims {it['model'].d_q, it['model'].d_r, it['model'].d_f} frame {it['pulse'].frame}",
                    tol)
        assert np.max(np.abs(lr.from_device(it["B"]) - Bo)) <= 1e-10


def test_transmon_model_rejections(lr):
    """Kind 1 runs packed only: a Context, a spread batch and a non-symmetric n_t are refused; d_q
    above the table size too."""
    from paper_2508_18114_amd import transmon
    m = transmon.paper_model(4, 3, 3)
    p = I.flattop_pulse(0.05, 0.2)
    with pytest.raises(lr.LrError):
        lr.Context(m, 2)
    with pytest.raises(lr.LrError):
        lr.Batch([_tm_items(lr, m, 2, p, 1e-3, 10, 5)])
    nt = list(m.n_t)
    nt[1] += 0.5
    with pytest.raises(lr.LrError):
        lr.Batch([_tm_items(lr, m.replace(n_t=tuple(nt)), 2, p, 1e-3, 10, 5)], packed=True)
    with pytest.raises(ValueError):
        lr.model_struct(transmon.paper_model(9, 2, 2))


def test_transmon_model_adaptive_matches_oracle(lr):
    """The paper's set-up: its Hamiltonian (transmon eigenbasis) in the drive frame, adaptive
    Dormand-Prince steps, against the oracle's adaptive integration (same step counts, records)."""
    from oracle import adaptive
    from paper_2508_18114_amd import transmon
    m = transmon.paper_model(4, 8, 4).replace(kappa_f=0.3, gamma_1=0.02)
    p = I.stepwise_pulse(I.ghz(0.15) * np.array([1.0j, 0.8j]), 1.0, sigma=0.1,
                         w_d=transmon.PAPER_W_DRIVE).replace(frame=1)
    it = _tm_items(lr, m, 4, p, 0.1, 10, 2)
    b = lr.Batch([it], adaptive=(1e-9, 1e-12))
    b.run()
    rc, codes, _ = b.status()
    assert rc == lr.LR_OK, codes
    acc, rej = b.adaptive_stats()
    _, ref, acc_o, rej_o = adaptive.integrate(m, p, 0.0, 0.1, 10, it["B0"], 1e-9, 1e-12, obs_stride=2)
    print(f"[parity] transmon model adaptive drive frame: steps gpu {acc[0]}+{rej[0]}, oracle {acc_o}+{rej_o}")
    _assert_obs(it["obs"].cpu().numpy(), ref, "transmon model adaptive")
    assert abs(acc[0] - acc_o) <= 3 and abs(rej[0] - rej_o) <= 3


def test_spsa_on_the_paper_model_with_adaptive_steps(lr):
    """Two SPSA steps over the paper's Hamiltonian (transmon eigenbasis, drive frame, adaptive steps):
    finite losses, heights inside the bound."""
    from paper_2508_18114_amd import serve, transmon
    m = transmon.paper_model(4, 6, 4).replace(kappa_f=0.3, gamma_1=0.02)
    theta, hist = serve.spsa_optimize(m, 4, T=0.4, nh=3, iters=2, dt=0.1, obs_stride=1, seed=5,
                                      w_d=transmon.PAPER_W_DRIVE, adaptive=(1e-8, 1e-11))
    assert len(hist) == 2 and all(np.isfinite(h["loss_plus"]) and np.isfinite(h["loss_minus"]) for h in hist)
    assert np.all(np.abs(serve.heights_from(theta)) < I.ghz(0.4))


@pytest.mark.parametrize("d_r,M,frame", [(1, 1, 0), (2, 3, 1), (3, 8, 1)])
def test_transmon_model_few_layers(lr, d_r, M, frame):
    """The eigenbasis model with one to three resonator layers and rank 1, both frames, fixed and
    adaptive steps, against the oracle."""
    from oracle import adaptive
    from paper_2508_18114_amd import transmon
    m = transmon.paper_model(3, d_r, 4).replace(kappa_f=0.4, gamma_1=0.05)
    p = I.stepwise_pulse(I.ghz(0.15) * np.array([1.0j, 0.5]), 0.3, sigma=0.03,
                         w_d=transmon.PAPER_W_DRIVE).replace(frame=frame)
    it = _tm_items(lr, m, M, p, 2e-4 if frame == 0 else 1e-3, 300 if frame == 0 else 300, 60,
                   seed=110 + d_r)
    assert _run_packed(lr, [it])[0] == lr.LR_OK
    _, ref, tol = oracle_with_tol(m, p, 0.0, it["dt"], it["nsteps"], it["B0"], 60)
    _assert_obs(it["obs"].cpu().numpy(), ref, f"transmon d_r={d_r} M={M} frame={frame}", tol)
    ia = _tm_items(lr, m, M, p, 0.05, 4, 2, seed=110 + d_r)
    b = lr.Batch([ia], adaptive=(1e-9, 1e-12))
    b.run()
    assert b.status()[0] == lr.LR_OK
    acc, rej = b.adaptive_stats()
    _, refa, acc_o, rej_o = adaptive.integrate(m, p, 0.0, 0.05, 4, ia["B0"], 1e-9, 1e-12, obs_stride=2)
    _assert_obs(ia["obs"].cpu().numpy(), refa, f"transmon adaptive d_r={d_r} M={M} frame={frame}")
    assert abs(acc[0] - acc_o) <= 3 and abs(rej[0] - rej_o) <= 3


# ------------------------------------------------------------ the paper's Hamiltonian, normal-mode basis (kind 2)

def _nm_model(d_q, d_l, d_u, J=None, **kw):
    """Kind 2 at the paper's parameters; J (rad/ns) replaces the resonator-filter coupling (a larger J
    gives the filter operator larger creation admixtures s_21, s_22)."""
    from paper_2508_18114_amd import transmon
    m = transmon.paper_model_normal(d_q, d_l, d_u)
    if J is not None:
        wl, wu, S2 = transmon.normal_modes(I.ghz(7.2), I.ghz(7.21), J)
        m = m.replace(w_r=wl, w_f=wu, S=tuple(np.asarray(S2).ravel()))
    return m.replace(**kw)


def test_normal_model_packed_matches_oracle(lr):
    """The paper's Hamiltonian in the normal-mode basis (S2.D; the filter jump across layers, its
    creation terms and the non-diagonal -1/2 L_1^ L_1 over a five-layer window) in the packed kernel
    against the oracle, in the lab frame and the frame rotating at the drive: a small strongly damped
    model with a large resonator-filter coupling, and the paper's parameters at N_t = 5, N_u = 4."""
    from paper_2508_18114_amd import transmon
    small = _nm_model(4, 7, 4, J=1.1, kappa_f=0.6, gamma_1=0.05, g=0.9)
    paper = _nm_model(5, 14, 4)
    pw = I.stepwise_pulse(I.ghz(0.15) * np.array([1.0, 1.0j, 0.7]), 0.5, sigma=0.05, w_d=transmon.PAPER_W_DRIVE)
    cases = [(small, 4, _stepwise(8, 202, T=0.3).replace(w_d=transmon.PAPER_W_DRIVE), 1e-3, 240, 40),
             (paper, 8, pw, 5e-4, 600, 100),
             (small, 4, _stepwise(8, 203, T=0.3).replace(w_d=transmon.PAPER_W_DRIVE, frame=1), 1e-3, 240, 40),
             (paper, 8, pw.replace(frame=1), 5e-4, 600, 100)]
    items = [_tm_items(lr, m, M, p, dt, n, s) for (m, M, p, dt, n, s) in cases]
    rc, codes, _ = _run_packed(lr, items)
    assert rc == lr.LR_OK, codes
    for it in items:
        Bo, ref, tol = oracle_with_tol(it["model"], it["pulse"], 0.0, it["dt"], it["nsteps"], it["B0"],
                                       it["obs_stride"])
        _assert_obs(it["obs"].cpu().numpy(), ref,
                    f"normal-mode model dims {it['model'].d_q, it['model'].d_r, it['model'].d_f} "
                    f"frame {it['pulse'].frame}", tol)
        assert np.max(np.abs(lr.from_device(it["B"]) - Bo)) <= 1e-10


@pytest.mark.parametrize("d_l,d_u,M,frame", [(1, 4, 1, 0), (2, 3, 3, 1), (3, 1, 2, 1), (4, 2, 5, 0), (5, 5, 8, 1)])
def test_normal_model_few_layers(lr, d_l, d_u, M, frame):
    """The normal-mode model with one to five layers (the edges of the five-layer window), one or two
    upper-mode levels and rank 1, both frames, against the oracle; mixed in one batch with a kind-0
    trajectory (the two kernel families of one batch)."""
    from paper_2508_18114_amd import transmon
    m = _nm_model(3, d_l, d_u, J=1.1, kappa_f=0.5, gamma_1=0.05, g=0.8)
    p = I.stepwise_pulse(I.ghz(0.15) * np.array([1.0j, 0.5]), 0.3, sigma=0.03,
                         w_d=transmon.PAPER_W_DRIVE).replace(frame=frame)
    it = _tm_items(lr, m, M, p, 2e-4 if frame == 0 else 1e-3, 300, 60, seed=210 + d_l)
    m0 = I.readout_model(3, 4, 3)
    it0 = _tm_items(lr, m0, 2, I.flattop_pulse(0.05, 0.2, t_ramp=0.05), 1e-3, 100, 50, seed=7)
    assert _run_packed(lr, [it0, it])[0] == lr.LR_OK
    _, ref, tol = oracle_with_tol(m, p, 0.0, it["dt"], it["nsteps"], it["B0"], 60)
    _assert_obs(it["obs"].cpu().numpy(), ref, f"normal-mode d_l={d_l} d_u={d_u} M={M} frame={frame}", tol)
    _, ref0, tol0 = oracle_with_tol(m0, it0["pulse"], 0.0, 1e-3, 100, it0["B0"], 50)
    _assert_obs(it0["obs"].cpu().numpy(), ref0, "kind-0 trajectory beside the normal-mode one", tol0)


@pytest.mark.parametrize("M", [13, 20, 27, 32])
def test_normal_model_large_ranks(lr, M):
    """Kind 2 at the ranks of the bench and beyond (4M Gram-term columns: entry blocks of 5 to 16 rows,
    the kernels held to two workgroups per CU up to blocks of 8), both frames, against the oracle."""
    from paper_2508_18114_amd import transmon
    m = _nm_model(4, 6, 4, J=1.1, kappa_f=0.5, gamma_1=0.05, g=0.8)
    items = []
    for frame in (0, 1):
        p = I.stepwise_pulse(I.ghz(0.15) * np.array([1.0j, 0.6]), 0.2, sigma=0.02,
                             w_d=transmon.PAPER_W_DRIVE).replace(frame=frame)
        items.append(_tm_items(lr, m, M, p, 2e-4 if frame == 0 else 1e-3, 60, 30, seed=250 + M))
    assert _run_packed(lr, items)[0] == lr.LR_OK
    for it in items:
        Bo, ref, tol = oracle_with_tol(m, it["pulse"], 0.0, it["dt"], it["nsteps"], it["B0"], 30)
        _assert_obs(it["obs"].cpu().numpy(), ref, f"normal-mode M={M} frame {it['pulse'].frame}", tol)
        assert np.max(np.abs(lr.from_device(it["B"]) - Bo)) <= 1e-10


@pytest.mark.parametrize("d_l,frame", [(8, 1), (3, 0), (1, 1)])
def test_normal_model_adaptive_matches_oracle(lr, d_l, frame):
    """The paper's own set-up: its Hamiltonian in the normal-mode basis with adaptive Dormand-Prince
    steps (drive frame; also the lab frame and a single layer), against the oracle's adaptive
    integration: the same accepted and rejected step counts (within 3) and the records."""
    from oracle import adaptive
    from paper_2508_18114_amd import transmon
    m = _nm_model(4, d_l, 3, J=1.1, kappa_f=0.4, gamma_1=0.02, g=0.8)
    p = I.stepwise_pulse(I.ghz(0.15) * np.array([1.0j, 0.8j]), 1.0, sigma=0.1,
                         w_d=transmon.PAPER_W_DRIVE).replace(frame=frame)
    dt, n, stride = (0.1, 8, 2) if frame else (0.02, 4, 2)
    it = _tm_items(lr, m, 4, p, dt, n, stride, seed=230 + d_l)
    b = lr.Batch([it], adaptive=(1e-9, 1e-12))
    b.run()
    rc, codes, _ = b.status()
    assert rc == lr.LR_OK, codes
    acc, rej = b.adaptive_stats()
    _, ref, acc_o, rej_o = adaptive.integrate(m, p, 0.0, dt, n, it["B0"], 1e-9, 1e-12, obs_stride=stride)
    print(f"[parity] normal-mode adaptive d_l={d_l} frame {frame}: steps gpu {acc[0]}+{rej[0]}, "
          f"oracle {acc_o}+{rej_o}")
    _assert_obs(it["obs"].cpu().numpy(), ref, f"normal-mode adaptive d_l={d_l} frame {frame}")
    assert abs(acc[0] - acc_o) <= 3 and abs(rej[0] - rej_o) <= 3
    b.close()


def test_normal_model_rejections(lr):
    """Kind 2 runs in packed batches (fixed or adaptive steps) in FP64 only: a Context, a spread batch
    and reduced precision are refused, and so is a non-finite S."""
    m = _nm_model(3, 3, 3)
    p = I.flattop_pulse(0.05, 0.2)
    with pytest.raises(lr.LrError):
        lr.Context(m, 2)
    with pytest.raises(lr.LrError):
        lr.Batch([_tm_items(lr, m, 2, p, 1e-3, 10, 5)])
    it = _tm_items(lr, m, 2, p, 1e-3, 10, 5)
    it["precision"] = I.FP32
    with pytest.raises(lr.LrError):
        lr.Batch([it], packed=True)
    S = list(m.S)
    S[5] = float("nan")
    with pytest.raises(lr.LrError):
        lr.Batch([_tm_items(lr, m.replace(S=tuple(S)), 2, p, 1e-3, 10, 5)], packed=True)


# ------------------------------------------------------------ operator application on its own

@pytest.mark.parametrize("dims,ncols,frame", [((8, 50, 5), 40, 0), ((8, 50, 5), 40, 1), ((3, 7, 4), 13, 0),
                                              ((2, 1, 1), 3, 1), ((8, 75, 5), 64, 0), ((4, 10, 5), 1, 1)])
def test_apply_heff_matches_oracle(lr, dims, ncols, frame):
    """Z = H_eff(t) B (lr_apply_heff) against the oracle's mode-wise operators, lab and drive frame,
    several columns side by side (a ragged count included).  Each entry of Z is a sum of at most 11
    products: the bound is a few ulps of the largest entry."""
    m = I.readout_model(*dims).replace(kappa_f=0.7, gamma_1=0.3)
    p = I.flattop_pulse(0.09, 6.0).replace(frame=frame)
    B = _rand_B(m.N, ncols, 31 + ncols)
    Bd = lr.to_device(B)
    for t in (0.0, 1.3, 3.7):
        d_t = opulses.drive(p, t)
        ref = (lowrank.apply_heff_drive_frame(m, d_t, p.w_d, t, B) if frame else lowrank.apply_heff(m, d_t, B))
        got = lr.from_device(lr.apply_heff(m, p, t, Bd))
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"[parity] apply_heff dims={dims} ncols={ncols} frame={frame} t={t}: rel err {err:.3e}")
        assert err <= 1e-14


def test_apply_heff_full_width_sampled(lr):
    """The measured width: 512 factors of N = 2000, M = 20 side by side (10240 columns, 328 MB in and
    out); sampled columns against the oracle, applied column by column."""
    import torch
    m = I.readout_model(8, 50, 5)
    p = I.config_paper_size()[0].pulse
    ncols = 512 * 20
    gen = torch.Generator(device="cuda").manual_seed(5)
    Bd = torch.randn((ncols, m.N), dtype=torch.complex128, device="cuda", generator=gen)
    t = 7.25
    Z = lr.apply_heff(m, p, t, Bd)
    torch.cuda.synchronize()
    d_t = opulses.drive(p, t)
    rs = np.random.default_rng(6)
    for c in list(rs.choice(ncols, 12, replace=False)) + [0, ncols - 1]:
        b = Bd[c].cpu().numpy()[:, None]
        ref = lowrank.apply_heff(m, d_t, b)[:, 0]
        got = Z[c].cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref)), c


def test_apply_heff_rejections(lr):
    import torch
    m = I.readout_model(2, 3, 2)
    p = I.flattop_pulse(0.05, 1.0)
    B = torch.zeros((2, m.N), dtype=torch.complex128, device="cuda")
    with pytest.raises(lr.LrError):
        lr.apply_heff(m, I.flattop_pulse(0.5, 1.0), 0.0, B)        # drive above the bound
    big = I.readout_model(8, 300, 5)                                   # N = 12000 > 8192
    with pytest.raises(lr.LrError):
        lr.apply_heff(big, p, 0.0, torch.zeros((1, big.N), dtype=torch.complex128, device="cuda"))
    with pytest.raises(lr.LrError):                                    # B and Z overlap
        lr.apply_heff(m, p, 0.0, B, B)


# ------------------------------------------------------------ layer-split packed trajectories

def _run_split(lr, items, parts, adaptive=None):
    b = lr.Batch(items, packed=True, parts=parts, adaptive=adaptive)
    b.run()
    rc, codes, steps = b.status()
    stats = b.adaptive_stats() if adaptive is not None else None
    b.close()
    return rc, codes, stats


@pytest.mark.parametrize("parts", [2, 3, 13, 255])
def test_split_matches_oracle(lr, parts):
    """Packed trajectories split over `parts` workgroups each (ragged layer ranges; more parts than
    layers gives one layer per part; a one-layer model runs as one part), mixed shapes and ranks in one
    cooperative launch, a drive-frame stepwise pulse, against the oracle."""
    import torch
    items = _batch_items(lr, BATCH_SPECS)
    m = I.readout_model(3, 7, 4).replace(kappa_f=0.5, gamma_1=0.05)
    p = _stepwise(20, 83).replace(frame=1)
    B0 = I.initial_state(m, 4, "e", seed=84, scale=1e-3)
    items.append(dict(model=m, M=4, pulse=p, dt=1e-3, nsteps=203, B0=B0, B=lr.to_device(B0), obs_stride=7,
                      obs=torch.zeros((203 // 7 + 1, 6 + 3), dtype=torch.float64, device="cuda")))
    m1 = I.readout_model(4, 1, 5).replace(kappa_f=0.5, gamma_1=0.05)
    B1 = I.initial_state(m1, 3, "g", seed=85, scale=1e-2)
    items.append(dict(model=m1, M=3, pulse=p, dt=1e-3, nsteps=90, B0=B1, B=lr.to_device(B1), obs_stride=30,
                      obs=torch.zeros((4, 6 + 4), dtype=torch.float64, device="cuda")))
    rc, codes, _ = _run_split(lr, items, parts)
    assert rc == lr.LR_OK, codes
    for it in items:
        Bo, ref, tol = oracle_with_tol(it["model"], it["pulse"], 0.0, it["dt"], it["nsteps"], it["B0"],
                                       it["obs_stride"])
        err = np.max(np.abs(lr.from_device(it["B"]) - Bo))
        what = f"split x{parts} dims {it['model'].d_q, it['model'].d_r, it['model'].d_f} M={it['M']}"
        print(f"[parity] {what}: |dB| {err:.3e}")
        assert err <= 1e-10
        if it["obs_stride"]:
            _assert_obs(it["obs"].cpu().numpy(), ref, what, tol)


@pytest.mark.parametrize("parts", [2, 5, 255])
def test_split_model_kinds_1_2_match_oracle(lr, parts):
    """The paper's Hamiltonian with the transmon in its eigenbasis (kind 1) and in the normal-mode basis
    (kind 2: the cross-layer term Q across every part boundary, one-layer parts at 255), split over
    `parts` workgroups, both frames, against the oracle."""
    from paper_2508_18114_amd import transmon
    small1 = transmon.paper_model(4, 6, 4).replace(kappa_f=0.5, gamma_1=0.05, g=0.9, G=0.4)
    small2 = _nm_model(4, 7, 4, J=1.1, kappa_f=0.6, gamma_1=0.05, g=0.9)
    paper2 = _nm_model(5, 14, 4)
    pw = I.stepwise_pulse(I.ghz(0.15) * np.array([1.0, 1.0j, 0.7]), 0.5, sigma=0.05, w_d=transmon.PAPER_W_DRIVE)
    cases = [(small1, 4, _stepwise(8, 102, T=0.3).replace(w_d=transmon.PAPER_W_DRIVE), 1e-3, 240, 40),
             (small1, 4, _stepwise(8, 103, T=0.3).replace(w_d=transmon.PAPER_W_DRIVE, frame=1), 1e-3, 240, 40),
             (small2, 4, _stepwise(8, 202, T=0.3).replace(w_d=transmon.PAPER_W_DRIVE), 1e-3, 240, 40),
             (small2, 4, _stepwise(8, 203, T=0.3).replace(w_d=transmon.PAPER_W_DRIVE, frame=1), 1e-3, 240, 40),
             (paper2, 8, pw.replace(frame=1), 5e-4, 600, 100)]
    items = [_tm_items(lr, m, M, p, dt, n, s) for (m, M, p, dt, n, s) in cases]
    rc, codes, _ = _run_split(lr, items, parts)
    assert rc == lr.LR_OK, codes
    for it in items:
        Bo, ref, tol = oracle_with_tol(it["model"], it["pulse"], 0.0, it["dt"], it["nsteps"], it["B0"],
                                       it["obs_stride"])
        _assert_obs(it["obs"].cpu().numpy(), ref,
                    f"split x{parts} kind {it['model'].kind} dims {it['model'].d_q, it['model'].d_r, it['model'].d_f} "
                    f"frame {it['pulse'].frame}", tol)
        assert np.max(np.abs(lr.from_device(it["B"]) - Bo)) <= 1e-10


@pytest.mark.parametrize("parts", [2, 255])
def test_split_adaptive_matches_oracle(lr, parts):
    """Adaptive Dormand-Prince steps of split trajectories (kinds 0, 1 and 2; the error norm summed over
    the parts), against the oracle's adaptive integration: step counts within 3 and the records."""
    from oracle import adaptive
    from paper_2508_18114_amd import transmon
    it0 = _adaptive_case(lr, I.FRAME_DRIVE)
    m1 = transmon.paper_model(4, 8, 4).replace(kappa_f=0.3, gamma_1=0.02)
    p1 = I.stepwise_pulse(I.ghz(0.15) * np.array([1.0j, 0.8j]), 1.0, sigma=0.1,
                          w_d=transmon.PAPER_W_DRIVE).replace(frame=1)
    it1 = _tm_items(lr, m1, 4, p1, 0.1, 10, 2)
    m2 = _nm_model(4, 8, 3, J=1.1, kappa_f=0.4, gamma_1=0.02, g=0.8)
    it2 = _tm_items(lr, m2, 4, p1, 0.1, 8, 2, seed=238)
    items = [it0, it1, it2]
    rc, codes, (acc, rej) = _run_split(lr, items, parts, adaptive=(1e-9, 1e-12))
    assert rc == lr.LR_OK, codes
    for k, it in enumerate(items):
        _, ref, acc_o, rej_o = adaptive.integrate(it["model"], it["pulse"], 0.0, it["dt"], it["nsteps"], it["B0"],
                                                  1e-9, 1e-12, obs_stride=it["obs_stride"])
        what = f"split x{parts} adaptive kind {it['model'].kind}"
        print(f"[parity] {what}: steps gpu {acc[k]}+{rej[k]}, oracle {acc_o}+{rej_o}")
        got = it["obs"].cpu().numpy()
        if it["model"].kind == 0:  # the case of test_adaptive_matches_oracle: records to 1e-7
            scale = max(1.0, np.max(np.abs(ref[:, 0:4])))
            assert np.max(np.abs(got[:, 0:4] - ref[:, 0:4])) / scale <= 1e-7
            assert np.max(np.abs(got[:, 4:] - ref[:, 4:])) <= 1e-7
        else:
            _assert_obs(got, ref, what)
        assert abs(acc[k] - acc_o) <= 3 and abs(rej[k] - rej_o) <= 3


def test_split_paper_size_matches_oracle(lr):
    """Paper size (N = 2000, M = 20), g and e split over 25 workgroups each (two layers per part), the
    first 6000 RK4 steps against the cached oracle run with the paper-size floor tolerances; and 2 ns of
    adaptive steps in the drive frame over 50 parts against the cached adaptive oracle run."""
    import torch
    trajs = I.config_paper_size()
    gd = _golden("paper_size")
    tol = _golden_tol("paper_size")
    stride, n = int(gd["stride"]), 6000
    items = [dict(model=t.model, M=t.M, pulse=t.pulse, dt=t.dt, nsteps=n, B=lr.to_device(t.B0()),
                  obs_stride=stride, obs=torch.zeros((n // stride + 1, 6 + t.model.d_q), dtype=torch.float64,
                                                     device="cuda"))
             for t in trajs]
    rc, codes, _ = _run_split(lr, items, 25)
    assert rc == lr.LR_OK, codes
    for it, key in zip(items, ("obs_g", "obs_e")):
        _assert_obs(it["obs"].cpu().numpy(), gd[key][:n // stride + 1], f"split x25 paper size {key} (3 ns)", tol)
    ga = np.load(os.path.join(HERE, "golden", "adaptive_paper_size.npz"))
    dt, n, stride = float(ga["dt"]), int(ga["nsteps"]), int(ga["stride"])
    items = [dict(model=t.model, M=t.M, pulse=t.pulse.replace(frame=I.FRAME_DRIVE), dt=dt, nsteps=n,
                  B=lr.to_device(t.B0()), obs_stride=stride,
                  obs=torch.zeros((n // stride + 1, 6 + t.model.d_q), dtype=torch.float64, device="cuda"))
             for t in trajs]
    rc, codes, (acc, rej) = _run_split(lr, items, 50, adaptive=(float(ga["rtol"]), float(ga["atol"])))
    assert rc == lr.LR_OK, codes
    for k, (it, key) in enumerate(zip(items, ("g", "e"))):
        e = _obs_errors(it["obs"].cpu().numpy(), ga["obs_" + key])
        print(f"[adaptive] split x50 paper size 2 ns drive frame {key}: gpu {acc[k]} + {rej[k]} rejected, oracle "
              f"{int(ga['acc_' + key])} + {int(ga['rej_' + key])}; field err {e['field']:.3e}, populations err "
              f"{e['pop']:.3e}")
        assert abs(acc[k] - int(ga["acc_" + key])) <= 3 and abs(rej[k] - int(ga["rej_" + key])) <= 3
        assert e["field"] <= 1e-9 and e["pop"] <= 1e-9 and e["trace"] <= 1e-9


def test_split_rejections_and_graph(lr):
    """A split batch refuses graph capture (cooperative launches); reduced-precision trajectories stay
    one workgroup each in a split batch; unknown adaptive flags are refused."""
    import torch
    m = I.readout_model(4, 6, 5)
    p = I.flattop_pulse(0.05, 0.1, t_ramp=0.02)
    b = lr.Batch([dict(model=m, M=4, pulse=p, dt=1e-3, nsteps=10, B=lr.to_device(I.initial_state(m, 4, "e", 1)))],
                 packed=True, parts=3, stream=torch.cuda.Stream())
    with pytest.raises(lr.LrError):
        b.graph(True)
    b.close()
    its = [dict(model=m, M=6, pulse=p, dt=1e-3, nsteps=30, precision=prec,
                B=lr.to_device(I.initial_state(m, 6, "e", 92, scale=1e-2))) for prec in (0, 1)]
    rc, codes, _ = _run_split(lr, its, 3)
    assert rc == lr.LR_OK, codes
    with pytest.raises(lr.LrError):
        lr.Batch([_adaptive_case(lr, I.FRAME_DRIVE)], adaptive=(1e-8, 1e-11), flags=lr.LR_BATCH_PACKED_MFMA64)
