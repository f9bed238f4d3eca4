"""Throughput benchmark of the low-rank Lindblad RK4 integrator on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Workload: the paper-size readout case -- dims (d_q, d_r, d_f) = (8, 50, 5)
(N = 2000), rank M = 20, dt = 5e-4 ns, FP64, two trajectories (transmon
initially in g and in e) with the seeded flat-top drive, integrated together
as one batch (one cooperative launch of the persistent kernel).  One bench
step is one RK4 step of both trajectories; inputs are resident in HBM before
the timed region.  Prints one JSON line (metric: RK steps x trajectories / s).

The JSON also carries
  roofline      -- the persistent kernel k_persist (the whole RK4 path runs
                   inside it): algorithmic FP64 flops per launch / its mean
                   launch duration, timed with HIP events on its stream during
                   the timed region, against the FP64 vector peak
  cpu_baseline  -- the FP64 numpy oracle on a bounded sample of the same
                   workload on the host cores.
"""
import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-compare", action="store_true", help="skip the batched / single / dense comparisons")
    ap.add_argument("--cpu-steps", type=int, default=2000, help="oracle steps per trajectory in the CPU sample")
    ap.add_argument("--packed-sample", type=int, default=0, metavar="STEPS",
                    help="only run the packed schedule on 512 trajectories (N=2000, M=20) for STEPS steps "
                         "(a workload for kernel profiles) and print its rate")
    ap.add_argument("--packed-precision", type=int, default=0, choices=(0, 1, 2),
                    help="with --packed-sample: arithmetic of the Gram terms (0 FP64, 1 FP32, 2 BF16x3)")
    ap.add_argument("--packed-mfma64", action="store_true",
                    help="with --packed-sample: FP64 Gram terms on the matrix cores instead of the vector ALU")
    ap.add_argument("--paper-setup", type=int, default=0, metavar="PULSES",
                    help="only run the paper's own set-up (normal-mode basis, N=2000, M=20, drive frame, "
                         "tau=40 ns, adaptive steps) alone and for PULSES pulses x g/e, and print wall times")
    ap.add_argument("--paper-spsa", type=int, default=0, metavar="EPOCHS",
                    help="only run EPOCHS steps of the paper's SPSA loop on its own set-up (normal-mode basis, "
                         "N=2000, M=20, drive frame, tau=40 ns, adaptive steps; four trajectories per step, each "
                         "split over 50 workgroups) and print the wall time per step and the losses")
    ap.add_argument("--paper-setup-parts", type=int, default=100, metavar="P",
                    help="workgroups per trajectory of the lone g/e pair of --paper-setup (layer-split packed "
                         "kernel; 1: one workgroup)")
    ap.add_argument("--config4-subset", type=int, default=0, metavar="PULSES",
                    help="only run configuration 4 to completion on a stratified subset (PULSES pulses x g/e "
                         "per (d_r, M) stratum) and print its rate")
    ap.add_argument("--serving", type=int, default=0, metavar="REQUESTS",
                    help="only run the serving form on REQUESTS loss evaluations of the uncapped serving workload "
                         "(saturation, 50/s, 0.7 x capacity) and print its summary")
    ap.add_argument("--serving-only", choices=("saturation", "literal", "sub"), default=None,
                    help="with --serving: run one scenario only")
    ap.add_argument("--serving-policy", choices=("hybrid", "spread", "packed"), default="spread",
                    help="with --serving: schedule of the requests")
    ap.add_argument("--serving-layers", type=int, default=4,
                    help="with --serving: resonator layers per workgroup of the spread schedule")
    ap.add_argument("--serving-capacity", type=float, default=None, metavar="EVALS_PER_S",
                    help="with --serving-only sub: the capacity measured by a saturation run")
    ap.add_argument("--apply-sample", type=int, default=0, metavar="LAUNCHES",
                    help="only time the operator application lr_apply_heff on 512 factors of N=2000, M=20 "
                         "(10240 columns) for LAUNCHES launches (a workload for kernel profiles)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device three times (the reference that HBM byte "
                         "counters are calibrated against) and print the rate")
    return ap.parse_args()


def copy_calibration(torch, mib):
    """A plain device copy of a known size: FETCH_SIZE / WRITE_SIZE read for it give the factors that turn
    the counters into bytes moved."""
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        t0 = time.perf_counter()
        y.copy_(x)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(json.dumps({"copy_mib": mib, "ms": el * 1e3, "gb_per_s_read_plus_write": 2 * mib * (1 << 20) / el / 1e9}),
              flush=True)


def packed_sample(lr, I, torch, steps, precision=0, mfma64=False):
    """512 trajectories (256 piecewise pulses x g/e, N=2000, M=20) in the packed schedule, kernel time
    from HIP events on the batch stream; precision: arithmetic of the Gram terms (FP32 / BF16x3 on the
    matrix cores), mfma64: FP64 Gram terms on the matrix cores instead of the vector ALU."""
    tl = I.batch_uniform(256)
    # the reduced modes need the rank padding above their rounding: the paper's padding weight
    items = [dict(model=t.model, M=t.M, pulse=t.pulse, dt=t.dt, nsteps=steps, precision=precision,
                  B=lr.to_device(t.B0(I.PAPER_PAD_SCALE if precision else None))) for t in tl]
    b = lr.Batch(items, packed=True, flags=lr.LR_BATCH_PACKED_MFMA64 if mfma64 else 0)
    b.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if b.status()[0] != lr.LR_OK:
        raise RuntimeError("packed sample failed")
    ms, launches = b.profile_read()
    b.close()
    m, M = tl[0].model, tl[0].M
    fl = 4 * m.N * M * (58 + 40 * M) * steps * len(items)
    valu = precision == 0 and not mfma64
    kern = "k_packed<5>" if valu else ("k_packed_mg<%d>" % precision)
    print(json.dumps({"workload": f"packed schedule, {len(items)} trajectories, N={m.N}, M={M}, {steps} steps, "
                                  f"precision {precision}, Gram terms on the {'vector ALU' if valu else 'matrix cores'}",
                      "value": len(items) * steps / el, "unit": "RK steps*trajectories/s",
                      "kernel": kern, "kernel_ms": ms, "launches": launches,
                      "achieved_tflops": fl / (ms * 1e-3) / 1e12, "peak": 78.6}), flush=True)


def apply_sample(lr, I, torch, launches):
    """Operator application Z = H_eff(t) B on its own (lr_apply_heff) over 512 factors of the paper-size
    model side by side (N=2000, 10240 columns: 328 MB in, 328 MB out), timed with HIP events on the
    launch stream; HBM roofline from the algorithmic bytes (one read of B, one write of Z)."""
    m = I.readout_model(8, 50, 5)
    p = I.config_paper_size()[0].pulse
    ncols = 512 * 20
    gen = torch.Generator(device="cuda").manual_seed(3)
    B = torch.randn((ncols, m.N), dtype=torch.complex128, device="cuda", generator=gen)
    Z = torch.empty_like(B)
    for _ in range(3):
        lr.apply_heff(m, p, 1.0, B, Z)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(launches):
        lr.apply_heff(m, p, 1.0 + 1e-3 * k, B, Z)
    e1.record()
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / launches
    by = 32.0 * m.N * ncols
    return {"bound": "hbm", "achieved": by / (us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": by / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, "traffic": measured_apply_traffic_per_launch(),
            "kernel": "k_apply_heff", "kernel_mean_us": us,
            "bytes_per_launch": by, "launches": launches,
            "workload": f"Z = H_eff(t) B for 512 factors of N={m.N}, M=20 side by side ({ncols} columns), lab frame"}


def _oracle_worker(args):
    idx, nsteps = args
    from threadpoolctl import threadpool_limits
    from oracle import lowrank
    from paper_2508_18114_amd import inputs as I
    tr = I.config_paper_size()[idx]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        lowrank.integrate(tr.model, tr.pulse, 0.0, tr.dt, nsteps, tr.B0(), obs_stride=0)
        return time.perf_counter() - t0


def cpu_baseline(nsteps):
    """Oracle (plain numpy FP64, one BLAS thread per process), g and e in two processes."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(2) as pool:
        pool.map(_oracle_worker, [(0, nsteps), (1, nsteps)])
    wall = time.perf_counter() - t0
    return {"value": 2 * nsteps / wall, "unit": "RK steps*trajectories/s", "cores": 2, "kind": "oracle",
            "sample": f"{nsteps} RK4 steps of each of the g and e trajectories at N=2000, M=20 "
                      f"(one process and one BLAS thread each; {wall:.1f} s wall incl. process start)"}


def comparisons(lr, I, torch, stream, plain_value):
    """Throughput of the other forms on the same GPU (bounded samples)."""
    import numpy as np
    out = {}
    trajs = I.config_paper_size()
    m, M = trajs[0].model, trajs[0].M

    def run_batch(tr_list, nsteps_cap, packed=False, precision=0, flags=0):
        items = [dict(model=t.model, M=t.M, pulse=t.pulse, dt=t.dt, nsteps=min(t.nsteps, nsteps_cap),
                      B=lr.to_device(t.B0(I.PAPER_PAD_SCALE if precision else None)), precision=precision)
                 for t in tr_list]
        b = lr.Batch(items, stream=stream, packed=packed, flags=flags)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rc, codes, _ = b.status()
        b.close()
        if rc != lr.LR_OK:
            raise RuntimeError(f"batch failed: {lr.lr_strerror(rc)}")
        return sum(it["nsteps"] for it in items) / el, el

    # operator application on its own, 512 factors of N=2000, M=20 (HBM-bound streaming pass)
    out["operator_application"] = apply_sample(lr, I, torch, 20)
    # plain single trajectory (one Context, trajectory g)
    steps = 2000
    ctx = lr.Context(m, M, stream=stream)
    B = lr.to_device(trajs[0].B0())
    ctx.integrate(trajs[0].pulse, 0.0, trajs[0].dt, 200, B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.integrate(trajs[0].pulse, 0.0, trajs[0].dt, steps, B)
    torch.cuda.synchronize()
    single = steps / (time.perf_counter() - t0)
    ctx.close()
    out["plain_single"] = {"value": single, "unit": "RK steps*trajectories/s",
                           "workload": f"one trajectory (g), N={m.N}, M={M}, {steps} steps"}
    # batched, same shape: 16 piecewise pulses x {g, e} at N=2000, M=20
    npulse, steps = 16, 1000
    v, el = run_batch(I.batch_uniform(npulse), steps)
    out["batched_same_shape"] = {"value": v, "unit": "RK steps*trajectories/s",
                                 "vs_plain_g_e": v / plain_value, "vs_plain_single": v / single,
                                 "workload": f"{2 * npulse} trajectories ({npulse} piecewise pulses x g/e), "
                                             f"N=2000, M=20, {steps} steps each, one batch ({el:.2f} s)"}
    vp, elp = run_batch(I.batch_uniform(npulse), steps, packed=True)
    out["batched_same_shape_packed"] = {"value": vp, "unit": "RK steps*trajectories/s", "vs_spread": vp / v,
                                        "workload": f"as batched_same_shape, packed schedule ({elp:.2f} s)"}
    # 512 trajectories of one shape (256 pulses x g/e, N=2000, M=20): spread vs packed schedule
    n512 = I.batch_uniform(256)
    v_s, el_s = run_batch(n512, 40)
    v_p, el_p = run_batch(n512, 200, packed=True)
    # the same with the FP64 Gram terms on the matrix cores, and the reduced modes (Gram terms on the matrix cores)
    v_pm, _ = run_batch(n512, 200, packed=True, flags=lr.LR_BATCH_PACKED_MFMA64)
    v_p32, _ = run_batch(n512, 200, packed=True, precision=1)
    v_pbf, _ = run_batch(n512, 200, packed=True, precision=2)
    # algorithmic FP64 flops per RK step and trajectory (same count as the main line's roofline)
    fl = 4 * m.N * M * (58 + 40 * M)
    by = 17 * 16 * m.N * M
    out["batched_512_same_shape"] = {
        "spread": v_s, "packed": v_p, "packed_vs_spread": v_p / v_s, "packed_vs_plain_g_e": v_p / plain_value,
        "packed_fp64_mfma_gram": v_pm, "packed_fp32_gram": v_p32, "packed_bf16x3_gram": v_pbf,
        "packed_roofline": {"bound": "alu", "achieved": v_p * fl / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                            "frac": v_p * fl / 1e12 / 78.6,
                            "note": "whole-batch wall time (launch overhead and the prologue included)"},
        # the HBM side of the same run: 17 passes of 16 N M bytes per trajectory-step
        # (stage input 4, B_n and accumulator reads 6, stage output 4, accumulator writes 3)
        "packed_hbm": {"bound": "hbm", "achieved": v_p * by / 1e9, "peak": 8000.0, "unit": "GB/s",
                       "frac": v_p * by / 1e9 / 8000.0, "algorithmic_bytes_per_traj_step": by,
                       "traffic_per_traj_step": measured_packed_traffic_per_traj_step()},
        "unit": "RK steps*trajectories/s",
        "workload": f"512 trajectories (256 piecewise pulses x g/e), N=2000, M=20; spread: first 40 steps "
                    f"({el_s:.2f} s), packed: first 200 steps ({el_p:.2f} s)"}
    # HIP graph replay of a packed batch with many short chunks (records every 10 steps)
    gl = I.batch_uniform(64)
    gsteps, gstride = 400, 10
    gitems = [dict(model=t.model, M=t.M, pulse=t.pulse, dt=t.dt, nsteps=gsteps, B=lr.to_device(t.B0()),
                   obs_stride=gstride, obs=torch.zeros((gsteps // gstride + 1, 6 + t.model.d_q),
                                                       dtype=torch.float64, device="cuda")) for t in gl]
    gb = lr.Batch(gitems, stream=torch.cuda.Stream(), packed=True)  # a capturable stream
    gt = {}
    for mode in ("eager", "graph"):
        if mode == "graph":
            gb.graph(True)
            gb.run()  # capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            gb.run()
        torch.cuda.synchronize()
        gt[mode] = (time.perf_counter() - t0) / 3
        if gb.status()[0] != lr.LR_OK:
            raise RuntimeError("graph comparison failed")
    gb.close()
    out["graph_replay_packed"] = {"eager_s": gt["eager"], "graph_s": gt["graph"],
                                  "speedup": gt["eager"] / gt["graph"],
                                  "workload": f"{len(gitems)} packed trajectories, N=2000, M=20, {gsteps} steps, "
                                              f"records every {gstride} steps ({gsteps // gstride} chunks)"}
    # the paper's Hamiltonian (transmon eigenbasis, N_t = 6 levels; bare resonator 60 x filter 10,
    # N = 3600), 256 seeded stepwise pulses x g/e in the packed schedule
    from paper_2508_18114_amd import transmon
    pm = transmon.paper_model(6, 60, 10)
    rng = np.random.default_rng(11)
    pitems = []
    for k in range(256):
        hts = I.ghz(0.15) * rng.uniform(0.3, 1.0, 4) * np.exp(1j * rng.uniform(0, 2 * np.pi, 4))
        pp = I.stepwise_pulse(hts, 40.0, w_d=transmon.PAPER_W_DRIVE)
        for which in ("g", "e"):
            pitems.append(dict(model=pm, M=20, pulse=pp, dt=5e-4, nsteps=100,
                               B=lr.to_device(I.initial_state(pm, 20, which, 12 + k, I.PAPER_PAD_SCALE))))
    pb = lr.Batch(pitems, stream=stream, packed=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pb.run()
    torch.cuda.synchronize()
    pel = time.perf_counter() - t0
    if pb.status()[0] != lr.LR_OK:
        raise RuntimeError("paper model batch failed")
    pb.close()
    del pitems
    out["paper_model_packed"] = {"value": 512 * 100 / pel, "unit": "RK steps*trajectories/s",
                                 "workload": "the paper's Hamiltonian (transmon eigenbasis N_t=6, resonator 60, "
                                             "filter 10: N=3600), M=20, 256 stepwise pulses x g/e, 100 steps "
                                             f"each, packed schedule ({pel:.2f} s)"}
    # the paper's Hamiltonian in its normal-mode basis at the paper's own size (N_t = 5, lower mode 100,
    # upper mode 4: N = 2000), M = 20, in the frame rotating at the drive; 256 pulses x g/e
    nm = transmon.paper_model_normal(5, 100, 4)
    nitems = []
    for k in range(256):
        hts = I.ghz(0.15) * rng.uniform(0.3, 1.0, 4) * np.exp(1j * rng.uniform(0, 2 * np.pi, 4))
        pp = I.stepwise_pulse(hts, 40.0, w_d=transmon.PAPER_W_DRIVE).replace(frame=I.FRAME_DRIVE)
        for which in ("g", "e"):
            nitems.append(dict(model=nm, M=20, pulse=pp, dt=2e-3, nsteps=100,
                               B=lr.to_device(I.initial_state(nm, 20, which, 300 + k, I.PAPER_PAD_SCALE))))
    nb = lr.Batch(nitems, stream=stream, packed=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nb.run()
    torch.cuda.synchronize()
    nel = time.perf_counter() - t0
    if nb.status()[0] != lr.LR_OK:
        raise RuntimeError("normal-mode model batch failed")
    nb.close()
    del nitems
    out["paper_model_normal_packed"] = {"value": 512 * 100 / nel, "unit": "RK steps*trajectories/s",
                                        "workload": "the paper's Hamiltonian in its normal-mode basis at its own "
                                                    "size (N_t=5, lower mode 100, upper mode 4: N=2000), M=20, drive "
                                                    "frame, 256 stepwise pulses x g/e, 100 steps each, packed "
                                                    f"schedule ({nel:.2f} s)"}
    # batched mixed shapes: the 512 trajectories of the batched configuration, capped step count
    steps = 150
    c4 = I.config_batched()
    v, el = run_batch(c4, steps)
    vp, elp = run_batch(c4, steps, packed=True)
    from paper_2508_18114_amd import autotune
    titems = [dict(model=t.model, M=t.M, pulse=t.pulse, dt=t.dt, nsteps=min(t.nsteps, steps),
                   B=lr.to_device(t.B0())) for t in c4]
    tch = autotune.tune(titems, steps=10, stream=stream)
    out["autotune_c4"] = {"choice": f'{tch["schedule"]} (tile height {tch["layers"]})' if tch["schedule"] == "spread"
                          else "packed", "rates_10_steps": tch["rates"],
                          "workload": "the 512 trajectories of the batched configuration, 10 steps per candidate"}
    del titems
    out["batched_mixed_c4_sample"] = {"value": v, "unit": "RK steps*trajectories/s",
                                      "packed": vp, "packed_vs_spread": vp / v,
                                      "workload": f"{len(c4)} trajectories, N in {{1000,1520,2000,3000}}, "
                                                  f"M in [8,32], first {steps} steps of each (spread "
                                                  f"{el:.2f} s, packed {elp:.2f} s)"}
    # dense full-Lindblad RK4 at the same N, dt
    N = m.N
    rho = torch.zeros((N, N), dtype=torch.complex128, device="cuda")
    n0 = I.basis_index(m, 0, 0, 0)
    rho[n0, n0] = 1.0
    ws = lr.dense_integrate(m, trajs[0].pulse, 0.0, trajs[0].dt, 2, rho)
    dsteps = 20
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lr.dense_integrate(m, trajs[0].pulse, 0.0, trajs[0].dt, dsteps, rho, workspace=ws)
    torch.cuda.synchronize()
    dms = 1e3 * (time.perf_counter() - t0) / dsteps
    nfull = trajs[0].nsteps
    out["dense_lindblad_gpu"] = {
        "ms_per_step": dms, "unit": "ms per RK4 step (one trajectory)",
        "full_trajectory_s": dms * nfull / 1e3, "lowrank_plain_single_full_trajectory_s": nfull / single,
        "speedup_lowrank_vs_dense": (dms * 1e-3) * single,
        "workload": f"dense rho {N}x{N} FP64, same model/drive/dt, {dsteps} steps timed; full trajectory = "
                    f"{nfull} steps (extrapolated)"}
    # reduced-precision modes (paper padding weight), g + e batch, same step count
    steps = 2000
    for name, prec in (("fp64", 0), ("fp32", 1), ("bf16x3", 2)):
        tl = [dataclasses.replace(t, precision=prec) for t in I.config_paper_size_paper_padding()]
        items = [dict(model=t.model, M=t.M, pulse=t.pulse, dt=t.dt, nsteps=steps, precision=prec,
                      B=lr.to_device(t.B0())) for t in tl]
        b = lr.Batch(items, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if b.status()[0] != lr.LR_OK:
            raise RuntimeError(f"precision {name} failed")
        b.close()
        out.setdefault("precision_modes", {})[name] = {
            "value": 2 * steps / el, "unit": "RK steps*trajectories/s",
            "workload": f"g+e, N=2000, M=20, padding weight 1e-5, {steps} steps"}
    out["validity_rank_study"] = validity_study(lr, I, torch)
    out["drive_frame_step_size"] = drive_frame_study(lr, I, torch)
    # serving, a CAPPED sample (12 requests, at most 4000 steps each) that keeps this run short; the
    # uncapped serving workload is `bench.py --serving N`
    out["serving_capped_sample"] = serving(lr, I, torch, stream, 12, cap=4000, progress=False)
    return out


def serving(lr, I, torch, stream, n_req, cap=None, progress=True, only=None, capacity=None, policy="spread",
            spread_layers=4):
    """The serving form on the serving workload: n_req loss evaluations (g + e each) with the serving
    shapes (d_r 13-75, M 4-32, T 10-60 ns at dt 5e-4: 2e4 - 1.2e5 steps, FP32 / FP64), uncapped unless
    cap is given, with asynchronous cost-balanced ticks.  Three runs: saturation (every request at t = 0;
    its throughput gives the capacity), the literal 50 requests/s, and 0.7 x the capacity.  only: one of
    "saturation", "literal", "sub" (with capacity: requests/s from an earlier saturation run).  policy:
    "hybrid" (packed, spread above 60 s of packed time), "spread" or "packed" (every request).  Each run's
    statistics are printed as a JSON line when it ends."""
    import numpy as np
    from paper_2508_18114_amd import serve
    budget = 64 << 30
    steps = [r.nsteps for r in serve.serving_requests(5, n_req, 1.0, step_cap=cap)]
    schedule = {"spread": f"spread schedule ({spread_layers} resonator layers per workgroup)",
                "packed": "packed schedule",
                "hybrid": "packed schedule, spread for requests whose packed duration would exceed 60 s"}[policy]
    workload = (f"{n_req} loss evaluations (g+e each) with the serving shapes (d_r 13-75, M 4-32, FP32/FP64), "
                f"{'step count capped at %d' % cap if cap else 'full step counts'} ({min(steps)}-{max(steps)} "
                f"steps, {sum(steps) * 2:.3g} trajectory-steps), padding weight 1e-5, {schedule}, asynchronous "
                f"cost-balanced ticks (2000 paper-size packed steps), HBM budget {budget >> 30} GiB")

    def serve_run(rate, label):
        reqs = serve.serving_requests(5, n_req, rate, step_cap=cap)
        t0 = time.perf_counter()

        def on_tick(srv):
            if progress:
                done = sum(1 for res in srv.results.values() if "done" in res)
                print(f"[serving {label}] tick {srv.ticks} completed at {time.perf_counter() - t0:.1f} s: "
                      f"{len(srv.active) // 2} active, {len(srv.queue)} queued, {done} done, "
                      f"{srv.steps_done} trajectory-steps", file=sys.stderr, flush=True)

        srv = serve.Server(hbm_budget_bytes=budget, chunk=2000, stream=stream, on_tick=on_tick,
                           packed=policy != "spread", max_packed_s=float("inf") if policy == "packed" else 60.0,
                           spread_layers=spread_layers)

        def on_result(rid, res):
            if progress:
                print(f"[serving {label}] request {rid} arrival {res['arrival']:.1f} s latency "
                      f"{res.get('latency', float('nan')):.1f} s", file=sys.stderr, flush=True)

        st = srv.run(reqs, on_result=on_result)
        st["offered_rate_per_s"] = rate
        st["routed_spread"] = sum(1 for r in reqs if not srv._packs(r))
        if progress:
            print(json.dumps({"serving_run": label, **st, "workload": workload}), flush=True)
        return st

    out = {"capped": cap is not None, "workload": workload, "policy": policy, "spread_layers": spread_layers}
    if only in (None, "saturation"):
        out["saturation"] = sat = serve_run(1e9, "saturation")
        capacity = sat["requests"] / sat["wall_s"]
    if capacity is not None:
        out["capacity_evals_per_s"] = capacity
    if only in (None, "literal"):
        out["literal_50_per_s"] = serve_run(50.0, "50/s")
    if only in (None, "sub"):
        if capacity is None:
            raise ValueError("the 0.7 x capacity run needs the capacity of a saturation run")
        out["sub_saturation_0.7x"] = serve_run(0.7 * capacity, "0.7x capacity")
    return out


def config4_subset(lr, I, torch, per_stratum):
    """Configuration 4 run to completion on a stratified subset: the 512 trajectories (256 pulses x g/e)
    fall into 12 strata (d_r in {25, 38, 50, 75} x M in 8-15, 16-23, 24-32); the first per_stratum
    pulses of each stratum (with both g and e) are integrated over their whole step counts in one
    batch (spread schedule: with a few dozen trajectories one workgroup per layer is the faster form).
    Reports the rate beside the whole configuration's step total."""
    import numpy as np
    allt = I.config_batched()
    strata = {}
    for k in range(0, len(allt), 2):
        t = allt[k]
        key = (t.model.d_r, 0 if t.M < 16 else (1 if t.M < 24 else 2))
        strata.setdefault(key, []).append(k)
    pick = []
    for key in sorted(strata):
        for k in strata[key][:per_stratum]:
            pick += [allt[k], allt[k + 1]]
    items = [dict(model=t.model, M=t.M, pulse=t.pulse, dt=t.dt, nsteps=t.nsteps, B=lr.to_device(t.B0()))
             for t in pick]
    b = lr.Batch(items)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rc, codes, _ = b.status()
    b.close()
    if rc != lr.LR_OK:
        raise RuntimeError(f"config 4 subset failed: {lr.lr_strerror(rc)}")
    steps = sum(t.nsteps for t in pick)
    total = sum(t.nsteps for t in allt)
    return {"value": steps / el, "unit": "RK steps*trajectories/s", "wall_s": el, "trajectories": len(pick),
            "trajectory_steps": steps, "config4_trajectory_steps": total,
            "strata": {f"d_r={k[0]},M-bin={k[1]}": len(v) for k, v in sorted(strata.items())},
            "workload": f"stratified subset of configuration 4: {per_stratum} pulse(s) x g/e from each of the "
                        f"{len(strata)} (d_r, M) strata, {len(pick)} trajectories to completion "
                        f"({steps:.3g} of the configuration's {total:.3g} trajectory-steps), spread schedule"}


def paper_setup(lr, I, torch, n_pulses, rtol=1e-8, atol=1e-10, parts=100):
    """The paper's own set-up end to end: its Hamiltonian in the resonator-filter normal-mode basis at
    its size (N_t = 5, lower mode 100, upper mode 4: N = 2000), M = 20, the frame rotating at the
    drive, tau = 40 ns, adaptive Dormand-Prince steps.  n_pulses stepwise pulses (the square start of
    the SPSA loop and seeded variations of it) x g/e in one packed adaptive batch; also one pulse (g and
    e) alone, each trajectory split over `parts` workgroups (layer ranges), and one workgroup per
    trajectory in the batch.  Context only: the paper's figure for this workload is a CPU wall time per
    trajectory."""
    import numpy as np
    from paper_2508_18114_amd import serve, transmon
    nm = transmon.paper_model_normal(5, 100, 4)
    rng = np.random.default_rng(21)
    T, nh, grid = 40.0, 4, 0.5

    nseg = 8  # tau in segments of 5 ns (one adaptive batch each, continuing the state; progress lines)

    def run(npulse, label, split=0):
        items = []
        for k in range(npulse):
            theta = serve.square_start(nm, nh) * (1.0 + (0.3 * rng.uniform(-1, 1, 2 * nh) if k else 0.0))
            pp = I.stepwise_pulse(serve.heights_from(theta), T, sigma=0.5,
                                  w_d=transmon.PAPER_W_DRIVE).replace(frame=I.FRAME_DRIVE)
            for which in ("g", "e"):
                items.append(dict(model=nm, M=20, pulse=pp, dt=grid, nsteps=int(T / grid) // nseg, obs_stride=1,
                                  B=lr.to_device(I.initial_state(nm, 20, which, 700 + k, I.PAPER_PAD_SCALE))))
        el, acc_t, rej_t = 0.0, np.zeros(len(items)), np.zeros(len(items))
        for seg in range(nseg):
            for it in items:
                it["step0"] = seg * it["nsteps"]
                it["obs"] = torch.zeros((it["nsteps"] + 1, 6 + nm.d_q), dtype=torch.float64, device="cuda")
            b = lr.Batch(items, packed=True, adaptive=(rtol, atol), parts=split)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.run()
            torch.cuda.synchronize()
            el += time.perf_counter() - t0
            rc, codes, _ = b.status()
            acc, rej = b.adaptive_stats()
            b.close()
            if rc != lr.LR_OK:
                raise RuntimeError(f"paper set-up failed: {lr.lr_strerror(rc)}")
            acc_t += np.asarray(acc)
            rej_t += np.asarray(rej)
            print(f"[paper set-up {label}] {(seg + 1) * T / nseg:.0f} ns done, {el:.1f} s, steps per trajectory "
                  f"{np.mean(acc_t):.0f} accepted + {np.mean(rej_t):.0f} rejected", file=sys.stderr, flush=True)
        return el, float(np.mean(acc_t)), float(np.mean(rej_t))

    el1, a1, r1 = run(1, f"one pulse, {parts} parts per trajectory", parts)
    eln, an, rn = run(n_pulses, f"{n_pulses} pulses")
    return {"single_pair_wall_s": el1, "single_pair_steps": [a1, r1], "single_pair_parts": parts,
            "batch_trajectories": 2 * n_pulses, "batch_wall_s": eln, "batch_steps_mean": [an, rn],
            "batch_wall_per_trajectory_s": eln / (2 * n_pulses),
            "workload": f"the paper's Hamiltonian in its normal-mode basis, N_t=5, lower mode 100, upper mode 4 "
                        f"(N=2000), M=20, drive frame, tau=40 ns, adaptive Dormand-Prince (rtol {rtol}, atol "
                        f"{atol}), records every {grid} ns, in {nseg} batches of {T / nseg:.0f} ns; one pulse x g/e "
                        f"alone ({parts} workgroups per trajectory), and {n_pulses} pulses x g/e in one packed adaptive "
                        f"batch (one workgroup per trajectory)"}


def paper_spsa(lr, I, torch, epochs, parts=50, rtol=1e-8, atol=1e-10):
    """Steps of the paper's optimisation loop (supplement S3.C) on its own set-up: SPSA over the four
    complex heights of the smoothed stepwise pulse from the square start, each step two loss
    evaluations (theta +- c_k Delta) = four trajectories at N = 2000, M = 20 in one adaptive batch, each
    trajectory split over `parts` workgroups.  Context: the paper quotes about 1.2e4 s for O(100)
    epochs of two loss evaluations on a laptop CPU."""
    import numpy as np
    from paper_2508_18114_amd import serve, transmon
    nm = transmon.paper_model_normal(5, 100, 4)
    walls = []
    t_last = [time.perf_counter()]

    def on_step(rec):
        torch.cuda.synchronize()
        now = time.perf_counter()
        walls.append(now - t_last[0])
        t_last[0] = now
        print(f"[paper spsa] step {rec['k']}: {walls[-1]:.1f} s, loss +{rec['loss_plus']:.4f} "
              f"-{rec['loss_minus']:.4f}", file=sys.stderr, flush=True)

    theta, hist = serve.spsa_optimize(nm, 20, 40.0, 4, epochs, 0.5, 1, sigma=0.5, frame=I.FRAME_DRIVE,
                                      w_d=transmon.PAPER_W_DRIVE, adaptive=(rtol, atol), parts=parts,
                                      on_step=on_step)
    return {"epochs": epochs, "wall_per_epoch_s": walls, "mean_wall_per_epoch_s": float(np.mean(walls[1:] or walls)),
            "losses": [[h["loss_plus"], h["loss_minus"]] for h in hist],
            "eps_a": [[h["eps_a_plus"], h["eps_a_minus"]] for h in hist],
            "theta": [float(x) for x in theta], "parts_per_trajectory": parts,
            "workload": f"SPSA (supplement S3.C) on the paper's Hamiltonian in its normal-mode basis (N=2000), M=20, "
                        f"drive frame, tau=40 ns, four stepwise heights, adaptive Dormand-Prince (rtol {rtol}, atol "
                        f"{atol}), records every 0.5 ns; per step four trajectories in one batch, each over {parts} "
                        f"workgroups"}


def validity_study(lr, I, torch):
    """Supplement S1.B on the small readout model (N=200, flat-top drive, 1e4
    steps, padding weight 1e-5): the control quantity p_M/p_1 and the purity
    tr rho^2 / (tr rho)^2 of the low-rank state against the full master
    equation (dense GPU solve, its spectrum from numpy on the host), and the
    SNR and assignment error eps_a of the g/e pair against the full ones, for
    several ranks M.  (The padding adds (M-1) 1e-5 to tr rho, hence the
    normalised purity.)"""
    import numpy as np
    base = I.config_small_paper_padding()
    m, pulse, dt, nsteps = base[0].model, base[0].pulse, base[0].dt, base[0].nsteps
    stride, nck = 100, 5
    ck = nsteps // nck
    cs = ck // stride
    nrec = nsteps // stride + 1

    def full(which):
        n0 = I.basis_index(m, 0 if which == "g" else 1, 0, 0)
        rho = torch.zeros((m.N, m.N), dtype=torch.complex128, device="cuda")
        rho[n0, n0] = 1.0
        obs = torch.zeros((nrec, 6 + m.d_q), dtype=torch.float64, device="cuda")
        ws, ev = None, []
        for k in range(nck):
            ws = lr.dense_integrate(m, pulse, k * ck * dt, dt, ck, rho, stride, obs[k * cs:], workspace=ws)
            ev.append(np.sort(np.linalg.eigvalsh(rho.cpu().numpy()))[::-1])
        return obs, ev

    def lowrank(which, M):
        tr = I.Trajectory(m, M, pulse, which, seed=1, dt=dt, nsteps=nsteps, pad_scale=I.PAPER_PAD_SCALE)
        ctx = lr.Context(m, M)
        Bd = lr.to_device(tr.B0())
        obs = torch.zeros((nrec, 6 + m.d_q), dtype=torch.float64, device="cuda")
        sp = []
        for k in range(nck):
            ctx.integrate(pulse, k * ck * dt, dt, ck, Bd, stride, obs[k * cs:])
            sp.append(ctx.spectrum(Bd).cpu().numpy())
        rc, _ = ctx.status()
        if rc != lr.LR_OK:
            raise RuntimeError(f"validity study M={M}: {lr.lr_strerror(rc)}")
        ctx.close()
        return obs, sp

    h = stride * dt
    fg, evg = full("g")
    fe, eve = full("e")
    ref = lr.readout_loss(fg, fe, m.d_q, h, m.kappa_f, m.gamma_1)
    def npur(w):
        return float(np.sum(w ** 2) / np.sum(w) ** 2)

    out = {"full_eps_a": ref["eps_a"], "full_snr": ref["snr"],
           "checkpoints_ns": [round((k + 1) * ck * dt, 6) for k in range(nck)],
           "full_purity_g": [npur(w) for w in evg],
           "full_purity_e": [npur(w) for w in eve],
           "ranks": {},
           "workload": f"dims (4,10,5) N={m.N}, flat-top drive, dt={dt} ns, {nsteps} steps, g and e; "
                       f"full = dense master equation on the GPU"}
    for M in (2, 4, 8, 16, 32):
        og, spg = lowrank("g", M)
        oe, spe = lowrank("e", M)
        f = lr.readout_loss(og, oe, m.d_q, h, m.kappa_f, m.gamma_1)
        row = {"eps_a": f["eps_a"], "eps_a_rel_err": abs(f["eps_a"] - ref["eps_a"]) / ref["eps_a"],
               "snr": f["snr"], "snr_rel_err": abs(f["snr"] - ref["snr"]) / ref["snr"]}
        for which, sp, ev in (("g", spg, evg), ("e", spe, eve)):
            row[f"pM_over_p1_{which}"] = [float(p[-1] / p[0]) for p in sp]
            row[f"full_pM_over_p1_{which}"] = [float(w[M - 1] / w[0]) for w in ev]
            row[f"purity_rel_dev_{which}"] = [npur(p) / npur(w) - 1.0 for p, w in zip(sp, ev)]
        out["ranks"][str(M)] = row
    return out


def drive_frame_study(lr, I, torch):
    """Step size at equal accuracy, lab frame vs the frame rotating at the drive
    carrier (counter-rotating terms kept): paper-size model (8,50,5), M=20,
    flat-top drive, 10 ns, excited state.  Each run is compared with a
    drive-frame run at dt = 1.25e-4 ns on records every 0.5 ns: <f> (lab
    records turned to the rotating frame by e^{i w_d t}, exact) and the
    transmon populations.  Same kernel cost per step in both frames."""
    import numpy as np
    base = I.config_paper_size()[1]
    m, M = base.model, base.M
    T = 10.0
    lab = base.pulse.replace(T=T)
    rot = lab.replace(frame=I.FRAME_DRIVE)
    B0 = base.B0()

    def run(pulse, dt):
        nsteps = int(round(T / dt))
        stride = int(round(0.5 / dt))
        ctx = lr.Context(m, M)
        Bd = lr.to_device(B0)
        obs = ctx.new_obs(nsteps, stride)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.integrate(pulse, 0.0, dt, nsteps, Bd, stride, obs)
        rc, _ = ctx.status()
        el = time.perf_counter() - t0
        ctx.close()
        o = obs.cpu().numpy()
        tt = np.arange(o.shape[0]) * stride * dt
        f = o[:, 2] + 1j * o[:, 3]
        if pulse.frame == I.FRAME_LAB:
            f = f * np.exp(1j * pulse.w_d * tt)
        return rc, f, o[:, 6:], nsteps / el

    rc, fref, pref, _ = run(rot, 1.25e-4)
    if rc != lr.LR_OK:
        raise RuntimeError("drive frame reference failed")
    scale = float(np.max(np.abs(fref)))
    out = {"workload": f"dims (8,50,5) N={m.N}, M={M}, flat-top {lab.amp / (2 * np.pi):.3f} GHz, T={T} ns, "
                       f"state e; reference: drive frame at dt=1.25e-4 ns",
           "runs": {}}
    best = {}
    for name, pulse in (("lab", lab), ("drive", rot)):
        for dt in (2.5e-4, 5e-4, 1e-3, 2e-3, 4e-3):
            rc, f, pq, sps = run(pulse, dt)
            ok = rc == lr.LR_OK and np.all(np.isfinite(f))
            ef = float(np.max(np.abs(f - fref)) / scale) if ok else None
            ep = float(np.max(np.abs(pq - pref))) if ok else None
            out["runs"][f"{name}_dt{dt:g}"] = {"status": lr.lr_strerror(rc), "field_err_rel": ef,
                                               "population_err": ep, "steps_per_s": sps}
            if ok and ef <= 1e-6 and ep <= 1e-6:
                best[name] = max(best.get(name, 0.0), dt)
    out["largest_dt_ns_at_1e-6"] = best
    if "lab" in best and "drive" in best:
        out["physical_time_speedup_drive_vs_lab"] = best["drive"] / best["lab"]
    # adaptive Dormand-Prince 5(4) steps in the drive frame over the first 2 ns (one packed
    # workgroup), against the same reference records
    ad = {}
    for rtol in (1e-6, 1e-8):
        nrec = 4
        obs = torch.zeros((nrec + 1, 6 + m.d_q), dtype=torch.float64, device="cuda")
        it = dict(model=m, M=M, pulse=rot, dt=0.5, nsteps=nrec, B=lr.to_device(B0), obs_stride=1, obs=obs)
        b = lr.Batch([it], adaptive=(rtol, 1e-2 * rtol))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run()
        rc = b.status()[0]
        el = time.perf_counter() - t0
        acc, rej = b.adaptive_stats()
        o = obs.cpu().numpy()
        f = o[:, 2] + 1j * o[:, 3]
        ok = rc == lr.LR_OK
        ad[f"rtol{rtol:g}"] = {
            "status": lr.lr_strerror(rc), "accepted": acc[0], "rejected": rej[0],
            "rhs_evaluations": 6 * (acc[0] + rej[0]) + 1,
            "field_err_rel": float(np.max(np.abs(f - fref[:nrec + 1])) / scale) if ok else None,
            "population_err": float(np.max(np.abs(o[:, 6:] - pref[:nrec + 1]))) if ok else None,
            "wall_s": el,
            "fixed_rk4_rhs_evaluations_same_span": {k: 4 * int(round(2.0 / v)) for k, v in best.items()}}
        b.close()
    out["adaptive_drive_frame_2ns"] = ad
    return out


def _profiled_traffic(summary, key, sources):
    """HBM bytes `key` from a committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary
    under profiles/, or None when the kernel sources changed since the counters
    were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_b = re.search(r"^" + key + r": (\S+)$", txt, re.M)
    m_h = re.search(r"^source_sha256: (\S+)$", txt, re.M)
    if not (m_b and m_h):
        return None
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2508_18114_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return float(m_b.group(1)) if h.hexdigest() == m_h.group(1) else None


def measured_traffic_per_step():
    """HBM bytes per g+e RK4 step of k_persist (measured), or None."""
    return _profiled_traffic("k_persist_paper_size_traffic.md", "traffic_bytes_per_step",
                             ("lr_persistent.hip", "lr_device.h"))


def measured_apply_traffic_per_launch():
    """HBM bytes per k_apply_heff launch on 10240 columns of N=2000 (measured), or None."""
    return _profiled_traffic("k_apply_heff_512_factors_traffic.md", "traffic_bytes_per_launch",
                             ("lr_apply.hip", "lr_device.h"))


def measured_packed_traffic_per_traj_step():
    """HBM bytes per trajectory-step of k_packed on 512 trajectories (measured), or None."""
    return _profiled_traffic("k_packed_512_same_shape_traffic.md", "traffic_bytes_per_traj_step",
                             ("lr_packed.hip", "lr_device.h"))


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: runs on one GPU only (--gpus {a.gpus} requested); the multi-GPU "
              "sharding of the integrator is not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2508_18114_amd import inputs as I
    from paper_2508_18114_amd import lr

    torch.cuda.set_device(0)
    if a.copy_calibration > 0:
        copy_calibration(torch, a.copy_calibration)
        return
    if a.packed_sample > 0:
        packed_sample(lr, I, torch, a.packed_sample, a.packed_precision, a.packed_mfma64)
        return
    if a.apply_sample > 0:
        print(json.dumps(apply_sample(lr, I, torch, a.apply_sample)), flush=True)
        return
    if a.paper_spsa > 0:
        print(json.dumps(paper_spsa(lr, I, torch, a.paper_spsa)), flush=True)
        return
    if a.paper_setup > 0:
        print(json.dumps(paper_setup(lr, I, torch, a.paper_setup, parts=a.paper_setup_parts)), flush=True)
        return
    if a.config4_subset > 0:
        print(json.dumps(config4_subset(lr, I, torch, a.config4_subset)), flush=True)
        return
    if a.serving > 0:
        print(json.dumps(serving(lr, I, torch, torch.cuda.current_stream(), a.serving, only=a.serving_only,
                                 capacity=a.serving_capacity, policy=a.serving_policy,
                                 spread_layers=a.serving_layers)), flush=True)
        return
    trajs = I.config_paper_size()
    m, M = trajs[0].model, trajs[0].M
    stream = torch.cuda.current_stream()

    def make_batch(nsteps):
        items = [dict(model=t.model, M=t.M, pulse=t.pulse, dt=t.dt, nsteps=nsteps, B=lr.to_device(t.B0()))
                 for t in trajs]
        return lr.Batch(items, stream=stream), items

    def check(b):
        rc, codes, steps = b.status()
        if rc != lr.LR_OK:
            raise RuntimeError(f"device error {lr.lr_strerror(rc)} (codes {codes}, steps {steps})")

    # warmup: the same batch shape, W steps
    wb, _ = make_batch(a.warmup)
    wb.run()
    check(wb)
    wb.close()
    # timed region: K RK4 steps of both trajectories in one batch (inputs
    # resident in HBM); the persistent kernel's launches are bracketed by HIP
    # events on the batch stream
    tb, titems = make_batch(a.steps)
    tb.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tb.run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    check(tb)
    value = len(trajs) * a.steps / elapsed
    kernel_ms, launches = tb.profile_read()
    tb.close()
    launch_us = 1e3 * kernel_ms / max(launches, 1)
    steps_per_launch = a.steps / max(launches, 1)
    # algorithmic FP64 work of one trajectory-step: 4 stages x N x M elements x
    # (58 stencil/update + 16 M jump assembly + 24 M Gram/cross) flops
    flops_per_step = 4 * m.N * M * (58 + 40 * M)
    flops_per_launch = flops_per_step * steps_per_launch * len(trajs)
    achieved = flops_per_launch / (launch_us * 1e-6) / 1e12
    # measured HBM bytes per launch (rocprofv3 counters, calibrated by a copy)
    tps = measured_traffic_per_step()
    traffic = tps * steps_per_launch if tps is not None else None

    out = {
        "metric": "RK steps*trajectories/s at N=2000, M=20",
        "value": value,
        "unit": "RK steps*trajectories/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "readout model dims (8,50,5) N=2000, M=20, RK4 dt=5e-4 ns, "
                               "trajectories g and e integrated together (one batch)",
                   "N": m.N, "M": M, "trajectories": len(trajs), "dt_ns": trajs[0].dt},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFS, "traffic": traffic,
                     "kernel": "k_persist", "kernel_mean_us": launch_us, "launches_timed": launches,
                     "steps_per_launch": steps_per_launch, "trajectories_per_launch": len(trajs),
                     "flops_per_launch": flops_per_launch},
    }
    if not a.no_compare:
        out["comparisons"] = comparisons(lr, I, torch, stream, value)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(a.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
