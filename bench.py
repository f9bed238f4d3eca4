"""Throughput benchmark of the low-rank Lindblad RK4 integrator on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Workload: the paper-size readout case -- dims (d_q, d_r, d_f) = (8, 50, 5)
(N = 2000), rank M = 20, dt = 5e-4 ns, FP64, two trajectories (transmon
initially in g and in e) with the seeded flat-top drive.  One bench step is
one RK4 step of both trajectories; inputs are resident in HBM before the
timed region.  Prints one JSON line (metric: RK steps x trajectories / s).

The JSON also carries
  roofline      -- the streaming stage kernel: algorithmic state bytes per
                   launch / its mean duration (HIP events on its stream)
  cpu_baseline  -- the FP64 numpy oracle on a bounded sample of the same
                   workload on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=400, help="oracle steps per trajectory in the CPU sample")
    return ap.parse_args()


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


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (--gpus {a.gpus} requested); "
              "multi-GPU sharding is described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2508_18114_amd import inputs as I
    from paper_2508_18114_amd import lr

    torch.cuda.set_device(0)
    trajs = I.config_paper_size()
    m, M = trajs[0].model, trajs[0].M
    streams = [torch.cuda.Stream() for _ in trajs]
    ctxs = [lr.Context(t.model, t.M, stream=s) for t, s in zip(trajs, streams)]
    Bs = [lr.to_device(t.B0()) for t in trajs]
    torch.cuda.synchronize()

    def run(nsteps):
        for c, t, B in zip(ctxs, trajs, Bs):
            c.integrate(t.pulse, 0.0, t.dt, nsteps, B)

    run(a.warmup)
    torch.cuda.synchronize()
    for c in ctxs:
        rc, fs = c.status()
        if rc != lr.LR_OK:
            raise RuntimeError(f"device error {lr.lr_strerror(rc)} at step {fs}")

    # timed region: K RK4 steps of both trajectories
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(a.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for c in ctxs:
        rc, fs = c.status()
        if rc != lr.LR_OK:
            raise RuntimeError(f"device error {lr.lr_strerror(rc)} at step {fs}")
    value = len(trajs) * a.steps / elapsed

    # live kernel timing of the stage kernel (events on its own stream)
    prof_steps = min(1000, max(1, a.steps // 4))
    c0 = ctxs[0]
    lr.lr_profile_enable(c0.handle, True)
    c0.integrate(trajs[0].pulse, 0.0, trajs[0].dt, prof_steps, Bs[0])
    _, stage_ms, stage_n, solve_ms, solve_n = lr.lr_profile_read(c0.handle)
    lr.lr_profile_enable(c0.handle, False)
    stage_us = 1e3 * stage_ms / max(stage_n, 1)
    solve_us = 1e3 * solve_ms / max(solve_n, 1)
    # algorithmic state traffic of one trajectory-step: 10 reads + 7 writes of N x M complex FP64
    bytes_per_step = 17 * 16 * m.N * M
    bytes_per_launch = bytes_per_step / 4.0
    achieved = bytes_per_launch / (stage_us * 1e-6) / 1e9

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
                               "trajectories g and e (plain form, one context each)",
                   "N": m.N, "M": M, "trajectories": len(trajs), "dt_ns": trajs[0].dt},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_stage", "kernel_mean_us": stage_us, "launches_timed": stage_n,
                     "bytes_per_launch": bytes_per_launch, "solve_kernel_mean_us": solve_us},
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(a.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
