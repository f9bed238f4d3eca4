"""Serving loop for readout-loss evaluations: continuous batching of low-rank
trajectories on one GPU.

A request is one loss evaluation of a pulse candidate (supplement S3.B-C):
the transmon starts in g and in e, both trajectories are integrated with the
same drive, and the figures of merit of the pair (lr_readout_loss) are its
result.  The server keeps every admitted trajectory's state B and its
observation series resident on the device and advances all of them together
in ticks: each tick is one lr_batch_run over the active trajectories, each
moving ahead by up to `chunk` RK4 steps (`step0` continues the stage-time grid
exactly, so a trajectory's result is bitwise the same whether it runs alone or
in any mix, in one call or in many).  Between ticks, finished requests are
retired and queued ones are admitted while their HBM footprint fits the
budget and their workgroups fit the co-resident capacity.

`EvolutionStrategy` is the gradient-free request source: a (mu, lambda)
evolution strategy over the six Piecewise6 parameters that emits generations
of candidates and moves its mean to the best of each finished generation.
`SPSA` and `spsa_optimize` are the paper's own optimiser (supplement S3.C)
over the smoothed stepwise pulse.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Dict, List, Optional

import numpy as np

from . import inputs as I
from . import lr


@dataclasses.dataclass
class Request:
    rid: int
    model: I.ModelParams
    M: int
    pulse: I.PulseParams
    dt: float
    nsteps: int
    precision: int = I.FP64
    obs_stride: int = 200
    pad_scale: float = I.PAPER_PAD_SCALE
    seed: int = 0
    arrival: float = 0.0          # seconds, relative to the start of the run


@dataclasses.dataclass
class _Traj:
    req: Request
    which: str
    B: object                     # device tensor (M, N) complex128
    obs: object                   # device tensor (records, 6 + d_q)
    done: int = 0                 # steps of completed ticks
    enq: int = 0                  # steps enqueued


def trajectory_footprint(model: I.ModelParams, M: int, obs_records: int, packed: bool = False,
                         precision: int = I.FP64) -> int:
    """Device bytes of one resident trajectory: state, observation series and
    its share of a batch workspace (planned on the host, nothing allocated)."""
    import torch
    B = torch.empty((1,), dtype=torch.complex128)  # placeholder pointer, never dereferenced by planning
    t = lr.traj_struct(model, M, I.flattop_pulse(0.05, 1.0), 0.0, 1e-3, 1, B, 0, None, precision)
    h = lr.lr_batch_init([t], lr.LR_BATCH_PACKED if packed else 0)
    try:
        ws = lr.lr_batch_workspace_bytes(h)
    finally:
        lr.lr_batch_destroy(h)
    return ws + model.N * M * 16 + obs_records * (6 + model.d_q) * 8


# Per-step time models of the two schedules (seconds), for routing and for
# cost-balanced ticks: a packed workgroup takes about T_PACKED_REF per RK4 step
# on the paper-size trajectory (N = 2000, M = 20) and scales with the flop count
# N M (58 + 40 M); the spread schedule's step is latency-bound, about
# T_SPREAD_REF at M = 20 and roughly linear in M (the solve).
T_PACKED_REF = 2.0e-3
T_SPREAD_REF = 120e-6
COST_REF = 2000 * 20 * (58 + 40 * 20)


def step_cost(model: I.ModelParams, M: int) -> float:
    return float(model.N * M * (58 + 40 * M))


def packed_step_s(model: I.ModelParams, M: int) -> float:
    return T_PACKED_REF * step_cost(model, M) / COST_REF


def spread_step_s(model: I.ModelParams, M: int) -> float:
    return T_SPREAD_REF * max(M, 4) / 20.0


class Server:
    """Continuous batching of loss evaluations.

    Routing: with packed=True (the default) a request runs in the packed
    schedule (one workgroup per trajectory, LR_BATCH_PACKED: the most
    trajectory-steps per second, but one workgroup's pace per trajectory)
    unless its estimated packed duration exceeds max_packed_s; then it runs in
    the spread schedule (one workgroup per resonator layer, the shortest time
    per step).  packed=False: every request spread, in tiles of spread_layers
    resonator layers per workgroup (LR_BATCH_SPREAD_LAYERS).  A packed request
    counts two workgroups against the cap (default: two per CU, the packed
    kernel's occupancy), a spread one 2 ceil(d_r / spread_layers).

    Ticks are asynchronous and cost-balanced: tick k gives every active
    trajectory the steps that take about `chunk` steps of the paper-size
    packed trajectory in its schedule, is built and enqueued on one of two
    alternating streams (after an event of tick k - 1, whose states it
    continues) before tick k - 1 is synchronised and retired, and queued
    requests are admitted on the host while the GPU runs.  A trajectory's
    result does not depend on the tick lengths or the mix (step0 continues the
    stage-time grid exactly; both schedules sum in fixed orders)."""

    def __init__(self, hbm_budget_bytes: int, chunk: int = 2000, max_workgroups: Optional[int] = None,
                 stream=None, packed: bool = True, max_packed_s: float = 60.0, on_tick=None,
                 spread_layers: int = 1):
        import torch
        self.torch = torch
        self.packed = bool(packed)
        self.budget = int(hbm_budget_bytes)
        self.chunk = int(chunk)
        props = torch.cuda.get_device_properties(0)
        self.wg_cap = int(max_workgroups or props.multi_processor_count * (2 if self.packed else 1))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.tick_streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        self.queue: List[Request] = []
        self.active: List[_Traj] = []
        self.in_use = 0
        self.wg_in_use = 0
        self.results: Dict[int, dict] = {}
        self.t_start = None
        self.steps_done = 0
        self.ticks = 0
        self._last_event = None
        self.max_packed_s = float(max_packed_s)
        self.on_tick = on_tick
        self.spread_layers = max(1, int(spread_layers))

    # -------------------------------------------------------------- admission
    def _packs(self, r: Request) -> bool:
        if not self.packed or (r.precision != I.FP64 and getattr(r.model, "kind", 0) == I.MODEL_NORMAL):
            return False
        return r.nsteps * packed_step_s(r.model, r.M) <= self.max_packed_s

    def _tick_steps(self, r: Request) -> int:
        t_tick = self.chunk * T_PACKED_REF
        per = packed_step_s(r.model, r.M) if self._packs(r) else spread_step_s(r.model, r.M)
        return max(1, int(t_tick / per))

    def _need(self, r: Request):
        nrec = r.nsteps // r.obs_stride + 1
        packs = self._packs(r)
        fp = 2 * trajectory_footprint(r.model, r.M, nrec, packs, r.precision)
        # one workgroup per trajectory, or per tile of spread_layers resonator layers
        wgs = 2 if packs else 2 * -(-r.model.d_r // self.spread_layers)
        return fp, wgs

    def submit(self, r: Request):
        if r.nsteps % r.obs_stride:
            raise ValueError("nsteps must be a multiple of obs_stride")
        if self._need(r)[0] > self.budget:  # could never be admitted
            self.results[r.rid] = {"arrival": r.arrival, "error": "footprint exceeds the HBM budget"}
            return
        self.queue.append(r)

    def _admit(self, now: float):
        torch = self.torch
        keep = []
        for r in self.queue:
            fp, wgs = self._need(r)
            fits = (r.arrival <= now and self.in_use + fp <= self.budget and
                    (self.wg_in_use + wgs <= self.wg_cap or not self.active))
            if not fits:
                keep.append(r)
                continue
            nrec = r.nsteps // r.obs_stride + 1
            for which in ("g", "e"):
                B0 = I.initial_state(r.model, r.M, which, r.seed, r.pad_scale)
                obs = torch.zeros((nrec, 6 + r.model.d_q), dtype=torch.float64, device="cuda")
                t = _Traj(r, which, lr.to_device(B0), obs)
                self.active.append(t)
            self.in_use += fp
            self.wg_in_use += wgs
            self.results[r.rid] = {"arrival": r.arrival, "admitted": now}
        self.queue = keep

    # -------------------------------------------------------------- ticks
    def _enqueue(self):
        """Build and enqueue the next tick: every active trajectory with steps not yet enqueued moves
        ahead by up to `chunk` steps.  Returns the pending tick or None."""
        torch = self.torch
        items = []
        for t in self.active:
            r = t.req
            n = min(self._tick_steps(r), r.nsteps - t.enq)
            if n <= 0:
                continue
            if n < r.nsteps - t.enq:
                n -= n % r.obs_stride  # keep record boundaries aligned
                n = max(n, r.obs_stride)
            items.append((t, dict(model=r.model, M=r.M, pulse=r.pulse, t0=0.0, dt=r.dt, nsteps=n, B=t.B,
                                  obs_stride=r.obs_stride, obs=t.obs[t.enq // r.obs_stride:],
                                  precision=r.precision, step0=t.enq)))
        if not items:
            return None
        s = self.tick_streams[self.ticks % 2]
        # plan and bind first (binding synchronises this stream, which holds only finished ticks) ...
        items = [x for x in items if self._packs(x[0].req)] + [x for x in items if not self._packs(x[0].req)]
        npk = sum(1 for x in items if self._packs(x[0].req))
        batches = []
        if npk:
            batches.append((lr.Batch([it for _, it in items[:npk]], stream=s, packed=True), items[:npk]))
        if npk < len(items):
            batches.append((lr.Batch([it for _, it in items[npk:]], stream=s, packed=False,
                                     flags=lr.LR_BATCH_SPREAD_LAYERS(self.spread_layers)), items[npk:]))
        # ... then order the launches after the admissions' copies and the previous tick
        s.wait_stream(torch.cuda.current_stream())
        if self._last_event is not None:
            s.wait_event(self._last_event)
        for b, _ in batches:
            b.run()
        ev = torch.cuda.Event()
        ev.record(s)
        self._last_event = ev
        for t, it in items:
            t.enq += it["nsteps"]
            t.B.record_stream(s)
            t.obs.record_stream(s)
        self.ticks += 1
        return batches

    def _complete(self, tick):
        """Synchronise a tick (its stream only) and account its steps and errors."""
        for b, items in tick:
            rc, codes, steps = b.status()
            for (t, it), c in zip(items, codes):
                if c != lr.LR_OK:
                    self.results[t.req.rid]["error"] = lr.lr_strerror(c)
                    t.done = t.enq = t.req.nsteps
                else:
                    t.done += it["nsteps"]
                    self.steps_done += it["nsteps"]
            b.close()
        if self.on_tick is not None:
            self.on_tick(self)

    def tick(self):
        """One synchronous tick (enqueue and complete)."""
        pend = self._enqueue()
        if pend is not None:
            self._complete(pend)

    def _retire(self, now: float):
        by_req: Dict[int, List[_Traj]] = {}
        for t in self.active:
            by_req.setdefault(t.req.rid, []).append(t)
        still = []
        for rid, ts in by_req.items():
            r = ts[0].req
            if all(t.done >= r.nsteps for t in ts):
                res = self.results[rid]
                if "error" not in res:
                    tg = next(t for t in ts if t.which == "g")
                    te = next(t for t in ts if t.which == "e")
                    res["loss"] = lr.readout_loss(tg.obs, te.obs, r.model.d_q, r.obs_stride * r.dt,
                                                  r.model.kappa_f, r.model.gamma_1, stream=self.stream)
                    res["B_g"], res["B_e"] = tg.B, te.B
                    res["obs_g"], res["obs_e"] = tg.obs, te.obs
                res["done"] = now
                res["latency"] = now - r.arrival
                fp, wgs = self._need(r)
                self.in_use -= fp
                self.wg_in_use -= wgs
            else:
                still.extend(ts)
        self.active = still

    # -------------------------------------------------------------- run
    def run(self, requests: List[Request], on_result=None):
        """Serve requests with open-loop arrivals (Request.arrival, seconds from
        now).  on_result(rid, result) is called as results complete and may
        submit further requests.  Returns the statistics of the run."""
        for r in requests:
            self.submit(r)
        t0 = time.perf_counter()
        self.t_start = t0
        reported = set()
        pending = None
        while self.queue or self.active or pending is not None:
            now = time.perf_counter() - t0
            self._admit(now)  # host work while the pending tick runs
            nxt = self._enqueue() if self.active else None
            if pending is not None:
                self._complete(pending)
                self._retire(time.perf_counter() - t0)
                if on_result is not None:
                    for rid, res in list(self.results.items()):
                        if "done" in res and rid not in reported:
                            reported.add(rid)
                            on_result(rid, res)
            pending = nxt
            if pending is None and not self.active and self.queue:
                nxt_arr = min(r.arrival for r in self.queue)
                time.sleep(max(0.0, min(nxt_arr - (time.perf_counter() - t0), 0.05)))
        wall = time.perf_counter() - t0
        lat = np.array([res["latency"] for res in self.results.values() if "latency" in res])
        return {"requests": len(lat), "wall_s": wall, "traj_steps": self.steps_done,
                "traj_steps_per_s": self.steps_done / wall if wall > 0 else 0.0, "ticks": self.ticks,
                "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else math.nan,
                "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else math.nan,
                "errors": sum(1 for res in self.results.values() if "error" in res)}


class EvolutionStrategy:
    """(mu, lambda) evolution strategy over the Piecewise6 parameters
    (A_1, phi_1, Delta_1, A_2, phi_2, Delta_2) in rad/ns and rad."""

    LO = np.array([I.ghz(0.02), 0.0, I.ghz(-0.02), I.ghz(0.02), 0.0, I.ghz(-0.02)])
    HI = np.array([I.ghz(0.1), 2 * np.pi, I.ghz(0.02), I.ghz(0.1), 2 * np.pi, I.ghz(0.02)])

    def __init__(self, seed: int, lam: int = 32, mu: int = 8, sigma: float = 0.15):
        self.rng = I.rng(seed)
        self.lam, self.mu, self.sigma = lam, mu, sigma
        self.mean = 0.5 * (self.LO + self.HI)
        self.generation = 0

    def ask(self) -> List[np.ndarray]:
        span = self.HI - self.LO
        out = []
        for _ in range(self.lam):
            x = self.mean + self.sigma * span * self.rng.standard_normal(6)
            out.append(np.clip(x, self.LO, self.HI))
        return out

    def tell(self, cands: List[np.ndarray], losses: List[float]):
        order = np.argsort(np.asarray(losses))[: self.mu]
        self.mean = np.mean([cands[i] for i in order], axis=0)
        self.generation += 1


def spsa_gradient(loss_plus: float, loss_minus: float, ck: float, delta: np.ndarray) -> np.ndarray:
    """SPSA gradient estimate from the two losses at theta +- ck delta (delta_i = +-1)."""
    return (loss_plus - loss_minus) / (2.0 * ck) / delta


class SPSA:
    """Simultaneous perturbation stochastic approximation (supplement S3.C): step k
    draws a direction Delta with independent +-1 entries, the loss is evaluated at
    theta + c_k Delta and theta - c_k Delta (two loss evaluations, each a g/e
    pair), and theta moves by -a_k (L+ - L-) / (2 c_k) Delta^-1, with the usual
    gain sequences a_k = a / (k + 1 + A)^alpha and c_k = c / (k + 1)^gamma.
    `project` maps a parameter vector back into the admissible set."""

    def __init__(self, theta0, seed: int, a: float, c: float, A: float = 10.0, alpha: float = 0.602,
                 gamma: float = 0.101, project=None):
        self.theta = np.asarray(theta0, dtype=np.float64).copy()
        self.rng = I.rng(seed)
        self.a, self.c, self.A, self.alpha, self.gamma = a, c, A, alpha, gamma
        self.project = project if project is not None else (lambda x: x)
        self.k = 0
        self._delta = None

    def gains(self):
        return self.a / (self.k + 1 + self.A) ** self.alpha, self.c / (self.k + 1) ** self.gamma

    def ask(self):
        """The two parameter vectors of this step: theta + c_k Delta, theta - c_k Delta."""
        _, ck = self.gains()
        self._delta = self.rng.choice([-1.0, 1.0], size=self.theta.shape)
        return self.project(self.theta + ck * self._delta), self.project(self.theta - ck * self._delta)

    def tell(self, loss_plus: float, loss_minus: float):
        ak, ck = self.gains()
        ghat = spsa_gradient(loss_plus, loss_minus, ck, self._delta)
        self.theta = self.project(self.theta - ak * ghat)
        self.k += 1
        return ghat


def heights_from(theta: np.ndarray) -> np.ndarray:
    """Complex heights from the real parameter vector (re, im interleaved)."""
    return theta[0::2] + 1j * theta[1::2]


def project_heights(theta: np.ndarray, bound: float = I.ghz(0.4) * (1.0 - 1e-9)) -> np.ndarray:
    """Scale each complex height into the drive bound |h| < 2 pi 400 MHz."""
    h = heights_from(theta)
    a = np.abs(h)
    h = np.where(a > bound, h * (bound / np.maximum(a, 1e-300)), h)
    out = np.empty_like(theta)
    out[0::2], out[1::2] = h.real, h.imag
    return out


def pulse_loss_batch(model: I.ModelParams, M: int, pulses, dt: float, nsteps: int, obs_stride: int,
                     pad_scale: float = I.PAPER_PAD_SCALE, seed: int = 0, stream=None, packed=None,
                     adaptive=None, parts: int = 0):
    """Readout loss Lambda (and its figures of merit) of each pulse: the g and e
    trajectories of every pulse integrated together in one batch, the loss of
    each g/e pair formed on the device.  packed: the packed schedule (default:
    on for the paper's models, kinds 1 and 2, which run only there); adaptive:
    (rtol, atol) for adaptive steps, dt then being the output grid; parts: each
    FP64 trajectory split over that many workgroups (latency when few pulses
    are evaluated at once)."""
    if packed is None:
        packed = getattr(model, "kind", 0) in (I.MODEL_TRANSMON, I.MODEL_NORMAL)
    import torch
    items = []
    nrec = nsteps // obs_stride + 1
    for p in pulses:
        for which in ("g", "e"):
            B0 = I.initial_state(model, M, which, seed, pad_scale)
            items.append(dict(model=model, M=M, pulse=p, dt=dt, nsteps=nsteps, B=lr.to_device(B0),
                              obs_stride=obs_stride,
                              obs=torch.zeros((nrec, 6 + model.d_q), dtype=torch.float64, device="cuda")))
    b = lr.Batch(items, stream=stream, packed=packed, adaptive=adaptive, parts=parts)
    b.run()
    rc, codes, steps = b.status()
    if rc != lr.LR_OK:
        raise RuntimeError(f"loss batch failed: {lr.lr_strerror(rc)} (codes {codes})")
    b.close()
    out = []
    for i in range(len(pulses)):
        g, e = items[2 * i]["obs"], items[2 * i + 1]["obs"]
        out.append(lr.readout_loss(g, e, model.d_q, obs_stride * dt, model.kappa_f, model.gamma_1, stream=stream))
    return out


def square_start(model: I.ModelParams, nh: int, amp: float = I.ghz(0.15)) -> np.ndarray:
    """SPSA start: every height amp, the square pulse of supplement S3.C.  The
    paper's drive Omega_d(t) sin(w_d t) on i (f^ - f) (kinds 1 and 2, which put
    d(t) = Re[Omega e^{-i w_d t}] on that quadrature) is a real paper amplitude
    only for an imaginary height here (d = Im Omega sin(w_d t)); the Duffing
    model's drive on (f + f^) takes real heights (a cos carrier)."""
    theta = np.zeros(2 * nh)
    theta[(1 if getattr(model, "kind", 0) in (I.MODEL_TRANSMON, I.MODEL_NORMAL) else 0)::2] = amp
    return theta


def spsa_optimize(model: I.ModelParams, M: int, T: float, nh: int, iters: int, dt: float, obs_stride: int,
                  seed: int = 1, a: float = 0.05, c: float = 0.05, sigma: float = 0.5,
                  frame: int = I.FRAME_DRIVE, stream=None, w_d: float = I.W_DRIVE, adaptive=None, parts: int = 0,
                  on_step=None):
    """The optimisation loop of supplement S3.C on the device: SPSA over the nh
    complex heights of the smoothed stepwise pulse, started from the square shape
    of amplitude 2 pi 150 MHz (square_start), each step evaluating theta +- c_k
    Delta in one batch of four trajectories (each split over `parts` workgroups
    when given).  Returns (theta, history) with the loss at both probes of every
    step; on_step(record) is called after each step."""
    opt = SPSA(square_start(model, nh), seed, a=a, c=c, project=project_heights)
    hist = []
    for _ in range(iters):
        tp, tm = opt.ask()
        pulses = [I.stepwise_pulse(heights_from(x), T, sigma=sigma, w_d=w_d).replace(frame=frame) for x in (tp, tm)]
        fp, fm = pulse_loss_batch(model, M, pulses, dt, int(round(T / dt)), obs_stride, stream=stream,
                                  adaptive=adaptive, parts=parts)
        opt.tell(fp["loss"], fm["loss"])
        hist.append({"k": opt.k, "loss_plus": fp["loss"], "loss_minus": fm["loss"],
                     "eps_a_plus": fp["eps_a"], "eps_a_minus": fm["eps_a"]})
        if on_step is not None:
            on_step(hist[-1])
    return opt.theta, hist


def pulse_from(x: np.ndarray, T: float) -> I.PulseParams:
    return I.PulseParams(kind=I.PULSE_PIECEWISE6, w_d=I.W_DRIVE, amp=0.0, t_ramp=I.T_RAMP, T=T,
                         p=tuple(float(v) for v in x))


def serving_requests(seed: int, n: int, rate_per_s: float, dt: float = 5e-4, step_cap: Optional[int] = None,
                     obs_stride: int = 200, es_seed: int = 5) -> List[Request]:
    """n requests of the serving workload: shapes from inputs.serving_request_shapes
    (d_r in [13, 75], M in [4, 32], T in [10, 60] ns, FP32 / FP64), pulses from
    the evolution strategy's first generations, open-loop Poisson arrivals at
    rate_per_s.  step_cap (if given) bounds each request's step count."""
    shapes = I.serving_request_shapes(seed, n, dt)
    arr = I.poisson_arrivals(seed, n, rate_per_s)
    es = EvolutionStrategy(es_seed)
    cands: List[np.ndarray] = []
    out = []
    for k, sh in enumerate(shapes):
        if not cands:
            cands = es.ask()
        nsteps = sh["nsteps"] if step_cap is None else min(sh["nsteps"], step_cap)
        nsteps -= nsteps % obs_stride
        nsteps = max(nsteps, obs_stride)
        m = I.readout_model(8, sh["d_r"], 5)
        out.append(Request(rid=k, model=m, M=sh["M"], pulse=pulse_from(cands.pop(), nsteps * dt), dt=dt,
                           nsteps=nsteps, precision=sh["precision"], obs_stride=obs_stride,
                           seed=seed * 1000 + k, arrival=float(arr[k])))
    return out
