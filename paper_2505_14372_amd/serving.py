"""Continuous-batching reconstruction server on one GPU.

Many reconstructions (each with its own probe size N, mode count M, slice
count S, scan and noise model) are served at once, the way the paper's
server runs many jobs (Sec. 2.3), but sharing the GPU instead of queueing:

* admission: a request that has arrived is admitted as soon as its resident
  footprint (object, probe, positions, Adam moments, patterns, propagator
  tables and gradient buffers) fits in the HBM budget next to the requests
  already running, in arrival order;
* residency: an admitted request keeps its whole state on the device until
  its last iteration, then its result is copied out and its memory freed;
* shared launches: in every round, each running request contributes its next
  minibatch of positions (one stochastic-gradient step, Sec. 3.2), and the
  minibatches of all requests with the same N go into shared kernel
  launches (pty_group_reconstruct_step: up to 16 reconstructions per launch,
  mixed M, S, object size and loss); groups of different N run on separate
  HIP streams, so their work overlaps on the device;
* accounting: per-iteration latency (one iteration = one pass over all of a
  request's positions) is recorded for p50/p99, next to positions x
  iterations per second.

`run_fifo` serves the same requests one at a time (single-request
reconstruct_step, same minibatch order), the baseline the server is compared
with.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import torch

from . import api, synth

# tiles per shared launch for each probe size (workspace of one N group)
DEFAULT_GROUP_TILES = {64: 4096, 128: 2048, 192: 1024, 256: 512}
MAX_SLICES = 32


@dataclass
class ReconRequest:
    """One reconstruction job (state in host memory until it is admitted)."""
    rid: int
    N: int
    M: int
    S: int
    probe: np.ndarray
    obj: np.ndarray
    positions: np.ndarray
    patterns: np.ndarray
    dz: List[float]
    dx: float = 0.2
    wavelength: float = synth.LAMBDA_300KV
    loss: str = "poisson"
    eps: float = 0.8
    n_iters: int = 50
    batch: int = 256
    opt: api.Optimizer = field(default_factory=lambda: api.Optimizer(kind="adam", lr_object=1e-3,
                                                                     lr_probe=1e-3, lr_pos=0.0))
    arrival: float = 0.0
    seed: int = 0

    @property
    def J(self):
        return self.positions.shape[0]

    @property
    def H(self):
        return self.obj.shape[1]

    @property
    def W(self):
        return self.obj.shape[2]

    def minibatches(self, iteration: int) -> List[np.ndarray]:
        """Seeded shuffled minibatches of one iteration (Sec. 2.2: random groups, shuffled order)."""
        rng = np.random.default_rng((self.seed, iteration))
        perm = rng.permutation(self.J).astype(np.int32)
        return [np.sort(perm[a:a + self.batch]) for a in range(0, self.J, self.batch)]

    def resident_bytes(self) -> int:
        c64 = 8
        obj = self.S * self.H * self.W * c64
        probe = self.M * self.N * self.N * c64
        pos = self.J * 2 * 4
        state = 3 * (obj + probe + pos)
        pats = self.J * self.N * self.N * 4
        ctx = api.workspace_bytes(self.N, self.M, self.S, self.H, self.W, self.J, 0, 1, dx=self.dx,
                                  wavelength=self.wavelength, dz=self.dz, loss=self.loss, eps=self.eps)
        return state + pats + ctx


@dataclass
class Result:
    rid: int
    probe: np.ndarray
    obj: np.ndarray
    positions: np.ndarray
    losses: List[float]
    iter_latency_s: List[float]
    admitted_at: float
    finished_at: float


class _Running:
    def __init__(self, req: ReconRequest, dev, now, reduction="atomic"):
        self.req = req
        self.prob = api.Problem(req.N, req.M, req.S, req.H, req.W, req.J, dz=req.dz, dx=req.dx,
                                wavelength=req.wavelength, loss=req.loss, eps=req.eps, max_batch=0)
        self.prob.set_reduction(reduction)
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)  # noqa: E731
        self.state = api.ReconState(t(req.probe, np.complex64), t(req.obj, np.complex64),
                                    t(req.positions, np.float32), adam=req.opt.kind == "adam")
        self.patterns = t(req.patterns, np.float32)
        n_steps = -(-req.J // req.batch)
        self.loss_slots = torch.zeros(n_steps, dtype=torch.float64, device=dev)   # one per step of an iteration
        self.iteration = 0
        self.batches: List[torch.Tensor] = []
        self.cursor = 0
        self.iter_start: Optional[float] = None
        self.losses: List[float] = []
        self.latency: List[float] = []
        self.admitted_at = now
        self._next_iteration(dev)

    def _next_iteration(self, dev):
        self.batches = [torch.from_numpy(b).to(dev) for b in self.req.minibatches(self.iteration)]
        self.cursor = 0
        self.iter_start = None

    def done(self):
        return self.iteration >= self.req.n_iters


class Server:
    """Admits, batches and runs reconstructions; see the module docstring."""

    def __init__(self, hbm_budget: int, group_tiles: Optional[Dict[int, int]] = None, device="cuda",
                 max_per_launch: int = 16, reduction: str = "atomic"):
        self.dev = torch.device(device)
        self.reduction = reduction   # object-gradient accumulation of every reconstruction
        self.budget = int(hbm_budget)
        self.group_tiles = dict(DEFAULT_GROUP_TILES if group_tiles is None else group_tiles)
        self.max_per_launch = min(max_per_launch, 16)
        self.groups: Dict[int, api.Group] = {}
        self.streams: Dict[int, torch.cuda.Stream] = {}
        self.pending: List[ReconRequest] = []
        self.running: List[_Running] = []
        self.results: Dict[int, Result] = {}
        self.used = 0
        self.rounds = 0
        self.inflight: Dict[int, tuple] = {}   # N -> (event, requests stepped)

    # workspace of the shared launches of one N (allocated on first use, counted in the budget)
    def _group(self, N):
        if N not in self.groups:
            tiles = self.group_tiles[N]
            self.used += api.Group.workspace_bytes(N, tiles, tiles, tiles * MAX_SLICES)
            self.groups[N] = api.Group(N, max_items=tiles, max_tiles=tiles, max_ckpt_tiles=tiles * MAX_SLICES)
            self.streams[N] = torch.cuda.Stream(device=self.dev)
        return self.groups[N]

    def submit(self, req: ReconRequest):
        if req.S > MAX_SLICES:
            raise ValueError(f"at most {MAX_SLICES} slices per reconstruction")
        if req.batch * req.M > self.group_tiles[req.N]:
            raise ValueError("minibatch x modes exceeds the shared-launch workspace")
        self.pending.append(req)
        self.pending.sort(key=lambda r: (r.arrival, r.rid))

    def _admit(self, now):
        admitted = []
        for req in list(self.pending):
            if req.arrival > now:
                break
            need = req.resident_bytes()
            grp_need = 0 if req.N in self.groups else api.Group.workspace_bytes(
                req.N, self.group_tiles[req.N], self.group_tiles[req.N], self.group_tiles[req.N] * MAX_SLICES)
            if self.used + need + grp_need > self.budget:
                if not self.running and not admitted:
                    raise MemoryError(f"request {req.rid} needs {need + grp_need} bytes, over the budget")
                break          # arrival order: later requests wait too
            self._group(req.N)
            self.running.append(_Running(req, self.dev, now, self.reduction))
            self.used += need
            self.pending.remove(req)
            admitted.append(req.rid)
        if admitted:
            # state initialisation ran on the current stream; the group streams read it next
            torch.cuda.current_stream(self.dev).synchronize()
        self.peak_used = max(getattr(self, "peak_used", 0), self.used)
        return admitted

    def _launch_round(self, N, runs, now):
        """One step of every running request of size N, in shared launches on N's stream."""
        grp = self.groups[N]
        cap = self.group_tiles[N]
        stream = self.streams[N]
        stepped = []
        with torch.cuda.stream(stream):
            launch, tiles, cks = [], 0, 0
            for r in runs:
                b = r.batches[r.cursor]
                need_t = b.numel() * r.req.M
                need_c = need_t * r.req.S
                if launch and (len(launch) == self.max_per_launch or tiles + need_t > cap
                               or cks + need_c > cap * MAX_SLICES):
                    grp.step(launch)
                    launch, tiles, cks = [], 0, 0
                if r.iter_start is None:
                    r.iter_start = now
                launch.append((r.prob, r.state, r.patterns, b, r.req.opt, r.loss_slots[r.cursor:r.cursor + 1]))
                tiles += need_t
                cks += need_c
                stepped.append(r)
            if launch:
                grp.step(launch)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.rounds += 1
        return ev, stepped

    def _complete(self, stepped, now, log):
        for r in stepped:
            r.cursor += 1
            if r.cursor == len(r.batches):
                r.latency.append(now - r.iter_start)
                r.losses.append(float(r.loss_slots.sum().item()))
                r.iteration += 1
                if r.done():
                    self._finish(r, now)
                    if log:
                        log(f"request {r.req.rid} done at {now:.2f}s")
                else:
                    r._next_iteration(self.dev)

    def run(self, clock=time.perf_counter, log=None) -> Dict[int, Result]:
        """Serve until every submitted request has finished. Each probe size
        advances on its own stream: a new round of size N is launched as soon
        as N's previous round has completed, independently of other sizes."""
        t0 = clock()
        while self.pending or self.running or self.inflight:
            now = clock() - t0
            self._admit(now)
            busy = False
            for N in sorted({r.req.N for r in self.running} | set(self.inflight)):
                if N in self.inflight:
                    ev, stepped = self.inflight[N]
                    if not ev.query():
                        busy = True
                        continue
                    del self.inflight[N]
                    self._complete(stepped, clock() - t0, log)
                runs = [r for r in self.running if r.req.N == N]
                if runs:
                    self.inflight[N] = self._launch_round(N, runs, clock() - t0)
                    busy = True
            if not busy:
                if self.pending and not self.running:
                    wait = self.pending[0].arrival - (clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.05))
                continue
            time.sleep(0.0001)
        return self.results

    def _finish(self, r: _Running, now):
        st = r.state
        self.results[r.req.rid] = Result(
            rid=r.req.rid, probe=st.probe.cpu().numpy(), obj=st.object.cpu().numpy(),
            positions=st.positions.cpu().numpy(), losses=r.losses, iter_latency_s=r.latency,
            admitted_at=r.admitted_at, finished_at=now)
        self.running.remove(r)
        self.used -= r.req.resident_bytes()
        r.prob.close()
        del r.state, r.patterns


def run_fifo(requests: List[ReconRequest], device="cuda", clock=time.perf_counter,
             reduction: str = "atomic") -> Dict[int, Result]:
    """Baseline: one reconstruction at a time in arrival order (single-request
    reconstruct_step with the same minibatches), starting each at the later of
    its arrival and the previous one's end."""
    dev = torch.device(device)
    results = {}
    t0 = clock()
    for req in sorted(requests, key=lambda r: (r.arrival, r.rid)):
        now = clock() - t0
        if req.arrival > now:
            time.sleep(req.arrival - now)
        admitted = clock() - t0
        prob = api.Problem(req.N, req.M, req.S, req.H, req.W, req.J, dz=req.dz, dx=req.dx,
                           wavelength=req.wavelength, loss=req.loss, eps=req.eps, max_batch=req.batch)
        prob.set_reduction(reduction)
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)  # noqa: E731
        st = api.ReconState(t(req.probe, np.complex64), t(req.obj, np.complex64), t(req.positions, np.float32),
                            adam=req.opt.kind == "adam")
        pats = t(req.patterns, np.float32)
        slots = torch.zeros(-(-req.J // req.batch), dtype=torch.float64, device=dev)
        losses, lat = [], []
        for it in range(req.n_iters):
            ts = clock()
            for k, b in enumerate(req.minibatches(it)):
                prob.reconstruct_step(st, pats, torch.from_numpy(b).to(dev), req.opt, slots[k:k + 1])
            losses.append(float(slots.sum().item()))
            lat.append(clock() - ts)
        results[req.rid] = Result(rid=req.rid, probe=st.probe.cpu().numpy(), obj=st.object.cpu().numpy(),
                                  positions=st.positions.cpu().numpy(), losses=losses, iter_latency_s=lat,
                                  admitted_at=admitted, finished_at=clock() - t0)
        prob.close()
    return results


def make_request_stream(n: int, seed: int = 0, rate_per_s: float = 2.0, n_iters: int = 50,
                        sizes=(64, 128, 192, 256), max_modes: int = 6, max_slices: int = 16,
                        scans=(16, 64), steps=(4, 8), batch: int = 256) -> List[ReconRequest]:
    """Poisson arrivals of reconstructions of mixed N, M, S and scan size, each
    generated from its own seed like the single-reconstruction workloads."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += rng.exponential(1.0 / rate_per_s)
        N = int(rng.choice(sizes))
        M = int(rng.integers(1, max_modes + 1))
        S = int(rng.integers(1, max_slices + 1))
        scan = int(rng.integers(scans[0], scans[1] + 1))
        step = int(rng.integers(steps[0], steps[1] + 1))
        rs = 1000 + k
        simple = (M == 1 and S == 1)
        dose = 1e4 if simple else 1e5
        side = N + scan * step
        probe = synth.make_probe(N, M, dose)
        obj = synth.make_object(S, side, side, 0.3 if simple else 0.1, rs)
        pos = synth.make_scan(scan, step, 0.0 if simple else 0.5, rs)
        pats = synth.make_patterns(N, pos.shape[0], dose, rs, pool=64)
        out.append(ReconRequest(rid=k, N=N, M=M, S=S, probe=probe, obj=obj, positions=pos, patterns=pats,
                                dz=[2.0] * (S - 1), loss="amplitude" if simple else "poisson",
                                eps=0.0 if simple else 0.8, n_iters=n_iters,
                                batch=min(batch, DEFAULT_GROUP_TILES[N] // M), arrival=t, seed=rs))
    return out


def latency_stats(results: Dict[int, Result]):
    """p50 and p99 of the per-iteration latencies of every request."""
    lat = np.array([x for r in results.values() for x in r.iter_latency_s])
    return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))


def request_latency_stats(results: Dict[int, Result], requests: List[ReconRequest]):
    """p50 and p99 of each request's time from arrival to completion (both on
    the clock of the run that produced `results`)."""
    lat = np.array([results[r.rid].finished_at - r.arrival for r in requests])
    return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))
