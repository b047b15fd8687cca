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
* shared launches: a round of size N is one shared kernel launch
  (pty_group_reconstruct_step: up to 16 reconstructions, mixed M, S, object
  size and loss) filled in arrival order with the next minibatch (one
  stochastic-gradient step, Sec. 3.2) of each running request of that size
  until its workspace is full: the oldest requests step in every round, as
  they would alone, and the small ones behind them share the launch instead
  of waiting for a GPU they would leave mostly idle; groups of different N
  run on separate HIP streams, so their work overlaps on the device;
* pipelining: the state is resident and every step is stream-ordered, so the
  next round of a size class is enqueued before the previous one has
  finished (up to `depth` rounds in flight per size); the host polls only to
  account for completed rounds, so the device never idles for a host
  round trip between rounds;
* accounting: per-iteration latency (one iteration = one pass over all of a
  request's positions, from the launch of its first round to the observed
  completion of its last) is recorded for p50/p99, next to positions x
  iterations per second; iteration losses are summed on the device and read
  when a request finishes.

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
    truth: Optional[np.ndarray] = None   # true object the patterns were simulated from, if any

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
        # per-step losses of an iteration and the per-iteration sums, both written
        # on the device: an iteration's sum is taken on N's stream right after its
        # last step, so the next iteration's steps (later on that stream) cannot
        # overwrite the slots before they are summed
        self.loss_slots = torch.zeros(n_steps, dtype=torch.float64, device=dev)
        self.iter_losses = torch.zeros(req.n_iters, dtype=torch.float64, device=dev)
        # every iteration's minibatches copied to the device once, at admission
        # (no host-to-device copy between rounds)
        plan = [req.minibatches(it) for it in range(req.n_iters)]
        flat = torch.from_numpy(np.concatenate([b for bs in plan for b in bs]).astype(np.int32)).to(dev)
        self.plan: List[List[torch.Tensor]] = []
        off = 0
        for bs in plan:
            row = []
            for b in bs:
                row.append(flat[off:off + len(b)])
                off += len(b)
            self.plan.append(row)
        self.launch_iter = 0          # iteration of the next step to launch
        self.batches: List[torch.Tensor] = self.plan[0]
        self.cursor = 0               # next minibatch of launch_iter
        self.iter_start: Dict[int, float] = {}
        self.iterations_done = 0
        self.latency: List[float] = []
        self.admitted_at = now

    def _load_batches(self):
        self.batches = self.plan[self.launch_iter]
        self.cursor = 0

    def has_work(self):
        return self.launch_iter < self.req.n_iters

    def next_step(self, now):
        """(iteration, minibatch, loss slot, last step of the iteration) of the next
        step to launch; advances the launch cursor."""
        it, k = self.launch_iter, self.cursor
        if k == 0:
            self.iter_start[it] = now
        b = self.batches[k]
        slot = self.loss_slots[k:k + 1]
        last = k == len(self.batches) - 1
        self.cursor += 1
        if last:
            self.launch_iter += 1
            if self.has_work():
                self._load_batches()
        return it, b, slot, last

    def done(self):
        return self.iterations_done >= self.req.n_iters


class Server:
    """Admits, batches and runs reconstructions; see the module docstring."""

    def __init__(self, hbm_budget: int, group_tiles: Optional[Dict[int, int]] = None, device="cuda",
                 max_per_launch: int = 16, reduction: str = "atomic", depth: int = 2, fill_first: bool = True):
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
        self.depth = max(1, int(depth))        # rounds in flight per size class
        self.fill_first = bool(fill_first)      # one launch per round, filled in arrival order
        self.inflight: Dict[int, List[tuple]] = {}   # N -> [(event, steps launched)], oldest first

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
        """One step of the running requests of size N that have work left, in
        shared launches on N's stream; returns (event, steps launched). With
        fill_first, a round is one shared launch filled in arrival order: the
        oldest requests step every round, as they would alone, and younger
        ones take the room they leave; otherwise every request steps in every
        round (several launches when one does not hold them)."""
        grp = self.groups[N]
        cap = self.group_tiles[N]
        stream = self.streams[N]
        stepped = []
        with torch.cuda.stream(stream):
            launch, tiles, cks = [], 0, 0
            for r in runs:
                if not r.has_work():
                    continue
                need_t = r.batches[r.cursor].numel() * r.req.M
                need_c = need_t * r.req.S
                if launch and (len(launch) == self.max_per_launch or tiles + need_t > cap
                               or cks + need_c > cap * MAX_SLICES):
                    if self.fill_first:
                        break
                    grp.step(launch)
                    launch, tiles, cks = [], 0, 0
                it, b, slot, last = r.next_step(now)
                launch.append((r.prob, r.state, r.patterns, b, r.req.opt, slot))
                tiles += need_t
                cks += need_c
                stepped.append((r, it, last))
            if launch:
                grp.step(launch)
            # iteration losses summed on the device, in stream order after their steps
            for r, it, last in stepped:
                if last:
                    r.iter_losses[it:it + 1].copy_(r.loss_slots.sum().reshape(1))
            ev = torch.cuda.Event()
            ev.record(stream)
        self.rounds += 1
        return ev, stepped

    def _complete(self, stepped, now, log):
        for r, it, last in stepped:
            if not last:
                continue
            r.latency.append(now - r.iter_start.pop(it))
            r.iterations_done += 1
            if r.done():
                self._finish(r, now)
                if log:
                    log(f"request {r.req.rid} done at {now:.2f}s")

    def run(self, clock=time.perf_counter, log=None) -> Dict[int, Result]:
        """Serve until every submitted request has finished. Each probe size
        advances on its own stream with up to `depth` rounds in flight: a round
        is enqueued as soon as fewer are in flight (the steps are stream-ordered
        on device-resident state), and completed rounds are accounted for in
        launch order."""
        t0 = clock()
        while self.pending or self.running or any(self.inflight.values()):
            now = clock() - t0
            self._admit(now)
            busy = False
            for N in sorted({r.req.N for r in self.running} | set(self.inflight)):
                q = self.inflight.setdefault(N, [])
                while q and q[0][0].query():
                    _, stepped = q.pop(0)
                    self._complete(stepped, clock() - t0, log)
                runs = [r for r in self.running if r.req.N == N and r.has_work()]
                while runs and len(q) < self.depth:
                    q.append(self._launch_round(N, runs, clock() - t0))
                    runs = [r for r in runs if r.has_work()]
                busy = busy or bool(q)
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
        # every round of this request has completed (its last one was just observed)
        self.results[r.req.rid] = Result(
            rid=r.req.rid, probe=st.probe.cpu().numpy(), obj=st.object.cpu().numpy(),
            positions=st.positions.cpu().numpy(), losses=r.iter_losses.cpu().tolist(), iter_latency_s=r.latency,
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
        n_steps = -(-req.J // req.batch)
        slots = torch.zeros((req.n_iters, n_steps), dtype=torch.float64, device=dev)
        # iterations are enqueued back to back (nothing waits for the host);
        # their latencies come from device events at their boundaries
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(req.n_iters + 1)]
        evs[0].record()
        for it in range(req.n_iters):
            for k, b in enumerate(req.minibatches(it)):
                prob.reconstruct_step(st, pats, torch.from_numpy(b).to(dev), req.opt, slots[it, k:k + 1])
            evs[it + 1].record()
        losses = slots.sum(dim=1).cpu().tolist()   # waits for the request's last step
        lat = [evs[i].elapsed_time(evs[i + 1]) / 1000.0 for i in range(req.n_iters)]
        results[req.rid] = Result(rid=req.rid, probe=st.probe.cpu().numpy(), obj=st.object.cpu().numpy(),
                                  positions=st.positions.cpu().numpy(), losses=losses, iter_latency_s=lat,
                                  admitted_at=admitted, finished_at=clock() - t0)
        prob.close()
    return results


def simulate_patterns(req: ReconRequest, obj: np.ndarray, device="cuda") -> np.ndarray:
    """Poisson counts of the forward model's intensities (computed by the
    library on the device) at the request's probe and positions and the object
    `obj`, drawn on the host from the request's seed: patterns a
    reconstruction can be scored against."""
    dev = torch.device(device)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)  # noqa: E731
    # positions per forward call: a context's workspace stays near 2 GiB
    chunk = int(max(1, min(req.J, (2 << 30) // (req.M * req.N * req.N * 8 * (req.S + 2)))))
    prob = api.Problem(req.N, req.M, req.S, req.H, req.W, req.J, dz=req.dz, dx=req.dx,
                       wavelength=req.wavelength, loss=req.loss, eps=req.eps, max_batch=chunk)
    P, O, X = t(req.probe, np.complex64), t(obj, np.complex64), t(req.positions, np.float32)
    I = np.empty((req.J, req.N, req.N), dtype=np.float64)
    for a in range(0, req.J, chunk):
        b = torch.arange(a, min(a + chunk, req.J), dtype=torch.int32, device=dev)
        Ib, _ = prob.forward(P, O, X, b)
        I[a:a + len(b)] = Ib.cpu().numpy()
    prob.check()
    prob.close()
    rng = np.random.default_rng(req.seed + 104729)
    return rng.poisson(np.maximum(I, 0.0)).astype(np.float32)


def _scanned(req: ReconRequest):
    n = np.floor(np.asarray(req.positions, dtype=np.float64) + 0.5).astype(int)
    y0, x0 = n.min(axis=0)
    y1, x1 = n.max(axis=0) + req.N
    return slice(y0, y1), slice(x0, x1)


def object_error(obj: np.ndarray, req: ReconRequest) -> float:
    """Relative distance of a reconstructed object from the request's truth
    over the region its windows cover: |O - O_true| / |O_true - 1|."""
    ys, xs = _scanned(req)
    a = obj[:, ys, xs].astype(np.complex128)
    b = req.truth[:, ys, xs].astype(np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b - 1.0))


def projected_phase_error(obj: np.ndarray, req: ReconRequest) -> float:
    """Relative distance of the projected phase (sum over slices of arg O,
    mean removed: the part a thin specimen's data fix, free of how the phase
    is shared among slices and of a constant offset) from the truth's, over
    the region the windows cover."""
    ys, xs = _scanned(req)
    pa = np.angle(obj[:, ys, xs].astype(np.complex128)).sum(axis=0)
    pb = np.angle(req.truth[:, ys, xs].astype(np.complex128)).sum(axis=0)
    pa, pb = pa - pa.mean(), pb - pb.mean()
    return float(np.linalg.norm(pa - pb) / np.linalg.norm(pb))


def make_request_stream(n: int, seed: int = 0, rate_per_s: float = 2.0, n_iters: int = 50,
                        sizes=(64, 128, 192, 256), max_modes: int = 6, max_slices: int = 16,
                        scans=(16, 64), steps=(4, 8), batch: int = 256, from_model: bool = False,
                        device="cuda") -> List[ReconRequest]:
    """Poisson arrivals of reconstructions of mixed N, M, S and scan size, each
    generated from its own seed like the single-reconstruction workloads.
    With from_model, each request's patterns are Poisson counts of the forward
    model at its true object (simulate_patterns), the request starts from the
    vacuum object O = 1 with the true probe, and the truth is kept for
    object_error; otherwise the patterns are synthetic bright-field disks and
    the request starts from the true object."""
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
        req = ReconRequest(rid=k, N=N, M=M, S=S, probe=probe, obj=obj, positions=pos, patterns=pats,
                           dz=[2.0] * (S - 1), loss="amplitude" if simple else "poisson",
                           eps=0.0 if simple else 0.8, n_iters=n_iters,
                           batch=min(batch, DEFAULT_GROUP_TILES[N] // M), arrival=t, seed=rs)
        if from_model:
            req.patterns = simulate_patterns(req, obj, device)
            req.truth = obj.astype(np.complex64)
            req.obj = np.ones_like(obj)
        out.append(req)
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
