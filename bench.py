"""Throughput of the hot path on one MI355X: probe positions per second of one
gradient iteration (forward model, noise-model loss, exact adjoint to object,
probe and positions, Adam step) on the 256 x 256, 8-mode, 30-slice workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch 512]
                    [--no-cpu-baseline] [--cpu-positions n]
                    [--workload ms256_m8_s30|ms192_m6_s20|ms128_m4_s8|spoa64|serving]
                    [--engine adam|sgd|epie|lsqml|grad] [--regularize]
                    [--checkpoint-every k] [--checkpoint-half] [--strategy ...] [--chunk n] [--streams k]
                    [--profile-steps n] [--graph]
                    [--reduction auto|atomic|ordered]

A step is one reconstruct_step over one group of `batch` positions drawn
from a seeded permutation of the 128 x 128 scan (16384 positions = 32 groups
per epoch), with every input resident in HBM before the timed region; with
--engine grad it is one loss_and_grad call instead (forward model, loss and
adjoint with all three gradients, no update).
Prints one JSON line. The headline is the default: Adam, float32
checkpoints, no regularizers; the other options measure the conventional
engines, the regularizers and the storage and schedule variants on the
same workload.

Timing: by default 64 warmup groups (2 epochs) and 640 timed groups (20
epochs); per-group and per-epoch p50/p99 from HIP events. The last warmup step
times every kernel class once (HIP events around each launch, on its own
stream) to name the dominant kernel; the first 64 timed steps then time that
class's launches alone, which gives the roofline's average launch duration; a
separate pass after the timed region gives the per-class breakdown.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "probe positions/s per fwd+adjoint iteration (256², 8 modes, 30 slices); p50/p99"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3


ENGINES = {"adam": "Adam", "sgd": "SGD", "epie": "ePIE", "lsqml": "LSQML",
           "grad": "forward + adjoint only (loss and gradients, no update)"}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    # default: 2 epochs of warmup, 20 timed epochs of the 256^2 workload (32 groups each)
    p.add_argument("--steps", type=int, default=640)
    p.add_argument("--warmup", type=int, default=64)
    p.add_argument("--batch", type=int, default=0, help="positions per group (0: the workload's)")
    p.add_argument("--workload", default="ms256_m8_s30")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-positions", type=int, default=0,
                   help="positions in the oracle's CPU sample (0: 8 per host core)")
    p.add_argument("--checkpoint-every", type=int, default=1)
    p.add_argument("--chunk", type=int, default=0)
    p.add_argument("--streams", type=int, default=1,
                   help="run the chunks of a chunked schedule concurrently on this many streams")
    p.add_argument("--graph", action="store_true",
                   help="record the step once as a HIP graph and replay it (launch-bound workloads)")
    p.add_argument("--profile-steps", type=int, default=4,
                   help="steps of the separate per-kernel timing pass after the timed region; with 0 no "
                        "kernel is timed at all, also not the dominant one inside the timed steps")
    p.add_argument("--strategy", default="auto", choices=["auto", "two_pass", "resident"])
    p.add_argument("--reduction", default="auto", choices=["auto", "atomic", "ordered"],
                   help="object-gradient accumulation: float atomics or the bit-reproducible ordered sum; "
                        "auto takes the one measured faster for the workload (see FASTER_REDUCTION)")
    p.add_argument("--checkpoint-half", action="store_true",
                   help="store entry-wave checkpoints as IEEE half pairs (reduced-precision storage)")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="run one 1 GiB device-to-device copy first (reference for HBM byte counters)")
    p.add_argument("--engine", default="adam", choices=list(ENGINES),
                   help="group step: gradient descent with Adam (the headline) or SGD, the ePIE / LSQML "
                        "engines, or grad: the loss and gradients alone")
    p.add_argument("--regularize", action="store_true",
                   help="enable every cost regularizer and constraint in the step")
    p.add_argument("--requests", type=int, default=64, help="serving stream: number of reconstructions")
    p.add_argument("--max-scan", type=int, default=64, help="serving stream: largest scan side (16..max)")
    p.add_argument("--iters", type=int, default=50, help="serving stream: iterations per reconstruction")
    return p.parse_args()


def live_fraction(N, bandlimit, S):
    """Fraction of row-spectrum columns u_x that the circular band limit
    (fraction of Nyquist) keeps; the others are zero after a propagation and
    are never read (at N = 256 the passes write those that share a 128-byte
    line with live ones)."""
    if S < 2 or bandlimit <= 0:
        return 1.0
    k = np.fft.fftfreq(N) * N
    return float(np.mean(k * k <= (bandlimit * N / 2.0) ** 2 * (1 + 1e-9)))


def kernel_bytes_per_launch(name, N, M, B, S, ck_half=False, engine="adam", spectral=False, live=1.0,
                            ordered=False, chain=False):
    """Algorithmic HBM bytes one launch of a kernel class must move at an
    interior slice (complex64 tile T = 8 N^2 bytes, per launch over B
    positions and M modes; a checkpoint is T, or T/2 when stored as half
    floats; with spectral checkpoints the forward column pass writes the
    checkpoint as its output tile and the forward row pass stores nothing
    extra; of a band-limited row spectrum only the live fraction of columns
    moves; LSQML adds the read-modify-write of a float illumination sum, T per
    position; with the ordered reduction the adjoint row pass stores each
    position's object-gradient contribution, T, instead of adding it into the
    gradient, 2T); with chain (the final pass as kProbeSplit = 16 chains that
    keep the probe-gradient sums, N = 256 with 4 or more modes, unchunked) the
    final pass reads every tile and writes 16 partial tiles per mode, which the
    probe-gradient sum reads back."""
    T = 8 * N * N
    C = T // 2 if ck_half else T
    Tl = T * live
    if name == "row_fwd":      # read + write every mode tile (both band-limited), [write the checkpoint], read the object patch
        return int(B * (M * (2 * Tl + (0 if spectral else C)) + T))
    if name == "row_adj":      # read tile and checkpoint, write tile (all band-limited), read object patch, RMW gradient
        ck = Tl if spectral else C
        return int(B * (M * (2 * Tl + ck) + (2 if ordered else 3) * T) + (B * T if engine == "lsqml" else 0))
    if name in ("col_prop", "col_prop_adj"):   # read + write the live columns of every tile
        return int(B * 2 * M * Tl)
    if name == "far_loss":     # tiles read twice (the far field is recomputed, not stored), seed written; pattern read
        return B * (3 * M * T + T // 2)
    if name == "col_shift":    # write every tile (the probe spectrum stays in cache)
        return B * M * T
    if name == "col_final":    # read + write every tile, or read every tile and write the chain sums
        return B * M * T + 16 * M * T if chain else B * 2 * M * T
    if name == "probe_grad":   # read every tile, or the chain sums
        return 16 * M * T if chain else B * M * T
    return 0


def kernel_flops_per_launch(name, N, M, B, S, spectral=False):
    """FFT flops of one launch by the 5 n log2 n convention per 1D transform
    (the adjoint row pass transforms three lines per row with spectral
    checkpoints: g, the recovered entry wave and h)."""
    per_line = 5 * N * np.log2(N)
    lines = B * M * N
    n_fft = {"row_fwd": 2, "row_adj": 3 if spectral else 2, "col_prop": 2, "col_prop_adj": 2, "far_loss": 2,
             "col_shift": 1, "col_final": 1}.get(name, 0)
    return n_fft * lines * per_line


def method_flops_per_launch(name, N, M, B, S=1):
    """The method's own FFT flops in one launch (5 n log2 n per 1D line
    transform): each slice step is a 2D DFT and an inverse 2D DFT per mode,
    whose row halves run in the row passes and column halves in the column
    passes; an LDS-resident chain runs every slice in one launch (row halves of
    all S slices, column halves of the S - 1 propagations). Work a kernel does
    beyond that (the adjoint row pass recovering the entry wave from its
    spectral checkpoint, the far-field pass recomputing the far field) is
    design overhead and not counted."""
    per_line = 5 * N * np.log2(N)
    lines = B * M * N
    n_fft = {"row_fwd": 2, "row_adj": 2, "col_prop": 2, "col_prop_adj": 2, "far_loss": 2,
             "col_shift": 1, "col_final": 1, "res_fwd": 4 * S - 2, "res_adj": 4 * S - 2}.get(name, 0)
    return n_fft * lines * per_line


def step_roofline(N, M, S, t_meas_pos):
    """Roofline of the method's own work per position (the measurement plan's
    counts): flops = 4 S M 2D FFTs of 5 N^2 log2 N^2 each; bytes = the pattern
    plus the object patch read in the forward and again in the adjoint plus the
    object-gradient read-modify-write. T_roof = max(bytes / HBM peak, flops /
    FP32 peak); the step's fraction is T_roof / T_measured (seconds per
    position)."""
    flop_pos = 4 * S * M * 5 * N * N * np.log2(N * N)
    bytes_pos = N * N * 4 + 4 * S * N * N * 8
    t_alu, t_hbm = flop_pos / (FP32_PEAK_TFLOPS * 1e12), bytes_pos / (HBM_PEAK_GBS * 1e9)
    t_roof_pos = max(t_alu, t_hbm)
    return {"bound": "alu" if t_alu >= t_hbm else "hbm",
            "flops_per_position": flop_pos, "bytes_per_position": bytes_pos,
            "t_roof_us_per_position": round(t_roof_pos * 1e6, 3),
            "t_measured_us_per_position": round(t_meas_pos * 1e6, 3),
            "frac": round(t_roof_pos / t_meas_pos, 4),
            "achieved_tflops": round(flop_pos / t_meas_pos / 1e12, 2),
            "achieved_alg_GBps": round(bytes_pos / t_meas_pos / 1e9, 1)}


def method_bytes_per_launch(name, N, B, S=1):
    """The method's own HBM bytes in one launch: the object patch of the slice
    (read in the forward and again in the adjoint), the object-gradient
    read-modify-write in the adjoint and the pattern read by the loss; tiles
    are taken to stay on chip (an LDS-resident chain covers all S slices)."""
    T = 8 * N * N
    return {"row_fwd": B * T, "row_adj": 3 * B * T, "far_loss": B * 4 * N * N,
            "res_fwd": S * B * T, "res_adj": 3 * S * B * T}.get(name, 0)


# Object-gradient reduction measured faster per workload on one MI355X: the
# ordered sum pays one extra pass over the group's contributions and wins
# where atomics contend (a whole dense scan in one group, 128^2) or where the
# adjoint row pass runs one wave per SIMD (192^2); the served stream also
# becomes bit-identical to its one-at-a-time run.
FASTER_REDUCTION = {"ms256_m8_s30": "atomic", "ms192_m6_s20": "ordered", "ms128_m4_s8": "ordered",
                    "spoa64": "atomic", "serving": "ordered"}


DOM_STEPS = 64   # timed steps whose dominant-kernel launches are bracketed by events


def main():
    args = parse()
    if args.reduction == "auto":
        # the resident chains accumulate the object gradient with atomics only
        args.reduction = "atomic" if args.strategy == "resident" else FASTER_REDUCTION.get(args.workload, "atomic")
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 (how the path would shard "
                                   "over GPUs is described in the design notes)"}))
        sys.exit(2)
    import torch

    from paper_2505_14372_amd import _lib, api, synth

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    if args.workload == "serving":
        return bench_serving(args)
    dev = "cuda:0"
    t0 = time.time()
    wl = synth.make_workload(args.workload, pattern_pool=64)
    N, M, S, H, W, J = wl.N, wl.M, wl.S, wl.H, wl.W, wl.J
    B = args.batch if args.batch > 0 else wl.batch
    print(f"[bench] inputs built in {time.time() - t0:.1f}s: N={N} M={M} S={S} object {H}x{W}x{S} J={J} B={B}",
          file=sys.stderr, flush=True)
    probe = torch.from_numpy(wl.probe.astype(np.complex64)).to(dev)
    obj = torch.from_numpy(wl.obj.astype(np.complex64)).to(dev)
    pos = torch.from_numpy(wl.positions.astype(np.float32)).to(dev)
    pats = torch.empty((J, N, N), dtype=torch.float32, device=dev)
    chunk = 1024
    for s0 in range(0, J, chunk):
        pats[s0:s0 + chunk].copy_(torch.from_numpy(wl.patterns[s0:s0 + chunk]))
    prob = api.Problem(N, M, S, H, W, J, dz=wl.dz, dx=wl.dx, wavelength=wl.wavelength, loss=wl.loss, eps=wl.eps,
                       max_batch=B, checkpoint_every=args.checkpoint_every, checkpoint_half=args.checkpoint_half,
                       lsqml=args.engine == "lsqml")
    prob.set_chunk(args.chunk)
    prob.set_streams(args.streams)
    prob.set_strategy(args.strategy)
    prob.set_reduction(args.reduction)
    if args.regularize:
        k = np.fft.fftfreq(N) * N
        prob.set_regularizers(obj_l2=1e-3, probe_l2=1e-6, obj_l1=1e-3, obj_tikhonov=1e-2, obj_tv=1e-2,
                              layers_tikhonov=1e-2, layers_tv=1e-2, tv_delta=1e-2, amp_range=(0.0, 1.0),
                              probe_support=(k[:, None] ** 2 + k[None, :] ** 2) <= (N / 3) ** 2, layer_sigma=0.5,
                              obj_lowpass_sigma=0.5, phase_deramp=True)
    if args.graph and args.engine not in ("adam", "sgd", "epie"):
        raise SystemExit("--graph records reconstruct_step (engines adam, sgd, epie)")
    state = api.ReconState(probe, obj, pos, adam=args.engine == "adam", device_step=args.graph)
    rng = np.random.default_rng(12345)
    n_groups = J // B
    if args.engine == "lsqml":
        illum = api.IllumSums(S, H, W, N)
        counter = [0]

        def step(batch, loss):
            prob.lsqml_step(state, illum, pats, batch, loss=loss)
            counter[0] += 1
            if counter[0] % n_groups == 0:
                illum.end_iteration()
    elif args.engine == "grad":
        g_obj, g_probe = torch.empty_like(obj), torch.empty_like(probe)
        g_pos = torch.empty((B, 2), dtype=torch.float32, device=dev)

        def step(batch, loss):
            prob.loss_and_grad(probe, obj, pos, pats, batch, g_object=g_obj, g_probe=g_probe, g_pos=g_pos, loss=loss)
    else:
        opt = {"adam": api.Optimizer(kind="adam", lr_object=1e-3, lr_probe=1e-3, lr_pos=1e-2),
               "sgd": api.Optimizer(kind="sgd", lr_object=1e-8, lr_probe=1e-10, lr_pos=1e-8),
               "epie": api.Optimizer(kind="epie", lr_object=1.0, lr_probe=1.0)}[args.engine]

        def step(batch, loss):
            prob.reconstruct_step(state, pats, batch, opt, loss)

    step_eager = step
    if args.graph:
        # the step recorded once as a HIP graph; each step writes its group's
        # indices into the recorded index buffer and replays the graph
        g_batch = torch.empty(B, dtype=torch.int32, device=dev)
        g_loss = torch.zeros(1, dtype=torch.float64, device=dev)
        recorded = []

        def step(batch, loss):
            g_batch.copy_(batch)
            if not recorded:
                recorded.append(prob.record_step(state, pats, g_batch, opt, g_loss))
            recorded[0].replay()

    def groups():
        while True:
            perm = rng.permutation(J).astype(np.int32)
            for g in range(n_groups):
                yield torch.from_numpy(np.sort(perm[g * B:(g + 1) * B])).to(dev)

    gen = groups()
    batches = [next(gen) for _ in range(args.warmup + args.steps)]
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    lib = _lib.load()
    n_prof = min(args.profile_steps, args.steps)

    def collect():
        names = C.create_string_buffer(4096)
        tot = (C.c_double * 64)()
        cnt = (C.c_int64 * 64)()
        n_cls = lib.pty_profile_collect(names, 4096, tot, cnt, 64)
        return {nm: (tot[i], cnt[i]) for i, nm in enumerate(names.value.decode().split("\n")[:n_cls])}

    def dominant(classes):
        # the single-kernel class with the most time ("recompute" times a whole
        # segment's row and column passes together, so it has no per-launch model)
        cand = [k for k in classes if k != "recompute" and classes[k][1] > 0]
        return max(cand, key=lambda k: classes[k][0]) if cand else None

    dom = None
    for w in range(args.warmup):
        # the last warmup step times every kernel class once, to name the
        # dominant kernel whose launches the timed steps then time
        probe_step = n_prof > 0 and w == args.warmup - 1
        if probe_step:
            lib.pty_profile_select(None)
            lib.pty_profile_enable(1)
            collect()
        (step_eager if probe_step else step)(batches[w], loss)
        if probe_step:
            lib.pty_profile_enable(0)
            dom = dominant(collect())
        print(f"[bench] warmup step {w} done", file=sys.stderr, flush=True)
    prob.check()
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    # every launch of the dominant kernel class in the first DOM_STEPS timed
    # steps is bracketed by two HIP events on the stream it runs on (no other
    # class; the cap bounds the number of events held until they are read)
    if args.graph:
        dom = None   # replays record no events: the roofline takes the separate pass's timing
    dom_steps = min(args.steps, DOM_STEPS) if dom else 0
    if dom:
        if lib.pty_profile_select(dom.encode()) != 1:
            raise RuntimeError(f"unknown kernel class {dom}")
        lib.pty_profile_enable(1)
        collect()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        step(batches[args.warmup + k], loss)
        ends[k].record(stream)
        if k + 1 == dom_steps:
            lib.pty_profile_enable(0)
        if (k + 1) % 32 == 0 or k + 1 == args.steps:
            print(f"[bench] timed step {k + 1}/{args.steps} queued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    dom_timed = None
    if dom:
        lib.pty_profile_select(None)
        dom_timed = collect().get(dom)
    prob.check()
    step_ms = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    ms_per_step = t_total * 1000.0 / args.steps
    value = B * args.steps / t_total
    p50, p99 = np.percentile(step_ms, 50), np.percentile(step_ms, 99)
    # per-epoch timings: n_groups consecutive groups (the whole scan once)
    n_ep = args.steps // n_groups
    ep_ms = np.array([starts[e * n_groups].elapsed_time(ends[(e + 1) * n_groups - 1]) for e in range(n_ep)])

    # The per-class breakdown comes from a separate pass over the same groups
    # with every launch of every class bracketed by two HIP events.
    prof = {}
    prof_ms_per_step = None
    if n_prof > 0:
        lib.pty_profile_enable(1)
        collect()   # drop anything recorded before
        torch.cuda.synchronize()
        t_p = time.perf_counter()
        for k in range(n_prof):
            step_eager(batches[args.warmup + k], loss)
        torch.cuda.synchronize()
        prof_ms_per_step = (time.perf_counter() - t_p) * 1000.0 / n_prof
        lib.pty_profile_enable(0)
        prof = {nm: (v[0] / n_prof, v[1] / n_prof) for nm, v in collect().items()}
        prob.check()
        print(f"[bench] profiled pass: {n_prof} steps, {prof_ms_per_step:.2f} ms/step", file=sys.stderr, flush=True)

    step_roof = step_roofline(N, M, S, ms_per_step / 1000.0 / B)
    roof = None
    kernels = {}
    if prof:
        # the dominant kernel's average launch time over the timed steps (from
        # the separate pass only when no warmup step could name it first)
        if dom_timed and dom_timed[1] > 0:
            avg_s = dom_timed[0] / dom_timed[1] / 1000.0
            avg_src = "timed steps"
        else:
            dom = dominant(prof)
            avg_s = prof[dom][0] / prof[dom][1] / 1000.0
            avg_src = "separate pass"
        spectral = not prob.checkpoint_half and args.strategy != "resident"
        live = live_fraction(N, wl.bandlimit, S)
        n_launch = B if args.chunk <= 0 else min(args.chunk, B)   # positions one launch processes
        alg_flops = method_flops_per_launch(dom, N, M, n_launch, S)
        alg_bytes = method_bytes_per_launch(dom, N, n_launch, S)
        chain = N == 256 and M >= 4 and args.chunk <= 0
        design_bytes = kernel_bytes_per_launch(dom, N, M, n_launch, S, prob.checkpoint_half, args.engine, spectral,
                                               live, args.reduction == "ordered", chain)
        tfl = alg_flops / avg_s / 1e12
        gbs = alg_bytes / avg_s / 1e9
        if alg_flops / (FP32_PEAK_TFLOPS * 1e12) >= alg_bytes / (HBM_PEAK_GBS * 1e9):
            roof = {"bound": "alu", "achieved": round(tfl, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(tfl / FP32_PEAK_TFLOPS, 4)}
        else:
            roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4)}
        # the committed counter summary covers the default configuration only
        default_cfg = (args.workload == "ms256_m8_s30" and B == 512 and prob.checkpoint_every == 1 and
                       not prob.checkpoint_half and args.engine == "adam" and not args.regularize and
                       args.strategy != "resident" and args.chunk == 0 and args.reduction == "atomic")
        traffic = measured_traffic(dom) if default_cfg else None
        roof.update({"traffic": traffic, "kernel": dom, "avg_launch_ms": round(avg_s * 1000, 4),
                     "avg_launch_from": avg_src,
                     "launches_timed": int(dom_timed[1]) if dom_timed and avg_src == "timed steps" else None,
                     "positions_per_launch": n_launch, "algorithmic_flops": alg_flops,
                     "algorithmic_bytes": alg_bytes, "achieved_alg_GBps": round(gbs, 1),
                     "design_bytes": design_bytes, "stream_GBps": round(design_bytes / avg_s / 1e9, 1)})
        kernels = {k: {"ms_per_step": round(v[0], 3), "launches_per_step": round(v[1], 2),
                       "avg_ms": round(v[0] / v[1], 4), "share": round(v[0] / sum(x[0] for x in prof.values()), 4)}
                   for k, v in prof.items()}
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "positions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: probe {N}x{N}, {M} modes, {S} slices of {wl.dz[0] if S > 1 else 0} A, "
                               f"object {H}x{W}x{S} complex64, {J} positions, groups of {B}, {wl.loss} loss, "
                               f"{ENGINES[args.engine]}{', all regularizers' if args.regularize else ''}",
                   "global_batch": B, "checkpoint_every": prob.checkpoint_every,
                   "checkpoint_storage": "f16" if prob.checkpoint_half else "f32", "strategy": args.strategy,
                   "reduction": args.reduction, "engine": args.engine, "regularizers": bool(args.regularize),
                   "graph": bool(args.graph)},
        "p50_ms_per_group": round(float(p50), 3), "p99_ms_per_group": round(float(p99), 3),
        "positions_per_s_p50": round(B / (p50 / 1000.0), 1), "positions_per_s_p99": round(B / (p99 / 1000.0), 1),
        "epochs_timed": int(n_ep),
        "epoch_s_p50": round(float(np.percentile(ep_ms, 50)) / 1000.0, 4) if n_ep else None,
        "positions_per_s_epoch_p50": round(n_groups * B / (float(np.percentile(ep_ms, 50)) / 1000.0), 1) if n_ep else None,
        "positions_per_s_epoch_p99": round(n_groups * B / (float(np.percentile(ep_ms, 99)) / 1000.0), 1) if n_ep else None,
        "fft_tflops_per_s": round(step_roof["flops_per_position"] * value / 1e12, 2),
        "roofline": roof, "step_roofline": step_roof, "kernels": kernels,
        "profiled_pass_ms_per_step": round(prof_ms_per_step, 3) if prof_ms_per_step else None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_positions)
    print(json.dumps(out), flush=True)


def kernel_source_hash():
    """sha256 of the kernel sources with comments and whitespace removed, so
    that a comment edit does not orphan counters taken on the same code."""
    import hashlib
    import re
    h = hashlib.sha256()
    for p in ("pty_kernels.hip", "pty_fft.hpp", "pty_internal.h"):
        with open(os.path.join(ROOT, "paper_2505_14372_amd", "csrc", p)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_ms256_m8_s30_b512.md")
    try:
        text = open(path).read()
        data = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if data.get("source_sha256") != kernel_source_hash() or kernel not in data.get("kernels", {}):
        return None
    k = data["kernels"][kernel]
    return int(k["fetch_bytes"] + k["write_bytes"])


def bench_serving(args):
    """Served mixed-size stream against one reconstruction at a time (same
    requests, same minibatch order), on one GPU."""
    import torch

    from paper_2505_14372_amd import serving
    t0 = time.time()
    reqs = serving.make_request_stream(args.requests, seed=0, rate_per_s=2.0, n_iters=args.iters,
                                       scans=(16, args.max_scan), from_model=True)
    work = sum(r.J * r.n_iters for r in reqs)
    print(f"[bench] {len(reqs)} requests built in {time.time() - t0:.1f}s, "
          f"{work} position-iterations", file=sys.stderr, flush=True)
    srv = serving.Server(hbm_budget=int(0.5 * torch.cuda.get_device_properties(0).total_memory),
                         reduction=args.reduction)
    for r in reqs:
        srv.submit(r)
    t1 = time.perf_counter()
    served = srv.run(log=lambda m: print("[bench] served " + m, file=sys.stderr, flush=True))
    t_served = time.perf_counter() - t1
    print(f"[bench] served stream done in {t_served:.1f}s", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    fifo = serving.run_fifo(reqs, reduction=args.reduction)
    t_fifo = time.perf_counter() - t1
    print(f"[bench] one-at-a-time done in {t_fifo:.1f}s", file=sys.stderr, flush=True)
    p50, p99 = serving.latency_stats(served)
    f50, f99 = serving.latency_stats(fifo)
    q50, q99 = serving.request_latency_stats(served, reqs)
    g50, g99 = serving.request_latency_stats(fifo, reqs)
    diff = 0.0
    for r in reqs:
        a, b = served[r.rid].obj, fifo[r.rid].obj
        diff = max(diff, float(np.linalg.norm(a - b) / np.linalg.norm(b)))
    # accuracy: distance from the true object (patterns simulated from it, start at O = 1)
    err_s = np.array([serving.object_error(served[r.rid].obj, r) for r in reqs])
    err_f = np.array([serving.object_error(fifo[r.rid].obj, r) for r in reqs])
    err_0 = np.array([serving.object_error(r.obj, r) for r in reqs])
    perr_s = np.array([serving.projected_phase_error(served[r.rid].obj, r) for r in reqs])
    perr_f = np.array([serving.projected_phase_error(fifo[r.rid].obj, r) for r in reqs])
    fall = np.array([fifo[r.rid].losses[-1] / fifo[r.rid].losses[0] for r in reqs])
    fall_s = np.array([served[r.rid].losses[-1] / served[r.rid].losses[0] for r in reqs])
    out = {
        "metric": "probe positions x iterations/s of a served stream of mixed reconstructions",
        "value": round(work / t_served, 1), "unit": "position-iterations/s", "n_gpus": 1, "steps": len(reqs),
        "warmup": 0, "ms_per_step": round(1000 * t_served / len(reqs), 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"serving: {len(reqs)} Poisson arrivals (2/s), probe 64-256, 1-6 modes, "
                               f"1-16 slices, 16^2-{args.max_scan}^2 scans, {args.iters} Adam iterations each, "
                               "patterns simulated from each request's true object, start from vacuum",
                   "reduction": args.reduction},
        "iteration_latency_p50_s": round(p50, 4), "iteration_latency_p99_s": round(p99, 4),
        "request_latency_p50_s": round(q50, 3), "request_latency_p99_s": round(q99, 3),
        "one_at_a_time": {"value": round(work / t_fifo, 1), "iteration_latency_p50_s": round(f50, 4),
                          "iteration_latency_p99_s": round(f99, 4), "request_latency_p50_s": round(g50, 3),
                          "request_latency_p99_s": round(g99, 3), "wall_s": round(t_fifo, 2)},
        "served_over_one_at_a_time": round(t_fifo / t_served, 3),
        "max_rel_object_diff_served_vs_alone": diff, "rounds": srv.rounds,
        "accuracy": {"object_error_served_mean": round(float(err_s.mean()), 5),
                     "object_error_one_at_a_time_mean": round(float(err_f.mean()), 5),
                     "object_error_start_mean": round(float(err_0.mean()), 5),
                     "projected_phase_error_served_mean": round(float(perr_s.mean()), 5),
                     "projected_phase_error_one_at_a_time_mean": round(float(perr_f.mean()), 5),
                     "last_over_first_iteration_loss_served_mean": round(float(fall_s.mean()), 5),
                     "last_over_first_iteration_loss_one_at_a_time_mean": round(float(fall.mean()), 5),
                     "max_abs_diff_served_vs_alone": float(max(np.max(np.abs(err_s - err_f)),
                                                               np.max(np.abs(perr_s - perr_f)))),
                     "definition": "patterns are Poisson counts of the forward model at each request's true "
                                   "object, start O = 1; object error |O - O_true| / |O_true - 1| and projected "
                                   "phase error |sum_i arg O_i - truth's| / |truth's| (means removed) over the "
                                   "scanned region"},
    }
    print(json.dumps(out), flush=True)


CPU_SHARE = 16


def cpu_baseline(wl, n_pos):
    """The FP64 oracle on the host: loss and gradients of a small group of the
    same workload, one oracle call per position on a thread pool over every
    core this process may run on (numpy's FFTs release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle as orc
    geom = orc.Geometry(N=wl.N, dx=wl.dx, wavelength=wl.wavelength, dz=list(wl.dz), bandlimit=wl.bandlimit,
                        loss=wl.loss, eps=wl.eps, sigma=wl.sigma)
    # every core this process may run on, capped at the host share one GPU's
    # job is given (16 cores), whatever the affinity mask lists
    cores = min(len(os.sched_getaffinity(0)), CPU_SHARE)
    if n_pos <= 0:
        n_pos = 8 * cores
    idx = list(range(0, wl.J, max(1, wl.J // n_pos)))[:n_pos]
    parts = [idx[k::cores] for k in range(cores) if idx[k::cores]]
    P = wl.probe.astype(np.complex64).astype(np.complex128)
    O = wl.obj.astype(np.complex64).astype(np.complex128)
    X = wl.positions.astype(np.float32).astype(np.float64)
    pats = {j: wl.patterns[j].astype(np.float64) for j in idx}
    patt = _PatternView(pats)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=len(parts)) as ex:
        list(ex.map(lambda part: orc.loss_and_grad(P, O, X, patt, part, geom), parts))
    dt = time.perf_counter() - t0
    return {"value": round(len(idx) / dt, 3), "unit": "positions/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(idx)} positions of the same workload (all {wl.M} modes, {wl.S} slices) split "
                      f"over {len(parts)} threads, one oracle loss_and_grad call per thread, numpy FP64, "
                      f"{dt:.1f} s"}


class _PatternView:
    """Index-only view of the sampled patterns (the oracle reads patterns[j])."""

    def __init__(self, d):
        self.d = d

    def __getitem__(self, j):
        return self.d[int(j)]


if __name__ == "__main__":
    main()
