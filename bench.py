#!/usr/bin/env python3
"""Benchmark of the FireANTs dense matching step on one MI355X.

One *step* is one whole registration of the 160x192x224 tissue pair:
building the three-level pyramid (4x, 2x, 1x) and running 200/100/50
iterations of Algorithm 1 (warp, LNCC, adjoint, Adam, smoothing, composition,
level upsampling).  The metric is voxel-iterations per second,
sum_l N_l T_l / (seconds per step), with the input volumes already resident
in device memory when timing starts.

Prints one JSON line.  Besides the headline value it reports
* ``roofline``: the dominant kernel's algorithmic HBM bytes per launch over
  its average launch time, measured with HIP events on the pair's stream
  around every launch of two registrations run after the timed ones, against
  the 8 TB/s HBM peak;
* ``plain_torch``: the same algorithm written with stock PyTorch operators
  (grid_sample, conv3d, autograd, elementwise Adam) on the same GPU;
* ``batch``: aggregate throughput of several registrations (step sizes of
  the paper's grid search) advanced together, on separate streams and by
  batched launches (one launch per kernel for all of them), against the same
  registrations run one after another;
* ``grid_search``: a hyperparameter grid search as one fused batch: pairs of
  three sizes, each at four step sizes (96 registrations), against the same
  registrations run one after another;
* ``inverse``: the post hoc inverse of the result (psi = phi^{-1} fitted by
  the same loop on the inverse-consistency cost): time per fit and the final
  cost;
* ``lncc128``: the fused LNCC cost and gradient (the differentiable loss of
  fa_lncc.h) against PyTorch autograd of grid_sample + conv3d LNCC, 128^3,
  windows 5^3 and 9^3;
* ``microscopy512``: the 512^3 microscopy-like workload (LNCC 7^3, four
  levels): time per registration and the per-level kernel split;
* ``autotuned``: the same registration with launch shapes picked on this GPU
  by fa_pair_autotune (tuning outside the timed region);
* ``symmetric``: the symmetric registration (two half-way warps, then
  phi = phi_M o phi_F^{-1}): time per registration relative to the
  asymmetric one, and its accuracy;
* ``use_jac``: the same registration with Algorithm 1's use_jac on (the
  Eulerian direction J(phi)^T dU/dphi), its time relative to the default
  Jacobian-free form, and its accuracy;
* ``accuracy``: Dice of the transferred tissue labels and the fraction of
  singular voxels for the fused result and the plain PyTorch result (the
  "same accuracy" condition of the comparison);
* ``lung_ct_params``: the same registration with the paper's lung CT
  (EMPIRE10) hyperparameters, eta 0.25, sigma_grad 6, sigma_warp 0.4;
* ``cpu_baseline``: the FP64 NumPy oracle timed on the host, on a bounded
  sample of the same workload, on one core (with the host's core count) and
  as independent runs in parallel processes.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "voxel-iters/sec @160×192×224 fused vs plain per-op GPU, same accuracy"
HBM_PEAK_GBS = 8000.0
GRAD_BYTES_PER_VOXEL = 80   # reads I_f, I_m, d(3), m(3), v(3); writes m(3), v(3), a(3); fp32
# the counters depend on the kernels and on the launch shapes the runtime picks
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_2404_01249_amd", "csrc", f)
                   for f in ("fa_kernels.hip", "fa_runtime.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_grad_tissue160_traffic.json")
# Inverse fit inside the symmetric registration: half the iterations of the
# standalone inverse leg.  On the 160x192x224 workload it takes 22 ms against
# 44 ms, for Dice 0.9688 against 0.9693 and the same singular-voxel fraction.
SYM_INVERSE_ITERS = [50, 25, 12]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for src in TRAFFIC_SOURCES:
        with open(src, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the gradient kernel at the finest level, from
    the committed rocprofv3 counter summary, if it was taken on the current
    kernel and runtime sources (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def level_voxels(shape, scales, iters):
    out = []
    for s, t in zip(scales, iters):
        n = 1
        for dim in shape:
            n *= max(1, int(dim / float(s) + 0.5))
        out.append((n, t))
    return out


def run_fused(p, steps, warmup, params, prof_steps=2):
    """Times `steps` registrations after `warmup`, then runs `prof_steps` more
    with per-kernel HIP events (kept out of the timed region: recording the
    events costs GPU time of its own)."""
    import torch

    from paper_2404_01249_amd import Pair, fa
    fixed = torch.from_numpy(p.fixed).cuda()
    moving = torch.from_numpy(p.moving).cuda()
    stream = torch.cuda.current_stream()
    pr = Pair(fixed, moving, stream=stream, **params)
    for _ in range(warmup):
        pr.set_schedule(p.scales, p.iters)
        pr.run()
    torch.cuda.synchronize()
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    marks[0].record(stream)
    for k in range(steps):
        pr.set_schedule(p.scales, p.iters)
        pr.run()
        marks[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = marks[0].elapsed_time(marks[-1]) / steps
    per_run = sorted(marks[k].elapsed_time(marks[k + 1]) for k in range(steps))
    median_ms = per_run[steps // 2] if steps % 2 else 0.5 * (per_run[steps // 2 - 1] + per_run[steps // 2])
    loss = pr.loss_history()
    field = pr.field()
    fa.fa_pair_profile(pr.handle, True)
    for _ in range(prof_steps):
        pr.set_schedule(p.scales, p.iters)
        pr.run()
    prof = {}
    for lvl in range(len(p.scales)):
        prof[lvl] = [fa.fa_pair_get_profile(pr.handle, lvl, k) for k in range(4)]
    fa.fa_pair_profile(pr.handle, False)
    torch.cuda.synchronize()
    pr.close()
    return ms, median_ms, wall / steps, prof, loss, field


def run_steady_graph(p, params, short=10, long=60, reps=5):
    """Steady-state finest-level time per iteration from HIP-graph replay.

    One pair on a single-level schedule at scale 1 (more iterations than are
    run) is advanced through fa_batch_step_fused with graph capture on.  Each
    call runs its first iteration eagerly, captures the next and replays the
    rest, so a call of `long` iterations and one of `short` differ by
    long - short replayed iterations; their HIP-event times (on the pair's
    stream, which the call joins) differ by those alone.  Median over `reps`
    such differences after one warm-up pair of calls; microseconds."""
    import statistics

    import torch

    from paper_2404_01249_amd import Pair, run_batch
    fixed = torch.from_numpy(p.fixed).cuda()
    moving = torch.from_numpy(p.moving).cuda()
    stream = torch.cuda.current_stream()
    pr = Pair(fixed, moving, stream=stream, **params)
    pr.set_schedule([1.0], [1 << 20])

    def timed(n):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        run_batch([pr], max_iters=n, graphs=True)
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    timed(short)
    timed(long)
    diffs = []
    for _ in range(reps):
        t_short = timed(short)
        t_long = timed(long)
        diffs.append((t_long - t_short) / (long - short) * 1e3)
    pr.close()
    return statistics.median(diffs)


def run_use_jac(p, steps, params):
    """Whole registrations with Algorithm 1's use_jac on (Eulerian descent,
    Section 4.4.2): milliseconds per registration and the final loss."""
    import torch

    from paper_2404_01249_amd import Pair
    fixed = torch.from_numpy(p.fixed).cuda()
    moving = torch.from_numpy(p.moving).cuda()
    stream = torch.cuda.current_stream()
    pr = Pair(fixed, moving, stream=stream, use_jac=True, **params)
    pr.set_schedule(p.scales, p.iters)
    pr.run()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        pr.set_schedule(p.scales, p.iters)
        pr.run()
    end.record(stream)
    torch.cuda.synchronize()
    loss = pr.loss_history()
    field = pr.field()
    pr.close()
    return start.elapsed_time(end) / steps, float(loss[-1]), field


def run_inverse(field, steps, params):
    """The post hoc inverse of the registration's result (fa_inverse.h):
    psi = phi^{-1} fitted over scales 4, 2, 1 at 100, 50, 25 iterations with
    eta 0.2.  Returns milliseconds per fit (HIP events, after a warm-up fit),
    the voxel-iterations of one fit and the cost history."""
    import torch

    from paper_2404_01249_amd import Inverse
    scales, iters = [4.0, 2.0, 1.0], [100, 50, 25]
    stream = torch.cuda.current_stream()
    shp = tuple(int(n) for n in field.shape[1:])
    vox = sum(int(np.prod([max(1, int(np.floor(n / s + 0.5))) for n in shp])) * it for s, it in zip(scales, iters))
    inv = Inverse(field.contiguous(), eta=0.2, sigma_grad=params["sigma_grad"], sigma_warp=params["sigma_warp"],
                  stream=stream)
    inv.set_schedule(scales, iters)
    inv.run()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        inv.set_schedule(scales, iters)
        inv.run()
    end.record(stream)
    torch.cuda.synchronize()
    loss = inv.loss_history()
    inv.close()
    return start.elapsed_time(end) / steps, vox, loss


def run_autotuned(p, steps, params):
    """The workload with the launch shapes picked by fa_pair_autotune on this
    GPU (the best of three runs of 10 launches per candidate), tuned once; the timed registrations'
    schedules take the kept shapes.  Returns milliseconds per registration
    (HIP events, after a warm-up), the tuning time in seconds, the final loss
    and the chosen shapes per level.  The kept shapes are cleared at the
    end."""
    import torch

    from paper_2404_01249_amd import Pair
    fixed = torch.from_numpy(p.fixed).cuda()
    moving = torch.from_numpy(p.moving).cuda()
    stream = torch.cuda.current_stream()
    pr = Pair(fixed, moving, stream=stream, **params)
    from paper_2404_01249_amd import fa
    pr.set_schedule(p.scales, p.iters)
    t0 = time.perf_counter()
    pr.autotune(trials=10)
    tune_s = time.perf_counter() - t0
    pr.run()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        pr.set_schedule(p.scales, p.iters)
        pr.run()
    end.record(stream)
    torch.cuda.synchronize()
    shapes = {f"level{l}": [list(pr.tiling(l, k)) for k in range(4)] for l in range(len(p.scales))}
    loss = pr.loss_history()
    pr.close()
    fa.fa_autotune_clear()
    return start.elapsed_time(end) / steps, tune_s, float(loss[-1]), shapes


def run_lncc128(reps=20):
    """The fused LNCC cost and gradient (fa_lncc.h) on the 128^3 gradient-check
    pair at a seeded smooth displacement (max 2 voxels), windows 5^3 and 9^3,
    against the same cost written with PyTorch operators (grid_sample warp,
    conv3d window sums) and differentiated by autograd.  Per window:
    milliseconds per forward + backward for the fused autograd Function, for
    the single fused pass (loss_and_grad) and for PyTorch autograd (HIP
    events, mean of `reps` after a warm-up), and the relative L2 difference of
    the two gradients."""
    import torch

    import bench_plain
    from paper_2404_01249_amd import LNCC, synth
    p = synth.load("blobs128")
    fixed = torch.from_numpy(p.fixed).cuda()
    moving = torch.from_numpy(p.moving).cuda()
    d0 = torch.from_numpy(synth.smooth_field(p.fixed.shape, 31, sigma=6.0, max_norm=2.0)).cuda()
    stream = torch.cuda.current_stream()
    shape = tuple(p.fixed.shape)
    ident = torch.stack(torch.meshgrid(*[torch.arange(n, device="cuda", dtype=torch.float32) for n in shape],
                                       indexing="ij"))[None]
    out = {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(reps):
            r = fn()
        end.record(stream)
        torch.cuda.synchronize()
        return start.elapsed_time(end) / reps, r

    for w in (5, 9):
        lncc = LNCC(shape, window=w)
        n = bench_plain.box(torch.ones((1, 1) + shape, device="cuda"), w)
        If, Im = fixed[None, None], moving[None, None]

        def fused_autograd():
            d = d0.clone().requires_grad_(True)
            lncc(fixed, moving, d).backward()
            return d.grad

        def fused_pass():
            return lncc.loss_and_grad(fixed, moving, d0)[1]

        def torch_autograd():
            d = d0[None].clone().requires_grad_(True)
            J = bench_plain.warp(Im, ident + d)
            bench_plain.lncc_loss(If, J, w, 1e-5, n).backward()
            return d.grad[0]

        ms_f, g_f = timed(fused_autograd)
        ms_p, _ = timed(fused_pass)
        ms_t, g_t = timed(torch_autograd)
        rel = float((g_f - g_t).norm() / g_t.norm())
        out[f"window{w}"] = {"fused_autograd_ms": ms_f, "fused_single_pass_ms": ms_p, "torch_autograd_ms": ms_t,
                             "speedup_autograd": ms_t / ms_f, "grad_rel_l2_vs_torch": rel}
        lncc.close()
    return out


def run_microscopy512(steps, params):
    """The 512^3 microscopy-like workload (synth.microscopy_pair, seed 5):
    LNCC 7^3 over scales 8, 4, 2, 1 at 200, 200, 100, 50 iterations.  Returns
    milliseconds per registration (HIP events, after a warm-up), the
    voxel-iterations of one registration, the first and last loss, the
    generation time, the per-level kernel split (HIP events, one more
    registration) and the milliseconds per registration with launch shapes
    from fa_pair_autotune."""
    import torch

    from paper_2404_01249_amd import Pair, fa, synth
    t0 = time.perf_counter()
    mp = synth.microscopy_pair((512, 512, 512), seed=5)
    gen_s = time.perf_counter() - t0
    scales, iters = [8.0, 4.0, 2.0, 1.0], [200, 200, 100, 50]
    vox = sum(int(np.prod([max(1, int(np.floor(512 / s + 0.5)))] * 3)) * it for s, it in zip(scales, iters))
    fixed = torch.from_numpy(mp.fixed).cuda()
    moving = torch.from_numpy(mp.moving).cuda()
    del mp
    stream = torch.cuda.current_stream()
    kw = dict(params)
    kw["window"] = 7
    pr = Pair(fixed, moving, stream=stream, **kw)
    pr.set_schedule(scales, iters)
    pr.run()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        pr.set_schedule(scales, iters)
        pr.run()
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / steps
    loss = pr.loss_history()
    # the same with launch shapes tuned on this GPU (kept for the process until cleared)
    pr.set_schedule(scales, iters)
    pr.autotune(trials=5)
    pr.run()
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        pr.set_schedule(scales, iters)
        pr.run()
    end.record(stream)
    torch.cuda.synchronize()
    tuned_ms = start.elapsed_time(end) / steps
    fa.fa_autotune_clear()
    fa.fa_pair_profile(pr.handle, True)
    pr.set_schedule(scales, iters)
    pr.run()
    split = {}
    for lvl in range(len(scales)):
        row = {}
        for kind, name in ((0, "grad_adam"), (1, "smooth_max"), (3, "compose"), (2, "smooth_warp")):
            tot, n = fa.fa_pair_get_profile(pr.handle, lvl, kind)
            row[name] = round(tot / max(n, 1) * 1e3, 1)
        split[f"level{lvl}"] = row
    fa.fa_pair_profile(pr.handle, False)
    pr.close()
    return ms, vox, float(loss[0]), float(loss[-1]), gen_s, split, tuned_ms


def run_symmetric(p, steps, params):
    """Symmetric registration of the workload (fa_symmetric.h): the two
    half-way warps over the workload's schedule, then phi_F inverted over
    scales 4, 2, 1 at 50, 25, 12 (eta 0.2) and composed with phi_M.
    Returns milliseconds per registration (HIP events, after a warm-up), the
    half-way cost history and the final field."""
    import torch

    from paper_2404_01249_amd import Symmetric
    fixed = torch.from_numpy(p.fixed).cuda()
    moving = torch.from_numpy(p.moving).cuda()
    stream = torch.cuda.current_stream()
    sy = Symmetric(fixed, moving, stream=stream, **params)

    def once():
        sy.set_schedule(p.scales, p.iters)
        sy.run()
        return sy.finish([4.0, 2.0, 1.0], SYM_INVERSE_ITERS, eta=0.2, sigma_grad=params["sigma_grad"],
                         sigma_warp=params["sigma_warp"])

    once()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        d = once()
    end.record(stream)
    torch.cuda.synchronize()
    loss = sy.loss_history()
    sy.close()
    return start.elapsed_time(end) / steps, loss, d


def run_batch_compare(p, k, params):
    """k registrations of the workload, one per step size of the paper's
    grid-search range (eta in 0.25, 0.5, 1, 2): one after another on one
    stream, advanced together on k streams (fa_batch_step), and advanced
    together by batched launches (fa_batch_step_fused).  Returns the seconds
    of each form (HIP-synchronised wall clock) after a warm-up."""
    import torch

    from paper_2404_01249_amd import Pair, run_batch
    etas = [0.25, 0.5, 1.0, 2.0, 0.375, 0.75, 1.5, 3.0][:k]
    fixed = torch.from_numpy(p.fixed).cuda()
    moving = torch.from_numpy(p.moving).cuda()
    base = {kk: vv for kk, vv in params.items() if kk != "eta"}
    streams = [torch.cuda.Stream() for _ in etas]
    pairs = [Pair(fixed, moving, stream=st, eta=e, **base) for st, e in zip(streams, etas)]
    torch.cuda.synchronize()

    def sequential():
        for pr in pairs:
            pr.set_schedule(p.scales, p.iters)
            pr.run()
            pr.stream.synchronize()

    def together():
        for pr in pairs:
            pr.set_schedule(p.scales, p.iters)
        run_batch(pairs, fused=False)
        torch.cuda.synchronize()

    def fused():
        for pr in pairs:
            pr.set_schedule(p.scales, p.iters)
        run_batch(pairs, fused=True)
        torch.cuda.synchronize()

    out = {}
    for name, fn in (("sequential", sequential), ("batched", together), ("fused", fused)):
        fn()
        t0 = time.perf_counter()
        fn()
        out[name] = time.perf_counter() - t0
    for pr in pairs:
        pr.close()
    return out


GRID_SIZES = [(96, 96, 96), (128, 160, 128), (160, 192, 224)]


def _grid_pair(args):
    """Worker: one pair of the grid-search batch (blob volume as in the 64^3
    workload, blob widths scaled to the size), seed 400 + i."""
    shp, seed = args
    from paper_2404_01249_amd import synth
    sp = synth.blobs_pair(shp, seed=seed, n_blobs=20, sigma_range=(4.0 * min(shp) / 64, 8.0 * min(shp) / 64),
                          field_sigma=6.0, field_max=3.0)
    return sp.fixed, sp.moving


def grid_pairs(n_per_size, workers):
    """The n_per_size seeded pairs of each size (seeds 400 + i, i counting
    over all pairs), generated in a pool of worker processes."""
    jobs = [(shp, 400 + k * n_per_size + i) for k, shp in enumerate(GRID_SIZES) for i in range(n_per_size)]
    if workers <= 1:
        return jobs, [_grid_pair(j) for j in jobs]
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(workers) as pool:
        return jobs, pool.map(_grid_pair, jobs)


def run_grid_search(n_per_size, params, sequential_too=True, workers=8):
    """The grid-search batch: n_per_size seeded pairs of each of three sizes
    (96^3, 128x160x128, 160x192x224), each registered at four step sizes
    (eta 0.25, 0.5, 1, 2) over scales 2, 1 at 100, 50 iterations.  Returns the
    seconds of the registrations run one after another and as one fused batch
    (eager, with graph replay, and with launch shapes picked by the autotuner
    on one pair of each size), the voxel-iterations of the batch and the
    generation time."""
    import torch

    from paper_2404_01249_amd import Pair, fa, run_batch
    etas = [0.25, 0.5, 1.0, 2.0]
    scales, iters = [2.0, 1.0], [100, 50]
    base = {k: v for k, v in params.items() if k != "eta"}
    g0 = time.perf_counter()
    jobs, vols = grid_pairs(n_per_size, workers)
    gen_s = time.perf_counter() - g0
    pairs, vox_iters, firsts = [], 0, {}
    for (shp, _), (fx, mv) in zip(jobs, vols):
        f = torch.from_numpy(fx).cuda()
        m = torch.from_numpy(mv).cuda()
        for e in etas:
            pairs.append(Pair(f, m, eta=e, **base))
            firsts.setdefault(shp, pairs[-1])
            vox_iters += sum(int(np.prod([int(np.floor(n / s + 0.5)) for n in shp])) * it
                             for s, it in zip(scales, iters))
    del vols
    torch.cuda.synchronize()

    def sequential():
        for pr in pairs:
            pr.set_schedule(scales, iters)
            pr.run()
        torch.cuda.synchronize()

    def fused():
        for pr in pairs:
            pr.set_schedule(scales, iters)
        run_batch(pairs, fused=True)
        torch.cuda.synchronize()

    def fused_graphs():
        for pr in pairs:
            pr.set_schedule(scales, iters)
        run_batch(pairs, fused=True, graphs=True)
        torch.cuda.synchronize()

    out = {"registrations": len(pairs), "voxel_iters": vox_iters, "generation_s": gen_s}
    forms = (("sequential", sequential), ("fused", fused), ("fused_graphs", fused_graphs)) if sequential_too \
        else (("fused", fused),)
    for name, fn in forms:
        fn()
        t0 = time.perf_counter()
        fn()
        out[name] = time.perf_counter() - t0
    # autotuned: shapes timed on one pair of each size (kept per level grid, so
    # every pair of that size takes them; batched launches keep tuned chunks)
    t0 = time.perf_counter()
    for pr in firsts.values():
        pr.set_schedule(scales, iters)
        pr.autotune(trials=3)
    torch.cuda.synchronize()
    out["tuning_s"] = time.perf_counter() - t0
    fused()
    t0 = time.perf_counter()
    fused()
    out["fused_tuned"] = time.perf_counter() - t0
    fa.fa_autotune_clear()      # the kept shapes are process-wide
    for pr in pairs:
        pr.close()
    return out


def run_plain(p, steps, warmup, params):
    import torch

    import bench_plain
    fixed = torch.from_numpy(p.fixed).cuda()
    moving = torch.from_numpy(p.moving).cuda()
    for _ in range(warmup):
        bench_plain.register(fixed, moving, p.scales, p.iters, **params)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        d, losses = bench_plain.register(fixed, moving, p.scales, p.iters, **params)
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps, losses, d.contiguous()


def accuracy(p, d):
    """Dice of the moving labels transferred by d against the fixed labels
    (mean over the 4 tissue classes) and the singular-voxel fraction,
    computed by the library's evaluation kernels."""
    import torch

    from paper_2404_01249_amd import evaluate
    if p.fixed_labels is None:
        return {}
    fl = torch.from_numpy(p.fixed_labels).cuda()
    ml = torch.from_numpy(p.moving_labels).cuda()
    return {"dice": evaluate.dice(evaluate.warp_labels(ml, d), fl, 4),
            "singular_fraction": evaluate.singular_fraction(d)}


def _oracle_iterations(args):
    """Worker of the parallel oracle leg: n_it iterations of the FP64 oracle
    at the finest level from the identity state (one process, one thread).
    Returns (iterations, wall seconds, voxels)."""
    name, params, n_it = args
    import oracle as O
    from paper_2404_01249_amd import synth
    p = synth.load(name)
    P = O.Params(eta=params["eta"], sigma_grad=params["sigma_grad"], sigma_warp=params["sigma_warp"],
                 window=params["window"])
    f = p.fixed.astype(np.float64)
    mv = p.moving.astype(np.float64)
    d = np.zeros((3,) + f.shape)
    m = np.zeros_like(d)
    v = np.zeros_like(d)
    w0 = time.perf_counter()
    for k in range(n_it):
        d, m, v, _, _ = O.iterate(f, mv, d, m, v, k + 1, P)
    return n_it, time.perf_counter() - w0, f.size


def cpu_parallel(p, params, processes, n_it):
    """P independent oracle runs at once (P processes of one thread each, as
    independent registrations of a batch would run): aggregate
    voxel-iterations per second over the wall time of the whole pool."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")     # the parent has initialised the GPU: no fork
    w0 = time.perf_counter()
    with ctx.Pool(processes) as pool:
        res = pool.map(_oracle_iterations, [(p.name, params, n_it)] * processes)
    wall = time.perf_counter() - w0
    vox_its = sum(r[0] * r[2] for r in res)
    return {"processes": processes, "cores": processes, "value": vox_its / wall, "unit": "voxel-iters/s",
            "wall_s": wall, "per_process_s": [round(r[1], 2) for r in res],
            "sample": f"{processes} processes x {n_it} oracle iteration(s) at the finest level, one thread each "
                      f"(wall clock of the pool, process start and input loading included)"}


def cpu_baseline(p, params, budget_s=20.0, processes=0):
    """The FP64 oracle on a bounded sample: iterations at the finest level
    from the identity state until ~budget_s of CPU time is spent; then, with
    processes > 1, that many independent oracle runs at once."""
    import numpy as np

    import oracle as O
    P = O.Params(eta=params["eta"], sigma_grad=params["sigma_grad"], sigma_warp=params["sigma_warp"],
                 window=params["window"])
    f = p.fixed.astype(np.float64)
    m_ = p.moving.astype(np.float64)
    d = np.zeros((3,) + f.shape)
    m = np.zeros_like(d)
    v = np.zeros_like(d)
    n_it = 0
    t0 = time.process_time()
    w0 = time.perf_counter()
    while True:
        n_it += 1
        d, m, v, L, _ = O.iterate(f, m_, d, m, v, n_it, P)
        if time.process_time() - t0 >= budget_s or n_it >= 50:
            break
    cpu = time.process_time() - t0
    wall = time.perf_counter() - w0
    rate = f.size * n_it / wall
    out = {"value": rate, "unit": "voxel-iters/s", "cores": 1, "kind": "oracle",
           "host_cores": os.cpu_count(),
           "sample": f"{n_it} iteration(s) of Algorithm 1 at the finest 160x192x224 level from the "
                     f"identity state, FP64 NumPy, single thread ({wall:.1f} s wall, {cpu:.1f} s CPU), "
                     f"1 of {os.cpu_count()} host cores"}
    if processes > 1:
        try:
            out["parallel"] = cpu_parallel(p, params, processes, max(1, min(2, n_it)))
        except Exception as e:  # the parallel leg must not hide the single-core figure
            out["parallel"] = {"error": f"{type(e).__name__}: {e}"}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tissue160")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain PyTorch comparison")
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--batch", type=int, default=4,
                    help="registrations run together (streams, then batched launches) for the batch figure (0 skips)")
    ap.add_argument("--grid", type=int, default=8,
                    help="variants per size in the grid-search batch (8 gives 96 registrations; 0 skips)")
    ap.add_argument("--grid-fused-only", action="store_true",
                    help="grid-search batch: skip the sequential comparison (for kernel traces)")
    ap.add_argument("--inverse-steps", type=int, default=2,
                    help="timed fits of the post hoc inverse of the result (0 skips)")
    ap.add_argument("--no-lncc", action="store_true", help="skip the fused LNCC vs autograd timing (128^3)")
    ap.add_argument("--large-steps", type=int, default=1,
                    help="timed registrations of the 512^3 microscopy-like workload (0 skips)")
    ap.add_argument("--tune-steps", type=int, default=2,
                    help="timed registrations with autotuned launch shapes (0 skips)")
    ap.add_argument("--sym-steps", type=int, default=2,
                    help="timed symmetric registrations (0 skips)")
    ap.add_argument("--jac-steps", type=int, default=2,
                    help="registrations timed with use_jac on (0 skips)")
    ap.add_argument("--graph-reps", type=int, default=5,
                    help="repeats of the graph-replayed finest-level steady-state timing (0 skips)")
    ap.add_argument("--prof-steps", type=int, default=2,
                    help="registrations run with per-kernel HIP events after the timed ones")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--cpu-processes", type=int, default=16,
                    help="independent oracle runs at once for the parallel CPU figure (<= 1 skips)")
    ap.add_argument("--workers", type=int, default=8,
                    help="host processes generating the grid-search pairs")
    ap.add_argument("--lungct-steps", type=int, default=1,
                    help="timed registrations with the paper's lung CT hyperparameters (0 skips)")
    ap.add_argument("--calib", action="store_true",
                    help="first run a 256 MiB read + 256 MiB write elementwise kernel "
                         "(reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the dense matching step of one registration is not "
              "sharded across GPUs (use --gpus 1).", file=sys.stderr)
        sys.exit(2)
    os.environ.setdefault("OMP_NUM_THREADS", "1")

    import torch

    from paper_2404_01249_amd import synth
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.calib:
        x = torch.ones(64 * 1024 * 1024, device="cuda")
        y = torch.empty_like(x)
        torch.add(x, 1.0, out=y)
        torch.cuda.synchronize()
        del x, y
    p = synth.load(args.workload)
    params = dict(eta=0.5, sigma_grad=1.0, sigma_warp=0.5, window=p.window)
    lv = level_voxels(p.fixed.shape, p.scales, p.iters)
    vox_iters = sum(n * t for n, t in lv)

    ms, median_ms, wall_ms, prof, loss, field = run_fused(p, args.steps, args.warmup, params, args.prof_steps)
    value = vox_iters / (ms / 1e3)

    # dominant kernel: the fused gradient kernel at the finest level
    fin = len(p.scales) - 1
    n_fin = lv[fin][0]
    g_ms, g_n = prof[fin][0]
    roof = {"bound": "hbm", "kernel": "k_grad (warp+LNCC+adjoint+Adam), finest level", "achieved": None,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None, "traffic": measured_traffic(),
            "bytes_per_launch": GRAD_BYTES_PER_VOXEL * n_fin, "avg_launch_us": None, "launches": g_n}
    split, steady = {}, None
    if g_n > 0:
        per_launch_ms = g_ms / g_n
        achieved = GRAD_BYTES_PER_VOXEL * n_fin / (per_launch_ms / 1e3) / 1e9
        roof.update(achieved=achieved, frac=achieved / HBM_PEAK_GBS, avg_launch_us=per_launch_ms * 1e3)
        names = ["grad_adam", "smooth_max", "smooth_warp", "compose"]   # kernel kinds 0 to 3
        for lvl, rows in prof.items():
            split[f"level{lvl}"] = {names[k]: round(rows[k][0] / max(rows[k][1], 1) * 1e3, 2) for k in (0, 1, 3, 2)}
        iter_ms_fin = sum(r[0] for r in prof[fin]) / g_n
        steady = {"us_per_iteration": iter_ms_fin * 1e3, "voxel_iters_per_s": n_fin / (iter_ms_fin / 1e3),
                  "roofline_frac_80B": GRAD_BYTES_PER_VOXEL * n_fin / (iter_ms_fin / 1e3) / 1e9 / HBM_PEAK_GBS,
                  "source": "sum of the four kernels' average HIP-event times at the finest level"}
    if steady:
        roof["whole_iteration"] = {
            "us": steady["us_per_iteration"], "frac_80B": steady["roofline_frac_80B"],
            "note": "all launches of one finest-level iteration against the same 80 B/voxel algorithmic bytes"}
    if args.graph_reps > 0:
        g_us = run_steady_graph(p, params, reps=args.graph_reps)
        steady = dict(steady or {})
        steady["graph_replay"] = {
            "us_per_iteration": g_us, "voxel_iters_per_s": n_fin / (g_us / 1e6),
            "roofline_frac_80B": GRAD_BYTES_PER_VOXEL * n_fin / (g_us / 1e6) / 1e9 / HBM_PEAK_GBS,
            "method": "one pair at the finest level through fa_batch_step_fused with HIP-graph capture; "
                      "(60-iteration call - 10-iteration call) / 50, median of %d" % args.graph_reps}

    out = {
        "metric": METRIC, "value": value, "unit": "voxel-iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{p.name}: {'x'.join(map(str, p.fixed.shape))} fp32 pair, "
                               f"scales {p.scales} at {p.iters} iterations, LNCC {p.window}^3, "
                               f"eta 0.5, sigma_grad 1.0, sigma_warp 0.5",
                   "voxel_iters_per_step": vox_iters, "parallelism": "single GPU"},
        "roofline": roof,
        "steady_state_finest": steady,
        "kernel_us_by_level": split,
        "wall_ms_per_step": wall_ms * 1e3,
        "ms_per_step_median": median_ms,
        "final_loss": float(loss[-1]) if len(loss) else None,
    }
    acc = accuracy(p, field)
    if acc:
        import torch
        zero = torch.zeros_like(field)
        out["accuracy"] = {"fused": acc, "identity_dice": accuracy(p, zero)["dice"]}
        if p.true_field is not None:
            from paper_2404_01249_amd import evaluate
            g = torch.from_numpy(p.true_field).cuda()
            out["accuracy"]["endpoint_error_vs_true_warp"] = {
                "fused": evaluate.endpoint_error(field, g)[0], "identity": evaluate.endpoint_error(zero, g)[0]}
    if args.batch > 0:
        bt = run_batch_compare(p, min(args.batch, 8), params)
        nb = min(args.batch, 8)
        out["batch"] = {"registrations": nb, "etas": [0.25, 0.5, 1.0, 2.0, 0.375, 0.75, 1.5, 3.0][:nb],
                        "sequential_s": bt["sequential"], "streams_s": bt["batched"],
                        "fused_s": bt["fused"],
                        "sequential_voxel_iters_per_s": nb * vox_iters / bt["sequential"],
                        "streams_voxel_iters_per_s": nb * vox_iters / bt["batched"],
                        "fused_voxel_iters_per_s": nb * vox_iters / bt["fused"],
                        "streams_speedup": bt["sequential"] / bt["batched"],
                        "fused_speedup": bt["sequential"] / bt["fused"]}
    if args.grid > 0:
        g = run_grid_search(min(args.grid, 8), params, not args.grid_fused_only, workers=args.workers)
        out["grid_search"] = {
            "registrations": g["registrations"],
            "sizes": ["96x96x96", "128x160x128", "160x192x224"], "etas": [0.25, 0.5, 1.0, 2.0],
            "pairs": f"{min(args.grid, 8)} seeded pairs per size (seeds 400-{400 + 3 * min(args.grid, 8) - 1})",
            "schedule": "scales [2.0, 1.0] at [100, 50]", "voxel_iters": g["voxel_iters"],
            "generation_s": g["generation_s"],
            "fused_s": g["fused"], "fused_voxel_iters_per_s": g["voxel_iters"] / g["fused"],
            "fused_tuned_s": g["fused_tuned"], "fused_tuned_voxel_iters_per_s": g["voxel_iters"] / g["fused_tuned"],
            "tuning_s": g["tuning_s"]}
        if "sequential" in g:
            out["grid_search"].update({
                "fused_graphs_s": g["fused_graphs"],
                "sequential_s": g["sequential"],
                "sequential_voxel_iters_per_s": g["voxel_iters"] / g["sequential"],
                "fused_speedup": g["sequential"] / g["fused"]})
    if args.inverse_steps > 0:
        ims, ivox, iloss = run_inverse(field, args.inverse_steps, params)
        out["inverse"] = {"ms_per_fit": ims, "voxel_iters": ivox, "voxel_iters_per_s": ivox / (ims * 1e-3),
                          "schedule": "scales [4.0, 2.0, 1.0] at [100, 50, 25], eta 0.2",
                          "cost_first": float(iloss[0]), "cost_final": float(iloss[-1]),
                          "rms_residual_final": float(np.sqrt(iloss[-1] / 2.0))}
    if not args.no_lncc:
        out["lncc128"] = run_lncc128()
    if args.large_steps > 0:
        lms, lvox, l0, l1, gen_s, lsplit, ltuned = run_microscopy512(args.large_steps, params)
        out["microscopy512"] = {
            "workload": "512x512x512 microscopy-like pair (seed 5), LNCC 7^3, scales [8, 4, 2, 1] at "
                        "[200, 200, 100, 50] iterations, eta 0.5, sigma_grad 1.0, sigma_warp 0.5",
            "ms_per_step": lms, "voxel_iters": lvox, "voxel_iters_per_s": lvox / (lms * 1e-3),
            "loss_first": l0, "loss_final": l1, "generation_s": gen_s, "kernel_us_by_level": lsplit,
            "autotuned_ms_per_step": ltuned, "autotuned_speedup": lms / ltuned}
    if args.tune_steps > 0:
        tms, tune_s, tloss, shapes = run_autotuned(p, args.tune_steps, params)
        out["autotuned"] = {"ms_per_step": tms, "speedup": ms / tms, "tuning_s": tune_s, "final_loss": tloss,
                            "shapes_ty_tx_zc_brick": shapes}
    if args.sym_steps > 0:
        sms, sloss, sfield = run_symmetric(p, args.sym_steps, params)
        out["symmetric"] = {"ms_per_step": sms, "runtime_ratio": sms / ms, "final_halfway_loss": float(sloss[-1]),
                            "inverse": "scales [4.0, 2.0, 1.0] at %s, eta 0.2" % SYM_INVERSE_ITERS,
                            "accuracy": accuracy(p, sfield)}
    if args.lungct_steps > 0:
        lparams = dict(params, eta=0.25, sigma_grad=6.0, sigma_warp=0.4)
        lms, _, _, _, lloss, lfield = run_fused(p, args.lungct_steps, 1, lparams, 0)
        out["lung_ct_params"] = {
            "hyperparameters": "eta 0.25, sigma_grad 6.0, sigma_warp 0.4 (the paper's EMPIRE10 settings; "
                               "Gaussian radii 18 and 2)",
            "ms_per_step": lms, "runtime_ratio": lms / ms, "voxel_iters_per_s": vox_iters / (lms / 1e3),
            "final_loss": float(lloss[-1])}
        if acc:
            out["lung_ct_params"]["accuracy"] = accuracy(p, lfield)
    if args.jac_steps > 0:
        jms, jloss, jfield = run_use_jac(p, args.jac_steps, params)
        out["use_jac"] = {"ms_per_step": jms, "runtime_ratio": jms / ms, "final_loss": jloss}
        if acc:
            out["use_jac"]["accuracy"] = accuracy(p, jfield)
    if not args.no_plain:
        try:
            pms, plosses, pfield = run_plain(p, args.plain_steps, 0, params)
            out["plain_torch"] = {"value": vox_iters / (pms / 1e3), "ms_per_step": pms,
                                  "speedup_fused": pms / ms, "final_loss": float(plosses[-1])}
            if acc:
                pacc = accuracy(p, pfield)
                out["accuracy"]["plain_torch"] = pacc
                out["accuracy"]["dice_difference"] = acc["dice"] - pacc["dice"]
                if "endpoint_error_vs_true_warp" in out["accuracy"]:
                    import torch

                    from paper_2404_01249_amd import evaluate
                    g = torch.from_numpy(p.true_field).cuda()
                    out["accuracy"]["endpoint_error_vs_true_warp"]["plain_torch"] = \
                        evaluate.endpoint_error(pfield.contiguous(), g)[0]
        except Exception as e:  # the comparison must not hide the headline line
            out["plain_torch"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu_baseline:
        procs = min(args.cpu_processes, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(p, params, args.cpu_budget, procs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
