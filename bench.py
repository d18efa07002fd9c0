#!/usr/bin/env python3
"""Throughput of the KB-NUFFT hot path on one MI355X.

One step = one pass of the whole path over one batch of synthetic input:
  index pass (set_points) -> forward A x and omega-Jacobian (forward op,
  upstream gradient g given beforehand; one library call that derives the
  r^[0] channel from the unweighted one, --separate for two calls) ->
  adjoint A^H g,
for B images of 256 x 256 (complex64, N(0,1)) sharing one trajectory of 64
golden-angle radial spokes x 512 samples (M = 32768) with uniform +-pi/256
jitter; sigma = 2, J = 6, FP32 arithmetic.  value = B * M / step time
(non-uniform points per second, whole job).

Per-kernel durations come from HIP events recorded by the library on the
launch stream over the timed region; the dominant kernel class is reported
against the HBM peak using the algorithmic bytes of the model below.  The
CPU baseline times the FP64 oracle on a bounded sample on the host.

Other workloads (one JSON line each, not the default):
  --workload batch   32 uneven 2D SENSE instances + one 128^3 kooshball, the
                     same bundle per instance, batched (streams, one graph)
                     against the same kernels launched per instance/coil/op.
  --workload train   SENSE trajectory-learning step through the autograd
                     layer: 320x320, 8 images x 8 coils, 16 x 1280 spiral;
                     forward, loss, backward (x and omega gradients), SGD on
                     omega (so every step re-sorts the points).
  --workload serve   CG-SENSE requests (10 iterations, lambda 1e-3, 8 coils)
                     arriving as a Poisson process at 50/s: 80% 2D spiral
                     (N 192..384, M 20k..60k), 20% 96^3 kooshball; latency
                     p50/p99 of a continuous-batching server.
  --workload jacobian  the Gram and PSD-inverse Jacobian test case of
                     Sec. IV-A (time and memory tables): gradients of
                     ||f(x)||^2 w.r.t. omega and x for f = E^H E and
                     f = (E^H E + lambda I)^{-1} (20 CG iterations), 8 coils,
                     one radial spoke, images 40^2 and 400^2, plus the
                     memory case 200 x 200 x 100.

  --workload learn   trajectory learning as in Sec. IV-B: 320x320, mini-batch
                     12, 8 coils, 16 shots x 1280 samples on 40 quadratic
                     spline kernels, CG-SENSE (20 iterations) through the
                     inverse layer, gradient/slew penalties, one Adam step.
  --workload cg      one CG-SENSE request (10 iterations) of the serving
                     workload on a resident plan: 96^3 x 8 coils kooshball
                     (--cg-shape 3d) or 384^2 x 8 coils spiral (2d).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B]
                       [--workload step|batch|train|serve|jacobian|learn]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "nonuniform pts/s (fwd+adj+ω-Jacobian), % HBM peak; served recon p50/p99 ms"
HBM_PEAK_GBPS = 8000.0
C8 = 8  # bytes per complex64
# hardware-counter traffic of this workload's kernels (rocprofv3 FETCH_SIZE and
# WRITE_SIZE, calibrated against a device copy of known size); used only while
# its source hash matches the kernels being run
PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_2d256_M32768_B256.json")


def measured_traffic(cls: str, launches_per_step: float):
    """HBM bytes per launch of kernel class `cls` from the counter summary,
    or None when there is none or the kernels changed since it was taken."""
    from paper_2111_02912_amd.profsummary import sources_hash
    try:
        with open(PMC_SUMMARY) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    c = d.get("classes", {}).get(cls)
    if d.get("sources") != sources_hash() or c is None or launches_per_step <= 0:
        return None
    return (c["fetch_per_step"] + c["write_per_step"]) / launches_per_step


def algorithmic_bytes(N, K, M, B, D, fused=False):
    """Bytes per step that each kernel class must move (no halos, no re-reads).

    Point record = sorted index (4 B) + D cells (4 B) + D fractions (4 B).
    fused (2D forward plus omega-Jacobian in one call): the first pass reads
    each image once and writes the unweighted and r^[1] channels; the axis-0
    pass reads those two and writes three (r^[0] is derived from the
    unweighted channel's rows, a re-read counted as a cache hit).
    """
    pN = math.prod(N)
    pK = math.prod(K)
    rows = pN // N[-1]            # image rows along the last axis
    first_out = rows * K[-1]      # elements after the first (last-axis) pass
    prec = M * (4 + 8 * D)
    out = {}
    out["index"] = M * D * 4 + prec
    # forward (1 channel / image) and omega-Jacobian (D channels / image)
    out["fft_first"] = C8 * (B * pN + B * first_out) + C8 * (B * pN + D * B * first_out)
    mid = 0
    # mid passes expand axes D-2..0 one at a time: sizes before/after each pass
    sizes = []
    cur = list(N[:-1]) + [K[-1]]
    for d in range(D - 2, -1, -1):
        before = math.prod(cur)
        cur[d] = K[d]
        sizes.append((before, math.prod(cur)))
    for before, after in sizes:
        mid += C8 * (before + after)
    out["fft_mid_fwd"] = mid * B * (1 + D)
    if fused:
        assert D == 2, "the fused forward plus omega-Jacobian model is 2D"
        out["fft_first"] = C8 * (B * pN + D * B * first_out)
        (before, after), = sizes
        out["fft_mid_fwd"] = C8 * B * (D * before + (D + 1) * after)
    out["gather"] = C8 * (B * pK + B * M) + prec
    out["gather_jac"] = C8 * (D * B * pK + B * M) + prec + 4 * M * D  # + gradient write
    out["spread"] = C8 * (B * M + B * pK) + prec
    out["fft_mid_inv"] = mid * B
    out["fft_last_adj"] = C8 * (B * first_out + B * pN)
    return out


def _cpu_model() -> str:
    """Host CPU model name (from /proc/cpuinfo, as lscpu reports it)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(N, om, x, g, images=2):
    """The FP64 oracle on the host, exact (no extrapolation): for `images`
    images, the direct NUDFT forward, the D omega-Jacobian operands
    A(x r^[d]) and the adjoint of the upstream gradient, all points and
    pixels."""
    from oracle import ndft

    D = len(N)
    M = om.shape[0]
    xs = x[:images]
    gs = g[:images, 0]
    t0 = time.perf_counter()
    ndft.forward(om, xs, N)
    for d in range(D):
        ndft.forward(om, xs, N, wdim=d)
    t1 = time.perf_counter()
    ndft.adjoint(om, gs, N)
    t2 = time.perf_counter()
    return {
        "value": images * M / (t2 - t0),
        "unit": "pts/s",
        "cores": ndft.num_threads(),
        "cpu_model": _cpu_model(),
        "kind": "oracle",
        "sample": (f"{images} of the {N[0]}x{N[1]} images, all M={M} points: direct FP64 NUDFT "
                   f"forward + {D} omega-Jacobian operands ({t1 - t0:.1f} s) and adjoint over "
                   f"all pixels ({t2 - t1:.1f} s)"),
    }


def _wall_ms(fn, steps, warmup, pause_ms=0.0):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if pause_ms > 0:
        # an idle gap on the GPU timeline that marks where the timed steps begin
        time.sleep(pause_ms * 1e-3)
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def bench_batch(args):
    """Multi-instance bundle: per instance forward E x, omega-Jacobian with
    upstream gradient k, adjoint E^H k (B = 1, all coils)."""
    import numpy as np
    import torch

    from paper_2111_02912_amd import batch as KB
    from paper_2111_02912_amd import workloads as W
    from paper_2111_02912_amd.autotune import tune_plan
    from paper_2111_02912_amd.nufft import KbNufft

    dev = torch.device("cuda", 0)
    insts = W.multi_instance_case()
    items = []
    pts = 0
    bundle_bytes = 0  # algorithmic bytes of the bundle (the byte model per instance)
    t0 = time.perf_counter()
    choices = {}
    for i, inst in enumerate(insts):
        x, smaps, k = W.instance_data(inst, 4500 + 10 * i)
        N, C, M, D = tuple(inst["N"]), inst["coils"], inst["omega"].shape[0], len(inst["N"])
        om = torch.from_numpy(inst["omega"]).to(dev)
        xt = torch.from_numpy(x).to(dev)
        kt = torch.from_numpy(k).to(dev)
        st = torch.from_numpy(smaps).to(dev) if smaps is not None else None
        if args.autotune:
            plan, info = tune_plan(N, om, C, xt, st, kt)
            c = info["choice"]
            key = f"{c['tile'][0]}/{c['spread_tile']}"
            choices[key] = choices.get(key, 0) + 1
        else:
            plan = KbNufft(N, device=dev)
            plan.set_points(om)
        ab = algorithmic_bytes(N, plan.K, M, C, D)  # C coil channels per instance
        bundle_bytes += sum(v for k_, v in ab.items() if k_ != "index")
        items.append(dict(plan=plan, N=N, C=C, M=M, D=D, x=xt, k=kt, s=st,
                          y=torch.empty((1, C, M), dtype=torch.complex64, device=dev),
                          dom=torch.empty((M, D), dtype=torch.float32, device=dev),
                          xa=torch.empty((1,) + N, dtype=torch.complex64, device=dev),
                          xc=torch.empty((C,) + N, dtype=torch.complex64, device=dev)))
        pts += C * M
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    batched, percall = [], []
    for it in items:
        C, s = it["C"], it["s"]
        batched += [KB.Task(it["plan"], KB.FORWARD, 1, C, it["x"], it["y"], s),
                    KB.Task(it["plan"], KB.JAC_OMEGA_FWD, 1, C, it["x"], it["dom"], s, g=it["k"]),
                    KB.Task(it["plan"], KB.ADJOINT, 1, C, it["k"], it["xa"], s)]
        for c in range(C):
            sc = s[c:c + 1] if s is not None else None
            percall += [KB.Task(it["plan"], KB.FORWARD, 1, 1, it["x"], it["y"][:, c:c + 1], sc),
                        KB.Task(it["plan"], KB.JAC_OMEGA_FWD, 1, 1, it["x"], it["dom"], sc,
                                g=it["k"][:, c:c + 1], accumulate=c > 0),
                        KB.Task(it["plan"], KB.ADJOINT, 1, 1, it["k"][:, c:c + 1], it["xc"][c:c + 1], sc)]
    want = set(args.modes.split(","))
    modes = {}
    if "per_call" in want:
        b = KB.KbnBatch(percall, nstreams=1)
        modes["per_call"] = _wall_ms(b.run, args.steps, args.warmup)
        b.close()
    if "per_instance_one_stream" in want:
        b = KB.KbnBatch(batched, nstreams=1)
        modes["per_instance_one_stream"] = _wall_ms(b.run, args.steps, args.warmup)
        b.close()
    b = KB.KbnBatch(batched, nstreams=args.streams)
    if "streams" in want:
        modes["streams"] = _wall_ms(b.run, args.steps, args.warmup)
    if "graph" in want:
        b.capture()
        modes["graph"] = _wall_ms(b.launch, args.steps, args.warmup, args.pause_ms)
    b.close()
    if "fused" in want:
        # interpolation of the whole bundle in one launch per phase and kernel
        # shape (fused batches run eagerly)
        b = KB.KbnBatch(batched, nstreams=args.streams, fuse=True)
        modes["fused"] = _wall_ms(b.run, args.steps, args.warmup, args.pause_ms)
        b.close()
    best = min((m for m in ("streams", "graph", "fused") if m in modes), key=lambda m: modes[m])
    out = {
        "metric": "multi-instance bundle nonuniform pts/s (fwd+adj+omega-Jacobian)",
        "value": pts / (modes[best] * 1e-3),
        "unit": "pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": modes[best],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{len(insts) - 1} uneven 2D SENSE instances (N_d 128..384, M 8k..80k, "
                         "4..8 coils, radial/spiral) + one 128^3 kooshball (M = 1048576, 1 coil): "
                         "forward + omega-Jacobian + adjoint per instance"),
            "coil_samples_per_step": pts, "autotune": bool(args.autotune),
            "tile_choices": choices, "streams": args.streams, "setup_s": setup_s,
        },
        "mode_ms": modes,
        "best_mode": best,
        "roofline": {"bound": "hbm", "kernel": "whole bundle", "alg_bytes": bundle_bytes,
                     "achieved": bundle_bytes / (modes[best] * 1e-3) / 1e9, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": bundle_bytes / (modes[best] * 1e-3) / 1e9 / HBM_PEAK_GBPS},
        "speedup_vs_per_call": modes["per_call"] / modes[best] if "per_call" in modes else None,
        "speedup_vs_per_instance": (modes["per_instance_one_stream"] / modes[best]
                                    if "per_instance_one_stream" in modes else None),
    }
    print(json.dumps(out), flush=True)


def bench_train(args):
    import numpy as np
    import torch

    from paper_2111_02912_amd import workloads as W
    from paper_2111_02912_amd.autograd import nufft
    from paper_2111_02912_amd.nufft import KbNufft

    dev = torch.device("cuda", 0)
    N, om, x, smaps = W.spiral_sense_case()
    B, C, M = x.shape[0], smaps.shape[0], om.shape[0]
    plan = KbNufft(N, device=dev, accuracy=args.accuracy)
    xt = torch.from_numpy(x).to(dev).requires_grad_(True)
    st = torch.from_numpy(smaps).to(dev)
    omt = torch.from_numpy(om).to(dev).requires_grad_(True)
    # data from a perturbed trajectory, as when learning a trajectory
    with torch.no_grad():
        delta = torch.from_numpy(W.rng(3004).normal(0.0, 0.1, om.shape).astype(np.float32)).to(dev)
        plan.set_points(omt + delta)
        yt = plan.forward(xt, st)
    opt = torch.optim.SGD([omt], lr=1e-9)

    def step():
        opt.zero_grad(set_to_none=False)
        # |r|^2 summed as re^2 + im^2 (no square root and its division in backward)
        loss = torch.view_as_real(nufft(xt, omt, plan, st) - yt).square().sum()
        loss.backward()
        opt.step()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-class breakdown from as many extra steps with every launch bracketed
    # by events (kept out of the timed steps: the events cost ~4% of a step)
    plan.timing(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    plan.timing(False)
    kt = {k: round(ms / args.steps, 4) for k, (n, ms) in plan.timing_read().items() if n}
    ms = (t1 - t0) * 1e3 / args.steps
    out = {
        "metric": "SENSE training step nonuniform pts/s (forward + x/omega gradients + index pass)",
        "value": B * C * M / (ms * 1e-3), "unit": "pts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"SENSE trajectory learning: {N[0]}x{N[1]}, {B} images x {C} coils, "
                                f"16 x 1280 spiral (M = {M}), loss |E(omega) x - y|^2, autograd "
                                "backward to x and omega, SGD on omega"),
                   "sigma": plan.opts["sigma"], "J": plan.opts["J"], "K": list(plan.K)},
        "kernel_ms_per_step": kt,
    }
    print(json.dumps(out), flush=True)


# Sec. IV-A time and memory tables (RTX 2080 Ti, seconds; MB of
# torch.cuda.max_memory_allocated), the proposed method's column
PAPER_JAC_S = {"gram_40": 0.1, "gram_400": 0.2, "inverse_40": 0.9, "inverse_400": 2.5}
PAPER_JAC_MB = {"gram_40": 2.8, "gram_400": 267.5, "inverse_40": 2.9, "inverse_400": 272.0,
                "gram_3d": 10.1e3, "inverse_3d": 10.8e3}


def bench_jacobian(args):
    """Gram and PSD-inverse Jacobian test case: one step = index pass, f(x),
    loss ||f(x)||^2 and its backward to omega and x."""
    import numpy as np
    import torch

    from paper_2111_02912_amd import workloads as W
    from paper_2111_02912_amd.autograd import gram, inverse
    from paper_2111_02912_amd.nufft import KbNufft

    dev = torch.device("cuda", 0)
    C = 8
    cases = {}
    for size in (40, 400, "3d"):
        if size == "3d":
            N = (200, 200, 100)
            om = W.kooshball_3d(1, 400)
        else:
            N = (size, size)
            om = W.radial_2d(1, 2 * size)  # one spoke through the centre, 2N samples
        smaps = W.sense_maps(C, N).astype(np.complex64)
        x = W.complex_normal((1,) + N, 7001).astype(np.complex64)
        for op in ("gram", "inverse"):
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            torch.cuda.reset_peak_memory_stats()
            plan = KbNufft(N, device=dev)
            xt = torch.from_numpy(x).to(dev).requires_grad_(True)
            omt = torch.from_numpy(om).to(dev).requires_grad_(True)
            st = torch.from_numpy(smaps).to(dev)

            def step():
                xt.grad = None
                omt.grad = None
                plan.set_points(omt.detach())
                plan.ensure_points(omt)
                if op == "gram":
                    z = gram(xt, omt, plan, st)
                else:
                    z = inverse(xt, omt, plan, st, lam=1e-3, iters=20)
                loss = torch.view_as_real(z).pow(2).sum()
                loss.backward()

            steps = args.steps if size != "3d" else max(1, min(args.steps, 5))
            ms = _wall_ms(step, steps, max(1, min(args.warmup, 2)))
            torch.cuda.synchronize()
            key = f"{op}_{size}"
            # the plan allocates through PyTorch's caching allocator, so the
            # peak includes its buffers (plan_device_MB of it)
            peak = torch.cuda.max_memory_allocated(dev)
            cases[key] = {"N": list(N), "M": int(om.shape[0]), "coils": C, "s": ms * 1e-3,
                          "peak_MB": peak / 2 ** 20, "plan_device_MB": plan.info()["device_bytes"] / 2 ** 20,
                          "paper_s": PAPER_JAC_S.get(key), "paper_MB": PAPER_JAC_MB.get(key)}
            plan.close()
            del xt, omt, st
    value = cases["inverse_400"]["s"]
    out = {
        "metric": "PSD-inverse Jacobian test case time (s): gradients of ||f(x)||^2 w.r.t. omega and x",
        "value": value, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": value * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": value / PAPER_JAC_S["inverse_400"], "dtype": "f32", "data": "synthetic",
        "config": {"workload": ("Gram / PSD-inverse Jacobian test case: 400x400 image (also 40x40 and "
                                "200x200x100), 8 coils, one radial spoke of 2N samples, "
                                "f = (E^H E + 1e-3 I)^{-1} by 20 CG iterations forward and backward"),
                   "images": "complex64 N(0,1) stand-in for the phantom crop with random phase"},
        "baseline_hardware": "paper: RTX 2080 Ti (context only)",
        "cases": cases,
    }
    print(json.dumps(out), flush=True)


def bench_learn(args):
    """One Adam step of trajectory learning per step (Sec. IV-B sizes)."""
    import numpy as np
    import torch

    from paper_2111_02912_amd import workloads as W
    from paper_2111_02912_amd.learn import TrajectoryLearner

    dev = torch.device("cuda", 0)
    N, B, C = (320, 320), 12, 8
    x = torch.from_numpy(W.complex_normal((B,) + N, 8901)).to(dev)
    smaps = torch.from_numpy(W.sense_maps(C, N)).to(dev)
    tl = TrajectoryLearner(N, shots=16, samples=1280, knots=40, lam=1e-3, cg_iters=20, lr=1e-4,
                           accuracy=args.accuracy, device=dev)
    hist = []
    ms = _wall_ms(lambda: hist.append(tl.step(x, smaps)), args.steps, args.warmup)
    out = {
        "metric": "trajectory-learning Adam step, images/s",
        "value": B / (ms * 1e-3), "unit": "images/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": ("trajectory learning: 320x320, mini-batch 12, 8 coils, 16 shots x 1280 "
                                "samples (40 quadratic spline kernels per shot, radial start), CG-SENSE "
                                "lambda 1e-3 with 20 CG iterations through the inverse layer, gradient "
                                "5 G/cm and slew 15 G/cm/ms soft limits (mu 10), Adam lr 1e-4"),
                   "sigma": tl.plan.opts["sigma"], "J": tl.plan.opts["J"]},
        "loss_first_last": [hist[0][0], hist[-1][0]] if hist else None,
    }
    print(json.dumps(out), flush=True)


def serve_pool(dev, n2d, n3d, coils=8, seed=5001):
    """Resident problems: square 2D spirals and 96^3 kooshballs with
    Gaussian-bump maps and noiseless data y = E x_true."""
    import numpy as np
    import torch

    from paper_2111_02912_amd import workloads as W
    from paper_2111_02912_amd.nufft import KbNufft
    from paper_2111_02912_amd.serve import Problem

    g = W.rng(seed)
    specs = []
    for i in range(n2d):
        n = int(g.integers(192, 385))
        M = int(g.integers(20000, 60001))
        specs.append(((n, n), W.spiral_2d(16, -(-M // 16))[:M], "2d"))
    koosh = W.kooshball_3d(4096, 256)
    for i in range(n3d):
        specs.append(((96, 96, 96), koosh, "3d"))
    probs = []
    for pid, (N, om, kind) in enumerate(specs):
        om_t = torch.from_numpy(np.ascontiguousarray(om)).to(dev)
        sm = torch.from_numpy(W.sense_maps(coils, N)).to(dev)
        xt = torch.from_numpy(W.complex_normal((1,) + N, seed + 100 + pid)).to(dev)
        plan = KbNufft(N, device=dev)
        plan.set_points(om_t)
        y = plan.forward(xt, sm)[0].contiguous()
        plan.close()
        probs.append(Problem(pid, N, coils, om.shape[0], kind, {"omega": om_t, "smaps": sm, "y": y}))
    torch.cuda.synchronize()
    return probs


def cg_iteration_bytes(N, K, M, C, D):
    """Algorithmic bytes of one CG-SENSE iteration (E^H E p for C coils):
    the forward and adjoint classes of the byte model with C channels."""
    ab = algorithmic_bytes(N, K, M, C, D)
    pN = math.prod(N)
    first_out = (pN // N[-1]) * K[-1]
    fwd_first = C8 * (C * pN + C * first_out)
    mid_one = ab["fft_mid_inv"]  # one channel set of mid passes (= forward's for 1 weight channel)
    return fwd_first + mid_one + ab["gather"] + ab["spread"] + ab["fft_mid_inv"] + ab["fft_last_adj"]


def bench_cg(args):
    """One CG-SENSE request (10 iterations, lambda 1e-3) on a resident plan:
    the serving workload's 3D class (96^3, 8 coils, 4096 x 256 kooshball) or
    its largest 2D class (384^2, 8 coils, 16-interleave spiral, M = 60000)."""
    import torch

    from paper_2111_02912_amd import workloads as W
    from paper_2111_02912_amd.cg import CgSense
    from paper_2111_02912_amd.nufft import KbNufft

    dev = torch.device("cuda", 0)
    C = 8
    if args.cg_shape == "3d":
        N, om = (96, 96, 96), W.kooshball_3d(4096, 256)
    else:
        N, om = (384, 384), W.spiral_2d(16, 3750)[:60000]
    M, D = om.shape[0], len(N)
    smaps = torch.from_numpy(W.sense_maps(C, N)).to(dev)
    plan = KbNufft(N, device=dev)
    plan.set_points(torch.from_numpy(om).to(dev))
    y = plan.forward(torch.from_numpy(W.complex_normal((1,) + N, 5301)).to(dev), smaps)[0].contiguous()

    def request():
        return CgSense(plan, C).begin(y, smaps).step(args.cg_iters, 1e-3)

    ms = _wall_ms(request, args.steps, args.warmup)
    plan.timing(True)
    for _ in range(args.steps):
        request()
    torch.cuda.synchronize()
    plan.timing(False)
    kt = {k: round(t / args.steps, 4) for k, (n, t) in plan.timing_read().items() if n}
    it_bytes = cg_iteration_bytes(N, plan.K, M, C, D)
    req_bytes = it_bytes * (args.cg_iters + 0.5)  # the start applies E^H once
    out = {
        "metric": "CG-SENSE request latency (unloaded, resident plan)", "value": ms, "unit": "ms",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"CG-SENSE request, {'x'.join(map(str, N))} image, {C} coils, M={M} "
                                f"({'4096 x 256 kooshball' if D == 3 else '16-interleave spiral'}), "
                                f"{args.cg_iters} iterations, lambda 1e-3"),
                   "K": list(plan.K)},
        "alg_bytes_per_request": req_bytes,
        "roofline": {"bound": "hbm", "kernel": "whole request", "achieved": req_bytes / (ms * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": req_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS},
        "kernel_ms_per_request": kt,
    }
    plan.close()
    print(json.dumps(out), flush=True)


def _per_call_cg(plan, y, smaps, lam, iters):
    """CG-SENSE written with plain per-coil library calls: every E^H E p is
    one forward and one adjoint call per coil, the vector updates are
    PyTorch ops (the baseline for the served throughput)."""
    import torch
    C = smaps.shape[0]

    def ehe(v):
        acc = torch.zeros_like(v)
        for c in range(C):
            acc += plan.adjoint(plan.forward(v[None], smaps[c:c + 1]), smaps[c:c + 1])[0]
        return acc

    b = torch.zeros((1,) + plan.N, dtype=torch.complex64, device=plan.device)[0]
    for c in range(C):
        b += plan.adjoint(y[c:c + 1][None].contiguous(), smaps[c:c + 1])[0]
    x = torch.zeros_like(b)
    r = b.clone()
    pv = r.clone()
    rr = torch.vdot(r.flatten(), r.flatten()).real
    for _ in range(iters):
        q = ehe(pv) + lam * pv
        alpha = rr / torch.vdot(pv.flatten(), q.flatten()).real
        x += alpha * pv
        r -= alpha * q
        rr_new = torch.vdot(r.flatten(), r.flatten()).real
        pv = r + (rr_new / rr) * pv
        rr = rr_new
    return x


def serve_capacity(dev, p2, p3, n, frac_3d, iters, lanes, hbm_gb, seed=5201):
    """Throughput at saturation (every request queued at t = 0) of the
    continuous-batching server, against the same requests run one at a time
    with the library's CG calls (all coils per call) and with plain per-coil
    calls, resident plans in both."""
    import numpy as np
    import torch

    from paper_2111_02912_amd.cg import CgSense
    from paper_2111_02912_amd.nufft import KbNufft
    from paper_2111_02912_amd.serve import GpuExecutor, Request, Server

    g = np.random.default_rng(seed)
    probs = []
    for _ in range(n):
        pool = p3 if g.random() < frac_3d else p2
        probs.append(pool[int(g.integers(len(pool)))])
    # served, all arriving at once; the plans are made resident by a warm pass
    ex = GpuExecutor(dev, lanes=lanes, lam=1e-3)
    srv = lambda: Server(ex, hbm_budget=int(hbm_gb * (1 << 30)), lanes=lanes, chunk=1, depth=2,
                         max_active=64)
    srv().run([Request(i, 0.0, p, iters=iters) for i, p in enumerate({q.pid: q for q in probs}.values())])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = srv().run([Request(i, 0.0, p, iters=iters) for i, p in enumerate(probs)])
    torch.cuda.synchronize()
    served_s = time.perf_counter() - t0
    ex.close()
    plans = {}
    for p in probs:
        if p.pid not in plans:
            pl = KbNufft(p.N, device=dev)
            pl.set_points(p.data["omega"])
            plans[p.pid] = pl
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p in probs:
        CgSense(plans[p.pid], p.coils).begin(p.data["y"], p.data["smaps"]).step(iters, 1e-3)
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    for p in probs:
        _per_call_cg(plans[p.pid], p.data["y"], p.data["smaps"], 1e-3, iters)
    torch.cuda.synchronize()
    percall_s = time.perf_counter() - t0
    for pl in plans.values():
        pl.close()
    return {"requests": n, "frac_3d": frac_3d, "served_rps": n / served_s, "sequential_rps": n / seq_s,
            "per_call_rps": n / percall_s, "speedup_vs_per_call": percall_s / served_s,
            "speedup_vs_sequential": seq_s / served_s,
            "failed": sum(1 for r in done if r.error is not None)}


def bench_serve(args):
    import numpy as np
    import torch

    from paper_2111_02912_amd.serve import (GpuExecutor, Request, Server, latency_stats,
                                            poisson_arrivals)

    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    probs = serve_pool(dev, args.pool_2d, args.pool_3d)
    p2 = [p for p in probs if p.kind == "2d"]
    p3 = [p for p in probs if p.kind == "3d"]
    print(f"# pool ready: {len(p2)} 2D + {len(p3)} 3D problems in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    n = args.warm_requests + args.requests
    arr = poisson_arrivals(n, args.rate, seed=5101)
    g = np.random.default_rng(5102)
    reqs = []
    for i, t in enumerate(arr):
        pool = p3 if g.random() < args.frac_3d else p2
        reqs.append(Request(i, float(t), pool[int(g.integers(len(pool)))], iters=args.cg_iters))
    ex = GpuExecutor(dev, lanes=args.lanes, lam=1e-3)
    srv = Server(ex, hbm_budget=int(args.hbm_gb * (1 << 30)), lanes=args.lanes, chunk=args.chunk,
                 depth=2, max_active=64)
    t1 = time.perf_counter()
    done = srv.run(reqs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    done.sort(key=lambda r: r.rid)
    meas = done[args.warm_requests:]
    rel = np.array([float(r.result["rel"].item()) for r in meas if r.error is None])
    st = latency_stats(meas)
    per = {k: latency_stats([r for r in meas if r.problem.kind == k]) for k in ("2d", "3d")}
    # unloaded latency of one request of each class
    solo = {}
    for k, pool in (("2d", p2), ("3d", p3)):
        ex1 = GpuExecutor(dev, lanes=1, lam=1e-3)
        r1 = Server(ex1, hbm_budget=int(args.hbm_gb * (1 << 30)), lanes=1).run(
            [Request(0, 0.0, pool[0], iters=args.cg_iters)])
        r2 = Server(ex1, hbm_budget=int(args.hbm_gb * (1 << 30)), lanes=1).run(
            [Request(0, 0.0, pool[0], iters=args.cg_iters)])
        solo[k] = {"N": list(pool[0].N), "M": pool[0].M, "cold_ms": r1[0].latency * 1e3,
                   "resident_ms": r2[0].latency * 1e3}
        ex1.close()
    capacity = None
    if args.capacity_requests > 0:
        capacity = serve_capacity(dev, p2, p3, args.capacity_requests, args.frac_3d, args.cg_iters,
                                  args.lanes, args.hbm_gb)
    out = {
        "metric": "served CG-SENSE recon latency p50 (p99 alongside)",
        "value": st["p50_ms"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.requests,
        "warmup": args.warm_requests,
        "ms_per_step": st["mean_ms"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"CG-SENSE serving: Poisson {args.rate}/s, {int(100 * (1 - args.frac_3d))}% "
                         "2D spiral N 192..384 M 20k..60k, "
                         f"{int(100 * args.frac_3d)}% 96^3 kooshball M 1048576, 8 coils, "
                         f"{args.cg_iters} CG iterations, lambda 1e-3"),
            "pool": {"2d": len(p2), "3d": len(p3)}, "lanes": args.lanes, "chunk": args.chunk,
            "hbm_budget_gb": args.hbm_gb,
        },
        "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "max_ms": st["max_ms"],
        "per_class": per, "unloaded": solo,
        "requests_per_s": len(meas) / (max(r.t_done for r in meas) - min(r.arrival for r in meas)),
        "wall_s": wall, "plans_created": ex.plans_created, "resident_plan_hits": ex.plan_hits,
        "peak_active": srv.peak_active, "peak_bytes_gb": srv.peak_bytes / 2 ** 30,
        "residual_median": float(np.median(rel)), "residual_max": float(rel.max()),
        "failed_requests": len(srv.failed),
        "capacity": capacity,
    }
    ex.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--separate", action="store_true",
                    help="step workload: forward and omega-Jacobian as two calls")
    ap.add_argument("--cpu-images", type=int, default=2)
    ap.add_argument("--workload", choices=("step", "batch", "train", "serve", "jacobian", "learn", "cg"),
                    default="step")
    ap.add_argument("--cg-shape", choices=("3d", "2d"), default="3d",
                    help="cg workload: the 96^3 or the 384^2 serving problem")
    ap.add_argument("--requests", type=int, default=2000, help="serve workload: measured requests")
    ap.add_argument("--warm-requests", type=int, default=100, help="serve workload: unmeasured first requests")
    ap.add_argument("--rate", type=float, default=50.0, help="serve workload: arrivals per second")
    ap.add_argument("--frac-3d", type=float, default=0.2)
    ap.add_argument("--pool-2d", type=int, default=24)
    ap.add_argument("--pool-3d", type=int, default=4)
    ap.add_argument("--lanes", type=int, default=4)
    ap.add_argument("--chunk", type=int, default=1, help="serve workload: CG iterations per issue")
    ap.add_argument("--cg-iters", type=int, default=10)
    ap.add_argument("--hbm-gb", type=float, default=64.0)
    ap.add_argument("--capacity-requests", type=int, default=100,
                    help="serve workload: requests of the saturation / per-call comparison (0: skip)")
    ap.add_argument("--streams", type=int, default=8, help="batch workload: streams")
    ap.add_argument("--modes", default="per_call,per_instance_one_stream,streams,graph,fused",
                    help="batch workload: modes to time (comma list; one of streams, graph, fused "
                         "must be in it)")
    ap.add_argument("--pause-ms", type=float, default=0.0,
                    help="batch workload: host pause before the timed graph replays or fused runs "
                         "(marks them on a kernel trace)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="batch workload: default tiles instead of tuned ones")
    ap.add_argument("--accuracy", choices=("high", "low"), default="high",
                    help="step/train workloads: sigma 2, J 6 (high) or sigma 1.25, J 5 (low)")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="after the run, copy this many bytes device-to-device once (a "
                         "known-size reference dispatch for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); "
              "the path shards by image, coil and instance with no communication", file=sys.stderr)
        sys.exit(2)
    run = {"batch": bench_batch, "serve": bench_serve, "train": bench_train, "jacobian": bench_jacobian,
           "learn": bench_learn, "cg": bench_cg}.get(args.workload, bench_step)
    run(args)
    if args.copy_calib:
        # a known-size reference dispatch for hardware byte counters
        import torch
        dev = torch.device("cuda", 0)
        n = args.copy_calib // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()


def bench_step(args):
    """The headline step (see the module docstring)."""
    import numpy as np
    import torch

    from paper_2111_02912_amd import workloads as W
    from paper_2111_02912_amd.nufft import KbNufft

    dev = torch.device("cuda", 0)
    B = args.batch
    N, om, x = W.throughput_case(batch=B)
    M = om.shape[0]
    D = len(N)
    g = W.complex_normal((B, 1, M), 2101)
    p = KbNufft(N, device=dev, accuracy=args.accuracy)
    om_t = torch.from_numpy(om).to(dev)
    x_t = torch.from_numpy(x).to(dev)
    g_t = torch.from_numpy(g).to(dev)
    dom = torch.empty((M, D), dtype=torch.float32, device=dev)

    fused = not args.separate and D == 2

    def step():
        p.set_points(om_t)
        if fused:
            y, _ = p.forward_jac_omega(x_t, g_t, out=dom)
        else:
            y = p.forward(x_t)
            p.jac_omega_fwd(x_t, g_t, out=dom)
        xa = p.adjoint(g_t)
        return y, xa

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # per-class breakdown from `steps` extra steps with every launch bracketed
    # by events (the events themselves cost ~4% of a step, so the timed steps
    # below bracket only the dominant class, whose roofline is reported)
    p.timing(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    p.timing(False)
    kt = p.timing_read()
    alg = algorithmic_bytes(N, p.K, M, B, D, fused=fused)
    kernels = {}
    for name, (n, ms) in kt.items():
        if n == 0:
            continue
        b = alg.get(name, 0) * args.steps
        kernels[name] = {"launches": n, "avg_ms": ms / n,
                         "ms_per_step": ms / args.steps,
                         "alg_GBps": (b / (ms * 1e-3) / 1e9) if b else None}
    # the index pass runs on the plan's own stream beside the FFT passes: its
    # event spans include the time it waits for and shares the GPU with them
    dom_name = max((k for k in kernels if k != "index"), key=lambda k: kernels[k]["ms_per_step"])

    p.timing(True, classes=[dom_name])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    p.timing(False)
    n_dom, ms_dom = p.timing_read()[dom_name]
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = B * M / ((t1 - t0) / args.steps)
    # the dominant class as timed inside the timed steps
    dk = {"launches": n_dom, "avg_ms": ms_dom / n_dom}
    per_launch_bytes = alg[dom_name] * args.steps / dk["launches"]
    achieved = per_launch_bytes / (dk["avg_ms"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": achieved, "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                "traffic": measured_traffic(dom_name, dk["launches"] / args.steps),
                "alg_bytes_per_launch": per_launch_bytes, "avg_launch_ms": dk["avg_ms"]}
    total_alg = sum(alg.values())

    # achievable HBM bandwidth: a 1 GiB device-to-device copy (read + write),
    # larger than the 256 MB Infinity Cache, best of 5
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    copy_ms = []
    for _ in range(6):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        copy_ms.append(e0.elapsed_time(e1))
    copy_gbps = 2 * src.numel() * 8 / (min(copy_ms[1:]) * 1e-3) / 1e9
    del src, dst
    roofline["achievable_copy_GBps"] = copy_gbps

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(N, om, x, g, images=min(args.cpu_images, B))

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"2D KB-NUFFT step, {N[0]}x{N[1]} images, batch {B}, M={M}: index pass + "
                         "forward + omega-Jacobian + adjoint"),
            "forward_jacobian": "one call (kbn_forward_jac_omega)" if fused else "two calls",
            "N": list(N), "K": list(p.K), "M": M, "batch": B, "sigma": p.opts["sigma"], "J": p.opts["J"],
            "trajectory": "64 golden-angle radial spokes x 512 samples, uniform +-pi/256 jitter",
            "images": "complex64, re/im i.i.d. N(0,1)",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "step_alg_GBps": total_alg / (ms_step * 1e-3) / 1e9,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
