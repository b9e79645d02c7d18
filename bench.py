#!/usr/bin/env python3
"""Benchmark of the Gaussian-mixture interpolation hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

A step is one interp_forward + interp_backward (binning, forward gather,
backward prologue and adjoint; gradients w.r.t. positions, sigma and values)
on the 1024x1024, N=2^20, C=3, per-point-sigma workload, inputs resident in
HBM.  Prints ONE JSON line with the output Mpix/s of fwd+bwd (`value`), the
forward-only Mpix/s, the roofline of the dominant kernel, the CPU oracle
baseline and, when the serving loop is built, its p50/p99 latency.
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks and derived ALU issue rate (see the design notes)
HBM_PEAK_GBS = 8000.0
CU, SIMD_LANES_PER_CU, CLOCK_GHZ = 256, 64, 2.4
VALU_PEAK_TLANEOPS = CU * SIMD_LANES_PER_CU * CLOCK_GHZ / 1000.0   # 39.32 T lane-ops/s
# Algorithmic VALU lane-ops per pixel-point pair inside the radius.  The
# method's count (the roofline's `frac`): forward 8 + C (2 sub, a mul and an
# FMA for d2, 1 mul by the exponent scale, compare + select, 1 add for Z, C
# FMAs), backward 13 + 2C, with the one v_exp_f32 per pair and pass counted
# against its own rate.  The implementation's count (`frac_impl`) follows the
# float32 radius test, which rounds d2 without contraction (one more op), and
# counts the exp as a VALU op (measured, it overlaps fully with the rest):
#   forward  2 sub + 2 mul + 1 add (d2), 1 mul (exponent), 1 exp, 1 cmp,
#            1 select, 1 add (Z), C FMAs                       = 10 + C
#   backward 1 sub + 1 mul + 1 add (d2, the row term amortised), 1 cmp,
#            1 mul, 1 exp, C FMAs (A), C FMAs (dL/dc), 1 mul, 3 FMAs = 11 + 2C
FORWARD_SOURCES = ("common.hpp", "kernels.hpp", "single.hip")
FORWARD_PROFILE = os.path.join(ROOT, "profiles", "forward_1024x1024_n1M_c3.md")


def forward_source_hash() -> str:
    """sha256 of the code (comments and blank space removed) of the sources
    the forward kernel is built from."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in FORWARD_SOURCES:
        with open(os.path.join(ROOT, "paper_2012_13257_amd", "csrc", f)) as fh:
            code = re.sub(r"//[^\n]*", "", fh.read())
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()


def forward_traffic():
    """HBM bytes per forward launch from the committed counter summary, or None
    when the forward's sources changed since the counters were taken."""
    try:
        with open(FORWARD_PROFILE) as fh:
            kv = dict(line.split(": ", 1) for line in fh.read().splitlines()
                      if line.startswith("forward_") and ": " in line)
        if kv.get("forward_source_sha256", "").strip() != forward_source_hash():
            return None
        return int(kv["forward_fetch_bytes_per_launch"]) + int(kv["forward_write_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def fwd_ops(C):
    """Method count of the forward: VALU lane-ops per in-radius pair."""
    return 8 + C


def bwd_ops(C):
    """Method count of the adjoint: VALU lane-ops per in-radius pair."""
    return 13 + 2 * C


def fwd_ops_impl(C):
    return 10 + C


def bwd_ops_impl(C):
    return 11 + 2 * C


def algorithmic_bytes(B, N, C, H, W, per_point, backward, vbytes=4):
    """HBM bytes the method must move: inputs read once, outputs written once
    (forward: points, image and Z; backward: G, out and Z read, points read,
    gradients written).  vbytes: bytes per stored value (values, out, grad_out,
    grad_values: 4 for float32, 2 for bfloat16 / half)."""
    pts = B * N * (8 + 4 * per_point + vbytes * C)
    fwd = pts + B * H * W * vbytes * C + B * H * W * 4
    if not backward:
        return fwd
    bwd = B * H * W * (2 * vbytes * C + 4) + pts + B * N * (vbytes * C + 8 + 4 * per_point)
    return fwd + bwd


def pair_count(pos: np.ndarray, sigma: np.ndarray, H: int, W: int, radius: float) -> int:
    """Exact number of (pixel, point) pairs passing the float32 radius test,
    enumerated per point over its bounding box (the work unit of the roofline)."""
    total = 0
    B, N, _ = pos.shape
    f32 = np.float32
    for b in range(B):
        sig = sigma[b] if sigma.ndim == 2 else np.full(N, sigma[b], np.float32)
        rs = (f32(radius) * sig.astype(np.float32)).astype(np.float32)
        R2 = (rs * rs).astype(np.float32)
        reach = np.ceil(rs.astype(np.float64) + 1.0).astype(np.int64)
        x = pos[b, :, 0]
        y = pos[b, :, 1]
        for rch in np.unique(reach):
            sel = np.nonzero(reach == rch)[0]
            offs = np.arange(-rch, rch + 1)
            for chunk in range(0, sel.size, 65536):
                s = sel[chunk: chunk + 65536]
                u = np.floor(x[s]).astype(np.int64)[:, None] + offs[None, :]
                v = np.floor(y[s]).astype(np.int64)[:, None] + offs[None, :]
                dx = (u.astype(np.float32) - x[s, None]).astype(np.float32)
                dy = (v.astype(np.float32) - y[s, None]).astype(np.float32)
                dxx = (dx * dx).astype(np.float32)
                dyy = (dy * dy).astype(np.float32)
                okx = (u >= 0) & (u < W)
                oky = (v >= 0) & (v < H)
                d2 = (dxx[:, None, :] + dyy[:, :, None]).astype(np.float32)
                inc = (d2 <= R2[s, None, None]) & okx[:, None, :] & oky[:, :, None]
                total += int(inc.sum())
    return total


def _to_dev(wl):
    import torch
    return (torch.from_numpy(wl.pos).cuda(), torch.from_numpy(wl.sigma).cuda(),
            torch.from_numpy(wl.values).cuda())


def time_steps(fn, steps: int, warmup: int, profile: bool):
    import torch
    from paper_2012_13257_amd import _lib
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if profile:
        _lib.profile_enable(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop) / steps
    kernels = {}
    if profile:
        for name in ("bin_keys", "radix_hist", "radix_scan", "radix_scatter", "place_wide",
                     "bin_finish", "fwd_plan", "forward", "bwd_pixel", "bwd_point", "bwd_sigma_sum"):
            tot, n = _lib.profile_read(name)
            if n:
                kernels[name] = {"avg_us": 1000.0 * tot / n, "launches": n}
        _lib.profile_enable(False)
    return ms, wall, kernels


def capture(fn):
    """Captures fn's launches (issued on torch's current stream) into a HIP graph."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, G, budget_s: float):
    """The oracle as it stands, on a bounded sample of the same workload."""
    import oracle
    workers = oracle.default_workers()
    rng = np.random.default_rng(2024)
    # forward: a pixel sample sized to about half the budget (calibrated on 16 pixels)
    t0 = time.perf_counter()
    px = 16
    oracle.forward_pixels(wl.pos, wl.sigma, wl.values, wl.radius, np.zeros(px, np.int64),
                          rng.integers(0, wl.H, px), rng.integers(0, wl.W, px), workers=1)
    t_px1 = (time.perf_counter() - t0) / px
    n_px = int(max(64, min(20000, 0.5 * budget_s * workers / max(t_px1, 1e-6))))
    b = np.zeros(n_px, np.int64)
    v = rng.integers(0, wl.H, n_px)
    u = rng.integers(0, wl.W, n_px)
    t0 = time.perf_counter()
    oracle.forward_pixels(wl.pos, wl.sigma, wl.values, wl.radius, b, v, u, workers=workers)
    t_fwd = (time.perf_counter() - t0) / n_px
    # backward: a point sample (each point recomputes Z and out at its support)
    t0 = time.perf_counter()
    oracle.backward_points(wl.pos, wl.sigma, wl.values, G, wl.H, wl.W, wl.radius, 0, [0], workers=1)
    t_pt1 = time.perf_counter() - t0
    n_pt = int(max(4, min(4096, 0.5 * budget_s * workers / max(t_pt1, 1e-6))))
    pts = rng.choice(wl.N, n_pt, replace=False)
    t0 = time.perf_counter()
    oracle.backward_points(wl.pos, wl.sigma, wl.values, G, wl.H, wl.W, wl.radius, 0, pts,
                           workers=workers, block=max(1, n_pt // (4 * workers)))
    t_bwd = (time.perf_counter() - t0) / n_pt
    per_px = t_fwd + t_bwd * (wl.N / (wl.H * wl.W))
    return {"value": 1.0 / per_px / 1e6, "unit": "Mpix/s (fwd+bwd)", "cores": workers,
            "kind": "oracle", "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)),
            "threads_note": "oracle thread pool = the CPUs this process may run on, at most 16 "
                            "(the host share of one GPU)",
            "sample": f"{n_px} random pixels forward + {n_pt} random points backward of the "
                      f"{wl.H}x{wl.W} N={wl.N} workload, extrapolated linearly to the full image "
                      f"(fwd {t_fwd * 1e3:.2f} ms/pixel, bwd {t_bwd * 1e3:.1f} ms/point)",
            "fwd_mpix_s": 1.0 / t_fwd / 1e6}


def measure_peaks(log):
    """Measured ceilings: VALU FMA rate, v_exp_f32 rate, a 1 exp : 6 VALU mix,
    and an HBM copy (also the reference kernel of known size for the byte
    counters)."""
    import ctypes
    import torch
    from paper_2012_13257_amd.build import PEAK_LIB
    lib = ctypes.CDLL(PEAK_LIB)
    lib.gmm_peak_launch.restype = ctypes.c_double
    lib.gmm_peak_launch.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_longlong, ctypes.c_void_p]
    st = torch.cuda.current_stream().cuda_stream
    out = torch.zeros(1 << 16, device="cuda")
    n4 = (512 << 20) // 16
    src = torch.ones(n4 * 4, device="cuda")
    dst = torch.empty_like(src)
    res = {}
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    runs = [(0, 0, "fma"), (1, 0, "exp"), (2, 0, "mix"), (3, 0, "copy")]
    # streaming copy and read at 4, 8 and 16 workgroups per compute unit (best kept)
    runs += [(4, k * cus, f"copy_stream{k}") for k in (4, 8, 16)]
    runs += [(5, k * cus, f"read_stream{k}") for k in (4, 8, 16)]
    for which, blocks, name in runs:
        def go():
            v = lib.gmm_peak_launch(which, blocks, out.data_ptr(), src.data_ptr(), dst.data_ptr(),
                                    n4, st)
            if v < 0:
                raise RuntimeError("peak kernel launch failed")
            return v
        go()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        reps = 5
        for _ in range(reps):
            work = go()
        b.record()
        torch.cuda.synchronize()
        sec = a.elapsed_time(b) / 1e3 / reps
        res[name] = work / sec
    best_copy = max(v for k, v in res.items() if k.startswith("copy"))
    best_read = max(v for k, v in res.items() if k.startswith("read"))
    peaks = {"valu_fma_tlaneops": round(res["fma"] / 1e12, 2),
             "exp_tlaneops": round(res["exp"] / 1e12, 2),
             "mix_iter_per_ns_per_lane": None,
             "exp_issue_slots": round(res["fma"] / res["exp"], 2),
             "hbm_copy_gbs": round(best_copy / 1e9, 1),
             "hbm_read_gbs": round(best_read / 1e9, 1),
             "hbm_copy_variants_gbs": {k: round(v / 1e9, 1) for k, v in res.items()
                                       if k.startswith(("copy", "read"))}}
    # mix: 7 VALU instructions per chain-iteration, one of them exp
    mix_inst = res["mix"] * 7
    peaks["mix_tlaneops"] = round(mix_inst / 1e12, 2)
    peaks.pop("mix_iter_per_ns_per_lane")
    log(f"measured ceilings: {peaks}")
    del src, dst
    return peaks


def measure_workload(wl, steps: int, warmup: int, backward: bool, log, kernel: int = 0,
                     storage: str = "float32"):
    """Times one named workload through the C ABI (eager calls, inputs in HBM):
    ms per step (forward, + backward when asked), Mpix/s, per-kernel event
    averages, the exact in-radius pair count, and the fraction of the ALU and
    HBM ceilings the dominant kernels and the whole step reach.  kernel: the
    INTERP_KERNEL_* flags (the pair count and ALU fractions are those of the
    isotropic test, so a diagonal kernel reports times only); storage: the
    dtype of values, out, grad_out and grad_values."""
    import ctypes
    import torch
    from paper_2012_13257_amd import _lib, interp
    pos, sig, val = _to_dev(wl)
    val = val.to(getattr(torch, storage))
    prob = interp.problem(pos, sig, val, wl.H, wl.W, wl.radius, normalized=bool(kernel & 1),
                          anisotropic=bool(kernel & 2))
    L = _lib.lib()
    out = torch.empty((wl.B, wl.C, wl.H, wl.W), device="cuda", dtype=val.dtype)
    saved = interp.Saved(prob, pos.device)
    work = interp.Workspace(prob, pos.device)
    pb = ctypes.byref(prob)
    G = gp = gs = gv = None
    if backward:
        gen = torch.Generator(device="cuda")
        gen.manual_seed(wl.grad_seed)
        G = torch.randn((wl.B, wl.C, wl.H, wl.W), generator=gen, device="cuda").to(val.dtype)
        gp, gs, gv = torch.empty_like(pos), torch.empty_like(sig), torch.empty_like(val)

    def fwd():
        st = torch.cuda.current_stream().cuda_stream
        _lib.check("interp_forward", L.interp_forward(
            pb, pos.data_ptr(), sig.data_ptr(), val.data_ptr(), out.data_ptr(), saved.addr,
            saved.nbytes, work.addr, work.nbytes, st))

    def step():
        fwd()
        if backward:
            st = torch.cuda.current_stream().cuda_stream
            _lib.check("interp_backward", L.interp_backward(
                pb, pos.data_ptr(), sig.data_ptr(), val.data_ptr(), out.data_ptr(), saved.addr,
                saved.nbytes, G.data_ptr(), gp.data_ptr(), gs.data_ptr(), gv.data_ptr(), work.addr,
                work.nbytes, st))

    ms_step, _, _ = time_steps(step, steps, warmup, profile=False)
    ms_fwd, _, _ = time_steps(fwd, steps, warmup, profile=False)
    _, _, kernels = time_steps(step, steps, warmup, profile=True)
    pix = wl.B * wl.H * wl.W
    res = {"B": wl.B, "H": wl.H, "W": wl.W, "N": wl.N, "C": wl.C, "kernel": kernel,
           "storage": storage,
           "ms_per_step": round(ms_step, 4), "mpix_s": round(pix / (ms_step * 1e-3) / 1e6, 1),
           "fwd_ms": round(ms_fwd, 4), "fwd_mpix_s": round(pix / (ms_fwd * 1e-3) / 1e6, 1),
           "kernels_us": {k: round(v["avg_us"], 2) for k, v in kernels.items()}}
    if kernel & 2:
        log(f"{wl.name} (kernel {kernel}): {res}")
        del out, saved, work, G, gp, gs, gv, pos, sig, val
        torch.cuda.empty_cache()
        return res
    P = pair_count(wl.pos, wl.sigma, wl.H, wl.W, wl.radius)
    res["pairs_in_radius"] = P
    # ALU fraction of the two pair kernels (method count), HBM fraction of the
    # whole step (algorithmic bytes over the step time)
    for kname, ops in (("forward", fwd_ops(wl.C)), ("bwd_point", bwd_ops(wl.C))):
        if kname in kernels:
            a = P * ops / (kernels[kname]["avg_us"] * 1e-6) / 1e12
            res[kname + "_alu_frac"] = round(a / VALU_PEAK_TLANEOPS, 4)
    per_point = int(wl.sigma.ndim == 2)
    nbytes = algorithmic_bytes(wl.B, wl.N, wl.C, wl.H, wl.W, per_point, backward,
                               vbytes=val.element_size())
    res["algorithmic_bytes"] = nbytes
    res["step_hbm_frac"] = round(nbytes / (ms_step * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)
    # the step's own roofline: the larger of the ALU and HBM times at the peaks
    t_alu = P * (fwd_ops(wl.C) + (bwd_ops(wl.C) if backward else 0)) / (VALU_PEAK_TLANEOPS * 1e12)
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    res["step_roofline_us"] = round(max(t_alu, t_hbm) * 1e6, 2)
    res["step_bound"] = "alu" if t_alu >= t_hbm else "hbm"
    res["step_frac"] = round(max(t_alu, t_hbm) / (ms_step * 1e-3), 4)
    log(f"{wl.name}: {res}")
    del out, saved, work, G, gp, gs, gv, pos, sig, val
    torch.cuda.empty_cache()
    return res


def latency_small(wl, steps: int, warmup: int, log):
    """Forward latency of the small 64x64 workload: one C-ABI call per step,
    eager and replayed from a HIP graph (the call is launch-bound)."""
    import ctypes
    import torch
    from paper_2012_13257_amd import _lib, interp
    pos, sig, val = _to_dev(wl)
    prob = interp.problem(pos, sig, val, wl.H, wl.W, wl.radius)
    L = _lib.lib()
    out = torch.empty((wl.B, wl.C, wl.H, wl.W), device="cuda")
    saved = interp.Saved(prob, pos.device)
    work = interp.Workspace(prob, pos.device)
    pb = ctypes.byref(prob)

    def fwd():
        st = torch.cuda.current_stream().cuda_stream
        _lib.check("interp_forward", L.interp_forward(
            pb, pos.data_ptr(), sig.data_ptr(), val.data_ptr(), out.data_ptr(), saved.addr,
            saved.nbytes, work.addr, work.nbytes, st))

    ms_eager, wall, _ = time_steps(fwd, steps, warmup, profile=False)
    g = capture(fwd)
    ms_graph, _, _ = time_steps(g.replay, steps, warmup, profile=False)
    res = {"B": wl.B, "H": wl.H, "W": wl.W, "N": wl.N, "C": wl.C,
           "fwd_us_eager": round(ms_eager * 1e3, 2), "fwd_us_graph": round(ms_graph * 1e3, 2),
           "fwd_us_host_wall": round(wall / steps * 1e6, 2)}
    log(f"{wl.name}: {res}")
    return res


def optimisation_step_timing(steps: int, warmup: int, log, size: int = 1024,
                             n_points: int = 1 << 18):
    """One step of the point / sigma fitting (render through the autograd
    binding, L1 loss against a synthetic target, backward, Adam update) on a
    1024x1024 RGB target with 2^18 points and per-point sigma."""
    import torch
    from paper_2012_13257_amd import synth
    from paper_2012_13257_amd.optimize import PointFit, l1_loss
    target = torch.from_numpy(synth.natural_image(7, 3, size, size)).cuda()
    fit = PointFit.from_image(target, n_points, 1.0, seed=7, per_point_sigma=True,
                              learn_pos=True, learn_sigma=True)
    opt = torch.optim.Adam([{"params": [fit.pos], "lr": 0.05},
                            {"params": [fit.log_sigma], "lr": 0.02}])

    def step():
        opt.zero_grad(set_to_none=True)
        l1_loss(fit.render(), target).backward()
        opt.step()

    ms, _, _ = time_steps(step, steps, warmup, profile=False)
    res = {"H": size, "W": size, "C": 3, "N": n_points, "ms_per_step": round(ms, 4),
           "mpix_s": round(size * size / (ms * 1e-3) / 1e6, 1),
           "step": "render + L1 + backward (pos, per-point sigma) + Adam"}
    log(f"optimisation step: {res}")
    return res


def upsampling_timing(steps: int, warmup: int, log, B: int = 16, low: int = 64, s: int = 4):
    """Gaussian-mixture upsampling of a batch of 16 RGB 64x64 images by 4 (the
    reconstruction study's operation): one forward call per step."""
    import torch
    from paper_2012_13257_amd import reconstruct, synth
    img = torch.from_numpy(np.stack([synth.natural_image(100 + i, 3, low * s, low * s)
                                     for i in range(B)])).cuda()
    lowres = reconstruct.downsample(img, s)
    pos, val = reconstruct.gmm_points(lowres, s)
    sig = torch.full((B,), 0.5 * s, device="cuda")
    from paper_2012_13257_amd import interp
    with torch.no_grad():
        fn = lambda: interp.forward(pos, sig, val, low * s, low * s, 3.0)  # noqa: E731
        ms, _, _ = time_steps(fn, steps, warmup, profile=False)
    res = {"B": B, "in": low, "factor": s, "out": low * s, "N": low * low, "C": 3,
           "sigma": 0.5 * s, "ms_per_call": round(ms, 4),
           "mpix_s": round(B * (low * s) ** 2 / (ms * 1e-3) / 1e6, 1)}
    log(f"upsampling: {res}")
    return res


def serving_benchmark(log, n_requests: int = 4096, seed: int = 1004, budget_gb: float = 24.0,
                      slots: int = 256):
    """Serving stream (sides 64..1024, N = side^2 * U(0.25, 1), C in {1,3,4},
    shared sigma U(0.5, 1.5), 30% with backward): the batching server against
    one launch sequence per request on the same GPU, saturated and with
    Poisson arrivals at 0.8x the baseline's saturated request rate."""
    import ctypes
    import torch
    from paper_2012_13257_amd import _lib, interp, synth
    from paper_2012_13257_amd.server import Batch, Server

    trace = synth.config4_trace(n_requests, None, seed=seed)
    gen = torch.Generator(device="cuda")
    reqs = []
    for r in trace:
        gen.manual_seed(r.seed)
        pos = torch.rand((1, r.N, 2), generator=gen, device="cuda") * r.side
        pos.clamp_(max=float(np.nextafter(np.float32(r.side), np.float32(0))))
        val = torch.rand((1, r.N, r.C), generator=gen, device="cuda")
        sig = torch.full((1,), r.sigma, device="cuda")
        G = torch.randn((1, r.C, r.side, r.side), generator=gen, device="cuda") if r.backward else None
        prob = interp.problem(pos, sig, val, r.side, r.side, 3.0)
        out = torch.empty((1, r.C, r.side, r.side), device="cuda")
        grads = (torch.empty_like(pos), torch.empty_like(sig), torch.empty_like(val)) if r.backward else None
        reqs.append(dict(r=r, pos=pos, sig=sig, val=val, G=G, prob=prob, out=out, grads=grads))
    torch.cuda.synchronize()
    px = np.array([q["r"].side ** 2 for q in reqs], dtype=np.float64)
    total_px = float(px.sum())
    log(f"serving: {n_requests} requests, {total_px / 1e6:.1f} Mpix, "
        f"{sum(q['r'].backward for q in reqs)} with backward")

    # --- one launch sequence per request (single-call API, one stream) ---
    L = _lib.lib()
    big = max(reqs, key=lambda q: q["r"].side ** 2 * 8 + q["r"].N)["prob"]
    sb = max(L.interp_saved_bytes(ctypes.byref(q["prob"])) for q in reqs)
    wb = max(L.interp_workspace_bytes(ctypes.byref(q["prob"])) for q in reqs)
    del big
    sbuf, saddr = interp.aligned_buffer(sb, "cuda")
    wbuf, waddr = interp.aligned_buffer(wb, "cuda")
    stream = torch.cuda.current_stream().cuda_stream

    def launch_one(q):
        pb = ctypes.byref(q["prob"])
        _lib.check("interp_forward", L.interp_forward(
            pb, q["pos"].data_ptr(), q["sig"].data_ptr(), q["val"].data_ptr(), q["out"].data_ptr(),
            saddr, sb, waddr, wb, stream))
        if q["G"] is not None:
            gp, gs, gv = q["grads"]
            _lib.check("interp_backward", L.interp_backward(
                pb, q["pos"].data_ptr(), q["sig"].data_ptr(), q["val"].data_ptr(),
                q["out"].data_ptr(), saddr, sb, q["G"].data_ptr(), gp.data_ptr(), gs.data_ptr(),
                gv.data_ptr(), waddr, wb, stream))

    # The timed request loops run with Python's garbage collector paused, so a
    # collection in the driver loop does not show up as request latency.
    def baseline(arrivals):
        evs = [torch.cuda.Event(enable_timing=True) for _ in reqs]
        start = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        gc.collect()
        gc.disable()
        try:
            t0 = time.perf_counter()
            start.record()
            for q, a, e in zip(reqs, arrivals, evs):
                while time.perf_counter() - t0 < a:
                    pass
                launch_one(q)
                e.record()
            torch.cuda.synchronize()
        finally:
            gc.enable()
        done = np.array([start.elapsed_time(e) / 1e3 for e in evs])
        return done, done - arrivals

    def server_run(arrivals, many=False):
        """Every request is described ahead (Server.prepare: the descriptor and
        its buffers, as the baseline's are), so the timed loop pays only the
        submission.  many: all of them (all arriving at once) queued by one
        interp_submit_many call, so the Python submit loop does not pace the
        server."""
        srv = Server(budget_bytes=int(budget_gb * (1 << 30)), max_slots=slots)
        try:
            tickets = []
            prepared = [srv.prepare(q["pos"], q["sig"], q["val"], q["r"].side, q["r"].side, 3.0,
                                    grad_out=q["G"], out=q["out"],
                                    grad_buffers=None if q["grads"] is None else
                                    dict(zip(("pos", "sigma", "values"), q["grads"])))
                        for q in reqs]
            batch = Batch(prepared) if many else None
            torch.cuda.synchronize()
            gc.collect()
            gc.disable()
            try:
                t0 = time.monotonic_ns()
                if many:
                    tickets = srv.submit_many(batch)
                else:
                    for pr, a in zip(prepared, arrivals):
                        while time.monotonic_ns() - t0 < a * 1e9:
                            pass
                        tickets.append(srv.submit_prepared(pr))
                srv.drain()
            finally:
                gc.enable()
            res = [srv.result(t) for t in tickets]
            assert all(x["state"] == _lib.DONE for x in res)
            done = np.array([(x["t_done_ns"] - t0) / 1e9 for x in res])
            lag = np.array([(x["t_submit_ns"] - t0) / 1e9 for x in res]) - arrivals
            log(f"  server submit lag behind the schedule: p50 {np.percentile(lag, 50) * 1e3:.3f} ms, "
                f"p99 {np.percentile(lag, 99) * 1e3:.3f} ms, max {lag.max() * 1e3:.3f} ms")
            return done, done - arrivals
        finally:
            srv.close()

    def summary(done, lat):
        mk = float(done.max())
        return {"throughput_mpix_s": round(total_px / mk / 1e6, 1),
                "requests_per_s": round(len(done) / mk, 1), "makespan_s": round(mk, 4),
                "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3)}

    zero = np.zeros(len(reqs))
    launch_one(reqs[0])  # warm-up
    torch.cuda.synchronize()
    b_sat = summary(*baseline(zero))
    log(f"serving baseline saturated: {b_sat}")
    s_sat = summary(*server_run(zero))
    log(f"serving server saturated:   {s_sat}")
    s_many = summary(*server_run(zero, many=True))
    log(f"serving server saturated, one submit_many call: {s_many}")
    rate = 0.8 * b_sat["requests_per_s"]
    arr = np.array([r.arrival_s for r in synth.config4_trace(n_requests, rate, seed=seed)])
    b_poi = summary(*baseline(arr))
    log(f"serving baseline Poisson {rate:.0f}/s: {b_poi}")
    s_poi = summary(*server_run(arr))
    log(f"serving server   Poisson {rate:.0f}/s: {s_poi}")
    return {"requests": n_requests, "poisson_rate_per_s": round(rate, 1),
            "server": {"saturated": s_sat, "saturated_submit_many": s_many, "poisson": s_poi},
            "one_launch_per_request": {"saturated": b_sat, "poisson": b_poi},
            "saturated_speedup": round(s_sat["throughput_mpix_s"] / b_sat["throughput_mpix_s"], 3),
            "saturated_speedup_submit_many":
                round(s_many["throughput_mpix_s"] / b_sat["throughput_mpix_s"], 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of CPU work for the oracle baseline (0 disables)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (64x64 latency, 16x256x256, 2x4096x4096 C=16)")
    ap.add_argument("--serving-requests", type=int, default=4096)
    ap.add_argument("--workload", choices=("c16",), default=None,
                    help="time only the 2 x 4096^2, C = 16 forward + backward (for profiling "
                         "its kernels); prints that measurement instead of the benchmark line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload:
        import torch
        from paper_2012_13257_amd import synth
        if not torch.cuda.is_available():
            print("bench.py needs the ROCm device", file=sys.stderr)
            sys.exit(1)
        log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)  # noqa: E731
        r = measure_workload(synth.config5(), args.steps, args.warmup, True, log)
        print(json.dumps({"workload": "cfg5_2x4096x4096_n4M_c16_fwd_bwd", **r}), flush=True)
        return

    import torch
    from paper_2012_13257_amd import interp, synth, _lib

    if not torch.cuda.is_available():
        print("bench.py needs the ROCm device", file=sys.stderr)
        sys.exit(1)
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)  # noqa: E731

    peaks = measure_peaks(log)
    wl = synth.config3()
    G_np = wl.grad_out()
    log("workload", wl.name, "B", wl.B, "N", wl.N, "C", wl.C, "HxW", wl.H, wl.W)
    pos, sig, val = _to_dev(wl)
    G = torch.from_numpy(G_np).cuda()
    prob = interp.problem(pos, sig, val, wl.H, wl.W, wl.radius)
    import ctypes
    L = _lib.lib()
    out = torch.empty((wl.B, wl.C, wl.H, wl.W), device="cuda")
    saved = interp.Saved(prob, pos.device)
    work = interp.Workspace(prob, pos.device)
    gp = torch.empty_like(pos)
    gs = torch.empty_like(sig)
    gv = torch.empty_like(val)
    pb = ctypes.byref(prob)

    def fwd():
        st = torch.cuda.current_stream().cuda_stream
        _lib.check("interp_forward", L.interp_forward(
            pb, pos.data_ptr(), sig.data_ptr(), val.data_ptr(), out.data_ptr(), saved.addr,
            saved.nbytes, work.addr, work.nbytes, st))

    def bwd():
        st = torch.cuda.current_stream().cuda_stream
        _lib.check("interp_backward", L.interp_backward(
            pb, pos.data_ptr(), sig.data_ptr(), val.data_ptr(), out.data_ptr(), saved.addr,
            saved.nbytes, G.data_ptr(), gp.data_ptr(), gs.data_ptr(), gv.data_ptr(), work.addr,
            work.nbytes, st))

    def step():
        fwd()
        bwd()

    # eager: one C-ABI call per forward / backward, no per-kernel events
    ms_eager, wall, _ = time_steps(step, args.steps, args.warmup, profile=False)
    log(f"fwd+bwd eager {ms_eager * 1e3:.1f} us/step (wall {wall / args.steps * 1e6:.1f} us/step)")
    ref = [t.clone() for t in (out, gp, gs, gv)]
    ms_fwd_eager, _, _ = time_steps(fwd, args.steps, args.warmup, profile=False)
    # the same calls captured once into a HIP graph and replayed
    graph, graph_fwd = capture(step), capture(fwd)
    ms_graph, _, _ = time_steps(graph.replay, args.steps, args.warmup, profile=False)
    step()
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    graph_ok = all(torch.equal(a, b) for a, b in zip(ref, (out, gp, gs, gv)))
    ms_fwd_graph, _, _ = time_steps(graph_fwd.replay, args.steps, args.warmup, profile=False)
    log(f"fwd+bwd graph {ms_graph * 1e3:.1f} us/step, fwd eager {ms_fwd_eager * 1e3:.1f} "
        f"graph {ms_fwd_graph * 1e3:.1f}; graph replay bitwise equal to eager: {graph_ok}")
    if not graph_ok:
        raise RuntimeError("graph replay differs from the eager result")
    # per-kernel durations: a separate run with events around every launch
    _, _, kernels = time_steps(step, args.steps, args.warmup, profile=True)
    for k, v in kernels.items():
        log(f"  {k:16s} {v['avg_us']:9.2f} us x{v['launches']}")
    ms_step = min(ms_eager, ms_graph)
    ms_fwd = min(ms_fwd_eager, ms_fwd_graph)

    pix = wl.B * wl.H * wl.W
    value = pix / (ms_step * 1e-3) / 1e6
    fwd_mpix = pix / (ms_fwd * 1e-3) / 1e6

    t0 = time.perf_counter()
    P = pair_count(wl.pos, wl.sigma, wl.H, wl.W, wl.radius)
    log(f"pairs inside the radius P = {P} ({time.perf_counter() - t0:.1f} s to count)")
    C = wl.C
    ops = {"forward": (fwd_ops(C), fwd_ops_impl(C)), "bwd_point": (bwd_ops(C), bwd_ops_impl(C))}
    dom = max(kernels.items(), key=lambda kv: kv[1]["avg_us"])
    name, info = dom
    roof = None
    if name in ops:
        m, im = ops[name]
        achieved = P * m / (info["avg_us"] * 1e-6) / 1e12
        roof = {"bound": "alu", "kernel": name, "achieved": round(achieved, 3),
                "peak": round(VALU_PEAK_TLANEOPS, 2), "unit": "Tlaneop/s",
                "frac": round(achieved / VALU_PEAK_TLANEOPS, 4),
                "traffic": forward_traffic() if name == "forward" else None,
                "work_per_launch": f"P={P} pairs x {m} VALU lane-ops (method count)",
                "frac_impl": round(P * im / (info["avg_us"] * 1e-6) / 1e12 / VALU_PEAK_TLANEOPS, 4),
                "impl_ops_per_pair": im,
                "kernel_avg_us": round(info["avg_us"], 2)}
    other = {}
    for kname, (m, im) in ops.items():
        if kname in kernels:
            a = P * m / (kernels[kname]["avg_us"] * 1e-6) / 1e12
            other[kname] = {"avg_us": round(kernels[kname]["avg_us"], 2),
                            "alu_frac": round(a / VALU_PEAK_TLANEOPS, 4),
                            "alu_frac_impl": round(a * im / m / VALU_PEAK_TLANEOPS, 4)}
    binning = sum(kernels[k]["avg_us"] * kernels[k]["launches"] / args.steps
                  for k in ("bin_keys", "radix_hist", "radix_scan", "radix_scatter", "place_wide",
                            "bin_finish", "fwd_plan") if k in kernels)
    del out, saved, work, gp, gs, gv, G, graph, graph_fwd, ref
    torch.cuda.empty_cache()

    configs = None
    if not args.no_configs:
        configs = {
            "cfg1_64x64_n4096_c3": latency_small(synth.config1(), 200, 20, log),
            "cfg2_16x256x256_n65536_c3_fwd": measure_workload(synth.config2(), args.steps,
                                                              args.warmup, False, log),
            "cfg5_2x4096x4096_n4M_c16_fwd_bwd": measure_workload(synth.config5(), 5, 2, True, log),
            "cfg5_2x4096x4096_n4M_c16_bf16_fwd_bwd": measure_workload(
                synth.config5(), 5, 2, True, log, storage="bfloat16"),
            "cfg3_normalised_fwd_bwd": measure_workload(synth.config3(), args.steps, args.warmup,
                                                        True, log, kernel=1),
            "cfg3_anisotropic_diagonal_fwd_bwd": measure_workload(
                synth.config3_anisotropic(), args.steps, args.warmup, True, log, kernel=2),
            "optimise_1024x1024_n256k_pos_sigma": optimisation_step_timing(args.steps,
                                                                          args.warmup, log),
            "upsample_16x64x64_x4": upsampling_timing(args.steps, args.warmup, log),
        }

    cpu = None
    if args.cpu_budget > 0:
        log("timing the CPU oracle baseline ...")
        cpu = cpu_baseline(wl, G_np, args.cpu_budget)
        log(f"oracle {cpu['value']:.3g} Mpix/s fwd+bwd on {cpu['cores']} threads")

    serving = None
    if not args.no_serving:
        serving = serving_benchmark(log, n_requests=args.serving_requests)

    res = {
        "metric": "output Mpix/s fwd+bwd at 1024x1024, N=1M (fwd-only and serving p50/p99 alongside)",
        "value": round(value, 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "launch": "hip_graph" if ms_graph <= ms_eager else "eager",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded: 70% of points in 8 Gaussian blobs, 30% uniform)",
        "config": {"workload": wl.name, "B": wl.B, "H": wl.H, "W": wl.W, "N": wl.N, "C": wl.C,
                   "sigma": "per point, log-uniform [0.5, 2]", "radius": wl.radius, "tile": 8,
                   "pairs_in_radius": P},
        "fwd_mpix_s": round(fwd_mpix, 2),
        "fwd_ms": round(ms_fwd, 4),
        "eager_ms_per_step": round(ms_eager, 4),
        "graph_ms_per_step": round(ms_graph, 4),
        "fwd_eager_ms": round(ms_fwd_eager, 4),
        "fwd_graph_ms": round(ms_fwd_graph, 4),
        "kernels_us": {k: round(v["avg_us"], 2) for k, v in kernels.items()},
        "kernel_alu": other,
        "binning_us": round(binning, 2),
        "roofline": roof,
        "measured_ceilings": peaks,
        "cpu_baseline": cpu,
        "serving": serving,
        "configs": configs,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
