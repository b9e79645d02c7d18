"""Helpers shared by the GPU parity tests: run the HIP path on a synthetic
workload and compare it with the CPU oracle under the stated tolerances."""
from __future__ import annotations

import sys

import numpy as np

FWD_RTOL = 1e-5      # forward outputs, scale-aware relative error
Z_RTOL = 1e-5        # normaliser
GRAD_RTOL = 1e-3     # gradients, scale-aware relative error


def say(*a):
    """Names the case before each GPU step, flushed, so a failing run shows it."""
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def to_dev(wl, device="cuda"):
    import torch
    pos = torch.from_numpy(np.ascontiguousarray(wl.pos)).to(device)
    sig = torch.from_numpy(np.ascontiguousarray(wl.sigma)).to(device)
    val = torch.from_numpy(np.ascontiguousarray(wl.values)).to(device)
    return pos, sig, val


def saved_Z(saved):
    """The normaliser Z [B,H,W] stored at the start of the saved state."""
    import torch
    p = saved.prob
    off = saved.addr - saved.buf.data_ptr()
    n = p.B * p.H * p.W
    return saved.buf[off: off + 4 * n].view(torch.float32).reshape(p.B, p.H, p.W)


def saved_reach(saved):
    """The per-image reach [B] (largest f32(radius * sigma)) stored after Z."""
    import torch
    p = saved.prob
    off = saved.addr - saved.buf.data_ptr()
    zbytes = (4 * p.B * p.H * p.W + 255) // 256 * 256
    return saved.buf[off + zbytes: off + zbytes + 4 * p.B].view(torch.float32)


def run_forward(wl, tile=8):
    from paper_2012_13257_amd import interp
    import torch
    pos, sig, val = to_dev(wl)
    out, saved, work = interp.forward(pos, sig, val, wl.H, wl.W, wl.radius, tile)
    torch.cuda.synchronize()
    return out, saved, work, (pos, sig, val)


def check_forward_pixels(out_g, Z_g, ref, where=""):
    """out_g [n, C], Z_g [n] (GPU, float32) vs oracle dict (out [n,C], Z [n], S [n,C])."""
    o_ref = ref["out"]
    Z_ref = ref["Z"]
    out_g = np.asarray(out_g, np.float64)
    Z_g = np.asarray(Z_g, np.float64)
    empty = Z_ref == 0
    # the radius test is bit-exact on both sides, so empty pixels agree exactly
    assert np.array_equal(Z_g == 0, empty), f"{where}: Z==0 pattern differs " \
        f"({int(np.sum((Z_g == 0) != empty))} pixels)"
    assert np.all(out_g[empty] == 0), f"{where}: empty pixel with non-zero output"
    nz = ~empty
    zerr = np.abs(Z_g[nz] - Z_ref[nz]) / Z_ref[nz]
    assert zerr.size == 0 or zerr.max() <= Z_RTOL, f"{where}: Z rel err {zerr.max():.3g}"
    scale = np.maximum(np.abs(o_ref), ref["S"])
    err = np.abs(out_g - o_ref)
    bad = err > FWD_RTOL * scale
    assert not bad.any(), (f"{where}: {int(bad.sum())} outputs beyond tolerance; worst rel "
                           f"{float((err / np.maximum(scale, 1e-300)).max()):.3g}")
    rel = err[nz] / np.maximum(scale[nz], 1e-300)
    return float(rel.max()) if rel.size else 0.0


def check_out_only(out_g, ref, where=""):
    """out_g [n, C] (GPU) vs the oracle where the GPU's Z is not available:
    pixels the oracle leaves empty must be exactly 0, the others within the
    scale-aware tolerance."""
    o_ref = ref["out"]
    out_g = np.asarray(out_g, np.float64)
    empty = ref["Z"] == 0
    assert np.all(out_g[empty] == 0), f"{where}: empty pixel with non-zero output"
    scale = np.maximum(np.abs(o_ref), ref["S"])
    err = np.abs(out_g - o_ref)
    bad = err > FWD_RTOL * scale
    assert not bad.any(), (f"{where}: {int(bad.sum())} outputs beyond tolerance; worst rel "
                           f"{float((err / np.maximum(scale, 1e-300)).max()):.3g}")


def check_grad(g_gpu, g_ref, scale, where=""):
    g_gpu = np.asarray(g_gpu, np.float64)
    err = np.abs(g_gpu - g_ref)
    lim = GRAD_RTOL * np.maximum(np.abs(g_ref), scale)
    bad = err > lim + 1e-30
    if bad.any():
        idx = np.argwhere(bad)[:6]
        detail = "; ".join(f"{tuple(int(i) for i in ix)}: gpu {float(g_gpu[tuple(ix)]):.6g} "
                           f"ref {float(g_ref[tuple(ix)]):.6g} scale {float(scale[tuple(ix)]):.3g}"
                           for ix in idx)
        raise AssertionError(
            f"{where}: {int(bad.sum())}/{bad.size} gradients beyond tolerance; worst rel "
            f"{float((err / np.maximum(np.maximum(np.abs(g_ref), scale), 1e-300)).max()):.3g}; "
            f"first: {detail}")
    den = np.maximum(np.maximum(np.abs(g_ref), scale), 1e-300)
    return float((err / den).max()) if err.size else 0.0
