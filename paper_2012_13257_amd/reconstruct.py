"""Downsample / upsample reconstruction study (paper, Section 3, "Testing the
reconstruction quality"), on synthetic images.

An image is downsampled by an integer factor s (area average over s x s
pixels); every low-resolution pixel becomes a known point at the centre of
its s x s footprint in the full-resolution grid, carrying that pixel's
value; the full-resolution image is then reconstructed by Gaussian-mixture
interpolation (Eq. 1 and Eq. 2, radius truncation) with a shared sigma
proportional to s, and scored by its L1 distance to the original.  torch's
own resamplers (nearest, bilinear, bicubic) upsample the same low-resolution
image for comparison.  The paper's ImageNet images and PIL filters are not
available here: synthetic images with natural-image statistics
(synth.natural_image) stand in for the former, torch's resamplers for the
latter.

    python -m paper_2012_13257_amd.reconstruct [--size 512] [--images 8]

Every Gaussian-mixture interpolation runs in libgmminterp.so.
"""
from __future__ import annotations

import argparse
import json
from typing import Dict, Sequence

import numpy as np
import torch
import torch.nn.functional as F

from . import interp, synth

__all__ = ["downsample", "grid_points", "gmm_upsample", "study"]


def downsample(img: torch.Tensor, s: int) -> torch.Tensor:
    """Area average over s x s blocks: [B, C, H, W] -> [B, C, H//s, W//s]."""
    return F.avg_pool2d(img, s)


def grid_points(h: int, w: int, s: int, device) -> torch.Tensor:
    """Positions [h*w, 2] (x, y) of the low-resolution pixels in the
    full-resolution grid: the centre of each s x s footprint,
    ((j + 1/2) s - 1/2, (i + 1/2) s - 1/2), row-major."""
    ys = (torch.arange(h, dtype=torch.float32, device=device) + 0.5) * s - 0.5
    xs = (torch.arange(w, dtype=torch.float32, device=device) + 0.5) * s - 0.5
    gy, gx = torch.meshgrid(ys, xs, indexing="ij")
    return torch.stack([gx.reshape(-1), gy.reshape(-1)], dim=1).contiguous()


def gmm_points(low: torch.Tensor, s: int):
    """The known points of a low-resolution batch [B, C, h, w]: positions
    [B, h*w, 2] and values [B, h*w, C]."""
    B, C, h, w = low.shape
    pos = grid_points(h, w, s, low.device)[None].expand(B, -1, -1).contiguous()
    val = low.permute(0, 2, 3, 1).reshape(B, h * w, C).contiguous()
    return pos, val


def gmm_upsample(low: torch.Tensor, s: int, sigma_factor: float = 0.5,
                 radius: float = 3.0) -> torch.Tensor:
    """Gaussian-mixture upsampling of [B, C, h, w] by s: shared sigma =
    sigma_factor * s for every image."""
    B = low.shape[0]
    pos, val = gmm_points(low, s)
    sig = torch.full((B,), sigma_factor * s, dtype=torch.float32, device=low.device)
    return interp.interpolate(pos, sig, val, low.shape[2] * s, low.shape[3] * s, radius)


def torch_upsample(low: torch.Tensor, s: int, mode: str) -> torch.Tensor:
    if mode == "nearest":
        return F.interpolate(low, scale_factor=s, mode="nearest")
    return F.interpolate(low, scale_factor=s, mode=mode, align_corners=False).clamp(0.0, 1.0)


def l1(a: torch.Tensor, b: torch.Tensor) -> float:
    return float((a - b).abs().mean())


def study(size: int = 512, n_images: int = 8, C: int = 3, factors: Sequence[int] = (2, 3, 4, 6, 8),
          sigma_factors: Sequence[float] = (0.2, 0.25, 0.3, 0.35, 0.4, 0.5, 0.7, 1.0),
          seed: int = 11,
          device: str = "cuda") -> Dict:
    """L1 of the reconstruction per factor: Gaussian mixture at each sigma
    factor (and the best of them) against nearest, bilinear and bicubic."""
    imgs = torch.from_numpy(np.stack([synth.natural_image(seed + i, C, size, size)
                                      for i in range(n_images)])).to(device)
    res = {"size": size, "images": n_images, "C": C, "factors": {}}
    for s in factors:
        hs = (size // s) * s
        full = imgs[:, :, :hs, :hs].contiguous()
        low = downsample(full, s)
        row = {m: l1(torch_upsample(low, s, m), full) for m in ("nearest", "bilinear", "bicubic")}
        gm = {}
        for a in sigma_factors:
            gm[f"{a:g}"] = l1(gmm_upsample(low, s, a), full)
        row["gmm"] = gm
        best = min(gm, key=gm.get)
        row["gmm_best"] = gm[best]
        row["gmm_best_sigma_factor"] = float(best)
        res["factors"][str(s)] = row
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--images", type=int, default=8)
    a = ap.parse_args()
    print(json.dumps(study(a.size, a.images)), flush=True)


if __name__ == "__main__":
    main()
