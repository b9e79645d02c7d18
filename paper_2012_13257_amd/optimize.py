"""Fitting the known points to an image by gradient descent (paper, Section 3,
"Optimizing the points locations").

The points' positions (and, as an extension, their sigmas) become learnable
parameters: the image is interpolated from the points (Eq. 1 and Eq. 2 with the
radius truncation), the L1 distance to the target image is the loss, and its
gradients flow back through the HIP backward kernels of InterpFunction.  The
paper samples the points uniformly over the image, keeps their values, moves
their positions and finds that the positions barely move while the choice of
sigma matters far more; `study()` repeats that experiment on a synthetic
target.

    python -m paper_2012_13257_amd.optimize [--size 512] [--points 65536]

Every interpolation runs in libgmminterp.so; torch supplies the tensors, the
loss and the optimiser.
"""
from __future__ import annotations

import argparse
import json
import math
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import interp, synth

__all__ = ["PointFit", "l1_loss", "study"]


def l1_loss(out: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """Mean absolute error over every pixel and channel."""
    return (out - target).abs().mean()


@dataclass
class PointFit:
    """Learnable point cloud rendered by Gaussian-mixture interpolation.

    pos [1, N, 2] (x = column, y = row) and values [1, N, C] are fixed inputs
    except where learned; sigma is either one shared value or one per point,
    parametrised by its logarithm so that it stays positive."""
    pos: torch.Tensor
    values: torch.Tensor
    log_sigma: torch.Tensor
    H: int
    W: int
    radius: float = 3.0
    learn_pos: bool = True
    learn_sigma: bool = False
    history: List[float] = field(default_factory=list)

    @staticmethod
    def from_image(target: torch.Tensor, n_points: int, sigma: float, seed: int = 0,
                   per_point_sigma: bool = False, learn_pos: bool = True,
                   learn_sigma: bool = False, radius: float = 3.0) -> "PointFit":
        """n_points uniform over the image of target [C, H, W], each carrying the
        value of its nearest pixel (the sampling the paper describes)."""
        C, H, W = target.shape
        rng = np.random.default_rng(seed)
        pos, val = synth.sample_image_points(rng, target.detach().cpu().numpy(), n_points)
        dev = target.device
        pos_t = torch.from_numpy(pos)[None].to(dev)
        val_t = torch.from_numpy(val)[None].to(dev)
        shape = (1, n_points) if per_point_sigma else (1,)
        ls = torch.full(shape, math.log(sigma), dtype=torch.float32, device=dev)
        pos_t.requires_grad_(learn_pos)
        ls.requires_grad_(learn_sigma)
        return PointFit(pos_t, val_t, ls, H, W, radius, learn_pos, learn_sigma)

    def params(self) -> List[torch.Tensor]:
        out = []
        if self.learn_pos:
            out.append(self.pos)
        if self.learn_sigma:
            out.append(self.log_sigma)
        return out

    def render(self) -> torch.Tensor:
        """The interpolated image [C, H, W]."""
        sigma = self.log_sigma.exp()
        return interp.interpolate(self.pos, sigma, self.values, self.H, self.W, self.radius)[0]

    def step(self, target: torch.Tensor, opt: Optional[torch.optim.Optimizer]) -> float:
        """One optimisation step: render, L1 loss, backward, update.  Returns
        the loss (as a 0-d tensor's value, which synchronises)."""
        if opt is not None:
            opt.zero_grad(set_to_none=True)
        loss = l1_loss(self.render(), target)
        if opt is not None:
            loss.backward()
            opt.step()
        v = float(loss.detach())
        self.history.append(v)
        return v

    def fit(self, target: torch.Tensor, steps: int, lr_pos: float = 0.05,
            lr_sigma: float = 0.02) -> List[float]:
        """Adam on the learnable parameters for `steps` steps; returns the loss
        history (the loss of the state before each update, then the final one)."""
        groups = []
        if self.learn_pos:
            groups.append({"params": [self.pos], "lr": lr_pos})
        if self.learn_sigma:
            groups.append({"params": [self.log_sigma], "lr": lr_sigma})
        opt = torch.optim.Adam(groups) if groups else None
        for _ in range(steps):
            self.step(target, opt)
        with torch.no_grad():
            self.history.append(float(l1_loss(self.render(), target)))
        return self.history


def study(size: int = 512, n_points: int = 1 << 16, C: int = 3, steps: int = 200,
          sigmas=(0.35, 0.5, 0.7, 1.0, 1.4, 2.0, 2.8, 4.0), seed: int = 7,
          device: str = "cuda") -> dict:
    """The paper's experiment on a synthetic target: (1) the L1 error of the
    interpolation for a sweep of shared sigmas with the sampled positions;
    (2) Adam on the positions at a fixed sigma (the paper's setting), from the
    sweep's worst and best sigma; (3) Adam on per-point sigmas (and positions).
    Reports the errors and how far the points moved."""
    target = torch.from_numpy(synth.natural_image(seed, C, size, size)).to(device)
    res = {"size": size, "points": n_points, "C": C, "steps": steps, "sweep": {}}
    for s in sigmas:
        fit = PointFit.from_image(target, n_points, s, seed=seed, learn_pos=False)
        with torch.no_grad():
            res["sweep"][f"{s:g}"] = float(l1_loss(fit.render(), target))
    best = min(res["sweep"], key=res["sweep"].get)
    worst = max(res["sweep"], key=res["sweep"].get)
    runs = {}
    for tag, s, pp, lp, lsg in (("pos@worst_sigma", float(worst), False, True, False),
                               ("pos@best_sigma", float(best), False, True, False),
                               ("sigma_per_point@best", float(best), True, False, True),
                               ("pos+sigma_per_point@best", float(best), True, True, True)):
        fit = PointFit.from_image(target, n_points, s, seed=seed, per_point_sigma=pp,
                                  learn_pos=lp, learn_sigma=lsg)
        p0 = fit.pos.detach().clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = fit.fit(target, steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        disp = (fit.pos.detach() - p0).norm(dim=-1)
        sg = fit.log_sigma.detach().exp()
        runs[tag] = {"sigma0": s, "l1_start": hist[0], "l1_end": hist[-1],
                     "mean_disp_px": float(disp.mean()), "p99_disp_px": float(disp.quantile(0.99))
                     if disp.numel() <= 1 << 24 else None,
                     "sigma_mean_end": float(sg.mean()), "ms_per_step": 1e3 * dt / steps}
    res["best_sigma"] = float(best)
    res["worst_sigma"] = float(worst)
    res["runs"] = runs
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--points", type=int, default=1 << 16)
    ap.add_argument("--steps", type=int, default=200)
    a = ap.parse_args()
    print(json.dumps(study(a.size, a.points, steps=a.steps)), flush=True)


if __name__ == "__main__":
    main()
