"""Seeded synthetic workloads for Gaussian-mixture interpolation.

This module only draws random inputs (point positions, per-point sigma,
point values, upstream gradients, request traces).  It contains none of the
interpolation arithmetic, so both the GPU path and the CPU oracle can take
their inputs from here without sharing any of the method's code.

Coordinates follow the convention used throughout the package: a point is
``(x, y)`` in pixel units with ``x`` the column and ``y`` the row, and output
pixel ``(row v, col u)`` sits at ``(x=u, y=v)``.

Named workloads (seed = 1000 + index):

1. one 64x64 image, N=4096 uniform points, C=3 U[0,1] values, shared sigma 0.5
2. 16 images of 256x256, N=65536 jittered-grid points each, smooth RGB field,
   shared sigma 0.7
3. one 1024x1024 image, N=2**20 points (70% in 8 Gaussian blobs, 30% uniform),
   C=3 U[0,1], per-point sigma log-uniform in [0.5, 2]
4. a serving trace of requests of mixed size / channel count
5. 2 images of 4096x4096, N=2**22 points each (50% in 32 blobs), C=16 N(0,1),
   per-point sigma log-uniform in [0.5, 3]

All use truncation radius 3 sigma.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "Workload", "uniform_points", "blob_points", "random_workload",
    "config1", "config2", "config3", "config3_anisotropic", "config4_trace", "config5",
    "ServingRequest", "CONFIGS", "natural_image", "sample_image_points",
]


@dataclasses.dataclass
class Workload:
    """One batch of interpolation problems sharing H, W, C and radius."""
    name: str
    pos: np.ndarray            # [B, N, 2] float32, (x=col, y=row)
    sigma: np.ndarray          # [B, N] (per point) or [B] (shared) float32
    values: np.ndarray         # [B, N, C] float32
    H: int
    W: int
    radius: float
    grad_seed: int = 0         # seed of the upstream gradient stream

    @property
    def B(self) -> int:
        return int(self.pos.shape[0])

    @property
    def N(self) -> int:
        return int(self.pos.shape[1])

    @property
    def C(self) -> int:
        return int(self.values.shape[2])

    @property
    def sigma_per_point(self) -> bool:
        return self.sigma.ndim == 2

    def grad_out(self) -> np.ndarray:
        """Upstream gradient dL/dout, [B, C, H, W] float32 drawn from N(0, 1)."""
        rng = np.random.default_rng(self.grad_seed)
        return rng.standard_normal((self.B, self.C, self.H, self.W), dtype=np.float32)


def uniform_points(rng: np.random.Generator, n: int, H: int, W: int) -> np.ndarray:
    """n points uniform in [0, W) x [0, H), float32 [n, 2]."""
    out = np.empty((n, 2), dtype=np.float32)
    out[:, 0] = rng.random(n, dtype=np.float32) * np.float32(W)
    out[:, 1] = rng.random(n, dtype=np.float32) * np.float32(H)
    # rounding of u*W can land exactly on W; keep the half-open interval
    np.minimum(out[:, 0], np.nextafter(np.float32(W), np.float32(0)), out=out[:, 0])
    np.minimum(out[:, 1], np.nextafter(np.float32(H), np.float32(0)), out=out[:, 1])
    return out


def blob_points(rng: np.random.Generator, n: int, H: int, W: int, n_blobs: int,
                std_lo: float, std_hi: float) -> np.ndarray:
    """n points from n_blobs isotropic Gaussian blobs with equal shares.

    Blob centres are uniform in the image, blob std is U[std_lo, std_hi].
    Draws that fall outside [0, W) x [0, H) are rejected and redrawn.
    """
    centres = np.stack([rng.random(n_blobs) * W, rng.random(n_blobs) * H], axis=1)
    stds = rng.uniform(std_lo, std_hi, size=n_blobs)
    shares = np.full(n_blobs, n // n_blobs, dtype=np.int64)
    shares[: n % n_blobs] += 1
    parts = []
    for b in range(n_blobs):
        need = int(shares[b])
        got: List[np.ndarray] = []
        while need > 0:
            draw = centres[b] + stds[b] * rng.standard_normal((max(need * 2, 64), 2))
            ok = (draw[:, 0] >= 0) & (draw[:, 0] < W) & (draw[:, 1] >= 0) & (draw[:, 1] < H)
            draw = draw[ok][:need]
            got.append(draw)
            need -= draw.shape[0]
        parts.append(np.concatenate(got, axis=0))
    pts = np.concatenate(parts, axis=0).astype(np.float32)
    # float32 rounding may push a value onto the upper edge
    np.minimum(pts[:, 0], np.nextafter(np.float32(W), np.float32(0)), out=pts[:, 0])
    np.minimum(pts[:, 1], np.nextafter(np.float32(H), np.float32(0)), out=pts[:, 1])
    return pts


def _log_uniform(rng: np.random.Generator, size, lo: float, hi: float) -> np.ndarray:
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=size)).astype(np.float32)


def random_workload(seed: int, B: int, N: int, H: int, W: int, C: int = 3,
                    sigma=(0.5, 2.0), per_point: bool = True, radius: float = 3.0,
                    blob_frac: float = 0.0, n_blobs: int = 8, blob_std=(4.0, 12.0),
                    values: str = "uniform", name: str = "random") -> Workload:
    """General seeded workload used by the parity tests.

    sigma: (lo, hi) log-uniform range for per-point sigma, or a float for a
    shared sigma (then per_point is ignored and sigma has shape [B]).
    values: "uniform" (U[0,1]) or "normal" (N(0,1)).
    """
    rng = np.random.default_rng(seed)
    pos = np.empty((B, N, 2), dtype=np.float32)
    n_blob = int(round(N * blob_frac))
    for b in range(B):
        parts = []
        if n_blob:
            parts.append(blob_points(rng, n_blob, H, W, n_blobs, *blob_std))
        parts.append(uniform_points(rng, N - n_blob, H, W))
        p = np.concatenate(parts, axis=0)
        pos[b] = p[rng.permutation(N)] if N else p
    if isinstance(sigma, (int, float)):
        sig = np.full((B,), sigma, dtype=np.float32)
    elif per_point:
        sig = _log_uniform(rng, (B, N), *sigma)
    else:
        sig = _log_uniform(rng, (B,), *sigma)
    if values == "uniform":
        val = rng.random((B, N, C), dtype=np.float32)
    elif values == "normal":
        val = rng.standard_normal((B, N, C), dtype=np.float32)
    else:
        raise ValueError(values)
    return Workload(name, pos, sig, val, H, W, float(radius), grad_seed=seed + 7919)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def config1(seed: int = 1001) -> Workload:
    """64x64, N=4096 uniform points, C=3 U[0,1], shared sigma 0.5, r=3."""
    rng = np.random.default_rng(seed)
    pos = uniform_points(rng, 4096, 64, 64)[None]
    val = rng.random((1, 4096, 3), dtype=np.float32)
    return Workload("cfg1_64x64_n4096", pos, np.array([0.5], np.float32), val, 64, 64, 3.0,
                    grad_seed=seed + 7919)


def _smooth_field(rng: np.random.Generator, pts: np.ndarray, C: int, size: int) -> np.ndarray:
    """0.5 + sum of 8 random sinusoids per channel, plus U(-0.05, 0.05) noise."""
    out = np.empty((pts.shape[0], C), dtype=np.float32)
    p = pts.astype(np.float64)
    for c in range(C):
        acc = np.full(pts.shape[0], 0.5)
        for _ in range(8):
            a = rng.uniform(0.0, 0.06)
            f = rng.uniform(-4.0, 4.0, size=2)
            ph = rng.uniform(0.0, 2 * math.pi)
            acc += a * np.sin(2 * math.pi * (p @ f) / size + ph)
        acc += rng.uniform(-0.05, 0.05, size=pts.shape[0])
        out[:, c] = acc
    return out


def config2(seed: int = 1002, B: int = 16) -> Workload:
    """16 x 256x256, jittered grid (N(0,0.3^2) offsets, clamped to [0,255]), sigma 0.7."""
    rng = np.random.default_rng(seed)
    size = 256
    vv, uu = np.meshgrid(np.arange(size), np.arange(size), indexing="ij")
    nodes = np.stack([uu.ravel(), vv.ravel()], axis=1).astype(np.float64)
    pos = np.empty((B, size * size, 2), dtype=np.float32)
    val = np.empty((B, size * size, 3), dtype=np.float32)
    for b in range(B):
        p = np.clip(nodes + 0.3 * rng.standard_normal(nodes.shape), 0.0, size - 1.0)
        pos[b] = p.astype(np.float32)
        val[b] = _smooth_field(rng, pos[b], 3, size)
    sig = np.full((B,), 0.7, dtype=np.float32)
    return Workload("cfg2_16x256x256_n65536", pos, sig, val, size, size, 3.0, grad_seed=seed + 7919)


def config3(seed: int = 1003) -> Workload:
    """1024x1024, N=2**20 (70% in 8 blobs std U[40,120], 30% uniform), C=3,
    per-point sigma log-uniform [0.5, 2], r=3."""
    rng = np.random.default_rng(seed)
    N, H, W = 1 << 20, 1024, 1024
    n_blob = int(round(0.7 * N))
    p = np.concatenate([blob_points(rng, n_blob, H, W, 8, 40.0, 120.0),
                        uniform_points(rng, N - n_blob, H, W)], axis=0)
    pos = p[rng.permutation(N)][None]
    val = rng.random((1, N, 3), dtype=np.float32)
    sig = _log_uniform(rng, (1, N), 0.5, 2.0)
    return Workload("cfg3_1024x1024_n1M_c3", pos, sig, val, H, W, 3.0, grad_seed=seed + 7919)


def config3_anisotropic(seed: int = 1003) -> Workload:
    """The 1024x1024, N=2**20 workload with a diagonal covariance per point:
    (sigma_x, sigma_y) drawn independently log-uniform in [0.5, 2]."""
    wl = config3(seed)
    rng = np.random.default_rng(seed + 17)
    sig = _log_uniform(rng, (1, wl.N, 2), 0.5, 2.0)
    return Workload("cfg3_aniso_1024x1024_n1M_c3", wl.pos, sig, wl.values, wl.H, wl.W, 3.0,
                    grad_seed=wl.grad_seed)


def config5(seed: int = 1005, B: int = 2, size: int = 4096, N: int = 1 << 22) -> Workload:
    """2 x 4096x4096, N=2**22 per image (50% in 32 blobs std U[40,120]), C=16 N(0,1),
    per-point sigma log-uniform [0.5, 3], r=3."""
    rng = np.random.default_rng(seed)
    pos = np.empty((B, N, 2), dtype=np.float32)
    n_blob = N // 2
    for b in range(B):
        p = np.concatenate([blob_points(rng, n_blob, size, size, 32, 40.0, 120.0),
                            uniform_points(rng, N - n_blob, size, size)], axis=0)
        pos[b] = p[rng.permutation(N)]
    val = rng.standard_normal((B, N, 16), dtype=np.float32)
    sig = _log_uniform(rng, (B, N), 0.5, 3.0)
    return Workload(f"cfg5_{B}x{size}x{size}_n{N}_c16", pos, sig, val, size, size, 3.0,
                    grad_seed=seed + 7919)


@dataclasses.dataclass
class ServingRequest:
    """One request of the serving trace (B=1)."""
    index: int
    arrival_s: float           # scheduled arrival, seconds from trace start
    side: int                  # H = W = side
    N: int
    C: int
    sigma: float               # one shared sigma for the request
    backward: bool
    seed: int

    def workload(self) -> Workload:
        rng = np.random.default_rng(self.seed)
        pos = uniform_points(rng, self.N, self.side, self.side)[None]
        val = rng.random((1, self.N, self.C), dtype=np.float32)
        return Workload(f"req{self.index}", pos, np.array([self.sigma], np.float32), val,
                        self.side, self.side, 3.0, grad_seed=self.seed + 7919)


def config4_trace(n_requests: int = 4096, rate_per_s: Optional[float] = None,
                  seed: int = 1004, sides=(64, 128, 256, 512, 1024)) -> List[ServingRequest]:
    """Serving trace: side from `sides`, N = round(side^2 * U(0.25, 1)), C in {1,3,4},
    shared sigma U(0.5, 1.5), 30% ask for backward.  Arrivals are Poisson with the
    given rate; rate None puts every arrival at t=0 (saturated)."""
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    for i in range(n_requests):
        side = int(rng.choice(sides))
        n = int(round(side * side * rng.uniform(0.25, 1.0)))
        c = int(rng.choice([1, 3, 4]))
        s = float(np.float32(rng.uniform(0.5, 1.5)))
        bwd = bool(rng.random() < 0.3)
        if rate_per_s:
            t += float(rng.exponential(1.0 / rate_per_s))
        reqs.append(ServingRequest(i, t, side, n, c, s, bwd, seed * 100003 + i))
    return reqs


# --------------------------------------------------------------------------
# Synthetic images (targets of the point optimisation and of the
# downsample / upsample study)
# --------------------------------------------------------------------------

def natural_image(seed: int, C: int, H: int, W: int, n_shapes: int = 12) -> np.ndarray:
    """A [C, H, W] float32 image in [0, 1] with natural-image statistics: a
    1/f-amplitude random-phase field (smooth shading and texture at every
    scale) plus n_shapes flat-coloured rectangles and discs with sharp edges
    (walls, furniture, objects), lit by a smooth gradient."""
    rng = np.random.default_rng(seed)
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.rfftfreq(W)[None, :]
    f = np.sqrt(fx * fx + fy * fy)
    f[0, 0] = 1.0
    img = np.empty((C, H, W), dtype=np.float64)
    base = rng.uniform(0.2, 0.8, size=C)
    for c in range(C):
        spec = (rng.standard_normal(f.shape) + 1j * rng.standard_normal(f.shape)) / f
        spec[0, 0] = 0.0
        field = np.fft.irfft2(spec, s=(H, W))
        field *= 0.12 / max(field.std(), 1e-12)
        img[c] = base[c] + field
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    for _ in range(n_shapes):
        col = rng.uniform(0.0, 1.0, size=C)
        if rng.random() < 0.5:
            x0, x1 = np.sort(rng.uniform(0, W, 2))
            y0, y1 = np.sort(rng.uniform(0, H, 2))
            m = (xx >= x0) & (xx < x1) & (yy >= y0) & (yy < y1)
        else:
            cx, cy = rng.uniform(0, W), rng.uniform(0, H)
            rad = rng.uniform(0.03, 0.2) * min(H, W)
            m = (xx - cx) ** 2 + (yy - cy) ** 2 <= rad * rad
        tex = img[:, m] - base[:, None]
        img[:, m] = col[:, None] + 0.5 * tex
    g = rng.uniform(-1, 1, size=2)
    light = 0.85 + 0.15 * (g[0] * (xx / W - 0.5) + g[1] * (yy / H - 0.5))
    img *= light[None]
    return np.clip(img, 0.0, 1.0).astype(np.float32)


def sample_image_points(rng: np.random.Generator, img: np.ndarray, n: int):
    """n points uniform over [0, W-1] x [0, H-1] carrying the image's value at
    the nearest pixel: (pos [n, 2] float32 (x, y), values [n, C] float32)."""
    C, H, W = img.shape
    pos = np.empty((n, 2), dtype=np.float32)
    pos[:, 0] = (rng.random(n) * (W - 1)).astype(np.float32)
    pos[:, 1] = (rng.random(n) * (H - 1)).astype(np.float32)
    iu = np.rint(pos[:, 0]).astype(np.int64)
    iv = np.rint(pos[:, 1]).astype(np.int64)
    return pos, np.ascontiguousarray(img[:, iv, iu].T)


CONFIGS = {1: config1, 2: config2, 3: config3, 5: config5}
