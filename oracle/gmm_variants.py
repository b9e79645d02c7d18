"""CPU oracle for the kernel variants of the Gaussian-mixture interpolation
(TEST INFRASTRUCTURE ONLY: only the test-suite may import it; it shares no
code with the HIP kernels).

Eq. 1 of the paper (Section 2) weights every known point by the Gaussian
density N(q | mu_j, sigma^2 I) at the query location q.  The main oracle
(gmm_oracle.py) uses the unnormalised isotropic kernel, which equals Eq. 1
whenever sigma is shared because the density's normalising factor cancels in
the ratio of Eq. 1 / Eq. 2.  This module covers the two adjacent variants the
paper's notation suggests:

* normalised: the weight carries the density's factor
  zeta_j = 1 / (2 pi sigma_j^2) (isotropic) or 1 / (2 pi sigma_xj sigma_yj)
  (diagonal), so points with different sigmas weigh as densities do;
* diagonal (anisotropic, axis-aligned) covariance diag(sigma_x^2, sigma_y^2)
  in place of sigma^2 I: the weight is exp(-m / 2) with the squared
  Mahalanobis distance m = dx^2 / sigma_x^2 + dy^2 / sigma_y^2.

Readings (also in the design notes):

* Truncation ("close enough", the sentence after Eq. 2) is r in the kernel's
  own metric: |d| <= r sigma_j (isotropic, the main oracle's float32 test) and
  sqrt(m) <= r (diagonal), decided in float32 without fused multiply-add as
      ix = f32(1 / sigma_x), iy = f32(1 / sigma_y),
      qx = f32(f32(u - x) * ix), qy = f32(f32(v - y) * iy),
      m2 = f32(f32(qx * qx) + f32(qy * qy)),   include iff m2 <= f32(r * r).
  The weight itself is float64 from the exact inputs.
* Gradients follow from Eq. 1 by the quotient rule and the chain rule through
  the weight (alpha_i = 1/Z_i, beta_i = alpha_i sum_k G_ik o_ik,
  A_ij = alpha_i sum_k G_ik c_jk - beta_i):
      dL/dc_jk   = sum_i w_ij alpha_i G_ik
      dL/dx_j    = sum_i A_ij w_ij dx / sigma_x^2   (y likewise with sigma_y)
      dL/dsigma  = sum_i A_ij w_ij (d^2 / sigma^3 - 2 / sigma)   (isotropic;
                   the -2/sigma term only when normalised)
      dL/dsigma_x = sum_i A_ij w_ij (dx^2 / sigma_x^3 - 1 / sigma_x)   (diagonal;
                   the -1/sigma_x term only when normalised; y likewise)
  with dx = u - x, dy = v - y.  The tolerance scale of a gradient is the sum
  of the absolute values of the elementary products it expands into: A_ij as
  alpha_i sum_k (|G_ik c_jk| + |G_ik o_ik|), and the two terms of a
  normalised sigma derivative separately.

sigma layouts: isotropic [B, N] or [B]; diagonal [B, N, 2] or [B, 2]
((sigma_x, sigma_y) per point or shared).  grad_sigma has sigma's layout
(shared: summed over the image's points).
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np

from .gmm_oracle import predicate as _iso_predicate

__all__ = ["KERNELS", "predicate_diag", "forward_variant", "backward_variant"]

KERNELS = ("iso", "iso_norm", "diag", "diag_norm")


def _flags(kernel: str):
    if kernel not in KERNELS:
        raise ValueError(f"kernel must be one of {KERNELS}")
    return kernel.startswith("diag"), kernel.endswith("_norm")


def predicate_diag(u, v, x, y, sx, sy, radius: Optional[float]):
    """Mahalanobis truncation of the diagonal kernel, float32, no FMA."""
    x = np.asarray(x, np.float32)
    y = np.asarray(y, np.float32)
    sx = np.asarray(sx, np.float32)
    sy = np.asarray(sy, np.float32)
    uf = np.asarray(u, np.float32)
    vf = np.asarray(v, np.float32)
    if radius is None:
        return np.ones(np.broadcast_shapes(uf.shape, vf.shape, x.shape, y.shape, sx.shape),
                       dtype=bool)
    ix = (np.float32(1.0) / sx).astype(np.float32)
    iy = (np.float32(1.0) / sy).astype(np.float32)
    qx = ((uf - x).astype(np.float32) * ix).astype(np.float32)
    qy = ((vf - y).astype(np.float32) * iy).astype(np.float32)
    m2 = ((qx * qx).astype(np.float32) + (qy * qy).astype(np.float32)).astype(np.float32)
    r2 = np.float32(np.float32(radius) * np.float32(radius))
    return m2 <= r2


def _point_sigmas(sigma: np.ndarray, b: int, N: int, diag: bool):
    """(sx, sy) of every point of image b, as given (float32 or float64)."""
    s = np.asarray(sigma)
    if diag:
        if s.ndim == 3:
            return s[b, :, 0], s[b, :, 1]
        return np.full(N, s[b, 0], s.dtype), np.full(N, s[b, 1], s.dtype)
    if s.ndim == 2:
        return s[b], s[b]
    return np.full(N, s[b], s.dtype), np.full(N, s[b], s.dtype)


def _pair_terms(u, v, x, y, sx, sy, radius, diag, norm):
    """Inclusion mask and float64 weights of pixel(s) (u, v) against points."""
    if diag:
        inc = predicate_diag(u, v, x, y, sx, sy, radius)
    else:
        inc = _iso_predicate(u, v, x, y, sx, radius)
    sx64 = np.asarray(sx, np.float64)
    sy64 = np.asarray(sy, np.float64)
    dx = np.asarray(u, np.float64) - np.asarray(x, np.float64)
    dy = np.asarray(v, np.float64) - np.asarray(y, np.float64)
    m = dx * dx / (sx64 * sx64) + dy * dy / (sy64 * sy64)
    w = np.exp(-0.5 * m)
    if norm:
        w = w / (2.0 * math.pi * sx64 * sy64)
    return inc, w, dx, dy


def forward_variant(pos, sigma, values, H: int, W: int, radius: Optional[float],
                    kernel: str) -> Dict[str, np.ndarray]:
    """Full-image forward of a kernel variant: out [B,C,H,W], Z [B,H,W],
    S [B,C,H,W] (sum_j w |c_jk| / Z, the tolerance scale)."""
    diag, norm = _flags(kernel)
    pos = np.asarray(pos)
    values = np.asarray(values)
    B, N, _ = pos.shape
    C = values.shape[2]
    out = np.zeros((B, C, H, W))
    Z = np.zeros((B, H, W))
    S = np.zeros((B, C, H, W))
    for b in range(B):
        sx, sy = _point_sigmas(sigma, b, N, diag)
        x, y = pos[b, :, 0], pos[b, :, 1]
        val = values[b].astype(np.float64)
        for v in range(H):
            for u in range(W):
                inc, w, _, _ = _pair_terms(u, v, x, y, sx, sy, radius, diag, norm)
                idx = np.nonzero(inc)[0]
                if idx.size == 0:
                    continue
                wi = w[idx]
                z = math.fsum(wi)
                Z[b, v, u] = z
                for k in range(C):
                    out[b, k, v, u] = math.fsum(wi * val[idx, k]) / z
                    S[b, k, v, u] = math.fsum(wi * np.abs(val[idx, k])) / z
    return {"out": out, "Z": Z, "S": S}


def backward_variant(pos, sigma, values, G, H: int, W: int, radius: Optional[float],
                     kernel: str) -> Dict[str, np.ndarray]:
    """Full backward of a kernel variant with upstream gradient G [B,C,H,W]:
    grad_pos [B,N,2], grad_sigma (sigma's layout), grad_values [B,N,C] and
    the matching tolerance scales."""
    diag, norm = _flags(kernel)
    pos = np.asarray(pos)
    values = np.asarray(values)
    sigma = np.asarray(sigma)
    G = np.asarray(G, np.float64)
    B, N, _ = pos.shape
    C = values.shape[2]
    fwd = forward_variant(pos, sigma, values, H, W, radius, kernel)
    gp = np.zeros((B, N, 2))
    sp = np.zeros((B, N, 2))
    gv = np.zeros((B, N, C))
    sv = np.zeros((B, N, C))
    gs = np.zeros((B, N, 2))   # d/dsigma_x, d/dsigma_y (isotropic: column 0)
    ss = np.zeros((B, N, 2))
    vv, uu = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    for b in range(B):
        sx_all, sy_all = _point_sigmas(sigma, b, N, diag)
        Zb = fwd["Z"][b]
        ob = fwd["out"][b]
        for j in range(N):
            xj, yj = pos[b, j, 0], pos[b, j, 1]
            sx, sy = sx_all[j], sy_all[j]
            inc, w, dx, dy = _pair_terms(uu, vv, xj, yj, sx, sy, radius, diag, norm)
            inc &= Zb > 0
            vs, us = np.nonzero(inc)
            if vs.size == 0:
                continue
            w = w[vs, us]
            dx = dx[vs, us]
            dy = dy[vs, us]
            alpha = 1.0 / Zb[vs, us]
            Gi = G[b][:, vs, us].T                          # [m, C]
            oi = ob[:, vs, us].T
            beta = alpha * np.sum(Gi * oi, axis=1)
            cj = values[b, j].astype(np.float64)
            A = alpha * (Gi @ cj) - beta
            Aabs = alpha * (np.abs(Gi) @ np.abs(cj) + np.sum(np.abs(Gi * oi), axis=1))
            sx64, sy64 = np.float64(sx), np.float64(sy)
            fx = w * dx / (sx64 * sx64)
            fy = w * dy / (sy64 * sy64)
            gp[b, j] = (math.fsum(A * fx), math.fsum(A * fy))
            sp[b, j] = (math.fsum(Aabs * np.abs(fx)), math.fsum(Aabs * np.abs(fy)))
            for k in range(C):
                tc = w * alpha * Gi[:, k]
                gv[b, j, k] = math.fsum(tc)
                sv[b, j, k] = math.fsum(np.abs(tc))
            if diag:
                parts = [(w * dx * dx / sx64 ** 3, w / sx64), (w * dy * dy / sy64 ** 3, w / sy64)]
            else:
                parts = [(w * (dx * dx + dy * dy) / sx64 ** 3, 2.0 * w / sx64)]
            for a, (f1, f2) in enumerate(parts):
                gs[b, j, a] = math.fsum(A * f1) - (math.fsum(A * f2) if norm else 0.0)
                ss[b, j, a] = math.fsum(Aabs * f1) + (math.fsum(Aabs * f2) if norm else 0.0)
    if diag:
        if sigma.ndim == 3:
            g_sig, s_sig = gs, ss
        else:
            g_sig = np.array([[math.fsum(gs[b, :, a]) for a in range(2)] for b in range(B)])
            s_sig = np.array([[math.fsum(ss[b, :, a]) for a in range(2)] for b in range(B)])
    else:
        if sigma.ndim == 2:
            g_sig, s_sig = gs[:, :, 0], ss[:, :, 0]
        else:
            g_sig = np.array([math.fsum(gs[b, :, 0]) for b in range(B)])
            s_sig = np.array([math.fsum(ss[b, :, 0]) for b in range(B)])
    return {"grad_pos": gp, "grad_sigma": g_sig, "grad_values": gv, "scale_pos": sp,
            "scale_sigma": s_sig, "scale_values": sv, "fwd": fwd}
