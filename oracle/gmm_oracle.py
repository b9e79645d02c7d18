"""CPU oracle for Gaussian-mixture interpolation (TEST INFRASTRUCTURE ONLY).

This file is the plain, slow, brute-force definition of what the GPU path
computes.  It is test infrastructure: only the test-suite, the package's
smoke check and the benchmark's CPU-baseline leg may import it.  The product
path never calls it, and it shares no code with the HIP kernels.

Method (paper, Section 2 "Method", Eq. 1 and Eq. 2): every known point j is an
isotropic 2-D Gaussian centred at its position p_j carrying a value c_j.  The
value at a query location q is the posterior mean of c, i.e. the weighted mean
of the c_j with the Gaussian densities at q as weights, normalised by their
sum Z_q (Eq. 2).  Only points close enough to q take part (the sentence after
Eq. 2), and every channel is interpolated on its own (end of Section 2).

Readings of the paper used here (each also listed in the design notes):

* Weights are the unnormalised kernel w = exp(-|q - p_j|^2 / (2 sigma_j^2)).
  With the paper's single shared sigma this is identical to Eq. 1, because the
  density's 1/(2 pi sigma^2) factor cancels between numerator and Z_q; the
  per-point sigma_j generalises the paper's fixed sigma.
* "Close enough" is the disk of radius r * sigma_j, inclusive, decided in
  float32 without fused multiply-add:
      dx = f32(f32(u) - x), dy = f32(f32(v) - y),
      d2 = f32(f32(dx*dx) + f32(dy*dy)), rs = f32(r*sigma), R2 = f32(rs*rs),
      include  iff  d2 <= R2.
  The predicate is evaluated on the float32 values of the inputs (the GPU
  receives float32); everything after that decision is float64, on the inputs
  as given (float64 inputs are used by the finite-difference checks).
  radius=None means no truncation.
* Output pixel (row v, column u) sits at (x=u, y=v).  Output layout [B,C,H,W].
* A pixel with no point inside the radius (Z = 0) outputs 0 and receives and
  passes on no gradient.
* The gradient at the truncation boundary is the almost-everywhere one: the
  indicator's jump is not differentiated.

Gradients (derived from Eq. 1 by the quotient rule; the paper states the
backward exists but does not write it out), with G = dL/d out,
alpha_i = 1/Z_i and beta_i = alpha_i * sum_k G_ik o_ik:

    dL/dc_jk     = sum_i w_ij alpha_i G_ik
    A_ij         = alpha_i sum_k G_ik c_jk - beta_i
    dL/dx_j      = sum_i A_ij w_ij (u_i - x_j) / sigma_j^2
    dL/dy_j      = sum_i A_ij w_ij (v_i - y_j) / sigma_j^2
    dL/dsigma_j  = sum_i A_ij w_ij d2_ij / sigma_j^3

Parity is pinned by closed forms and invariants in the test-suite (two-point
sigmoid, single point, grid-node reproduction, separable normalised
convolution, tail bound, finite differences, partition of unity).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, Optional, Sequence

import numpy as np

__all__ = [
    "predicate", "weights", "forward_pixels", "forward", "backward_points", "backward",
    "bins", "pair_count", "reach", "halo_bins",
]


# --------------------------------------------------------------------------
# The truncation predicate and the weights
# --------------------------------------------------------------------------

def predicate(u, v, x, y, sigma, radius: Optional[float]):
    """Is point (x, y, sigma) close enough to pixel (u, v)?  float32, no FMA.

    u, v, x, y, sigma broadcast against each other.  radius None: always True.
    numpy evaluates every float32 operation below separately with
    round-to-nearest-even, which is the specified operation sequence.
    """
    x = np.asarray(x, dtype=np.float32)
    y = np.asarray(y, dtype=np.float32)
    sigma = np.asarray(sigma, dtype=np.float32)
    uf = np.asarray(u, dtype=np.float32)
    vf = np.asarray(v, dtype=np.float32)
    if radius is None:
        return np.ones(np.broadcast_shapes(uf.shape, vf.shape, x.shape, y.shape, sigma.shape),
                       dtype=bool)
    dx = (uf - x).astype(np.float32)
    dy = (vf - y).astype(np.float32)
    dxx = (dx * dx).astype(np.float32)
    dyy = (dy * dy).astype(np.float32)
    d2 = (dxx + dyy).astype(np.float32)
    rs = (np.float32(radius) * sigma).astype(np.float32)
    R2 = (rs * rs).astype(np.float32)
    return d2 <= R2


def weights(u, v, x, y, sigma):
    """Unnormalised Gaussian weight exp(-d^2 / (2 sigma^2)) in float64."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)
    d2 = (np.asarray(u, np.float64) - x) ** 2 + (np.asarray(v, np.float64) - y) ** 2
    return np.exp(-d2 / (2.0 * s * s))


def _sigma_of(sigma: np.ndarray, b: int, N: int) -> np.ndarray:
    """Per-point sigma of image b (a shared sigma is broadcast to all N)."""
    if sigma.ndim == 2:
        return sigma[b]
    return np.full(N, sigma[b], dtype=sigma.dtype)


# --------------------------------------------------------------------------
# Forward
# --------------------------------------------------------------------------

def _forward_block(args):
    pos_b, sig_b, val_b, us, vs, radius = args
    x = pos_b[:, 0]
    y = pos_b[:, 1]
    n_pix = us.shape[0]
    C = val_b.shape[1]
    out = np.zeros((n_pix, C))
    Z = np.zeros(n_pix)
    S = np.zeros((n_pix, C))
    P = 0
    absval = np.abs(val_b.astype(np.float64))
    val64 = val_b.astype(np.float64)
    for t in range(n_pix):
        inc = predicate(us[t], vs[t], x, y, sig_b, radius)
        idx = np.nonzero(inc)[0]
        P += idx.size
        if idx.size == 0:
            continue
        w = weights(us[t], vs[t], x[idx], y[idx], sig_b[idx])
        z = math.fsum(w)
        Z[t] = z
        for k in range(C):
            out[t, k] = math.fsum(w * val64[idx, k]) / z
            S[t, k] = math.fsum(w * absval[idx, k]) / z
    return out, Z, S, P


def _pool_map(fn, jobs, workers):
    # threads, not processes: the heavy work is large numpy array operations,
    # which release the GIL, and a thread pool is safe in a process that has
    # already initialised a GPU
    if workers <= 1 or len(jobs) <= 1:
        return [fn(j) for j in jobs]
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, jobs))


def default_workers() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:  # pragma: no cover
        return max(1, min(16, os.cpu_count() or 1))


def forward_pixels(pos, sigma, values, radius: Optional[float], b_idx, v_idx, u_idx,
                   workers: int = 1, block: int = 256) -> Dict[str, np.ndarray]:
    """Forward at an arbitrary list of pixels (b, row v, col u), brute force over all N.

    Returns out [n, C] (float64), Z [n], S [n, C] (the scale sum_j w|c_jk| / Z used
    by the tolerance) and P (number of included pixel-point pairs).
    """
    pos = np.asarray(pos)
    values = np.asarray(values)
    sigma = np.asarray(sigma)
    B, N, _ = pos.shape
    C = values.shape[2]
    b_idx = np.asarray(b_idx, np.int64)
    v_idx = np.asarray(v_idx, np.int64)
    u_idx = np.asarray(u_idx, np.int64)
    n = b_idx.shape[0]
    out = np.zeros((n, C))
    Z = np.zeros(n)
    S = np.zeros((n, C))
    P = 0
    jobs, slots = [], []
    for b in np.unique(b_idx):
        sel = np.nonzero(b_idx == b)[0]
        sig_b = _sigma_of(sigma, int(b), N)
        for s in range(0, sel.size, block):
            part = sel[s:s + block]
            jobs.append((pos[b], sig_b, values[b], u_idx[part], v_idx[part], radius))
            slots.append(part)
    for part, (o, z, sc, p) in zip(slots, _pool_map(_forward_block, jobs, workers)):
        out[part] = o
        Z[part] = z
        S[part] = sc
        P += p
    return {"out": out, "Z": Z, "S": S, "P": P}


def forward(pos, sigma, values, H: int, W: int, radius: Optional[float],
            workers: int = 1) -> Dict[str, np.ndarray]:
    """Full-image forward: out [B,C,H,W], Z [B,H,W], S [B,C,H,W], P."""
    pos = np.asarray(pos)
    B = pos.shape[0]
    C = np.asarray(values).shape[2]
    bb, vv, uu = np.meshgrid(np.arange(B), np.arange(H), np.arange(W), indexing="ij")
    r = forward_pixels(pos, sigma, values, radius, bb.ravel(), vv.ravel(), uu.ravel(),
                       workers=workers)
    return {
        "out": r["out"].reshape(B, H, W, C).transpose(0, 3, 1, 2).copy(),
        "Z": r["Z"].reshape(B, H, W),
        "S": r["S"].reshape(B, H, W, C).transpose(0, 3, 1, 2).copy(),
        "P": r["P"],
    }


def pair_count(pos, sigma, H: int, W: int, radius: float, b: int = 0) -> int:
    """Number of (pixel, point) pairs inside the radius for image b (all pixels)."""
    pos = np.asarray(pos, np.float32)
    N = pos.shape[1]
    sig_b = _sigma_of(np.asarray(sigma, np.float32), b, N)
    total = 0
    for v in range(H):
        uu = np.arange(W, dtype=np.float32)[:, None]
        total += int(predicate(uu, np.float32(v), pos[b, :, 0][None], pos[b, :, 1][None],
                               sig_b[None], radius).sum())
    return total


# --------------------------------------------------------------------------
# Backward
# --------------------------------------------------------------------------

def _backward_block(args):
    (pos_b, sig_b, val_b, G_b, H, W, radius, js, zmap, omap) = args
    C = val_b.shape[1]
    N = pos_b.shape[0]
    x_all = pos_b[:, 0]
    y_all = pos_b[:, 1]
    n = js.shape[0]
    gpos = np.zeros((n, 2))
    gsig = np.zeros(n)
    gval = np.zeros((n, C))
    spos = np.zeros((n, 2))
    ssig = np.zeros(n)
    sval = np.zeros((n, C))
    uu_all = np.arange(W)
    vv_all = np.arange(H)
    for t, j in enumerate(js):
        xj, yj, sj = pos_b[j, 0], pos_b[j, 1], sig_b[j]
        # every pixel of the image is tested against point j
        inc = predicate(uu_all[None, :], vv_all[:, None], xj, yj, sj, radius)
        vs, us = np.nonzero(inc)
        if vs.size == 0:
            continue
        # Z and o at those pixels: given (full-image oracle) or brute force here
        if zmap is not None:
            Zi = zmap[vs, us]
            oi = omap[:, vs, us].T
        else:
            Zi = np.zeros(vs.size)
            oi = np.zeros((vs.size, C))
            for q in range(vs.size):
                inc_q = predicate(us[q], vs[q], x_all, y_all, sig_b, radius)
                idx = np.nonzero(inc_q)[0]
                w = weights(us[q], vs[q], x_all[idx], y_all[idx], sig_b[idx])
                z = math.fsum(w)
                Zi[q] = z
                for k in range(C):
                    oi[q, k] = math.fsum(w * val_b[idx, k].astype(np.float64)) / z
        keep = Zi > 0
        vs, us, Zi, oi = vs[keep], us[keep], Zi[keep], oi[keep]
        Gi = G_b[:, vs, us].T.astype(np.float64)            # [m, C]
        w = weights(us, vs, xj, yj, sj)                      # [m]
        alpha = 1.0 / Zi
        beta = alpha * np.sum(Gi * oi, axis=1)
        cj = val_b[j].astype(np.float64)
        A = alpha * (Gi @ cj) - beta
        # |A| expanded into its elementary products: alpha sum_k |G c| + |G o|
        Aabs = alpha * (np.abs(Gi) @ np.abs(cj) + np.sum(np.abs(Gi * oi), axis=1))
        s64 = np.float64(sj)
        dxu = us - np.float64(xj)
        dyv = vs - np.float64(yj)
        d2 = dxu * dxu + dyv * dyv
        fx = w * dxu / (s64 * s64)
        fy = w * dyv / (s64 * s64)
        fs = w * d2 / (s64 ** 3)
        gpos[t, 0] = math.fsum(A * fx)
        gpos[t, 1] = math.fsum(A * fy)
        gsig[t] = math.fsum(A * fs)
        spos[t, 0] = math.fsum(Aabs * np.abs(fx))
        spos[t, 1] = math.fsum(Aabs * np.abs(fy))
        ssig[t] = math.fsum(Aabs * fs)
        for k in range(C):
            tc = w * alpha * Gi[:, k]
            gval[t, k] = math.fsum(tc)
            sval[t, k] = math.fsum(np.abs(tc))
    return gpos, gsig, gval, spos, ssig, sval


def backward_points(pos, sigma, values, G, H: int, W: int, radius: Optional[float],
                    b: int, points: Sequence[int], fwd: Optional[Dict] = None,
                    workers: int = 1, block: int = 16) -> Dict[str, np.ndarray]:
    """Per-point gradients of image b for the listed points.

    fwd: optional full-image forward result of this oracle (out, Z) to reuse;
    otherwise Z and o are recomputed brute force at every pixel in each
    point's support.  Returns grad_pos [n,2], grad_sigma [n] (the per-point
    derivative, also for a shared sigma), grad_values [n,C] and the matching
    scales used by the tolerance: the sum of the absolute values of the
    elementary products each gradient expands into (A_ij counted as
    alpha_i sum_k (|G_ik c_jk| + |G_ik o_ik|), so that a point whose A_ij
    cancels exactly still has the scale of the float32 terms that cancel).
    """
    pos = np.asarray(pos)
    values = np.asarray(values)
    sigma = np.asarray(sigma)
    G = np.asarray(G)
    N = pos.shape[1]
    sig_b = _sigma_of(sigma, b, N)
    pts = np.asarray(points, dtype=np.int64)
    zmap = omap = None
    if fwd is not None:
        zmap = fwd["Z"][b]
        omap = fwd["out"][b]
    jobs = []
    for s in range(0, pts.size, block):
        jobs.append((pos[b], sig_b, values[b], G[b], H, W, radius, pts[s:s + block], zmap, omap))
    parts = _pool_map(_backward_block, jobs, workers)
    cat = [np.concatenate([p[i] for p in parts], axis=0) if parts else None for i in range(6)]
    C = values.shape[2]
    if not parts:
        cat = [np.zeros((0, 2)), np.zeros(0), np.zeros((0, C)), np.zeros((0, 2)),
               np.zeros(0), np.zeros((0, C))]
    return {"grad_pos": cat[0], "grad_sigma": cat[1], "grad_values": cat[2],
            "scale_pos": cat[3], "scale_sigma": cat[4], "scale_values": cat[5]}


def backward(pos, sigma, values, G, H: int, W: int, radius: Optional[float],
             workers: int = 1) -> Dict[str, np.ndarray]:
    """Full backward of every image and point.

    grad_sigma is [B, N] for per-point sigma and [B] (the sum over the image's
    points) for a shared sigma.
    """
    pos = np.asarray(pos)
    sigma = np.asarray(sigma)
    B, N, _ = pos.shape
    C = np.asarray(values).shape[2]
    fwd = forward(pos, sigma, values, H, W, radius, workers=workers)
    gp = np.zeros((B, N, 2))
    gs = np.zeros((B, N))
    gv = np.zeros((B, N, C))
    sp = np.zeros((B, N, 2))
    ss = np.zeros((B, N))
    sv = np.zeros((B, N, C))
    for b in range(B):
        r = backward_points(pos, sigma, values, G, H, W, radius, b, np.arange(N), fwd=fwd,
                            workers=workers, block=max(1, min(256, N // max(1, workers) + 1)))
        gp[b], gs[b], gv[b] = r["grad_pos"], r["grad_sigma"], r["grad_values"]
        sp[b], ss[b], sv[b] = r["scale_pos"], r["scale_sigma"], r["scale_values"]
    if sigma.ndim == 1:
        gs_out = np.array([math.fsum(gs[b]) for b in range(B)])
        ss_out = np.array([math.fsum(ss[b]) for b in range(B)])
    else:
        gs_out, ss_out = gs, ss
    return {"grad_pos": gp, "grad_sigma": gs_out, "grad_values": gv,
            "scale_pos": sp, "scale_sigma": ss_out, "scale_values": sv, "fwd": fwd}


# --------------------------------------------------------------------------
# Spatial bins (the counting sort the GPU path uses to find near points)
# --------------------------------------------------------------------------

def reach(sigma, radius: float, N: int) -> np.ndarray:
    """Per-image largest truncation radius max_j f32(radius * sigma_j) (float32).

    sigma is [B, N] (per point) or [B] (shared).  An image without points has
    reach 0.  This is the distance beyond which no point of the image has
    weight (the truncation sentence after Eq. 2), so it bounds the bins a
    pixel must look at.
    """
    sigma = np.asarray(sigma, np.float32)
    B = sigma.shape[0]
    out = np.zeros(B, np.float32)
    for b in range(B):
        if N == 0:
            continue
        s = sigma[b] if sigma.ndim == 2 else sigma[b:b + 1]
        out[b] = np.max((np.float32(radius) * s).astype(np.float32))
    return out


def halo_bins(sigma, radius: float, N: int, tile: int) -> np.ndarray:
    """Bins of halo K per image: floor((reach + 2^-10) / tile) + 1.

    Every point with weight at a pixel lies in a bin at most K bins away (in x
    and in y) from the pixel's own bin: |x - u| <= reach, so the bin columns
    differ by at most ceil(reach / tile) <= K, with the 2^-10 margin covering
    the float32 rounding of the radius test.
    """
    r = reach(sigma, radius, N).astype(np.float64)
    return (np.floor((r + 2.0 ** -10) / tile) + 1).astype(np.int64)


def bins(pos, H: int, W: int, tile: int) -> Dict[str, np.ndarray]:
    """Bin of every point and the stable counting-sort order, per image.

    A point belongs to bin (bx, by) with bx = floor(x / tile) clamped to
    [0, ceil(W/tile) - 1] (by likewise from y) and bin id by * ceil(W/tile) + bx.
    count[b] is the number of points per bin, offset[b] its exclusive prefix sum
    with offset[nb] = N, and perm the stable order: sorted by bin id, ties by the
    original point index.
    """
    pos = np.asarray(pos, np.float32)
    B, N, _ = pos.shape
    nbx = -(-W // tile)
    nby = -(-H // tile)
    nb = nbx * nby
    bin_of = np.zeros((B, N), np.int32)
    count = np.zeros((B, nb), np.int32)
    offset = np.zeros((B, nb + 1), np.int32)
    perm = np.zeros((B, N), np.int32)
    for b in range(B):
        fx = np.floor(pos[b, :, 0].astype(np.float64) / tile)
        fy = np.floor(pos[b, :, 1].astype(np.float64) / tile)
        bx = np.clip(fx, 0, nbx - 1).astype(np.int64)
        by = np.clip(fy, 0, nby - 1).astype(np.int64)
        key = by * nbx + bx
        bin_of[b] = key
        count[b] = np.bincount(key, minlength=nb)
        offset[b, 1:] = np.cumsum(count[b])
        perm[b] = np.lexsort((np.arange(N), key))
    return {"bin_of": bin_of, "count": count, "offset": offset, "perm": perm,
            "nbx": nbx, "nby": nby}
