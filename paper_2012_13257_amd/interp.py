"""PyTorch binding of the HIP Gaussian-mixture interpolation.

    out = interpolate(pos, sigma, values, H, W, radius=3.0)

pos [B,N,2] (x = column, y = row), sigma [B,N] (per point) or [B] (shared),
values [B,N,C]; all float32, contiguous, on the ROCm device.  out is
[B,C,H,W].  The operation is Eq. 1-2 of the paper with a radius*sigma
truncation; gradients flow to pos, sigma and values through the hand-written
backward kernels.  Every step runs in libgmminterp.so on the current torch
stream; torch only provides memory and the stream.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import torch

from . import _lib

__all__ = ["interpolate", "InterpFunction", "forward", "forward_noalloc", "backward", "debug_bins",
           "problem", "aligned_buffer"]

DEFAULT_TILE = 8

# storage type of values, out, grad_out and grad_values, from values' dtype
_STORAGE = {torch.float32: _lib.STORAGE_F32, torch.bfloat16: _lib.STORAGE_BF16,
            torch.float16: _lib.STORAGE_F16}


def problem(pos: torch.Tensor, sigma: torch.Tensor, values: torch.Tensor, H: int, W: int,
            radius: float = 3.0, tile: int = DEFAULT_TILE, normalized: bool = False,
            anisotropic: bool = False) -> _lib.InterpProblem:
    """The C-ABI problem descriptor of these tensors.  normalized keeps the
    density factor in each weight; anisotropic takes a diagonal covariance,
    sigma then holding (sigma_x, sigma_y) pairs: [B, N, 2] or [B, 2].  The
    dtype of values (float32, bfloat16 or float16) is the storage type of
    values, out, grad_out and grad_values; sums are float32 throughout."""
    if pos.dim() != 3 or pos.shape[2] != 2:
        raise ValueError("pos must be [B, N, 2]")
    B, N = int(pos.shape[0]), int(pos.shape[1])
    if values.dim() != 3 or values.shape[0] != B or values.shape[1] != N:
        raise ValueError("values must be [B, N, C]")
    k = 2 if anisotropic else 1
    tail = (2,) if anisotropic else ()
    if tuple(sigma.shape) == (B, N) + tail:
        per_point = 1
    elif tuple(sigma.shape) == (B,) + tail:
        per_point = 0
    else:
        raise ValueError("sigma must be [B, N] or [B]" if k == 1 else
                         "anisotropic sigma must be [B, N, 2] or [B, 2]")
    for name, t in (("pos", pos), ("sigma", sigma), ("values", values)):
        if name != "values" and t.dtype != torch.float32:
            raise ValueError(f"{name} must be float32")
        if not t.is_cuda:
            raise ValueError(f"{name} must be on the ROCm device")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    if values.dtype not in _STORAGE:
        raise ValueError("values must be float32, bfloat16 or float16")
    kernel = (_lib.KERNEL_NORMALIZED if normalized else 0) | (_lib.KERNEL_DIAGONAL if anisotropic else 0)
    return _lib.InterpProblem(B, N, int(values.shape[2]), int(H), int(W), float(radius), int(tile),
                              per_point, kernel, _STORAGE[values.dtype])


def aligned_buffer(nbytes: int, device) -> Tuple[torch.Tensor, int]:
    """A byte tensor holding a 256-byte aligned region of nbytes; returns (tensor, address)."""
    buf = torch.empty(max(1, nbytes) + 256, dtype=torch.uint8, device=device)
    addr = (buf.data_ptr() + 255) // 256 * 256
    return buf, addr


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Saved:
    """State kept from the forward for the backward (device buffer)."""

    def __init__(self, prob: _lib.InterpProblem, device):
        L = _lib.lib()
        self.prob = prob
        self.nbytes = L.interp_saved_bytes(ctypes.byref(prob))
        if self.nbytes == 0:
            raise ValueError(_lib.last_error())
        self.buf, self.addr = aligned_buffer(self.nbytes, device)


class Workspace:
    def __init__(self, prob: _lib.InterpProblem, device):
        L = _lib.lib()
        self.nbytes = L.interp_workspace_bytes(ctypes.byref(prob))
        if self.nbytes == 0:
            raise ValueError(_lib.last_error())
        self.buf, self.addr = aligned_buffer(self.nbytes, device)


def forward(pos, sigma, values, H, W, radius=3.0, tile=DEFAULT_TILE, normalized=False,
            anisotropic=False):
    """Runs interp_forward; returns (out, saved, workspace)."""
    prob = problem(pos, sigma, values, H, W, radius, tile, normalized, anisotropic)
    dev = pos.device
    out = torch.empty((prob.B, prob.C, prob.H, prob.W), dtype=values.dtype, device=dev)
    saved = Saved(prob, dev)
    work = Workspace(prob, dev)
    rc = _lib.lib().interp_forward(ctypes.byref(prob), _ptr(pos), _ptr(sigma), _ptr(values),
                                   _ptr(out), saved.addr, saved.nbytes, work.addr, work.nbytes,
                                   _stream(dev))
    _lib.check("interp_forward", rc)
    return out, saved, work


def forward_noalloc(pos, sigma, values, out, saved: Saved, H, W, radius=3.0, tile=DEFAULT_TILE,
                    normalized=False, anisotropic=False):
    """Runs interp_forward_noalloc into the caller's out [B,C,H,W] and saved
    state: the library allocates nothing and uses its static per-GPU scratch
    as the workspace.  Returns out."""
    prob = problem(pos, sigma, values, H, W, radius, tile, normalized, anisotropic)
    if (out.dtype != values.dtype or not out.is_cuda or not out.is_contiguous()
            or tuple(out.shape) != (prob.B, prob.C, prob.H, prob.W)):
        raise ValueError("out must be a contiguous [B, C, H, W] tensor of values' dtype on the device")
    rc = _lib.lib().interp_forward_noalloc(ctypes.byref(prob), _ptr(pos), _ptr(sigma),
                                           _ptr(values), _ptr(out), saved.addr, saved.nbytes,
                                           _stream(pos.device))
    _lib.check("interp_forward_noalloc", rc)
    return out


def backward(pos, sigma, values, out, saved: Saved, grad_out, need_pos=True, need_sigma=True,
             need_values=True, work: Optional[Workspace] = None):
    """Runs interp_backward; returns (grad_pos, grad_sigma, grad_values) (None where not needed)."""
    prob = saved.prob
    dev = pos.device
    if grad_out.dtype != values.dtype or not grad_out.is_cuda:
        raise ValueError("grad_out must have the dtype of values and be on the ROCm device")
    grad_out = grad_out.contiguous()
    if tuple(grad_out.shape) != (prob.B, prob.C, prob.H, prob.W):
        raise ValueError("grad_out must be [B, C, H, W]")
    gp = torch.empty_like(pos) if need_pos else None
    gs = torch.empty_like(sigma) if need_sigma else None
    gv = torch.empty_like(values) if need_values else None
    if work is None:
        work = Workspace(prob, dev)
    rc = _lib.lib().interp_backward(ctypes.byref(prob), _ptr(pos), _ptr(sigma), _ptr(values),
                                    _ptr(out), saved.addr, saved.nbytes, _ptr(grad_out), _ptr(gp),
                                    _ptr(gs), _ptr(gv), work.addr, work.nbytes, _stream(dev))
    _lib.check("interp_backward", rc)
    return gp, gs, gv


def debug_bins(saved: Saved, work: Workspace):
    """Binning state of a forward call: (bin_of [B,N], count [B,nb], offset [B,nb+1], perm [B,N])."""
    p = saved.prob
    T = p.tile or DEFAULT_TILE
    nb = ((p.W + T - 1) // T) * ((p.H + T - 1) // T)
    dev = saved.buf.device
    bin_of = torch.empty((p.B, p.N), dtype=torch.int32, device=dev)
    count = torch.empty((p.B, nb), dtype=torch.int32, device=dev)
    offset = torch.empty((p.B, nb + 1), dtype=torch.int32, device=dev)
    perm = torch.empty((p.B, p.N), dtype=torch.int32, device=dev)
    rc = _lib.lib().interp_debug_bins(ctypes.byref(p), saved.addr, saved.nbytes, work.addr,
                                      work.nbytes, _ptr(bin_of), _ptr(count), _ptr(offset),
                                      _ptr(perm), _stream(dev))
    _lib.check("interp_debug_bins", rc)
    return bin_of, count, offset, perm


class InterpFunction(torch.autograd.Function):
    """Differentiable Gaussian-mixture interpolation (forward and backward in HIP)."""

    @staticmethod
    def forward(ctx, pos, sigma, values, H, W, radius, tile, normalized=False, anisotropic=False):
        out, saved, work = forward(pos, sigma, values, H, W, radius, tile, normalized, anisotropic)
        ctx.saved_state = saved
        ctx.work = work  # the backward reuses the forward's workspace
        ctx.save_for_backward(pos, sigma, values, out)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        pos, sigma, values, out = ctx.saved_tensors
        need = ctx.needs_input_grad
        if not (need[0] or need[1] or need[2]):
            return (None,) * 9
        gp, gs, gv = backward(pos, sigma, values, out, ctx.saved_state, grad_out.to(values.dtype),
                              need_pos=need[0], need_sigma=need[1], need_values=need[2],
                              work=ctx.work)
        return (gp, gs, gv) + (None,) * 6


def interpolate(pos: torch.Tensor, sigma: torch.Tensor, values: torch.Tensor, H: int, W: int,
                radius: float = 3.0, tile: int = DEFAULT_TILE, normalized: bool = False,
                anisotropic: bool = False) -> torch.Tensor:
    """Gaussian-mixture interpolation of scattered points onto an H x W grid (Eq. 1-2).

    normalized: keep the normal density's factor in each weight (Eq. 1 with
    per-point sigmas); anisotropic: diagonal covariance, sigma = (sigma_x,
    sigma_y) pairs [B, N, 2] or [B, 2]."""
    return InterpFunction.apply(pos, sigma, values, int(H), int(W), float(radius), int(tile),
                                bool(normalized), bool(anisotropic))
