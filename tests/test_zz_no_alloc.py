"""interp_forward_noalloc (the forward on the library's static per-GPU scratch)
against interp_forward with a caller workspace, through the C ABI: two calls
in a row, the second on a smaller problem, each bit for bit equal to the
regular entry point (same kernels, same summation order), and a backward
from its saved state equal to the backward from the regular one."""
import ctypes

import numpy as np
import pytest

from paper_2012_13257_amd import synth
from gpu_helpers import say, to_dev

pytestmark = pytest.mark.gpu


def _both(wl, tile=8):
    import torch
    from paper_2012_13257_amd import _lib, interp
    L = _lib.lib()
    pos, sig, val = to_dev(wl)
    prob = interp.problem(pos, sig, val, wl.H, wl.W, wl.radius, tile)
    pb = ctypes.byref(prob)
    st = torch.cuda.current_stream().cuda_stream
    out_r = torch.full((wl.B, wl.C, wl.H, wl.W), float("nan"), device="cuda")
    out_n = torch.full_like(out_r, float("nan"))
    saved_r = interp.Saved(prob, pos.device)
    saved_n = interp.Saved(prob, pos.device)
    # the alignment padding between the saved arrays is never written: start
    # both buffers from the same bytes so that the comparison sees only data
    saved_r.buf.zero_()
    saved_n.buf.zero_()
    work = interp.Workspace(prob, pos.device)
    say("noalloc", wl.name, wl.B, wl.N, wl.C, wl.H, wl.W)
    _lib.check("interp_forward", L.interp_forward(
        pb, pos.data_ptr(), sig.data_ptr(), val.data_ptr(), out_r.data_ptr(), saved_r.addr,
        saved_r.nbytes, work.addr, work.nbytes, st))
    _lib.check("interp_forward_noalloc", L.interp_forward_noalloc(
        pb, pos.data_ptr(), sig.data_ptr(), val.data_ptr(), out_n.data_ptr(), saved_n.addr,
        saved_n.nbytes, st))
    torch.cuda.synchronize()
    assert torch.equal(out_r, out_n), "outputs differ"
    # the saved state (Z, reach, offsets, perm, sorted records) bit for bit
    n = saved_r.nbytes
    a = saved_r.buf[saved_r.addr - saved_r.buf.data_ptr():][:n]
    b = saved_n.buf[saved_n.addr - saved_n.buf.data_ptr():][:n]
    assert torch.equal(a, b), "saved states differ"
    # a backward from either saved state gives the same gradients
    G = torch.from_numpy(wl.grad_out()).cuda()
    g_r = interp.backward(pos, sig, val, out_r, saved_r, G, work=work)
    g_n = interp.backward(pos, sig, val, out_n, saved_n, G, work=work)
    torch.cuda.synchronize()
    for x, y in zip(g_r, g_n):
        assert torch.equal(x, y), "gradients differ"
    return out_n


def test_noalloc_matches_forward_two_calls_second_smaller():
    big = synth.random_workload(9101, 1, 120000, 500, 430, C=3, sigma=(0.5, 2.0),
                                blob_frac=0.6, blob_std=(10.0, 40.0))
    small = synth.random_workload(9102, 2, 3000, 70, 90, C=5, sigma=1.1, per_point=False,
                                  values="normal")
    _both(big)
    _both(small)


def test_noalloc_rejects_a_problem_beyond_the_scratch():
    import torch
    from paper_2012_13257_amd import _lib
    L = _lib.lib()
    # 2^22 points: the radix buffers alone exceed 64 MiB
    prob = _lib.InterpProblem(1, 1 << 22, 3, 2048, 2048, 3.0, 8, 1)
    need = L.interp_workspace_bytes(ctypes.byref(prob))
    assert need > _lib.NOALLOC_SCRATCH_BYTES
    dummy = torch.empty(256, dtype=torch.uint8, device="cuda")
    p = dummy.data_ptr()
    rc = L.interp_forward_noalloc(ctypes.byref(prob), p, p, p, p, p, 256,
                                  torch.cuda.current_stream().cuda_stream)
    assert rc == _lib.INTERP_EINVAL
    assert "static scratch" in _lib.last_error()
