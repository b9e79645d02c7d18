"""The C-ABI forward + backward captured into a HIP graph: every replay, with
eager work and synchronisations between replays, must reproduce the eager
result bit for bit (the library records no memset or host synchronisation)."""
import ctypes

import numpy as np
import pytest

from paper_2012_13257_amd import synth
from gpu_helpers import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("per_point", [True, False])
def test_graph_replay_matches_eager(per_point):
    import torch
    from paper_2012_13257_amd import _lib, interp
    wl = synth.random_workload(4242, 2, 30000, 200, 328, C=3, sigma=(0.5, 2.0) if per_point else 1.2,
                               per_point=per_point, blob_frac=0.5, blob_std=(5.0, 20.0))
    say("graph replay", wl.name, wl.B, wl.N, wl.H, wl.W, "per_point", per_point)
    pos, sig, val = to_dev(wl)
    G = torch.from_numpy(wl.grad_out()).cuda()
    prob = interp.problem(pos, sig, val, wl.H, wl.W, wl.radius)
    saved = interp.Saved(prob, pos.device)
    work = interp.Workspace(prob, pos.device)
    out = torch.empty((wl.B, wl.C, wl.H, wl.W), device="cuda")
    gp, gs, gv = torch.empty_like(pos), torch.empty_like(sig), torch.empty_like(val)
    L = _lib.lib()
    pb = ctypes.byref(prob)

    def step():
        st = torch.cuda.current_stream().cuda_stream
        _lib.check("interp_forward", L.interp_forward(
            pb, pos.data_ptr(), sig.data_ptr(), val.data_ptr(), out.data_ptr(), saved.addr,
            saved.nbytes, work.addr, work.nbytes, st))
        _lib.check("interp_backward", L.interp_backward(
            pb, pos.data_ptr(), sig.data_ptr(), val.data_ptr(), out.data_ptr(), saved.addr,
            saved.nbytes, G.data_ptr(), gp.data_ptr(), gs.data_ptr(), gv.data_ptr(), work.addr,
            work.nbytes, st))

    step()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (out, gp, gs, gv)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    for rep in range(4):
        for t in (out, gp, gs, gv):
            t.fill_(float("nan"))
        # eager work on the same buffers between replays
        work.buf.fill_(0x5A)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for name, a, b in zip(("out", "grad_pos", "grad_sigma", "grad_values"), ref,
                              (out, gp, gs, gv)):
            assert torch.equal(a, b), f"replay {rep}: {name} differs from the eager result"
        step()
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(ref, (out, gp, gs, gv)))
    assert np.isfinite(ref[0].cpu().numpy()).all()


@pytest.mark.parametrize("kern,dtype", [("diag_norm", "float32"), ("iso", "bfloat16")])
def test_graph_replay_variants_and_storage(kern, dtype):
    """The same for a normalised diagonal kernel and for bfloat16 storage."""
    import torch
    from paper_2012_13257_amd import _lib, interp
    wl = synth.random_workload(4343, 1, 20000, 160, 200, C=3, sigma=(0.5, 2.0),
                               blob_frac=0.5, blob_std=(5.0, 20.0))
    say("graph replay", kern, dtype)
    norm, aniso = kern.endswith("_norm"), kern.startswith("diag")
    pos, sig, val = to_dev(wl)
    if aniso:
        sig = torch.stack([sig, sig.flip(-1)], dim=-1).contiguous()
    val = val.to(getattr(torch, dtype))
    G = torch.from_numpy(wl.grad_out()).cuda().to(val.dtype)
    prob = interp.problem(pos, sig, val, wl.H, wl.W, wl.radius, 8, norm, aniso)
    saved = interp.Saved(prob, pos.device)
    work = interp.Workspace(prob, pos.device)
    out = torch.empty((wl.B, wl.C, wl.H, wl.W), device="cuda", dtype=val.dtype)
    gp, gs, gv = torch.empty_like(pos), torch.empty_like(sig), torch.empty_like(val)
    L = _lib.lib()
    pb = ctypes.byref(prob)

    def step():
        st = torch.cuda.current_stream().cuda_stream
        _lib.check("interp_forward", L.interp_forward(
            pb, pos.data_ptr(), sig.data_ptr(), val.data_ptr(), out.data_ptr(), saved.addr,
            saved.nbytes, work.addr, work.nbytes, st))
        _lib.check("interp_backward", L.interp_backward(
            pb, pos.data_ptr(), sig.data_ptr(), val.data_ptr(), out.data_ptr(), saved.addr,
            saved.nbytes, G.data_ptr(), gp.data_ptr(), gs.data_ptr(), gv.data_ptr(), work.addr,
            work.nbytes, st))

    step()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (out, gp, gs, gv)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        for t in (out, gp, gs, gv):
            t.fill_(float("nan"))
        work.buf.fill_(0x5A)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for name, a, b in zip(("out", "grad_pos", "grad_sigma", "grad_values"), ref,
                              (out, gp, gs, gv)):
            assert torch.equal(a, b), f"replay {rep}: {name} differs from the eager result"
