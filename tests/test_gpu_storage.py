"""GPU parity of bfloat16 / half storage of the value arrays (values, out,
grad_out, grad_values) against the oracle on the same (rounded) inputs.

Sums are float32 on the GPU, so the float32 tolerances hold before the one
rounding of out and grad_values to the storage type; the bound adds half a
unit in the last place of that type (relative 2^-8 for bfloat16, 2^-11 for
half, plus half's smallest subnormal step)."""
import numpy as np
import pytest

import oracle
from paper_2012_13257_amd import synth
from gpu_helpers import FWD_RTOL, GRAD_RTOL, check_grad, say, saved_Z

pytestmark = pytest.mark.gpu

HALF_ULP = {"bfloat16": (2.0 ** -8, 0.0), "float16": (2.0 ** -11, 2.0 ** -25)}


def _dtype(name):
    import torch
    return getattr(torch, name)


def _check_rounded(got, ref, scale, rtol, dt, where):
    rel, absl = HALF_ULP[dt]
    got = np.asarray(got, np.float64)
    lim = rtol * scale * (1 + rel) + rel * np.abs(ref) + absl
    bad = np.abs(got - ref) > lim
    assert not bad.any(), (f"{where}: {int(bad.sum())}/{bad.size} beyond the {dt} bound; worst "
                           f"{float(np.max(np.abs(got - ref) / np.maximum(lim, 1e-300))):.3g}")


@pytest.mark.parametrize("dt", ["bfloat16", "float16"])
@pytest.mark.parametrize("C", [3, 16])
def test_storage_forward_and_backward_match_oracle(dt, C):
    import torch
    from paper_2012_13257_amd import interp
    wl = synth.random_workload(1200 + C, 2, 300, 29, 34, C=C, sigma=(0.5, 2.2), values="normal",
                               blob_frac=0.4, blob_std=(2.0, 5.0))
    say("storage", dt, "C", C)
    t = _dtype(dt)
    pos = torch.from_numpy(wl.pos).cuda()
    sig = torch.from_numpy(wl.sigma).cuda()
    val = torch.from_numpy(wl.values).cuda().to(t)
    G = torch.from_numpy(wl.grad_out()).cuda().to(t)
    out, saved, work = interp.forward(pos, sig, val, wl.H, wl.W, wl.radius)
    assert out.dtype == t
    gp, gs, gv = interp.backward(pos, sig, val, out, saved, G, work=work)
    torch.cuda.synchronize()
    assert gv.dtype == t and gp.dtype == torch.float32
    # the oracle on exactly the stored inputs
    vals = val.float().cpu().numpy()
    Gn = G.float().cpu().numpy()
    ref = oracle.backward(wl.pos, wl.sigma, vals, Gn, wl.H, wl.W, wl.radius,
                          workers=oracle.default_workers())
    f = ref["fwd"]
    Zg = saved_Z(saved).cpu().numpy()
    assert np.array_equal(Zg == 0, f["Z"] == 0)
    nz = f["Z"] > 0
    assert np.max(np.abs(Zg[nz] - f["Z"][nz]) / f["Z"][nz]) <= 1e-5
    o = out.float().cpu().numpy()
    for b in range(wl.B):
        assert np.all(o[b][:, ~nz[b]] == 0)
    _check_rounded(o, f["out"], np.maximum(np.abs(f["out"]), f["S"]), FWD_RTOL, dt, "out")
    check_grad(gp.cpu().numpy(), ref["grad_pos"], ref["scale_pos"], dt + " pos")
    check_grad(gs.cpu().numpy(), ref["grad_sigma"], ref["scale_sigma"], dt + " sigma")
    _check_rounded(gv.float().cpu().numpy(), ref["grad_values"],
                   np.maximum(np.abs(ref["grad_values"]), ref["scale_values"]), GRAD_RTOL, dt,
                   "grad_values")


def test_bfloat16_storage_at_full_size_c16_sampled():
    """The 2 x 4096^2, C = 16 workload in bfloat16 (the launch configuration
    the benchmark times): 1024 random pixels of the forward against the
    oracle on the rounded values."""
    import torch
    from paper_2012_13257_amd import interp
    wl = synth.config5()
    say("storage bf16 full size", wl.name)
    pos = torch.from_numpy(wl.pos).cuda()
    sig = torch.from_numpy(wl.sigma).cuda()
    val = torch.from_numpy(wl.values).cuda().to(torch.bfloat16)
    out, saved, _ = interp.forward(pos, sig, val, wl.H, wl.W, wl.radius)
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    b = rng.integers(0, wl.B, 1024)
    v = rng.integers(0, wl.H, 1024)
    u = rng.integers(0, wl.W, 1024)
    got = out.float()[torch.from_numpy(b).cuda(), :, torch.from_numpy(v).cuda(),
                      torch.from_numpy(u).cuda()].cpu().numpy()
    vals = val.float().cpu().numpy()
    del out, saved, val
    ref = oracle.forward_pixels(wl.pos, wl.sigma, vals, wl.radius, b, v, u,
                                workers=oracle.default_workers())
    _check_rounded(got, ref["out"], np.maximum(np.abs(ref["out"]), ref["S"]), FWD_RTOL,
                   "bfloat16", "cfg5 bf16 out")
