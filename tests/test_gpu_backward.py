"""GPU parity of the backward (adjoint) kernels against the oracle's analytic
gradient, finite differences, and the autograd binding."""
import numpy as np
import pytest

import oracle
from paper_2012_13257_amd import synth
from gpu_helpers import check_grad, run_forward, say, to_dev

pytestmark = pytest.mark.gpu


def _gpu_grads(wl, G, tile=8):
    import torch
    from paper_2012_13257_amd import interp
    out, saved, work, (pos, sig, val) = run_forward(wl, tile)
    Gt = torch.from_numpy(np.ascontiguousarray(G)).cuda()
    gp, gs, gv = interp.backward(pos, sig, val, out, saved, Gt)
    torch.cuda.synchronize()
    return gp.cpu().numpy(), gs.cpu().numpy(), gv.cpu().numpy()


def _full_backward_check(wl, tile=8):
    say("backward full", wl.name, wl.B, wl.N, wl.C, wl.H, wl.W)
    G = wl.grad_out()
    gp, gs, gv = _gpu_grads(wl, G, tile)
    ref = oracle.backward(wl.pos, wl.sigma, wl.values, G, wl.H, wl.W, wl.radius,
                          workers=oracle.default_workers())
    e1 = check_grad(gp, ref["grad_pos"], ref["scale_pos"], wl.name + " pos")
    e2 = check_grad(gv, ref["grad_values"], ref["scale_values"], wl.name + " values")
    e3 = check_grad(gs, ref["grad_sigma"], ref["scale_sigma"], wl.name + " sigma")
    return e1, e2, e3


def test_backward_cfg1_full():
    _full_backward_check(synth.config1())


@pytest.mark.parametrize("C", [1, 3, 4, 8, 16, 32])
def test_backward_per_point_sigma_multitile(C):
    _full_backward_check(synth.random_workload(700 + C, 2, 500, 26, 37, C=C, sigma=(0.5, 2.0),
                                               values="normal", blob_frac=0.5, blob_std=(2.0, 5.0)))


@pytest.mark.parametrize("C", [3, 8])
def test_backward_single_radix_pass_nine_bit_keys(C):
    """The backward after a one-pass sort of 9-bit keys (160 x 200 image)."""
    _full_backward_check(synth.random_workload(320 + C, 1, 3000, 160, 200, C=C, sigma=(0.5, 2.0),
                                               values="normal", blob_frac=0.5, blob_std=(4.0, 12.0)))


@pytest.mark.parametrize("C", [3, 12])
def test_backward_shared_sigma_batch(C):
    """Shared sigma: the per-unit partial sums of dL/dsigma and their
    fixed-order total (C = 12 runs the eight-lanes-per-point adjoint)."""
    _full_backward_check(synth.random_workload(751 + C, 3, 400, 24, 30, C=C, sigma=0.9))


def _densest_bin_points(wl, b, k, tile=8):
    """k points of image b taken from its most populated tile x tile bins."""
    key = (np.floor(wl.pos[b, :, 1] / tile).astype(np.int64) * (wl.W // tile + 1)
           + np.floor(wl.pos[b, :, 0] / tile).astype(np.int64))
    vals, counts = np.unique(key, return_counts=True)
    dense = vals[np.argsort(counts)[::-1][:4]]
    members = np.nonzero(np.isin(key, dense))[0]
    return np.random.default_rng(k).choice(members, k, replace=False)


def test_backward_cfg3_sampled_points():
    """256 points of the 1024x1024 workload: random ones, the 16 with the
    largest sigma and 32 from the four densest bins."""
    wl = synth.config3()
    say("backward cfg3 sampled")
    G = wl.grad_out()
    gp, gs, gv = _gpu_grads(wl, G)
    rng = np.random.default_rng(77)
    special = np.concatenate([np.argsort(wl.sigma[0])[-16:], _densest_bin_points(wl, 0, 32)])
    rest = rng.choice(np.setdiff1d(np.arange(wl.N), special), 256 - np.unique(special).size,
                      replace=False)
    pts = np.unique(np.concatenate([special, rest]))
    assert pts.size == 256
    ref = oracle.backward_points(wl.pos, wl.sigma, wl.values, G, wl.H, wl.W, wl.radius, 0, pts,
                                 workers=oracle.default_workers(), block=4)
    check_grad(gp[0, pts], ref["grad_pos"], ref["scale_pos"], "cfg3 pos")
    check_grad(gv[0, pts], ref["grad_values"], ref["scale_values"], "cfg3 values")
    check_grad(gs[0, pts], ref["grad_sigma"], ref["scale_sigma"], "cfg3 sigma")


def test_backward_cfg5_sampled_points():
    """2 x 4096x4096, C=16, sigma up to 3: 32 points of the second image (the
    batch offset) -- random ones, the four with the largest disks and four
    from the densest bins -- against the oracle's per-point brute force."""
    wl = synth.config5()
    say("backward cfg5 sampled")
    G = wl.grad_out()
    gp, gs, gv = _gpu_grads(wl, G)
    rng = np.random.default_rng(78)
    special = np.concatenate([np.argsort(wl.sigma[1])[-4:], _densest_bin_points(wl, 1, 4)])
    rest = rng.choice(np.setdiff1d(np.arange(wl.N), special), 32 - np.unique(special).size,
                      replace=False)
    pts = np.unique(np.concatenate([special, rest]))
    assert pts.size == 32
    ref = oracle.backward_points(wl.pos, wl.sigma, wl.values, G, wl.H, wl.W, wl.radius, 1, pts,
                                 workers=oracle.default_workers(), block=1)
    check_grad(gp[1, pts], ref["grad_pos"], ref["scale_pos"], "cfg5 pos")
    check_grad(gv[1, pts], ref["grad_values"], ref["scale_values"], "cfg5 values")
    check_grad(gs[1, pts], ref["grad_sigma"], ref["scale_sigma"], "cfg5 sigma")


@pytest.mark.parametrize("C,sigma", [(3, (0.5, 2.5)), (3, 1.3), (8, (0.5, 2.5))])
def test_backward_points_outside_image_and_dense_bin(C, sigma):
    """Points just outside the border whose disks reach in, far-away points,
    a 5000-point bin: every gradient of the image against the oracle."""
    from test_gpu_forward import _outside_workload
    wl = _outside_workload(95 + C, C, sigma, values="normal" if C > 4 else "uniform")
    _full_backward_check(wl)


def test_backward_empty_and_single_point():
    say("backward N=0")
    for sig in (np.zeros((2, 0), np.float32), np.array([0.8, 1.1], np.float32)):
        wl0 = synth.Workload("empty", np.zeros((2, 0, 2), np.float32), sig,
                             np.zeros((2, 0, 3), np.float32), 17, 9, 3.0, grad_seed=3)
        gp, gs, gv = _gpu_grads(wl0, wl0.grad_out())
        assert gp.shape == (2, 0, 2) and gv.shape == (2, 0, 3)
        assert gs.shape == sig.shape and np.all(gs == 0)
    say("backward N=1")
    rng = np.random.default_rng(2)
    for sig in (np.array([[1.2]], np.float32), np.array([1.2], np.float32)):
        wl1 = synth.Workload("one", np.array([[[4.3, 5.6]]], np.float32), sig,
                             rng.random((1, 1, 3), dtype=np.float32), 12, 11, 3.0, grad_seed=4)
        # one point: out = c wherever Z > 0, so the exact position and sigma
        # gradients vanish; the GPU's float32 cancellation is held to the
        # scale of the terms that cancel
        _full_backward_check(wl1)


def test_backward_partition_of_unity_cfg3():
    """sum_j dL/dc_jk equals the sum of G over pixels with Z > 0 (any size)."""
    import torch
    from gpu_helpers import saved_Z
    from paper_2012_13257_amd import interp
    wl = synth.config3()
    G = wl.grad_out()
    out, saved, work, (pos, sig, val) = run_forward(wl)
    Gt = torch.from_numpy(G).cuda()
    _, _, gv = interp.backward(pos, sig, val, out, saved, Gt, need_pos=False, need_sigma=False)
    m = (saved_Z(saved) > 0).double()
    lhs = gv.double().sum(dim=1)[0]
    rhs = (Gt.double() * m[:, None]).sum(dim=(2, 3))[0]
    absG = (Gt.double().abs() * m[:, None]).sum(dim=(2, 3))[0]
    assert torch.all((lhs - rhs).abs() <= 1e-4 * absG)


def test_backward_matches_gpu_finite_differences():
    """Directional FD of the GPU forward itself (float32, loose tolerance): the
    backward is the derivative of what the forward computes."""
    import torch
    from paper_2012_13257_amd import interp
    wl = synth.random_workload(801, 1, 300, 24, 24, C=2, sigma=(0.8, 2.0))
    pos, sig, val = to_dev(wl)
    G = torch.from_numpy(wl.grad_out()).cuda()
    out, saved, _ = interp.forward(pos, sig, val, wl.H, wl.W, 3.0)
    gp, gs, gv = interp.backward(pos, sig, val, out, saved, G)
    rng = np.random.default_rng(9)
    d = torch.from_numpy(rng.standard_normal(wl.values.shape).astype(np.float32)).cuda()
    h = 1e-2
    lp = (interp.forward(pos, sig, val + h * d, wl.H, wl.W, 3.0)[0].double() * G).sum()
    lm = (interp.forward(pos, sig, val - h * d, wl.H, wl.W, 3.0)[0].double() * G).sum()
    fd = float((lp - lm) / (2 * h))
    an = float((gv.double() * d).sum())
    assert fd == pytest.approx(an, rel=2e-3)


def test_autograd_function_matches_backward():
    import torch
    from paper_2012_13257_amd import interp
    wl = synth.random_workload(811, 2, 400, 20, 28, C=3, sigma=(0.5, 1.5))
    pos, sig, val = to_dev(wl)
    pos.requires_grad_(True)
    sig.requires_grad_(True)
    val.requires_grad_(True)
    out = interp.interpolate(pos, sig, val, wl.H, wl.W, 3.0)
    G = torch.from_numpy(wl.grad_out()).cuda()
    (out * G).sum().backward()
    out2, saved, _ = interp.forward(pos.detach(), sig.detach(), val.detach(), wl.H, wl.W, 3.0)
    gp, gs, gv = interp.backward(pos.detach(), sig.detach(), val.detach(), out2, saved, G)
    assert torch.equal(out, out2)
    assert torch.equal(pos.grad, gp) and torch.equal(sig.grad, gs) and torch.equal(val.grad, gv)
    # only the values need a gradient: the others are not computed
    v2 = val.detach().clone().requires_grad_(True)
    interp.interpolate(pos.detach(), sig.detach(), v2, wl.H, wl.W, 3.0).mul(G).sum().backward()
    assert torch.equal(v2.grad, gv)


def test_backward_deterministic():
    wl = synth.random_workload(821, 1, 5000, 64, 64, C=3, sigma=(0.5, 2.0), blob_frac=0.6,
                               blob_std=(4.0, 9.0))
    G = wl.grad_out()
    a = _gpu_grads(wl, G)
    b = _gpu_grads(wl, G)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
