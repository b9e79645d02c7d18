"""GPU parity of the two experiments built on the interpolation: one step of
the point / sigma optimisation (paper, Section 3, "Optimizing the points
locations") and the Gaussian-mixture upsampling of the reconstruction study
("Testing the reconstruction quality"), each against the oracle."""
import numpy as np
import pytest

import oracle
from paper_2012_13257_amd import synth
from gpu_helpers import check_grad, check_out_only, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("per_point", [True, False])
def test_optimisation_step_matches_oracle(per_point):
    import torch
    from paper_2012_13257_amd.optimize import PointFit, l1_loss
    say("optimisation step, per-point sigma", per_point)
    target = torch.from_numpy(synth.natural_image(5, 3, 40, 48)).cuda()
    fit = PointFit.from_image(target, 300, 1.2, seed=3, per_point_sigma=per_point,
                              learn_pos=True, learn_sigma=True)
    pos0 = fit.pos.detach().clone()
    ls0 = fit.log_sigma.detach().clone()
    lr = 0.25
    opt = torch.optim.SGD([fit.pos, fit.log_sigma], lr=lr)
    out = fit.render()
    loss = l1_loss(out, target)
    opt.zero_grad()
    loss.backward()
    gpos = fit.pos.grad.detach().clone()
    gls = fit.log_sigma.grad.detach().clone()
    opt.step()
    torch.cuda.synchronize()
    # the same float32 inputs on the CPU
    P = pos0.cpu().numpy()
    S = ls0.exp().cpu().numpy()
    V = fit.values.cpu().numpy()
    # dL/dout of the mean absolute error, from the GPU's output (the upstream
    # gradient is an input of the backward)
    G = (torch.sign(out.detach() - target) / out.numel())[None].cpu().numpy()
    ref = oracle.backward(P, S, V, G, 40, 48, 3.0)
    check_out_only(out.detach().cpu().numpy().reshape(3, -1).T,
                   {"out": ref["fwd"]["out"][0].reshape(3, -1).T, "Z": ref["fwd"]["Z"][0].ravel(),
                    "S": ref["fwd"]["S"][0].reshape(3, -1).T}, "render")
    check_grad(gpos.cpu().numpy(), ref["grad_pos"], ref["scale_pos"], "d loss / d pos")
    # d/d log(sigma) = sigma * d/d sigma
    s64 = S.astype(np.float64)
    check_grad(gls.cpu().numpy(), s64 * ref["grad_sigma"], s64 * ref["scale_sigma"],
               "d loss / d log sigma")
    # the SGD update moved every position by -lr * its gradient
    moved = (fit.pos.detach() - pos0).cpu().numpy().astype(np.float64)
    lim = lr * 1e-3 * np.maximum(np.abs(ref["grad_pos"]), ref["scale_pos"]) + 4e-6 * (1 + np.abs(P))
    assert np.all(np.abs(moved + lr * ref["grad_pos"]) <= lim)


def test_gmm_upsampling_matches_oracle():
    import torch
    from paper_2012_13257_amd import reconstruct
    say("gmm upsampling 3x")
    img = torch.from_numpy(synth.natural_image(8, 3, 36, 42))[None].cuda()
    low = reconstruct.downsample(img, 3)
    # the area average is the plain block mean
    ref_low = img.cpu().numpy().reshape(1, 3, 12, 3, 14, 3).mean(axis=(3, 5))
    assert np.allclose(low.cpu().numpy(), ref_low, atol=1e-6)
    for a in (0.4, 0.7):
        up = reconstruct.gmm_upsample(low, 3, a)
        pos, val = reconstruct.gmm_points(low, 3)
        sig = np.array([a * 3], np.float32)
        ref = oracle.forward(pos.cpu().numpy(), sig, val.cpu().numpy(), 36, 42, 3.0)
        check_out_only(up.cpu().numpy()[0].reshape(3, -1).T,
                       {"out": ref["out"][0].reshape(3, -1).T, "Z": ref["Z"][0].ravel(),
                        "S": ref["S"][0].reshape(3, -1).T}, f"upsample sigma {a} s")
