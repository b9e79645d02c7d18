"""GPU parity of the kernel variants (normalised density, diagonal
covariance) against the variant oracle: full images forward (outputs and Z)
and every point's gradients, per-point and shared sigma, narrow and wide
channel counts, points outside the image."""
import numpy as np
import pytest

from oracle.gmm_variants import KERNELS, backward_variant
from gpu_helpers import check_forward_pixels, check_grad, say

pytestmark = pytest.mark.gpu


def _workload(seed, kern, per_point, B=2, N=300, H=23, W=37, C=3):
    rng = np.random.default_rng(seed)
    pos = np.empty((B, N, 2), np.float32)
    pos[..., 0] = rng.uniform(-3.0, W + 3.0, (B, N))
    pos[..., 1] = rng.uniform(-3.0, H + 3.0, (B, N))
    # a tight cluster so that some bins are dense
    pos[:, : N // 4] = (np.array([W * 0.3, H * 0.6]) + rng.normal(0, 1.5, (B, N // 4, 2)))
    shape = ((B, N) if per_point else (B,)) + ((2,) if kern.startswith("diag") else ())
    sig = np.exp(rng.uniform(np.log(0.5), np.log(2.2), shape)).astype(np.float32)
    val = rng.standard_normal((B, N, C)).astype(np.float32)
    G = rng.standard_normal((B, C, H, W)).astype(np.float32)
    return pos, sig, val, G, H, W


@pytest.mark.parametrize("kern", KERNELS)
@pytest.mark.parametrize("per_point", [True, False])
@pytest.mark.parametrize("C", [1, 3, 6])
def test_variant_forward_and_backward_match_oracle(kern, per_point, C):
    _check_variant(kern, per_point, C)


def _check_variant(kern, per_point, C):
    import torch
    from paper_2012_13257_amd import interp
    pos, sig, val, G, H, W = _workload(900 + 7 * C + 3 * KERNELS.index(kern) + per_point,
                                       kern, per_point, C=C)
    say("variant", kern, "per_point", per_point, "C", C)
    norm, aniso = kern.endswith("_norm"), kern.startswith("diag")
    P, S, V = (torch.from_numpy(a).cuda() for a in (pos, sig, val))
    out, saved, work = interp.forward(P, S, V, H, W, 3.0, 8, norm, aniso)
    gp, gs, gv = interp.backward(P, S, V, out, saved, torch.from_numpy(G).cuda(), work=work)
    torch.cuda.synchronize()
    from gpu_helpers import saved_Z
    ref = backward_variant(pos, sig, val, G, H, W, 3.0, kern)
    f = ref["fwd"]
    for b in range(pos.shape[0]):
        check_forward_pixels(out[b].cpu().numpy().reshape(C, -1).T,
                             saved_Z(saved)[b].cpu().numpy().ravel(),
                             {"out": f["out"][b].reshape(C, -1).T, "Z": f["Z"][b].ravel(),
                              "S": f["S"][b].reshape(C, -1).T}, f"{kern} image {b}")
    check_grad(gp.cpu().numpy(), ref["grad_pos"], ref["scale_pos"], kern + " pos")
    check_grad(gv.cpu().numpy(), ref["grad_values"], ref["scale_values"], kern + " values")
    check_grad(gs.cpu().numpy(), ref["grad_sigma"], ref["scale_sigma"], kern + " sigma")


@pytest.mark.parametrize("kern", ["iso_norm", "diag_norm"])
@pytest.mark.parametrize("C", [4, 32])
def test_normalised_four_and_thirty_two_channels(kern, C):
    """The normalised kernel with C = 4 (the four-value records of the narrow
    path) and C = 32 (the widest records) against the variant oracle."""
    _check_variant(kern, True, C)


@pytest.mark.parametrize("kern", ["iso_norm", "diag"])
def test_variant_through_autograd_and_small_tile(kern):
    """The autograd binding and a 4-pixel tile give the same gradients."""
    import torch
    from paper_2012_13257_amd import interp
    pos, sig, val, G, H, W = _workload(77, kern, True, B=1, N=200, H=19, W=26, C=2)
    norm, aniso = kern.endswith("_norm"), kern.startswith("diag")
    P, S, V = (torch.from_numpy(a).cuda().requires_grad_(True) for a in (pos, sig, val))
    out = interp.interpolate(P, S, V, H, W, 3.0, 4, normalized=norm, anisotropic=aniso)
    (out * torch.from_numpy(G).cuda()).sum().backward()
    ref = backward_variant(pos, sig, val, G, H, W, 3.0, kern)
    check_grad(P.grad.cpu().numpy(), ref["grad_pos"], ref["scale_pos"], "autograd pos")
    check_grad(S.grad.cpu().numpy(), ref["grad_sigma"], ref["scale_sigma"], "autograd sigma")
    check_grad(V.grad.cpu().numpy(), ref["grad_values"], ref["scale_values"], "autograd values")
