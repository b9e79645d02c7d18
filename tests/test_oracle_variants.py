"""Pins of the kernel-variant oracle (normalised density, diagonal covariance)
against closed forms, library routines, invariants and finite differences.

Each test ties oracle/gmm_variants.py to something other than its own
formulas, so that a dropped normalising factor, a swapped sigma_x / sigma_y,
a wrong power or sign in a gradient, or a wrong truncation metric fails at
least one of them."""
import math

import numpy as np
import pytest

from oracle import gmm_oracle
from oracle.gmm_variants import KERNELS, backward_variant, forward_variant, predicate_diag


def _sigmoid(t):
    return 1.0 / (1.0 + math.exp(-t))


def test_diagonal_with_equal_sigmas_is_the_isotropic_kernel():
    """sigma_x = sigma_y = sigma: the diagonal kernel is the isotropic one (no
    truncation, where the two float32 tests cannot differ).  The unnormalised
    case is compared with the main oracle, the normalised one with the
    isotropic normalised variant; d/dsigma_x + d/dsigma_y = d/dsigma."""
    rng = np.random.default_rng(1)
    B, N, H, W, C = 1, 40, 9, 11, 2
    pos = rng.uniform(-1, 12, (B, N, 2))
    s = rng.uniform(0.6, 2.0, (B, N))
    val = rng.standard_normal((B, N, C))
    G = rng.standard_normal((B, C, H, W))
    for kern, ref in (("diag", gmm_oracle.backward(pos, s, val, G, H, W, None)),
                      ("diag_norm", backward_variant(pos, s, val, G, H, W, None, "iso_norm"))):
        d = backward_variant(pos, np.stack([s, s], -1), val, G, H, W, None, kern)
        np.testing.assert_allclose(d["fwd"]["out"], ref["fwd"]["out"], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(d["grad_pos"], ref["grad_pos"], rtol=1e-10, atol=1e-13)
        np.testing.assert_allclose(d["grad_sigma"].sum(-1), ref["grad_sigma"], rtol=1e-10,
                                   atol=1e-13)
        np.testing.assert_allclose(d["grad_values"], ref["grad_values"], rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("norm", [False, True])
def test_diagonal_uniform_grid_is_separable_normalised_convolution(norm):
    """Unit grid, one point per node, shared (sigma_x, sigma_y), no truncation:
    the output is the ratio of two separable Gaussian filterings (sigma_x
    along rows, sigma_y along columns) of the values and of ones, computed
    with numpy.convolve."""
    H, W = 10, 13
    sx, sy = 1.3, 0.7
    rng = np.random.default_rng(2)
    c = rng.random((H, W))
    vv, uu = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    pos = np.stack([uu.ravel(), vv.ravel()], 1).astype(np.float64)[None]
    kern = "diag_norm" if norm else "diag"
    r = forward_variant(pos, np.array([[sx, sy]]), c.reshape(1, -1, 1), H, W, None, kern)
    gx = np.exp(-np.arange(-(W - 1), W) ** 2 / (2 * sx * sx))
    gy = np.exp(-np.arange(-(H - 1), H) ** 2 / (2 * sy * sy))

    def sep(a):
        rows = np.array([np.convolve(a[i], gx, mode="full")[W - 1: 2 * W - 1] for i in range(H)])
        return np.array([np.convolve(rows[:, j], gy, mode="full")[H - 1: 2 * H - 1]
                         for j in range(W)]).T

    expect = sep(c) / sep(np.ones_like(c))
    np.testing.assert_allclose(r["out"][0, 0], expect, rtol=1e-12)
    z = sep(np.ones_like(c)) / ((2 * math.pi * sx * sy) if norm else 1.0)
    np.testing.assert_allclose(r["Z"][0], z, rtol=1e-12)


def test_diagonal_two_points_on_a_row_follow_the_sigmoid_in_sigma_x():
    """Two points at x=a and a+1 on one row: sigma_y scales both weights alike
    at any pixel row, so o = c0 + (c1 - c0) sigmoid((2(u - a) - 1) / (2 sigma_x^2))."""
    a, sx, sy = 2.25, 0.9, 2.7
    c0, c1 = 0.2, 1.7
    W, H = 7, 3
    pos = np.array([[[a, 1.4], [a + 1.0, 1.4]]])
    for kern in ("diag", "diag_norm"):
        r = forward_variant(pos, np.array([[[sx, sy], [sx, sy]]]), np.array([[[c0], [c1]]]),
                            H, W, None, kern)
        for v in range(H):
            for u in range(W):
                t = (2 * (u - a) - 1) / (2 * sx * sx)
                assert abs(r["out"][0, 0, v, u] - (c0 + (c1 - c0) * _sigmoid(t))) < 1e-13


@pytest.mark.parametrize("kern", ["iso", "diag"])
def test_normalisation_cancels_for_a_shared_sigma(kern):
    rng = np.random.default_rng(4)
    B, N, H, W, C = 2, 30, 8, 9, 2
    pos = rng.uniform(0, 9, (B, N, 2))
    sig = rng.uniform(0.7, 1.6, (B, 2)) if kern == "diag" else rng.uniform(0.7, 1.6, B)
    val = rng.standard_normal((B, N, C))
    a = forward_variant(pos, sig, val, H, W, 3.0, kern)
    b = forward_variant(pos, sig, val, H, W, 3.0, kern + "_norm")
    np.testing.assert_allclose(b["out"], a["out"], rtol=1e-13, atol=1e-14)
    zeta = 1 / (2 * math.pi * (sig[:, 0] * sig[:, 1] if kern == "diag" else sig ** 2))
    np.testing.assert_allclose(b["Z"], a["Z"] * zeta[:, None, None], rtol=1e-13)


@pytest.mark.parametrize("kern,sig", [("iso_norm", 1.1), ("diag_norm", (1.2, 1.7))])
def test_normalised_density_sums_to_one_over_a_unit_grid(kern, sig):
    """One point per node of a unit grid, no truncation: far from the border
    the normalised weights at a pixel are a Riemann sum of a 2-D normal
    density, so Z = 1 up to the Poisson-summation error exp(-2 pi^2 sigma^2)
    (< 1e-8 here) and the border cut-off (< 1e-9 at 9 sigma)."""
    H = W = 40
    vv, uu = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    pos = np.stack([uu.ravel(), vv.ravel()], 1).astype(np.float64)[None]
    s = np.array([sig]) if kern == "diag_norm" else np.array([sig])
    N = H * W
    # only the centre pixels: evaluate on a small window of the full problem
    r = forward_variant(pos, s, np.ones((1, N, 1)), H, W, None, kern)
    centre = r["Z"][0, 17:23, 17:23]
    np.testing.assert_allclose(centre, 1.0, atol=2e-8)


@pytest.mark.parametrize("kern", ["iso_norm", "diag_norm"])
def test_normalised_coincident_points_give_the_precision_weighted_mean(kern):
    """Points at the same place with different sigmas: at that place every
    exponential is 1, so the output is the mean weighted by the densities'
    peak heights 1 / (2 pi sigma_x sigma_y) (inverse-variance weighting)."""
    s = np.array([0.6, 1.0, 1.9])
    sy = np.array([0.9, 1.3, 0.8])
    c = np.array([1.0, -2.0, 5.0])
    pos = np.tile(np.array([[3.0, 2.0]]), (3, 1))[None]
    if kern == "diag_norm":
        sig = np.stack([s, sy], -1)[None]
        wt = 1 / (s * sy)
    else:
        sig = s[None]
        wt = 1 / s ** 2
    r = forward_variant(pos, sig, c[None, :, None], 5, 6, None, kern)
    assert abs(r["out"][0, 0, 2, 3] - np.sum(wt * c) / np.sum(wt)) < 1e-13


def test_diagonal_predicate_matches_the_exact_metric_away_from_the_boundary():
    rng = np.random.default_rng(5)
    u = rng.integers(0, 40, 20000).astype(np.float64)
    v = rng.integers(0, 40, 20000).astype(np.float64)
    x = rng.uniform(0, 40, 20000).astype(np.float32)
    y = rng.uniform(0, 40, 20000).astype(np.float32)
    sx = rng.uniform(0.5, 4, 20000).astype(np.float32)
    sy = rng.uniform(0.5, 4, 20000).astype(np.float32)
    m = ((u - x.astype(np.float64)) / sx) ** 2 + ((v - y.astype(np.float64)) / sy) ** 2
    far = np.abs(m - 9.0) > 1e-4 * 9.0
    got = predicate_diag(u, v, x, y, sx, sy, 3.0)
    assert np.array_equal(got[far], (m <= 9.0)[far])
    assert got.sum() > 100 and (~got).sum() > 100
    # it is inclusive and uses sigma_x along x: a pixel exactly 3 sigma_x away
    assert predicate_diag(np.float32(7.0), np.float32(0.0), np.float32(1.0), np.float32(0.0),
                          np.float32(2.0), np.float32(0.5), 3.0)
    assert not predicate_diag(np.float32(0.0), np.float32(7.0), np.float32(0.0), np.float32(1.0),
                              np.float32(2.0), np.float32(0.5), 3.0)


@pytest.mark.parametrize("kern", KERNELS)
@pytest.mark.parametrize("per_point", [True, False])
def test_variant_gradients_match_finite_differences(kern, per_point):
    rng = np.random.default_rng(6 + KERNELS.index(kern) + 10 * per_point)
    B, N, H, W, C = 1, 6, 6, 7, 2
    pos = rng.uniform(0, 7, (B, N, 2))
    diag = kern.startswith("diag")
    if diag:
        sig = rng.uniform(0.8, 1.8, (B, N, 2)) if per_point else rng.uniform(0.8, 1.8, (B, 2))
    else:
        sig = rng.uniform(0.8, 1.8, (B, N)) if per_point else rng.uniform(0.8, 1.8, (B,))
    val = rng.standard_normal((B, N, C))
    G = rng.standard_normal((B, C, H, W))

    def loss(p, s, c):
        return float(np.sum(forward_variant(p, s, c, H, W, None, kern)["out"] * G))

    g = backward_variant(pos, sig, val, G, H, W, None, kern)
    h = 1e-6
    for arr, grad in ((pos, g["grad_pos"]), (sig, g["grad_sigma"]), (val, g["grad_values"])):
        flat = arr.reshape(-1)
        gflat = np.asarray(grad).reshape(-1)
        for i in range(flat.size):
            old = flat[i]
            flat[i] = old + h
            lp = loss(pos, sig, val)
            flat[i] = old - h
            lm = loss(pos, sig, val)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gflat[i]) <= 1e-6 * max(1.0, abs(fd)), (kern, i, fd, gflat[i])


@pytest.mark.parametrize("kern", KERNELS)
def test_variant_partition_of_unity_constant_colour_and_scales(kern):
    rng = np.random.default_rng(9)
    B, N, H, W, C = 1, 25, 9, 10, 2
    pos = rng.uniform(0, 10, (B, N, 2))
    diag = kern.startswith("diag")
    sig = rng.uniform(0.6, 1.5, (B, N, 2)) if diag else rng.uniform(0.6, 1.5, (B, N))
    val = rng.standard_normal((B, N, C))
    G = rng.standard_normal((B, C, H, W))
    g = backward_variant(pos, sig, val, G, H, W, 3.0, kern)
    mask = g["fwd"]["Z"][0] > 0
    for k in range(C):
        assert abs(g["grad_values"][0, :, k].sum() - G[0, k][mask].sum()) < 1e-10
    for name in ("pos", "sigma", "values"):
        assert np.all(np.abs(g["grad_" + name]) <= g["scale_" + name] * (1 + 1e-12) + 1e-15)
    const = np.full_like(val, 0.75)
    h = backward_variant(pos, sig, const, G, H, W, 3.0, kern)
    assert np.abs(h["grad_pos"]).max() < 1e-12 and np.abs(h["grad_sigma"]).max() < 1e-12


@pytest.mark.parametrize("kern", KERNELS)
def test_variant_scales_against_log_normaliser_when_terms_share_a_sign(kern):
    """A point left of and above the image carrying the largest value, G = 1,
    C = 1, no truncation: A_ij = alpha_i (c_0 - o_i) > 0 with expansion
    magnitude alpha_i (c_0 + o_i), so scale + grad = 2 c_0 d/dtheta sum_i
    log Z_i for the position (and, unnormalised, the sigmas), checked by
    central differences of the variant's Z."""
    rng = np.random.default_rng(11)
    B, N, H, W, C = 1, 20, 8, 9, 1
    pos = rng.uniform(1, 8, (B, N, 2))
    pos[0, 0] = (-0.6, -0.8)
    diag = kern.startswith("diag")
    sig = rng.uniform(0.8, 1.5, (B, N, 2)) if diag else rng.uniform(0.8, 1.5, (B, N))
    val = rng.uniform(0, 1, (B, N, C))
    val[0, 0] = 2.0
    G = np.ones((B, C, H, W))
    g = backward_variant(pos, sig, val, G, H, W, None, kern)

    def slz(p, s):
        return float(np.sum(np.log(forward_variant(p, s, val, H, W, None, kern)["Z"])))

    h = 1e-6
    targets = [(pos, (0, 0, a), g["scale_pos"][0, 0, a] + g["grad_pos"][0, 0, a])
               for a in range(2)]
    if not kern.endswith("_norm"):
        gsig = np.asarray(g["grad_sigma"])[0, 0]
        ssig = np.asarray(g["scale_sigma"])[0, 0]
        if diag:
            targets += [(sig, (0, 0, a), ssig[a] + gsig[a]) for a in range(2)]
        else:
            targets += [(sig, (0, 0), ssig + gsig)]
    for arr, ix, lhs in targets:
        old = arr[ix]
        arr[ix] = old + h
        lp = slz(pos, sig)
        arr[ix] = old - h
        lm = slz(pos, sig)
        arr[ix] = old
        assert lhs == pytest.approx(2 * 2.0 * (lp - lm) / (2 * h), rel=1e-7), (kern, ix)


@pytest.mark.parametrize("kern", ["iso", "diag"])
def test_normalised_gradients_equal_unnormalised_for_a_shared_sigma(kern):
    """With one shared sigma the density factor cancels in every output, so
    every gradient -- sigma's included -- is that of the unnormalised kernel."""
    rng = np.random.default_rng(12)
    B, N, H, W, C = 1, 15, 7, 8, 2
    pos = rng.uniform(0, 8, (B, N, 2))
    sig = rng.uniform(0.8, 1.5, (B, 2)) if kern == "diag" else rng.uniform(0.8, 1.5, B)
    val = rng.standard_normal((B, N, C))
    G = rng.standard_normal((B, C, H, W))
    a = backward_variant(pos, sig, val, G, H, W, 3.0, kern)
    b = backward_variant(pos, sig, val, G, H, W, 3.0, kern + "_norm")
    for name in ("grad_pos", "grad_sigma", "grad_values"):
        np.testing.assert_allclose(b[name], a[name], rtol=1e-9, atol=1e-12)
