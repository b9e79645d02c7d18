"""GPU parity of binning and the forward gather against the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_2012_13257_amd import synth
from gpu_helpers import check_forward_pixels, run_forward, saved_Z, say

pytestmark = pytest.mark.gpu


def _bins_gpu(saved, work):
    from paper_2012_13257_amd import interp
    import torch
    r = interp.debug_bins(saved, work)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in r]


def _check_bins(wl, tile=8):
    say("bins", wl.name, wl.B, wl.N, wl.H, wl.W, "tile", tile)
    out, saved, work, _ = run_forward(wl, tile)
    bin_of, count, offset, perm = _bins_gpu(saved, work)
    ref = oracle.bins(wl.pos, wl.H, wl.W, tile)
    assert np.array_equal(bin_of, ref["bin_of"])
    assert np.array_equal(count, ref["count"])
    assert np.array_equal(offset, ref["offset"])
    assert np.array_equal(perm, ref["perm"])


def test_bins_cfg1():
    _check_bins(synth.config1())


@pytest.mark.parametrize("tile", [4, 8, 16, 32, 64])
def test_bins_tiles_ragged(tile):
    _check_bins(synth.random_workload(101, 2, 3000, 37, 53, C=2, sigma=(0.5, 2.0), blob_frac=0.5,
                                      blob_std=(2.0, 6.0)), tile)


def test_bins_edges_borders_outside_and_one_big_bin():
    rng = np.random.default_rng(7)
    H, W = 40, 50
    pts = [[8.0, 8.0], [16.0, 0.0], [7.9999995, 15.9999995], [-5.0, 3.0], [60.0, 45.0],
           [49.99, 39.99], [-1e6, -1e6], [1e6, 2.0], [0.0, 1e6]]
    # one bin holding 5000 points (exercises the merge path of the in-bin sort)
    big = np.column_stack([rng.uniform(16.0, 23.99, 5000), rng.uniform(8.0, 15.99, 5000)])
    allp = np.concatenate([np.array(pts), big, rng.random((500, 2)) * [W, H]]).astype(np.float32)
    allp = allp[rng.permutation(allp.shape[0])]
    N = allp.shape[0]
    wl = synth.Workload("edges", allp[None], np.full((1, N), 0.8, np.float32),
                        rng.random((1, N, 3), dtype=np.float32), H, W, 3.0)
    _check_bins(wl)


def test_bins_cfg3_full():
    _check_bins(synth.config3())


def _full_forward_check(wl, tile=8):
    say("forward full", wl.name, wl.B, wl.N, wl.C, wl.H, wl.W)
    out, saved, work, _ = run_forward(wl, tile)
    ref = oracle.forward(wl.pos, wl.sigma, wl.values, wl.H, wl.W, wl.radius,
                         workers=oracle.default_workers())
    og = out.cpu().numpy().transpose(0, 2, 3, 1).reshape(-1, wl.C)
    Zg = saved_Z(saved).cpu().numpy().ravel()
    r = {"out": ref["out"].transpose(0, 2, 3, 1).reshape(-1, wl.C), "Z": ref["Z"].ravel(),
         "S": ref["S"].transpose(0, 2, 3, 1).reshape(-1, wl.C)}
    return check_forward_pixels(og, Zg, r, wl.name)


def test_forward_cfg1_full():
    _full_forward_check(synth.config1())


@pytest.mark.parametrize("C", [1, 2, 3, 4, 5, 8, 16, 17, 32])
def test_forward_channels_ragged_multitile(C):
    _full_forward_check(synth.random_workload(200 + C, 2, 700, 29, 43, C=C, sigma=(0.4, 2.5),
                                              values="normal", blob_frac=0.4, blob_std=(2.0, 5.0)))


@pytest.mark.parametrize("tile", [4, 16, 64])
def test_forward_other_tiles_shared_sigma(tile):
    _full_forward_check(synth.random_workload(300 + tile, 1, 900, 40, 33, C=3, sigma=1.3), tile)


def test_forward_large_sigma_and_radius():
    # reach beyond one bin in every direction, r = 3.5
    wl = synth.random_workload(401, 1, 400, 48, 40, C=2, sigma=(2.0, 6.0), radius=3.5)
    _full_forward_check(wl)


def test_forward_empty_and_single_point():
    rng = np.random.default_rng(1)
    wl0 = synth.Workload("empty", np.zeros((2, 0, 2), np.float32), np.zeros((2, 0), np.float32),
                         np.zeros((2, 0, 3), np.float32), 17, 9, 3.0)
    out, saved, _, _ = run_forward(wl0)
    assert np.all(out.cpu().numpy() == 0) and np.all(saved_Z(saved).cpu().numpy() == 0)
    wl1 = synth.Workload("one", np.array([[[4.3, 5.6]]], np.float32), np.array([1.2], np.float32),
                         rng.random((1, 1, 3), dtype=np.float32), 12, 11, 3.0)
    _full_forward_check(wl1)


def test_forward_cfg2_one_image_full_and_batch_sampled():
    wl = synth.config2()
    say("forward cfg2", wl.B, wl.N)
    out, saved, _, _ = run_forward(wl)
    out = out.cpu().numpy()
    Zg = saved_Z(saved).cpu().numpy()
    rng = np.random.default_rng(5)
    n = 2048
    b = rng.integers(0, wl.B, n)
    v = rng.integers(0, wl.H, n)
    u = rng.integers(0, wl.W, n)
    ref = oracle.forward_pixels(wl.pos, wl.sigma, wl.values, wl.radius, b, v, u,
                                workers=oracle.default_workers())
    check_forward_pixels(out[b, :, v, u], Zg[b, v, u], ref, "cfg2 sampled")


def _densest_block(wl, b):
    cnt, _, _ = np.histogram2d(wl.pos[b, :, 1], wl.pos[b, :, 0], bins=[wl.H // 8, wl.W // 8],
                               range=[[0, wl.H // 8 * 8], [0, wl.W // 8 * 8]])
    by, bx = np.unravel_index(np.argmax(cnt), cnt.shape)
    return by * 8, bx * 8


def _sampled_check(wl, n_random, seed, tile=8):
    say("forward sampled", wl.name, "tile", tile)
    out, saved, _, _ = run_forward(wl, tile)
    out = out.cpu().numpy()
    Zg = saved_Z(saved).cpu().numpy()
    rng = np.random.default_rng(seed)
    bs, vs, us = [], [], []
    bs.append(rng.integers(0, wl.B, n_random))
    vs.append(rng.integers(0, wl.H, n_random))
    us.append(rng.integers(0, wl.W, n_random))
    for b in range(wl.B):
        v0, u0 = _densest_block(wl, b)
        vv, uu = np.meshgrid(np.arange(v0, v0 + 8), np.arange(u0, u0 + 8), indexing="ij")
        bs.append(np.full(64, b))
        vs.append(vv.ravel())
        us.append(uu.ravel())
    # the last row and column (ragged tail of the block grid at odd sizes)
    bs.append(np.zeros(16, np.int64))
    vs.append(np.full(16, wl.H - 1))
    us.append(rng.integers(0, wl.W, 16))
    b = np.concatenate(bs)
    v = np.concatenate(vs)
    u = np.concatenate(us)
    ref = oracle.forward_pixels(wl.pos, wl.sigma, wl.values, wl.radius, b, v, u,
                                workers=oracle.default_workers())
    return check_forward_pixels(out[b, :, v, u], Zg[b, v, u], ref, wl.name)


def test_forward_cfg3_sampled():
    _sampled_check(synth.config3(), 1024, 33)


def test_forward_cfg5_sampled():
    _sampled_check(synth.config5(), 192, 55)


def test_three_radix_passes_bins_and_sampled_forward():
    # 4-pixel bins on a 2047 x 2050 image: 513 x 512 bins need 18 key bits,
    # so the sort takes three passes (and both sets of between-pass records)
    wl = synth.random_workload(4711, 1, 60000, 2047, 2050, C=3, sigma=(0.5, 2.0), blob_frac=0.5,
                               blob_std=(20.0, 80.0))
    _check_bins(wl, 4)
    _sampled_check(wl, 512, 77, tile=4)


def test_single_bin_needs_no_radix_pass():
    # a 7 x 6 image is one 8 x 8 bin: the point order is the sorted order
    wl = synth.random_workload(4712, 2, 300, 7, 6, C=4, sigma=(0.5, 2.0))
    _check_bins(wl)
    _full_forward_check(wl)


# ---------------------------------------------------------------------------
# Exactness checks
# ---------------------------------------------------------------------------

def test_constant_power_of_two_colour_is_bitwise():
    wl = synth.random_workload(501, 1, 3000, 64, 80, C=4, sigma=(0.5, 2.0))
    wl.values[:] = 0.25
    out, saved, _, _ = run_forward(wl)
    out = out.cpu().numpy()
    Zg = saved_Z(saved).cpu().numpy()
    m = Zg[0] > 0
    assert m.sum() > 1000
    assert np.all(out[0][:, m] == np.float32(0.25))
    assert np.all(out[0][:, ~m] == 0)


def test_uniform_grid_small_sigma_reproduces_nodes_bitwise():
    H, W = 45, 70
    vv, uu = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    pos = np.stack([uu.ravel(), vv.ravel()], 1).astype(np.float32)[None]
    rng = np.random.default_rng(3)
    val = rng.standard_normal((1, H * W, 3)).astype(np.float32)
    wl = synth.Workload("grid", pos, np.array([0.3], np.float32), val, H, W, 3.0)
    out, saved, _, _ = run_forward(wl)
    expect = val[0].reshape(H, W, 3).transpose(2, 0, 1)
    assert np.array_equal(out.cpu().numpy()[0], expect)
    assert np.all(saved_Z(saved).cpu().numpy() == 1.0)


def test_forward_deterministic():
    wl = synth.random_workload(601, 2, 20000, 96, 80, C=3, sigma=(0.5, 2.0), blob_frac=0.7,
                               blob_std=(4.0, 10.0))
    o1, s1, _, _ = run_forward(wl)
    o2, s2, _, _ = run_forward(wl)
    assert np.array_equal(o1.cpu().numpy(), o2.cpu().numpy())
    assert np.array_equal(saved_Z(s1).cpu().numpy(), saved_Z(s2).cpu().numpy())
