"""GPU parity of binning and the forward gather against the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_2012_13257_amd import synth
from gpu_helpers import check_forward_pixels, run_forward, saved_reach, saved_Z, say

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


@pytest.mark.parametrize("H,W,N", [(160, 200, 20000), (256, 256, 70000), (120, 72, 900)])
def test_bins_single_pass_nine_and_ten_bit_keys(H, W, N):
    """500 and 1024 bins (keys of 9 and 10 bits: one radix pass of up to 1024
    digits, scan by one wavefront per digit), and 135 bins with fewer points
    than one radix tile."""
    _check_bins(synth.random_workload(H + W + N, 2, N, H, W, C=3, sigma=(0.5, 2.0), blob_frac=0.5,
                                      blob_std=(4.0, 12.0)))


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


@pytest.mark.parametrize("C", [3, 8])
def test_forward_single_radix_pass_nine_bit_keys(C):
    """A 160 x 200 image (500 bins: one radix pass over 9-bit keys), narrow
    records carried through the pass and wide records placed afterwards."""
    _full_forward_check(synth.random_workload(300 + C, 1, 4000, 160, 200, C=C, sigma=(0.5, 2.0),
                                              values="normal", blob_frac=0.5, blob_std=(4.0, 12.0)))


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


def test_forward_cfg2_one_image_full():
    """Image 0 of the 16 x 256x256 jittered-grid batch, every pixel against
    the oracle's brute force over all 65536 points of that image."""
    wl = synth.config2()
    say("forward cfg2 image 0 full", wl.B, wl.N)
    out, saved, _, _ = run_forward(wl)
    out = out.cpu().numpy()[0]
    Zg = saved_Z(saved).cpu().numpy()[0]
    ref = oracle.forward(wl.pos[:1], wl.sigma[:1], wl.values[:1], wl.H, wl.W, wl.radius,
                         workers=oracle.default_workers())
    r = {"out": ref["out"][0].transpose(1, 2, 0).reshape(-1, wl.C), "Z": ref["Z"][0].ravel(),
         "S": ref["S"][0].transpose(1, 2, 0).reshape(-1, wl.C)}
    check_forward_pixels(out.transpose(1, 2, 0).reshape(-1, wl.C), Zg.ravel(), r, "cfg2 image 0")


def test_forward_cfg2_batch_sampled():
    """2048 pixels drawn over all 16 images of the batch (the batch offsets)."""
    wl = synth.config2()
    say("forward cfg2 batch sampled", wl.B, wl.N)
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


def _densest_tiles(wl, b, side, k):
    """Top-left corners (row, col) of the k most populated side x side tiles of image b."""
    cnt, _, _ = np.histogram2d(wl.pos[b, :, 1], wl.pos[b, :, 0],
                               bins=[wl.H // side, wl.W // side],
                               range=[[0, wl.H // side * side], [0, wl.W // side * side]])
    flat = np.argsort(cnt.ravel())[::-1][:k]
    return [(int(i // cnt.shape[1]) * side, int(i % cnt.shape[1]) * side) for i in flat]


def _sampled_check(wl, n_random, seed, tile=8, dense_tiles=1, dense_side=8):
    """n_random random pixels over the batch, every pixel of the dense_tiles
    most populated dense_side x dense_side tiles of each image, and part of
    the last row (the ragged tail of the block grid at odd sizes)."""
    say("forward sampled", wl.name, "tile", tile, "pixels", n_random)
    out, saved, _, _ = run_forward(wl, tile)
    out = out.cpu().numpy()
    Zg = saved_Z(saved).cpu().numpy()
    rng = np.random.default_rng(seed)
    bs, vs, us = [], [], []
    bs.append(rng.integers(0, wl.B, n_random))
    vs.append(rng.integers(0, wl.H, n_random))
    us.append(rng.integers(0, wl.W, n_random))
    for b in range(wl.B):
        for v0, u0 in _densest_tiles(wl, b, dense_side, dense_tiles):
            vv, uu = np.meshgrid(np.arange(v0, v0 + dense_side), np.arange(u0, u0 + dense_side),
                                 indexing="ij")
            bs.append(np.full(vv.size, b))
            vs.append(vv.ravel())
            us.append(uu.ravel())
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
    """4096 random pixels plus every pixel of the 4 densest 16x16 tiles."""
    _sampled_check(synth.config3(), 4096, 33, dense_tiles=4, dense_side=16)


def test_forward_cfg5_sampled():
    """4096 random pixels over both images plus the densest 16x16 tile of each."""
    _sampled_check(synth.config5(), 4096, 55, dense_tiles=1, dense_side=16)


def test_reach_is_bit_exact():
    """The stored per-image reach is the largest f32(radius * sigma) (a max is
    order-free, so it is exact), for per-point and shared sigma."""
    for wl in (synth.random_workload(91, 3, 2000, 40, 50, C=2, sigma=(0.5, 3.0)),
               synth.random_workload(92, 2, 300, 30, 20, C=1, sigma=1.7),
               synth.config3()):
        say("reach", wl.name, wl.B, wl.N)
        _, saved, _, _ = run_forward(wl)
        got = saved_reach(saved).cpu().numpy()
        assert np.array_equal(got, oracle.reach(wl.sigma, wl.radius, wl.N))


def _outside_workload(seed, C, sigma, values="uniform"):
    """Points inside, on the border, just outside (whose disks reach in) and
    far away, plus one 8x8 bin holding 5000 points, on a 40 x 50 image."""
    rng = np.random.default_rng(seed)
    H, W = 40, 50
    pts = [[-1.5, 10.2], [W + 0.7, 20.4], [25.3, H + 1.0], [12.0, -2.25], [-0.5, -0.5],
           [W - 0.01, H - 0.01], [W + 2.0, H + 2.0], [8.0, 8.0], [16.0, 0.0],
           [-1e6, -1e6], [1e6, 2.0], [0.0, 1e6], [-7.5, 30.0]]
    big = np.column_stack([rng.uniform(16.0, 23.99, 5000), rng.uniform(8.0, 15.99, 5000)])
    allp = np.concatenate([np.array(pts), big, rng.random((600, 2)) * [W, H]]).astype(np.float32)
    allp = allp[rng.permutation(allp.shape[0])]
    N = allp.shape[0]
    if isinstance(sigma, float):
        sig = np.full((1,), sigma, np.float32)
    else:
        sig = rng.uniform(sigma[0], sigma[1], (1, N)).astype(np.float32)
    if values == "normal":
        val = rng.standard_normal((1, N, C)).astype(np.float32)
    else:
        val = rng.random((1, N, C), dtype=np.float32)
    return synth.Workload(f"outside_c{C}", allp[None], sig, val, H, W, 3.0, grad_seed=seed + 1)


@pytest.mark.parametrize("C,sigma", [(3, (0.5, 2.5)), (3, 1.3), (8, (0.5, 2.5))])
def test_forward_points_outside_image_and_dense_bin(C, sigma):
    wl = _outside_workload(95 + C, C, sigma, values="normal" if C > 4 else "uniform")
    _check_bins(wl)
    _full_forward_check(wl)


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
