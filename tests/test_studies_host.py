"""Host-side pieces of the two experiments (no GPU): the synthetic images and
point sampling, and the grid of known points of the upsampling study."""
import numpy as np

from paper_2012_13257_amd import synth


def test_natural_image_is_seeded_and_in_range():
    a = synth.natural_image(3, 3, 50, 70)
    b = synth.natural_image(3, 3, 50, 70)
    assert a.shape == (3, 50, 70) and a.dtype == np.float32
    assert np.array_equal(a, b)
    assert a.min() >= 0.0 and a.max() <= 1.0 and a.std() > 0.05
    assert not np.array_equal(a, synth.natural_image(4, 3, 50, 70))


def test_sampled_points_carry_the_nearest_pixel():
    img = synth.natural_image(1, 2, 30, 40)
    pos, val = synth.sample_image_points(np.random.default_rng(0), img, 500)
    assert pos.shape == (500, 2) and val.shape == (500, 2)
    assert pos[:, 0].min() >= 0 and pos[:, 0].max() <= 39
    assert pos[:, 1].min() >= 0 and pos[:, 1].max() <= 29
    for k in range(0, 500, 37):
        u, v = int(round(float(pos[k, 0]))), int(round(float(pos[k, 1])))
        assert np.array_equal(val[k], img[:, v, u])


def test_grid_points_sit_at_footprint_centres():
    import torch
    from paper_2012_13257_amd.reconstruct import gmm_points, grid_points
    g = grid_points(3, 4, 5, "cpu").numpy()
    assert g.shape == (12, 2)
    # low-res pixel (i=1, j=2) covers full-res rows 5..9 and columns 10..14
    assert np.array_equal(g[1 * 4 + 2], [12.0, 7.0])
    low = torch.arange(2 * 3 * 4, dtype=torch.float32).reshape(1, 2, 3, 4)
    pos, val = gmm_points(low, 5)
    assert pos.shape == (1, 12, 2) and val.shape == (1, 12, 2)
    assert float(val[0, 1 * 4 + 2, 1]) == float(low[0, 1, 1, 2])
