"""Seeded input generators (CPU): the travelling source sequence is the GRF
pattern translated in space."""
import numpy as np

from paper_2604_01800_amd import inputs


def test_travelling_grf_is_a_translation():
    g = inputs.make_grid(48, 40, 1.3)
    s, d = 0.02, np.array([0.6, 0.8])
    fs = inputs.travelling_grf(g, 4, 4, shift=s, direction=d)
    assert fs.shape == (4, 40, 48) and fs.dtype == np.float32
    np.testing.assert_array_equal(fs[0], inputs.grf(g, 4).astype(np.float32))
    feats = inputs.grf_features(np.random.default_rng(4))
    for t in range(1, 4):
        # the step-0 field read at the cell centres moved back by t * s along d
        ref = inputs.grf_eval(g.xc - t * s * d[0], g.yc - t * s * d[1], feats)
        np.testing.assert_allclose(fs[t], ref, rtol=0, atol=2e-5 * np.abs(ref).max())
        assert np.linalg.norm(fs[t] - fs[t - 1]) > 1e-3 * np.linalg.norm(fs[t])
