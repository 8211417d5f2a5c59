"""The seeded input recipes: shapes, spacing and determinism."""
import numpy as np

import workloads as W


def test_spacing_follows_unknown_counts():
    assert np.isclose(W.C1_FHN.h[0], 2.5 / 63)
    assert np.isclose(W.C2_GS.h[0], 2.0 / 512)
    assert np.isclose(W.C3_SCHNAK_DIR.h[0], 1.0 / 129)
    assert np.isclose(W.C4_GM_ADJ.h[0], 2.0 / 255)
    assert np.isclose(W.C5_SCHNAK_NEU.h[0], 1.0 / 255)
    assert np.isclose(W.C3_SCHNAK_DIR.coords(0)[0], 1.0 / 129)


def test_initial_fields_are_seeded():
    for wl in (W.C1_FHN, W.C2_GS, W.C4_GM_ADJ):
        a, b = W.initial_fields(wl), W.initial_fields(wl)
        assert a.shape == (2,) + wl.shape and a.dtype == np.float64
        assert np.array_equal(a, b)
    small = W.small(W.C3_SCHNAK_DIR, (8, 9, 10))
    u = W.initial_fields(small)
    assert u.shape == (2, 8, 9, 10) and abs(u.mean() - 0.9) < 0.01
    gs = W.initial_fields(W.C2_GS)
    assert abs(gs[0, 256, 256] - 0.5) <= 0.01 and abs(gs[0, 0, 0] - 1.0) <= 0.01
