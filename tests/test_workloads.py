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


def test_paper_presets_follow_section_5_2():
    """Initial data and constants of the paper's applications (Section 5.2)."""
    fhn = W.initial_fields(W.PAPER_FHN)
    h = 2.5 / 256
    assert np.isclose(W.PAPER_FHN.h[0], h)
    # u = 1 exactly on the nodes with 0 < x, y <= 12 h (0.125 = 12.8 h)
    assert fhn[0].sum() == 144 and fhn[0, 1, 1] == 1.0 and fhn[0, 0, 1] == 0.0
    assert fhn[0, 12, 12] == 1.0 and fhn[0, 13, 12] == 0.0
    assert fhn[1, 12, 0] == 0.0 and fhn[1, 13, 0] == 0.1
    gm = W.initial_fields(W.PAPER_GM)
    assert W.PAPER_GM.shape == (65, 65) and np.isclose(W.PAPER_GM.h[0], 2.0 / 64)
    assert np.isclose(gm[0, 32, 32], 0.51)                      # centre: (1 + 0.02)/2
    assert np.isclose(gm[1, 32, 32], 1.0 / 3.0)                 # cosh(1)/(3 cosh 1)
    assert np.isclose(gm[1, 0, 0], np.cosh(1 - np.sqrt(2)) / (3 * np.cosh(1)))
    mu, eps = 0.1, 0.04
    assert np.allclose(W.PAPER_GM.params, (0.0, 1.0, 1.0, 1 / (eps * mu), 1 / mu))
    assert np.allclose(W.PAPER_GM.kappa, (eps ** 2, 0.0162 / mu))
    gs = W.initial_fields(W.PAPER_GS)
    c = np.argmin(np.abs(W.PAPER_GS.coords(0) - 0.5))
    assert gs[0, c, c] == 0.5 and gs[1, c, c] == 0.25 and gs[0, 0, 0] == 1.0
    sch = W.initial_fields(W.PAPER_SCHNAK)
    assert np.isclose(sch[0, 16, 16, 16], 0.0) and np.isclose(sch[1, 16, 16, 16], 1.0)
    assert np.isclose(sch[1, 16, 17, 16], np.exp(-10 * 2 * (10 / 32) ** 2))
