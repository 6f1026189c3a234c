"""Host logic of the adaptive pruning and densification (no GPU)."""
import numpy as np

from paper_2503_16424_amd import adaptive as ad
from paper_2503_16424_amd import scenes


def _closed(ctrls, colors, opas, W=128, H=128, K=8, R=2):
    n = len(ctrls)
    return scenes._assemble(W, H, [1] * n, [1] * n, [K] * n, [R] * n,
                            [np.asarray(c, np.float64) for c in ctrls], np.zeros(n),
                            np.asarray(colors, np.float64), [[o] for o in opas], np.arange(n))


LENS = [[20, 40], [30, 30], [50, 30], [60, 40], [30, 50], [50, 50]]


def test_threshold_decreases_linearly():
    cfg = ad.AdaptiveConfig()
    assert ad.opacity_threshold(0, 1000, cfg) == cfg.opacity_start
    assert abs(ad.opacity_threshold(500, 1000, cfg) - 0.5 * (0.2 + 0.02)) < 1e-12
    assert abs(ad.opacity_threshold(1000, 1000, cfg) - cfg.opacity_end) < 1e-15


def test_pruning_criteria():
    far = (np.asarray(LENS) + [50, 50]).tolist()
    sc = _closed([LENS, LENS, far, far, (np.asarray(LENS) + [0, 60]).tolist()],
                 [[0.2, 0.3, 0.4], [0.21, 0.3, 0.4], [0.9, 0.1, 0.1], [0.1, 0.9, 0.1],
                  [0.5, 0.5, 0.5]],
                 [0.9, 0.9, 0.9, 0.9, 0.05])
    area = np.array([500.0, 500.0, 500.0, 2.0, 500.0])
    rep = ad.PassReport(step=0)
    keep = ad.prune_mask(sc, area, 0, 1000, ad.AdaptiveConfig(), rep)
    # 1 duplicates 0 (same box, colour distance 0.01): the later-drawn one goes;
    # 2 and 3 share a box but not a colour; 3 is too small; 4 is too faint
    assert keep.tolist() == [True, False, True, False, False]
    assert (rep.pruned_opacity, rep.pruned_area, rep.pruned_overlap) == (1, 1, 1)


def test_split_rule_and_subdivision():
    sc = scenes._assemble(64, 64, [0, 0], [3, 3], [12, 12], [0, 0],
                          [np.linspace([0, 0], [30, 30], 10), np.linspace([0, 5], [30, 35], 10)],
                          [2.0, 2.0], [[0.5] * 3] * 2, [[0.9, 0.1, 0.8], [0.9, 0.6, 0.9]], [0, 1])
    assert ad.split_candidates(sc, ad.AdaptiveConfig()) == [0]
    # subdividing a cubic reproduces it: the pieces meet the original at u = s / S
    P = np.array([[0.0, 0.0], [10.0, 30.0], [40.0, -10.0], [50.0, 20.0]])
    Q = ad._subdivide(P, 3)
    assert Q.shape == (10, 2)

    def bez(C, t):
        return ((1 - t) ** 3) * C[0] + 3 * (1 - t) ** 2 * t * C[1] + 3 * (1 - t) * t ** 2 * C[2] \
            + t ** 3 * C[3]
    for s in range(3):
        for t in (0.0, 0.3, 1.0):
            assert np.allclose(bez(Q[3 * s: 3 * s + 4], t), bez(P, (s + t) / 3.0), atol=1e-12)


def test_error_regions_largest_first():
    tgt = np.zeros((3, 40, 60))
    img = np.zeros((3, 40, 60))
    img[:, 5:15, 5:25] = 1.0          # 200 px
    img[:, 30:34, 40:44] = 1.0        # 16 px
    tgt[0] = 0.25
    regs = ad.error_regions(img, tgt, 0.5)
    assert [r[0] for r in regs] == [200, 16]
    assert abs(regs[0][1] - 15.0) < 1e-9 and abs(regs[0][2] - 10.0) < 1e-9
    assert np.allclose(regs[0][3], [0.25, 0.0, 0.0])


def test_pass_keeps_the_budget_and_puts_new_curves_in_front():
    sc = _closed([LENS, LENS, (np.asarray(LENS) + [40, 40]).tolist()],
                 [[0.2, 0.3, 0.4], [0.2, 0.3, 0.4], [0.5, 0.5, 0.5]], [0.9, 0.9, 0.9])
    sc.rank = np.array([2, 1, 0], np.int32)
    img = np.zeros((3, 128, 128))
    tgt = np.zeros((3, 128, 128))
    tgt[:, 90:110, 90:120] = 1.0
    out, rep = ad.adapt(sc, np.full(3, 500.0), img, tgt, 400, 1000, ad.AdaptiveConfig())
    assert out.n_curves == 3 and rep.added == 1 and rep.pruned_overlap == 1
    assert out.rank[0] == 0                       # the new curve is drawn first
    c = out.ctrl[out.ctrl_off[0]: out.ctrl_off[1]].astype(np.float64)
    assert np.allclose(c[[0, 3]].mean(0), [105.0, 100.0], atol=1.0)    # at the error region
    assert np.allclose(out.color[0], [1.0, 1.0, 1.0])
    # survivors keep their relative draw order (2 in front of 0)
    assert out.rank[1] > out.rank[0] and out.rank[2] > out.rank[0]
