"""CPU pins of the min-cut oracle (oracle/mincut.py): brute force over every labelling
of tiny grids (value and the largest-object minimiser), the cut's energy equals the
flow on larger grids, closed forms without n-links and with dominating n-links, the
FP32 round-half-even quantisation, and planted mistakes."""
import numpy as np
import pytest

from oracle import mincut as MC


def _caps(rng, H, W, hi=10, pw_hi=6):
    cs = rng.integers(0, hi, (H, W)).astype(np.int64)
    ct = rng.integers(0, hi, (H, W)).astype(np.int64)
    pw = rng.integers(0, pw_hi, (4, H, W)).astype(np.int64)
    return cs, ct, pw


@pytest.mark.parametrize("H,W,seed", [(1, 5, 0), (2, 2, 1), (2, 3, 2), (3, 3, 3), (3, 4, 4), (4, 3, 5), (2, 6, 6)])
def test_brute_force_value_and_largest_object(H, W, seed):
    rng = np.random.default_rng(seed)
    for trial in range(4):
        cs, ct, pw = _caps(rng, H, W, hi=6 if trial % 2 else 10, pw_hi=3 if trial < 2 else 8)
        flow, lab = MC.min_cut(cs, ct, pw)
        best, union = MC.min_cut_brute(cs, ct, pw)
        assert flow == best
        assert np.array_equal(lab, union)
        assert MC.energy(lab, cs, ct, pw) == flow


@pytest.mark.parametrize("H,W,seed", [(16, 16, 7), (30, 40, 8), (9, 57, 9)])
def test_cut_energy_equals_flow(H, W, seed):
    rng = np.random.default_rng(seed)
    cs, ct, pw = _caps(rng, H, W, hi=200, pw_hi=60)
    left = (np.arange(W) < W // 2)[None, :]
    cs = cs + 250 * left          # the left half prefers the object, the right half the background
    ct = ct + 250 * ~left
    flow, lab = MC.min_cut(cs, ct, pw)
    assert 0 < lab.sum() < H * W   # the cut has a boundary
    assert MC.energy(lab, cs, ct, pw) == flow
    # flipping any single pixel never lowers the energy of a minimum cut
    for y, x in [(0, 0), (H // 2, W // 2), (H - 1, W - 1)]:
        l2 = lab.copy()
        l2[y, x] ^= 1
        assert MC.energy(l2, cs, ct, pw) >= flow


def test_ties_go_to_the_largest_object():
    # equal t-links and no n-links: every labelling is a minimum cut; the brute force and
    # the residual search both return the whole frame as object
    cs = np.full((3, 3), 4, np.int64)
    pw = np.zeros((4, 3, 3), np.int64)
    flow, lab = MC.min_cut(cs, cs.copy(), pw)
    best, union = MC.min_cut_brute(cs, cs.copy(), pw)
    assert flow == best == 36
    assert np.array_equal(lab, union) and np.all(lab == 1)
    # one n-link ring of equal costs: a tie between all-object and all-background
    pw2 = np.full((4, 2, 2), 3, np.int64)
    cs2 = np.array([[5, 0], [0, 5]], np.int64)
    ct2 = np.array([[0, 5], [5, 0]], np.int64)
    flow2, lab2 = MC.min_cut(cs2, ct2, pw2)
    best2, union2 = MC.min_cut_brute(cs2, ct2, pw2)
    assert flow2 == best2 and np.array_equal(lab2, union2)


def test_without_nlinks_each_pixel_takes_its_cheaper_label():
    rng = np.random.default_rng(10)
    cs, ct, _ = _caps(rng, 7, 9)
    pw = np.zeros((4, 7, 9), np.int64)
    flow, lab = MC.min_cut(cs, ct, pw)
    assert flow == int(np.minimum(cs, ct).sum())
    assert np.array_equal(lab, (ct <= cs).astype(np.uint8))   # ties go to the object


def test_dominating_nlinks_give_one_label():
    rng = np.random.default_rng(11)
    cs, ct, _ = _caps(rng, 5, 6)
    pw = np.full((4, 5, 6), 10_000, np.int64)
    flow, lab = MC.min_cut(cs, ct, pw)
    assert flow == min(int(cs.sum()), int(ct.sum()))
    assert np.all(lab == (1 if ct.sum() <= cs.sum() else 0))


def test_quantisation_rounds_half_to_even_in_fp32():
    q = MC.quantise(np.array([0.5, 1.5, 2.5, -3.0, 1e9, 0.49999997]), 1.0)
    assert q.tolist() == [0, 2, 2, 0, 1 << 24, 0]
    x = np.float32(0.1)
    assert MC.quantise(np.array([x]), 256.0)[0] == int(np.rint(np.float32(x) * np.float32(256.0)))


def test_planted_mistakes_fail_the_pins(monkeypatch):
    orig = MC.min_cut

    def smallest_object(cs, ct, pw):        # the minimal source side instead of the maximal
        flow, lab = orig(cs, ct, pw)
        H, W = cs.shape
        best = None
        for k in range(1 << (H * W)):
            l2 = np.array([(k >> i) & 1 for i in range(H * W)], np.uint8).reshape(H, W)
            if MC.energy(l2, cs, ct, pw) == flow and (best is None or l2.sum() < best.sum()):
                best = l2
        return flow, best
    monkeypatch.setattr(MC, "min_cut", smallest_object)
    with pytest.raises(AssertionError):
        test_ties_go_to_the_largest_object()
    monkeypatch.undo()
    monkeypatch.setattr(MC, "min_cut", lambda cs, ct, pw: orig(ct, cs, pw))   # t-links swapped
    with pytest.raises(AssertionError):
        test_without_nlinks_each_pixel_takes_its_cheaper_label()
    monkeypatch.undo()
    orig_e = MC.energy

    def double_pairs(labels, cs, ct, pw):   # each differing pair counted twice
        return orig_e(labels, cs, ct, 2 * pw) - orig_e(labels, cs, ct, 0 * pw) + orig_e(labels, cs, ct, 0 * pw)
    monkeypatch.setattr(MC, "energy", double_pairs)
    with pytest.raises(AssertionError):
        test_cut_energy_equals_flow(16, 16, 7)
