"""Pins of the CPU ranking-similarity reference (oracle/rank.py): values worked by
hand from the definition of isim_K (Sec. 6), the closed form of a reversed ranking,
identity, symmetry, bounds, the tie rule, and a set-based brute force."""
import numpy as np
import pytest

from oracle import rank


def test_hand_worked_example():
    # x ranks nodes 0,1,2,3; y ranks 1,0,3,2:
    # i=1: {0} vs {1} -> |delta| 2 -> 2/2; i=2: equal; i=3: {0,1,2} vs {0,1,3} -> 2/6; i=4: equal
    x = [4.0, 3.0, 2.0, 1.0]
    y = [3.0, 4.0, 1.0, 2.0]
    assert rank.isim(x, y) == pytest.approx((1.0 + 0.0 + 1.0 / 3.0 + 0.0) / 4.0, rel=1e-15)
    assert rank.isim(x, y, 2) == pytest.approx(0.5, rel=1e-15)
    assert rank.isim(x, y, 1) == 1.0


@pytest.mark.parametrize("n", [1, 2, 7, 10, 101])
def test_reversed_ranking_closed_form(n):
    x = np.arange(n, dtype=float)
    y = -x
    h = n // 2
    expect = (h + sum((n - i) / i for i in range(h + 1, n + 1))) / n
    assert rank.isim(x, y) == pytest.approx(expect, rel=1e-13)


def test_identity_symmetry_bounds():
    rng = np.random.default_rng(1)
    for _ in range(20):
        n = int(rng.integers(1, 60))
        x = rng.normal(size=n)
        y = x + rng.normal(scale=0.3, size=n)
        for k in (1, max(1, n // 3), n):
            assert rank.isim(x, x, k) == 0.0
            a, b = rank.isim(x, y, k), rank.isim(y, x, k)
            assert a == pytest.approx(b, rel=1e-15, abs=1e-15)
            assert 0.0 <= a <= 1.0


def test_tie_rule_and_signed_zero():
    assert list(rank.ranking([1.0, 1.0, 0.0, 2.0])) == [3, 0, 1, 2]
    assert list(rank.ranking([0.0, -0.0, -1.0])) == [0, 1, 2]
    assert list(rank.ranking([-0.0, 0.0, -1.0])) == [0, 1, 2]
    assert rank.isim([0.0, -0.0], [-0.0, 0.0]) == 0.0


def test_matches_set_brute_force():
    rng = np.random.default_rng(2)
    for _ in range(30):
        n = int(rng.integers(1, 40))
        x = np.round(rng.normal(size=n), 1)       # ties
        y = np.round(rng.normal(size=n), 1)
        k = int(rng.integers(1, n + 1))
        ox = sorted(range(n), key=lambda j: (-x[j], j))
        oy = sorted(range(n), key=lambda j: (-y[j], j))
        brute = sum(len(set(ox[:i]) ^ set(oy[:i])) / (2.0 * i) for i in range(1, k + 1)) / k
        assert rank.isim(x, y, k) == pytest.approx(brute, rel=1e-14, abs=1e-15)


def test_rejects_bad_input():
    with pytest.raises(ValueError):
        rank.isim([1.0, np.nan], [1.0, 2.0])
    with pytest.raises(ValueError):
        rank.isim([1.0, 2.0], [1.0, 2.0], 3)
