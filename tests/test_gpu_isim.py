"""GPU parity of mc_isim (the ranking similarity of Sec. 6) with the CPU reference,
through the C ABI: random vectors with ties and signed zeros, every K from 1 to n,
a reversed ranking, and the error codes."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import rank
import paper_1904_12759_amd as mc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 2, 333, 5000])
def test_isim_matches_reference(n):
    rng = np.random.default_rng(n)
    x = np.round(rng.normal(size=n), 2)                 # ties
    y = np.round(x + rng.normal(scale=0.05, size=n), 2)
    x[: n // 10] = -0.0                                  # signed zeros among ties
    y[n // 20: n // 10] = 0.0
    for k in sorted({1, 2, max(1, n // 10), max(1, n // 2), n}):
        if k > n:
            continue
        g = mc.isim(x, y, k)
        c = rank.isim(x, y, k)
        assert g == pytest.approx(c, rel=1e-12, abs=1e-15), (n, k)
    assert mc.isim(x, x) == 0.0


def test_isim_reversed_and_large():
    n = 200_001
    x = np.arange(n, dtype=np.float64)
    h = n // 2
    expect = (h + sum((n - i) / i for i in range(h + 1, n + 1))) / n
    assert mc.isim(x, -x) == pytest.approx(expect, rel=1e-12)
    rng = np.random.default_rng(7)
    a = rng.random(n)
    b = a + rng.normal(scale=1e-3, size=n)
    assert mc.isim(a, b, n // 10) == pytest.approx(rank.isim(a, b, n // 10), rel=1e-12)


def test_isim_errors():
    x = np.arange(10, dtype=np.float64)
    with pytest.raises(mc.MCError) as ei:
        mc.isim(x, x, 0)
    assert ei.value.code == 1
    with pytest.raises(mc.MCError) as ei:
        mc.isim(x, x, 11)
    assert ei.value.code == 1
    y = x.copy()
    y[3] = np.nan
    with pytest.raises(mc.MCError) as ei:
        mc.isim(x, y)
    assert ei.value.code == 3


def test_isim_extreme_values_and_constant_vectors():
    """Keys across the whole double range (largest and smallest magnitudes of both
    signs, subnormals, signed zeros) in a vector longer than two sort tiles and not a
    multiple of one, and constant vectors (every node tied)."""
    rng = np.random.default_rng(11)
    n = 9001
    vals = np.array([-1.7e308, -1.0, -5e-324, -0.0, 0.0, 5e-324, 1e-300, 1.0, 1.7e308])
    x = rng.choice(vals, n)
    y = rng.choice(vals, n)
    for k in (1, 17, n // 3, n):
        assert mc.isim(x, y, k) == pytest.approx(rank.isim(x, y, k), rel=1e-12, abs=1e-15), k
    z = np.full(n, 3.5)
    assert mc.isim(z, z) == 0.0
    assert mc.isim(z, -np.arange(n, dtype=np.float64), n // 2) == \
        pytest.approx(rank.isim(z, -np.arange(n, dtype=np.float64), n // 2), rel=1e-12)
