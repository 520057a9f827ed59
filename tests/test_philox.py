"""Checks of the oracle's counter-based normal generator.

The paper does not name its random number generator.  This build uses
Philox4x32-R (Salmon et al., SC'11) with Box-Muller; no published known-answer
vectors are available in this environment, so the bit stream itself is parity
unpinned.  What is checked here: the uniforms lie on the 24-bit grid and are
uniform, the normals have the moments and distribution of N(0, 1), the Box-Muller
pairing follows the documented counter layout, and draws at neighbouring
counters (node, step, call) are uncorrelated.
"""
import numpy as np
import pytest
from scipy import stats


def draw(ora, nodes, step=0, seed=1, stream=0, rounds=10):
    return np.array([ora.normals(seed, stream, rounds, n, step) for n in nodes])


def test_uniforms_on_24_bit_grid(ora):
    u = np.concatenate([ora.uniforms(7, 0, 10, n, 3) for n in range(2000)])
    q = u * 2 ** 24 - 1
    np.testing.assert_array_equal(q, np.round(q))
    assert u.min() > 0 and u.max() <= 1
    # every value is exact in single precision (24-bit significand)
    np.testing.assert_array_equal(u.astype(np.float32).astype(np.float64), u)
    assert stats.kstest(u, "uniform").pvalue > 1e-4


def test_box_muller_pairing(ora):
    for n in range(50):
        u = ora.uniforms(3, 1, 10, n, 9)
        z = ora.normals(3, 1, 10, n, 9)
        r2 = z[0::2] ** 2 + z[1::2] ** 2
        np.testing.assert_allclose(r2, -2 * np.log(u[0::2]), rtol=1e-13)
        ang = np.arctan2(z[1::2], z[0::2]) % (2 * np.pi)
        np.testing.assert_allclose(ang, (2 * np.pi * u[1::2]) % (2 * np.pi), atol=1e-9)


def test_normal_moments_and_distribution(ora):
    z = draw(ora, range(20000))[:, :23].ravel()
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(stats.kurtosis(z)) < 5 * np.sqrt(24 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_per_mode_normals_are_standard(ora):
    z = draw(ora, range(20000))
    for k in range(23):
        assert abs(z[:, k].mean()) < 5 / np.sqrt(len(z))
        assert abs(z[:, k].var() - 1) < 5 * np.sqrt(2 / len(z))


@pytest.mark.parametrize("which", ["node", "step", "mode", "stream"])
def test_neighbouring_counters_uncorrelated(ora, which):
    m = 8000
    if which == "node":
        a, b = draw(ora, range(0, 2 * m, 2)), draw(ora, range(1, 2 * m, 2))
    elif which == "step":
        a, b = draw(ora, range(m), step=5), draw(ora, range(m), step=6)
    elif which == "stream":
        a, b = draw(ora, range(m), stream=0), draw(ora, range(m), stream=1)
    else:
        z = draw(ora, range(m))
        a, b = z[:, :-1], z[:, 1:]
    r = np.corrcoef(a.ravel(), b.ravel())[0, 1]
    assert abs(r) < 5 / np.sqrt(a.size)


def test_key_rounds_and_determinism(ora):
    base = ora.normals(1, 0, 10, 123, 4)
    np.testing.assert_array_equal(base, ora.normals(1, 0, 10, 123, 4))
    assert not np.array_equal(base, ora.normals(2, 0, 10, 123, 4))
    assert not np.array_equal(base, ora.normals(1 + (1 << 32), 0, 10, 123, 4))  # high key word
    assert not np.array_equal(base, ora.normals(1, 0, 7, 123, 4))
    out = ora.philox4x32([0, 0, 0, 0], [0, 0], 10)
    assert out.dtype == np.uint32 and np.any(out != 0)


def test_seven_round_variant_is_also_normal(ora):
    z = draw(ora, range(10000), rounds=7)[:, :23].ravel()
    assert stats.kstest(z, "norm").pvalue > 1e-4
