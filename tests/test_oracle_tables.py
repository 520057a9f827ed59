"""Pins of the oracle's lattice tables to Tables I and II of the paper (Sec. II).

Every check compares the oracle with something other than itself: the printed
tables under tests/golden/, closed-form identities of Hermite polynomials, or
linear-algebra identities the paper states (orthogonality, Eq. normal_fact,
the b_k / multiplicity relation, the inverse matrix of Eq. backtrasf).
"""
import math
import os

import numpy as np

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load_rows(name):
    rows = []
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_table1_velocity_classes_and_weights(ora):
    t = ora.tables()
    c = t["c"]
    assert set(np.unique(c)) == {-1, 0, 1}
    assert len({tuple(v) for v in c}) == 27
    c2 = (c ** 2).sum(axis=1)
    rows = load_rows("table1_d3q27.txt")
    assert sum(int(r[1]) for r in rows) == 27
    for cls, count, num, den in rows:
        sel = c2 == int(cls)
        assert sel.sum() == int(count)
        np.testing.assert_allclose(t["w"][sel], int(num) / int(den), rtol=0, atol=1e-16)
    # canonical order: population 26 - i is the opposite of i, 13 is the rest particle
    assert np.array_equal(c[::-1], -c)
    assert np.array_equal(c[13], [0, 0, 0])
    # isotropy of the weights: sum w = 1, sum w c_a c_b = cs2 delta_ab
    assert abs(t["w"].sum() - 1.0) < 1e-15
    np.testing.assert_allclose((t["w"][:, None, None] * c[:, :, None] * c[:, None, :]).sum(0),
                               np.eye(3) / 3.0, atol=1e-15)


def test_table2_orders_multiplicities_and_norms(ora):
    t = ora.tables()
    rows = load_rows("table2_hermite.txt")
    assert len(rows) == 27
    for k, sym, n, mu, bn, bd in rows:
        k, n, mu = int(k), int(n), int(mu)
        sub = "" if sym == "-" else sym
        assert t["order"][k] == n
        assert t["mult"][k] == mu
        # the order is the rank of the Hermite tensor, i.e. the subscript length
        assert len(sub) == n
        # the multiplicity counts the distinct orderings of the subscript
        counts = [sub.count(a) for a in "xyz"]
        assert mu == math.factorial(n) // math.prod(math.factorial(m) for m in counts)
        # b_k of Eq. normal_fact equals the printed value ...
        assert abs(t["b"][k] - int(bn) / int(bd)) < 1e-15
        # ... and the printed relation b_k = n_k! cs^(2 n_k) / mu_k
        assert abs(t["b"][k] - math.factorial(n) * (1.0 / 3.0) ** n / mu) < 1e-15
        # the Hermite-sum coefficient mu_k / (cs^(2n) n!) of Eq. hermite_feq2 is 1/b_k
        assert abs(t["hcoef"][k] * t["b"][k] - 1.0) < 1e-14


def test_table2_polynomials_match_hermite_symbols(ora):
    """e_ki (typed from the polynomial column) equals the Hermite tensor named
    by the symbol column: a product over axes of the scaled 1-D Hermite
    polynomials He_m(c / cs) cs^m, m the number of times the axis appears:
    1, c, c^2 - cs2 for m = 0, 1, 2."""
    t = ora.tables()
    c = t["c"].astype(np.float64)
    one_d = [lambda v: np.ones_like(v), lambda v: v, lambda v: v * v - 1.0 / 3.0]
    for k, sym, *_ in load_rows("table2_hermite.txt"):
        sub = "" if sym == "-" else sym
        expect = np.ones(27)
        for a, axis in enumerate("xyz"):
            expect *= one_d[sub.count(axis)](c[:, a])
        np.testing.assert_allclose(t["e"][int(k)], expect, rtol=0, atol=1e-15)


def test_orthogonality_inverse_and_completeness(ora):
    t = ora.tables()
    e, w, b = t["e"], t["w"], t["b"]
    # sum_i w_i e_ki e_li = b_k delta_kl (Sec. II.A)
    np.testing.assert_allclose(e @ np.diag(w) @ e.T, np.diag(b), atol=1e-15)
    # M^-1_ik = w_i e_ki / b_k is the inverse of M_ki = e_ki (Eq. backtrasf, Sec. II.B)
    minv = (w[:, None] * e.T) / b[None, :]
    np.testing.assert_allclose(minv @ e, np.eye(27), atol=1e-13)
    np.testing.assert_allclose(e @ minv, np.eye(27), atol=1e-13)
    # completeness: sum_k e_ki e_kj / b_k = delta_ij / w_i
    np.testing.assert_allclose(e.T @ np.diag(1.0 / b) @ e, np.diag(1.0 / w), atol=1e-12)


def test_conserved_modes_are_mass_and_momentum(ora):
    t = ora.tables()
    np.testing.assert_array_equal(t["e"][0], np.ones(27))
    for a in range(3):
        np.testing.assert_array_equal(t["e"][1 + a], t["c"][:, a])


def test_table3_fixture_matches_benchmark_taus():
    """The Table III fixture holds 14 taus, the ones the benchmark's Table III
    mode runs, with BGK values from tau = 0.505 on (Sec. III)."""
    import bench
    paper = bench.paper_table3()
    reg = sorted(t for m, t in paper if m == "reg")
    bgk = sorted(t for m, t in paper if m == "bgk")
    assert tuple(reg) == bench.TABLE3_TAUS
    assert tuple(bgk) == bench.TABLE3_TAUS[3:]
    assert paper[("reg", 0.5001)] == [1.037, 1.052, 1.072, 1.048]
    assert paper[("bgk", 50.0)] == [0.953, 1.001, 0.930, 1.000]
