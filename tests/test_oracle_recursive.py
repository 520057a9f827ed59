"""Pins of the oracle's recursive ghost non-equilibrium (Sec. II.B, Eq. recursive_eq).

Model "rec" rebuilds the non-equilibrium Hermite coefficients of the ghost
modes (orders 3..6) from the second-order ones and u by the recursion of
Eq. recursive_eq, and relaxes them with omega_g in Eq. r-flbe.  Checked here
against things other than the oracle's own recursion:

- the closed sum over index pairs that the recursion unrolls to;
- the continuous-velocity Hermite coefficients of the first-order
  Chapman-Enskog shape (a Gaussian shifted by u times a second-degree Hermite
  polynomial), which the recursion is built to reproduce, by Gauss-Hermite
  quadrature (numpy);
- the paper's setting omega_g = 1, where it must equal plain Reg-FLBM;
- the moments of the post-collision populations (the relaxed recursive
  coefficient lands on the ghost modes, nowhere else);
- the linearised fluctuation-dissipation residual, which for this reading has
  the closed form -mu b_k (1 - omega_g)^2 on each ghost mode (its deterministic
  ghost part is quadratic in the fluctuations, while Eq. fluct_phi scales the
  ghost noise by omega_g (2 - omega_g)).
"""
import itertools
import os

import numpy as np
import pytest

CS2 = 1.0 / 3.0
GOLD = os.path.join(os.path.dirname(__file__), "golden")
PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def index_strings():
    """Hermite subscripts of Table II (tests/golden/table2_hermite.txt)."""
    subs = {}
    with open(os.path.join(GOLD, "table2_hermite.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                k, sym = line.split()[:2]
                subs[int(k)] = "" if sym == "-" else sym
    return subs


def a2_matrix(a2v):
    a = np.zeros((3, 3))
    for v, (i, j) in zip(a2v, PAIRS):
        a[i, j] = a[j, i] = v
    return a


def pair_sum(sub, a2, u):
    """sum over index pairs i < j of a2[s_i, s_j] prod_{l != i, j} u[s_l]."""
    ax = ["xyz".index(ch) for ch in sub]
    total = 0.0
    for i, j in itertools.combinations(range(len(ax)), 2):
        term = a2[ax[i], ax[j]]
        for l in range(len(ax)):
            if l not in (i, j):
                term *= u[ax[l]]
        total += term
    return total


@pytest.mark.parametrize("seed", range(4))
def test_recursion_equals_sum_over_index_pairs(ora, seed):
    rng = np.random.default_rng(seed)
    a2v = rng.standard_normal(6)
    u = rng.uniform(-0.3, 0.3, 3)
    got = ora.ghost_recursive(a2v, u)
    subs = index_strings()
    a2 = a2_matrix(a2v)
    for k in range(10, 27):
        assert abs(got[k] - pair_sum(subs[k], a2, u)) < 1e-14, k
    assert not got[:10].any()


def hermite_1d(p, xi):
    """Degree-p factor of a Table II polynomial in a continuous velocity: 1, xi, xi^2 - cs2."""
    return np.ones_like(xi) if p == 0 else (xi if p == 1 else xi * xi - CS2)


@pytest.mark.parametrize("seed", range(3))
def test_recursion_reproduces_continuous_hermite_coefficients(ora, seed):
    """For f(xi) = M(xi - u) A : H2(xi - u) / (2 cs^4), M the unit Gaussian of
    variance cs2 per axis, the Hermite coefficient of every ghost polynomial
    (integral of f H_k over continuous velocities) equals the recursion's
    value; the quadrature is exact for these polynomial degrees."""
    rng = np.random.default_rng(50 + seed)
    a2v = rng.standard_normal(6)
    a2 = a2_matrix(a2v)
    u = rng.uniform(-0.2, 0.2, 3)
    t, wt = np.polynomial.hermite_e.hermegauss(8)  # weight exp(-t^2/2)
    x1 = np.sqrt(CS2) * t
    w1 = wt / np.sqrt(2 * np.pi)
    X, Y, Z = np.meshgrid(x1, x1, x1, indexing="ij")
    W = w1[:, None, None] * w1[None, :, None] * w1[None, None, :]
    x = [X, Y, Z]
    h2 = sum(a2[a, b] * (x[a] * x[b] - (CS2 if a == b else 0.0)) for a in range(3) for b in range(3))
    fw = W * h2 / (2 * CS2 ** 2)
    got = ora.ghost_recursive(a2v, u)
    subs = index_strings()
    for k in range(4, 27):
        p = [subs[k].count(ch) for ch in "xyz"]
        hk = hermite_1d(p[0], X + u[0]) * hermite_1d(p[1], Y + u[1]) * hermite_1d(p[2], Z + u[2])
        coef = float((fw * hk).sum())
        if k < 10:
            i, j = PAIRS[k - 4]
            assert abs(coef - a2[i, j]) < 1e-12  # a2 itself is the second-order coefficient
        else:
            assert abs(got[k] - coef) < 1e-12, k


def perturbed(ora, rng, amp=5e-3):
    rho = 1.0 + 0.05 * rng.uniform(-1, 1)
    u = 0.08 * rng.uniform(-1, 1, 3)
    w = ora.tables()["w"]
    return ora.equilibrium(rho, u) + amp * w * rng.standard_normal(27)


@pytest.mark.parametrize("seed", range(3))
def test_recursive_ghosts_equal_reg_at_unit_ghost_rate(ora, seed):
    """omega_g = 1 (the paper's setting): the relaxed ghost part vanishes in both
    readings, so "rec" and "reg" give the same post-collision populations."""
    rng = np.random.default_rng(seed)
    f = perturbed(ora, rng)
    r = rng.standard_normal(23)
    kw = dict(kT=1e-4, tau_shear=rng.uniform(0.51, 2), tau_bulk=rng.uniform(0.51, 2), tau_ghost=1.0)
    reg = ora.collide(ora.make_params(model="reg", **kw), f, r)
    rec = ora.collide(ora.make_params(model="rec", **kw), f, r)
    np.testing.assert_allclose(rec, reg, rtol=0, atol=1e-16)


@pytest.mark.parametrize("seed", range(3))
def test_recursive_ghost_moments_after_collision(ora, seed):
    """Without noise, the post-collision moments are: conserved ones unchanged,
    second-order ones as in Reg, ghosts at m_eq + (1 - omega_g,k) a1_rec,k."""
    rng = np.random.default_rng(20 + seed)
    f = perturbed(ora, rng, amp=2e-2)
    t = ora.tables()
    e, c = t["e"], t["c"].astype(np.float64)
    tau_g = rng.uniform(0.6, 1.9, 17)
    kw = dict(kT=0.0, tau_shear=0.8, tau_bulk=1.3, tau_ghost=tau_g)
    rec = ora.collide(ora.make_params(model="rec", **kw), f, np.zeros(23))
    reg = ora.collide(ora.make_params(model="reg", **kw), f, np.zeros(23))
    rho = f.sum()
    u = (c.T @ f) / rho
    feq = ora.equilibrium(rho, u)
    m_in, m_eq = e @ f, e @ feq
    a2v = (e @ (f - feq))[4:10]
    a_rec = ora.ghost_recursive(a2v, u)
    m_rec, m_reg = e @ rec, e @ reg
    np.testing.assert_allclose(m_rec[:4], m_in[:4], rtol=0, atol=1e-15)
    np.testing.assert_allclose(m_rec[4:10], m_reg[4:10], rtol=0, atol=1e-15)
    expect = m_eq[10:] + (1 - 1 / tau_g) * a_rec[10:]
    np.testing.assert_allclose(m_rec[10:], expect, rtol=0, atol=1e-15)
    # the reading differs from the projected (MRT) one when omega_g != 1
    assert np.abs(m_rec[10:] - m_reg[10:]).max() > 1e-6


def linearised(ora, params, rho0=1.0, h=1e-6):
    """C = d f*/d f at rest (central differences) and B with f*(r) - f*(0) = B r."""
    w = ora.tables()["w"]
    f_rest = rho0 * w
    zero = np.zeros(23)
    quiet = ora.make_params(kT=0.0, tau_shear=params.tau_shear, tau_bulk=params.tau_bulk,
                            tau_ghost=list(params.tau_ghost),
                            model={v: k for k, v in ora.MODELS.items()}[params.model])
    cmat = np.zeros((27, 27))
    for j in range(27):
        d = np.zeros(27)
        d[j] = h
        cmat[:, j] = (ora.collide(quiet, f_rest + d, zero) - ora.collide(quiet, f_rest - d, zero)) / (2 * h)
    base = ora.collide(params, f_rest, zero)
    bmat = np.zeros((27, 23))
    for k in range(23):
        r = np.zeros(23)
        r[k] = 1.0
        bmat[:, k] = ora.collide(params, f_rest, r) - base
    return cmat, bmat, w


@pytest.mark.parametrize("tau_g", [0.55, 1.25, 1.5 ** -1, 1.9])
def test_linearised_fdt_residual_closed_form(ora, tau_g):
    """At rest the recursive ghost coefficients are quadratic in the
    fluctuations, so the linear collision drives every ghost to 0 (as at
    omega_g = 1), while the ghost noise carries omega_g (2 - omega_g).  In
    moment space the one-collision Lyapunov residual C S C^T + B B^T - S,
    S = mu W, is therefore diagonal: 0 on modes 0..9 and -mu b_k (1 - omega_g)^2
    on each ghost."""
    kT, rho0 = 1e-4, 1.0
    p = ora.make_params(kT=kT, tau_shear=0.7, tau_bulk=1.1, tau_ghost=tau_g, model="rec")
    cmat, bmat, w = linearised(ora, p, rho0)
    t = ora.tables()
    e, b = t["e"], t["b"]
    mu = rho0 * kT / CS2
    sigma = mu * np.diag(w)
    resid = e @ (cmat @ sigma @ cmat.T + bmat @ bmat.T - sigma) @ e.T
    om = 1.0 / tau_g
    expect = np.zeros(27)
    expect[10:] = -mu * b[10:] * (1 - om) ** 2
    np.testing.assert_allclose(resid, np.diag(expect), rtol=0, atol=1e-9 * mu)
    # the deterministic linear part equals the one of Reg at omega_g = 1
    reg1 = ora.make_params(kT=kT, tau_shear=0.7, tau_bulk=1.1, tau_ghost=1.0, model="reg")
    creg, _, _ = linearised(ora, reg1, rho0)
    np.testing.assert_allclose(cmat, creg, rtol=0, atol=1e-9)
