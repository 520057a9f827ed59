"""Pins of the oracle's equilibrium and collision (Sec. II) to closed forms.

- equilibrium: the product form of the full-Hermite equilibrium, its
  second-order truncation equal to Eq. classicfeq, and its first moments;
- collision: exact mass and momentum conservation, the tau = 1 limit, the
  zero-noise limit against the textbook population-space regularisation
  (f* = f0 + (1 - omega) w_i H2_i : Pi_neq / (2 cs^4)), equality of Reg and BGK
  when the non-equilibrium part is purely second order, and the linearised
  fluctuation-dissipation balance (the discrete Lyapunov equation
  C (mu W) C^T + Q = mu W, which fixes every noise amplitude of Eq. fluct_phi).
"""
import numpy as np
import pytest

CS2 = 1.0 / 3.0


def vel():
    i = np.arange(27)
    return np.stack([i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1], axis=1).astype(np.float64)


def axis_weight(ca):
    return np.where(ca == 0, 2.0 / 3.0, 1.0 / 6.0)


def product_form(rho, u):
    """rho prod_a w1(c_a) [1 + c_a u_a / cs2 + (c_a^2 - cs2) u_a^2 / (2 cs2^2)]."""
    c = vel()
    out = rho * np.ones(27)
    for a in range(3):
        ca = c[:, a]
        out *= axis_weight(ca) * (1 + ca * u[a] / CS2 + (ca * ca - CS2) * u[a] ** 2 / (2 * CS2 ** 2))
    return out


def classic_feq(rho, u):
    """Eq. classicfeq."""
    c = vel()
    w = axis_weight(c[:, 0]) * axis_weight(c[:, 1]) * axis_weight(c[:, 2])
    cu = c @ u
    return w * rho * (1 + cu / CS2 + cu ** 2 / (2 * CS2 ** 2) - (u @ u) / (2 * CS2))


def random_state(rng, amp=0.05):
    rho = 1.0 + 0.05 * rng.uniform(-1, 1)
    u = 0.05 * rng.uniform(-1, 1, 3)
    return rho, u


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_product_form(ora, seed):
    rho, u = random_state(np.random.default_rng(seed))
    np.testing.assert_allclose(ora.equilibrium(rho, u), product_form(rho, u), rtol=0, atol=1e-15)


def test_equilibrium_second_order_truncation_is_classic(ora):
    # f0(eps u) - classic(eps u) = O(eps^3): the ratio to eps^3 converges.
    rng = np.random.default_rng(7)
    u = rng.uniform(-1, 1, 3)
    ratios = []
    for eps in (1e-2, 5e-3):
        d = ora.equilibrium(1.0, eps * u) - classic_feq(1.0, eps * u)
        ratios.append(d / eps ** 3)
    np.testing.assert_allclose(ratios[0], ratios[1], rtol=0, atol=2e-2 * np.abs(ratios[1]).max())
    assert np.abs(ratios[1]).max() > 1e-3  # the cubic term is really there


@pytest.mark.parametrize("seed", range(3))
def test_equilibrium_moments(ora, seed):
    rho, u = random_state(np.random.default_rng(100 + seed))
    f = ora.equilibrium(rho, u)
    c = vel()
    assert abs(f.sum() - rho) < 1e-15
    np.testing.assert_allclose(c.T @ f, rho * u, atol=1e-16)
    second = np.einsum("i,ia,ib->ab", f, c, c)
    np.testing.assert_allclose(second, rho * np.outer(u, u) + rho * CS2 * np.eye(3), atol=1e-15)


def perturbed(ora, rng, amp=1e-3):
    rho, u = random_state(rng)
    f0 = ora.equilibrium(rho, u)
    c = vel()
    w = axis_weight(c[:, 0]) * axis_weight(c[:, 1]) * axis_weight(c[:, 2])
    return f0 + amp * w * rng.standard_normal(27)


@pytest.mark.parametrize("model", ["reg", "bgk"])
@pytest.mark.parametrize("seed", range(4))
def test_collision_conserves_mass_and_momentum(ora, model, seed):
    rng = np.random.default_rng(seed)
    f = perturbed(ora, rng)
    p = ora.make_params(kT=1e-4, tau_shear=rng.uniform(0.51, 3), tau_bulk=rng.uniform(0.51, 3),
                        tau_ghost=rng.uniform(0.6, 2, 17), model=model)
    out = ora.collide(p, f, rng.standard_normal(23))
    c = vel()
    assert abs(out.sum() - f.sum()) < 1e-15
    np.testing.assert_allclose(c.T @ out, c.T @ f, rtol=0, atol=1e-16)


@pytest.mark.parametrize("model", ["reg", "bgk"])
def test_tau_one_no_noise_gives_equilibrium(ora, model):
    rng = np.random.default_rng(3)
    f = perturbed(ora, rng, amp=1e-2)
    c = vel()
    rho = f.sum()
    u = (c.T @ f) / rho
    p = ora.make_params(kT=0.0, tau_shear=1.0, model=model)
    np.testing.assert_allclose(ora.collide(p, f, np.zeros(23)), product_form(rho, u),
                               rtol=0, atol=1e-15)


@pytest.mark.parametrize("tau", [0.5001, 0.6, 0.8, 1.7, 100.0])
def test_zero_noise_is_textbook_regularisation(ora, tau):
    """kT = 0, ghosts at omega_g = 1: Eq. r-flbe2 reduces to the population-space
    regularised update f* = f0 + (1 - omega) w_i /(2 cs^4) H2_i,ab Pi_neq,ab,
    Pi_neq,ab = sum_i (f_i - f0_i) c_ia c_ib."""
    rng = np.random.default_rng(11)
    f = perturbed(ora, rng, amp=5e-3)
    c = vel()
    rho = f.sum()
    u = (c.T @ f) / rho
    f0 = product_form(rho, u)
    pi_neq = np.einsum("i,ia,ib->ab", f - f0, c, c)
    h2 = np.einsum("ia,ib->iab", c, c) - CS2 * np.eye(3)[None]
    w = axis_weight(c[:, 0]) * axis_weight(c[:, 1]) * axis_weight(c[:, 2])
    expect = f0 + (1 - 1 / tau) * w / (2 * CS2 ** 2) * np.einsum("iab,ab->i", h2, pi_neq)
    p = ora.make_params(kT=0.0, tau_shear=tau)
    np.testing.assert_allclose(ora.collide(p, f, np.zeros(23)), expect, rtol=0, atol=2e-15)


def test_reg_equals_bgk_for_second_order_nonequilibrium(ora):
    """If f - f0 lies in the span of the second-order Hermite modes, projecting
    it (regularisation) changes nothing, so Reg and BGK give the same update."""
    rng = np.random.default_rng(5)
    rho, u = random_state(rng)
    c = vel()
    w = axis_weight(c[:, 0]) * axis_weight(c[:, 1]) * axis_weight(c[:, 2])
    h2 = np.einsum("ia,ib->iab", c, c) - CS2 * np.eye(3)[None]
    a = rng.standard_normal((3, 3)) * 1e-3
    a = a + a.T
    f = ora.equilibrium(rho, u) + w / (2 * CS2 ** 2) * np.einsum("iab,ab->i", h2, a)
    for tau in (0.55, 2.0):
        reg = ora.collide(ora.make_params(tau_shear=tau, model="reg"), f, np.zeros(23))
        bgk = ora.collide(ora.make_params(tau_shear=tau, model="bgk"), f, np.zeros(23))
        np.testing.assert_allclose(reg, bgk, rtol=0, atol=1e-15)


def linearised(ora, params, rho0=1.0, h=1e-6):
    """C = d f* / d f at the rest state (central differences) and the noise
    matrix B with f*(r) - f*(0) = B r at the rest state."""
    c = vel()
    w = axis_weight(c[:, 0]) * axis_weight(c[:, 1]) * axis_weight(c[:, 2])
    f_rest = rho0 * w
    zero = np.zeros(23)
    cmat = np.zeros((27, 27))
    quiet = ora.make_params(kT=0.0, tau_shear=params.tau_shear, tau_bulk=params.tau_bulk,
                            tau_ghost=list(params.tau_ghost), model=("reg", "bgk")[params.model])
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


@pytest.mark.parametrize("model,tau_s,tau_b,tau_g,rho0", [
    ("reg", 1.0, 1.0, 1.0, 1.0),
    ("reg", 0.8, 1.0, 1.0, 1.0),
    ("reg", 0.5001, 0.5001, 1.0, 1.0),
    ("reg", 100.0, 100.0, 1.0, 1.0),
    ("reg", 0.6, 2.5, 1.5, 2.5),
    ("reg", 0.7, 0.7, 1.0, 0.4),
    ("bgk", 0.7, 0.7, 1.0, 1.7),
])
def test_linear_fluctuation_dissipation_balance(ora, model, tau_s, tau_b, tau_g, rho0):
    """With Sigma = mu W, mu = rho0 kT / cs2 (the equilibrium covariance of the
    populations), one collision maps Sigma to itself: C Sigma C^T + B B^T = Sigma.
    Streaming is a permutation in real space (a diagonal phase in Fourier
    space) and leaves diagonal Sigma unchanged, so this holds at every
    wavevector.  A wrong b_k, omega(2 - omega) factor or projector fails it."""
    kT = 1e-4
    p = ora.make_params(kT=kT, tau_shear=tau_s, tau_bulk=tau_b, tau_ghost=tau_g, model=model)
    cmat, bmat, w = linearised(ora, p, rho0=rho0)
    sigma = (rho0 * kT / CS2) * np.diag(w)
    resid = cmat @ sigma @ cmat.T + bmat @ bmat.T - sigma
    assert np.abs(resid).max() < 1e-9 * (rho0 * kT / CS2)


@pytest.mark.parametrize("rho", [0.5, 1.0, 3.0])
def test_noise_covariance_scales_with_local_density(ora, rho):
    """phi_k^2 is proportional to the density of the node (Eq. fluct_phi): the
    covariance of the injected noise at a node of density rho is rho times the
    one at density 1, whatever the reference density."""
    p = ora.make_params(kT=1e-4, tau_shear=0.7, tau_bulk=1.1, tau_ghost=1.4, rho0=1.0)
    _, b1, _ = linearised(ora, p, rho0=1.0)
    _, br, _ = linearised(ora, p, rho0=rho)
    np.testing.assert_allclose(br @ br.T, rho * (b1 @ b1.T), rtol=0, atol=1e-14)


def test_linear_collision_spectrum(ora):
    """The linearised Reg collision has eigenvalue 1 on the 4 conserved modes,
    1 - omega_s on the 5 deviatoric second-order modes, 1 - omega_b on the
    trace, and 1 - omega_g on the 17 ghosts."""
    tau_s, tau_b, tau_g = 0.8, 1.3, 1.6
    p = ora.make_params(kT=0.0, tau_shear=tau_s, tau_bulk=tau_b, tau_ghost=tau_g)
    cmat, _, _ = linearised(ora, p)
    ev = np.sort(np.linalg.eigvals(cmat).real)
    expect = np.sort([1.0] * 4 + [1 - 1 / tau_s] * 5 + [1 - 1 / tau_b] + [1 - 1 / tau_g] * 17)
    np.testing.assert_allclose(ev, expect, atol=1e-8)
