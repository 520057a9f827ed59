"""Pins of the oracle's whole-lattice dynamics to the physics the paper fixes.

- shear-wave decay at the viscosity nu = cs2 (tau - 1/2) of Sec. II.A, and at
  the exact rate of the linearised lattice operator (numpy eigenvalues);
- equipartition: <d rho^2> = rho0 kT / cs2, <j_a^2> = rho0 kT, <u_a^2> = kT /
  rho0, <d Pi_aa^2> = mu b_4, <d Pi_ab^2> = mu b_7 (mu = rho0 kT / cs2), the
  variances of the modes under the stationary covariance mu w_i delta_ij that
  the fluctuation-dissipation balance of Eq. fluct_phi gives;
- a flat static structure factor S(|k|) of the normalised FFT (Sec. III).
"""
import numpy as np
import pytest

import workloads as wl

CS2 = 1.0 / 3.0


def shear_run(ora, tau, L, steps=200):
    dims = (2, 2, L)
    rho, u = wl.shear_wave(dims, 1e-3)
    f = ora.init_equilibrium(dims, rho, u)
    p = ora.make_params(kT=0.0, tau_shear=tau, tau_bulk=1.0)
    _, _, z = wl.grid(dims)
    s = np.sin(2 * np.pi * z / L)
    amps = []
    for t in range(steps + 1):
        m = ora.moments(f)
        amps.append(2 * np.mean(m["j"][0] / m["rho"] * s))
        if t < steps:
            f = ora.step(p, dims, f, t)
    amps = np.asarray(amps)
    t0 = steps // 4
    rate = -np.polyfit(np.arange(t0, steps + 1), np.log(amps[t0:]), 1)[0]
    return rate, p


def lattice_shear_rate(ora, params, L):
    """-ln|lambda| of the shear eigenmode of S(k) C at k = (0, 0, 2 pi / L)."""
    c = np.stack([np.arange(27) % 3 - 1, (np.arange(27) // 3) % 3 - 1, np.arange(27) // 9 - 1], 1)
    w = np.where(c == 0, 2 / 3, 1 / 6).prod(axis=1)
    h = 1e-6
    cmat = np.zeros((27, 27))
    for j in range(27):
        d = np.zeros(27)
        d[j] = h
        cmat[:, j] = (ora.collide(params, w + d, np.zeros(23)) -
                      ora.collide(params, w - d, np.zeros(23))) / (2 * h)
    k = 2 * np.pi / L
    # push streaming f_i(x + c_i) = f*_i(x): a plane wave picks up exp(-i k.c_i)
    a = np.diag(np.exp(-1j * k * c[:, 2])) @ cmat
    ev, vecs = np.linalg.eig(a)
    jx = np.abs(c[:, 0] @ vecs)  # x-momentum content of each eigenvector
    shear = np.argmax(jx * (np.abs(ev) > 0.5))
    return -np.log(np.abs(ev[shear]))


@pytest.mark.parametrize("tau,tol", [(0.8, 1e-3), (2.0, 1e-2), (0.55, 1e-3)])
def test_shear_wave_decays_at_lattice_viscosity(ora, tau, tol):
    L = 64
    rate, p = shear_run(ora, tau, L)
    nu_k2 = CS2 * (tau - 0.5) * (2 * np.pi / L) ** 2
    assert abs(rate / nu_k2 - 1) < tol
    assert abs(rate / lattice_shear_rate(ora, p, L) - 1) < 1e-5


def thermal_state(ora, dims, kT, seed, rho0=1.0):
    """Populations drawn from the stationary covariance: w_i rho0 + sqrt(mu w_i) xi."""
    w = ora.tables()["w"]
    n = int(np.prod(dims))
    xi = wl.normal_array((27, n), seed)
    return rho0 * w[:, None] + np.sqrt(rho0 * kT / CS2 * w)[:, None] * xi


def sample_run(ora, dims, params, f, steps, every, sk_every):
    acc = {"rho": [], "j": [], "u2": [], "pi_d": [], "pi_o": []}
    spectra = []
    for t in range(steps):
        if t % every == 0:
            m = ora.moments(f)
            acc["rho"].append(np.var(m["rho"]))
            acc["j"].append(np.mean(m["j"] ** 2, axis=1))
            acc["u2"].append(np.mean((m["j"] / m["rho"]) ** 2, axis=1))
            acc["pi_d"].append(np.var(m["pi"][:3], axis=1))
            acc["pi_o"].append(np.var(m["pi"][3:], axis=1))
            if t % sk_every == 0:
                spectra.append([ora.shell_spectrum(m["rho"], dims)[0],
                                sum(ora.shell_spectrum(m["j"][a], dims)[0] for a in range(3))])
        f = ora.step(params, dims, f, t)
    return {k: np.mean(v, axis=0) for k, v in acc.items()}, np.mean(spectra, axis=0)


@pytest.mark.parametrize("tau_s,tau_b", [(1.0, 1.0), (0.6, 1.0)])
def test_equipartition_and_flat_structure_factor(ora, tau_s, tau_b):
    dims = (16, 16, 16)
    kT, rho0 = 1e-4, 1.0
    p = ora.make_params(kT=kT, tau_shear=tau_s, tau_bulk=tau_b, seed=1)
    f = thermal_state(ora, dims, kT, seed=42)
    mean, spec = sample_run(ora, dims, p, f, steps=400, every=2, sk_every=20)
    mu = rho0 * kT / CS2
    np.testing.assert_allclose(mean["rho"] / (rho0 * kT / CS2), 1.0, atol=0.01)
    np.testing.assert_allclose(mean["j"] / (rho0 * kT), 1.0, atol=0.01)
    np.testing.assert_allclose(mean["u2"] / (kT / rho0), 1.0, atol=0.01)
    np.testing.assert_allclose(mean["pi_d"] / (mu * 2 / 9), 1.0, atol=0.01)
    np.testing.assert_allclose(mean["pi_o"] / (mu * 1 / 9), 1.0, atol=0.01)
    # flat S(|k|): every shell 1..13 of the density and momentum spectra
    _, counts = ora.shell_spectrum(np.zeros(int(np.prod(dims))), dims)
    nsnap = 400 // 20
    for field, theory in ((0, rho0 * kT / CS2), (1, 3 * rho0 * kT)):
        s = spec[field][1:14] / counts[1:14] / theory
        # each |F(n)|^2 of a real Gaussian field is exponential; n and -n are one
        # sample, so the shell mean has relative error sqrt(2 / count) per snapshot
        sig = np.sqrt(2.0 / (counts[1:14] * (3 if field else 1) * nsnap))
        assert np.all(np.abs(s - 1) < np.maximum(0.02, 5 * sig)), (field, s)


def test_zero_temperature_state_stays_deterministic(ora):
    dims = (4, 4, 4)
    rho, u = wl.random_velocity(dims, seed=3)
    f = ora.init_equilibrium(dims, rho, u)
    p = ora.make_params(kT=0.0, tau_shear=0.7, seed=1)
    q = ora.make_params(kT=0.0, tau_shear=0.7, seed=99)
    np.testing.assert_array_equal(ora.run(p, dims, f, 0, 5), ora.run(q, dims, f, 0, 5))


def test_lattice_conserves_mass_and_momentum(ora):
    dims = (5, 6, 7)
    rho, u = wl.random_velocity(dims, seed=4)
    f = ora.init_equilibrium(dims, rho, u)
    p = ora.make_params(kT=1e-4, tau_shear=0.55, tau_bulk=0.9, tau_ghost=1.3, seed=8)
    g = ora.run(p, dims, f, 0, 20)
    m0, m1 = ora.moments(f), ora.moments(g)
    assert abs(m1["rho"].sum() / m0["rho"].sum() - 1) < 1e-13
    np.testing.assert_allclose(m1["j"].sum(axis=1), m0["j"].sum(axis=1), rtol=0,
                               atol=1e-13 * m0["rho"].sum())


def test_streaming_moves_population_along_its_velocity(ora):
    """One step at tau = 1, kT = 0 from a state whose only non-uniformity is
    in f at one node: population i lands at x + c_i (Eq. eq:streaming)."""
    dims = (5, 4, 3)
    n = 60
    w = ora.tables()["w"]
    f = np.tile(w[:, None], (1, n))
    x0, y0, z0 = 1, 2, 0
    node = x0 + 5 * (y0 + 4 * z0)
    f[:, node] *= 1.01  # a pure density bump: f* = f0(1.01, 0) = 1.01 w
    p = ora.make_params(kT=0.0, tau_shear=1.0)
    g = ora.step(p, dims, f, 0)
    c = np.stack([np.arange(27) % 3 - 1, (np.arange(27) // 3) % 3 - 1, np.arange(27) // 9 - 1], 1)
    for i in range(27):
        xd, yd, zd = (x0 + c[i, 0]) % 5, (y0 + c[i, 1]) % 4, (z0 + c[i, 2]) % 3
        d = xd + 5 * (yd + 4 * zd)
        assert abs(g[i, d] - 1.01 * w[i]) < 1e-15
        others = np.delete(g[i], d)
        np.testing.assert_allclose(others, w[i], rtol=0, atol=1e-15)


def test_thermal_start_has_stationary_covariance(ora):
    """The thermalised start has mean f^(0) and covariance rho0 kT w_i / cs2
    per population, independent across populations and nodes."""
    dims = (24, 24, 24)
    kT, rho0 = 1e-4, 1.3
    p = ora.make_params(kT=kT, rho0=rho0, seed=9, stream_id=2)
    f = ora.init_thermal(p, dims)
    w = ora.tables()["w"]
    n = f.shape[1]
    d = f - rho0 * w[:, None]
    np.testing.assert_allclose(d.mean(axis=1) / np.sqrt(rho0 * kT / CS2 * w), 0, atol=5 / np.sqrt(n))
    var = d.var(axis=1) / (rho0 * kT / CS2 * w)
    np.testing.assert_allclose(var, 1, atol=5 * np.sqrt(2 / n))
    cc = np.corrcoef(d / np.sqrt(w)[:, None])
    assert np.abs(cc - np.eye(27)).max() < 5 / np.sqrt(n)
    # a different seed or stream gives a different draw
    q = ora.make_params(kT=kT, rho0=rho0, seed=9, stream_id=3)
    assert not np.array_equal(ora.init_thermal(q, dims), f)


def test_thermal_start_stays_thermal(ora):
    """Started from the stationary covariance, the equipartition ratios hold
    from the first step on (no transient)."""
    dims = (16, 16, 16)
    kT = 1e-4
    p = ora.make_params(kT=kT, tau_shear=0.6, tau_bulk=1.0, seed=4)
    f = ora.init_thermal(p, dims)
    mean, _ = sample_run(ora, dims, p, f, steps=60, every=2, sk_every=1000)
    np.testing.assert_allclose(mean["u2"] / kT, 1.0, atol=0.02)
    np.testing.assert_allclose(mean["rho"] / (kT / CS2), 1.0, atol=0.02)
