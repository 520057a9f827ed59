"""Stationary fluctuation statistics of the linearised update (test helper).

Around the rest state the update of the population deviations is linear:
one collision dfp = C df + B r (C, B from the oracle by differentiation), then
streaming, which at wavevector q multiplies population i by exp(-i q . c_i).
The stationary covariance at q solves the discrete Lyapunov equation
Sigma_q = A_q Sigma_q A_q^H + D_q B B^T D_q^H with A_q = D_q C.  The spatial
variance of a moment m = o . df is (1/N) sum over q of o Sigma_q o^T; the
equilibration ratio is that over the fluctuation-dissipation value o (mu W) o^T.
"""
import numpy as np
from scipy.linalg import solve_discrete_lyapunov

CS2 = 1.0 / 3.0
PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def linearised(ora, params, rho0=1.0, h=1e-6):
    w = ora.tables()["w"]
    f_rest = rho0 * w
    zero = np.zeros(23)
    name = {v: k for k, v in ora.MODELS.items()}[params.model]
    quiet = ora.make_params(kT=0.0, tau_shear=params.tau_shear, tau_bulk=params.tau_bulk,
                            tau_ghost=list(params.tau_ghost), model=name)
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


def observables():
    """Population-space vectors of rho, j_a and Pi_ab (xx, yy, zz, xy, xz, yz)."""
    i = np.arange(27)
    c = np.stack([i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1], axis=1).astype(np.float64)
    obs = {"rho": np.ones(27)}
    for a, name in enumerate("xyz"):
        obs["j" + name] = c[:, a]
    for a, b in PAIRS:
        obs["pi_" + "xyz"[a] + "xyz"[b]] = c[:, a] * c[:, b] - (CS2 if a == b else 0.0)
    return c, obs


def predicted_er(ora, params, dims, rho0=1.0):
    """ER of each observable (spatial variance over its FDT value), averaged over
    the wavevectors q != 0 of the periodic box.  Wavevectors where the linear
    update has an undamped mode (|eigenvalue| = 1; on even boxes the lattice's
    spurious invariants at q = (pi, 0, 0) and its permutations) are left out:
    there the stationary variance is set by the initial state, not the noise."""
    kT = params.kT
    cmat, bmat, w = linearised(ora, params, rho0)
    q_noise = bmat @ bmat.T
    c, obs = observables()
    sigma_th = rho0 * kT / CS2 * np.diag(w)
    o = np.stack(list(obs.values()))
    theory = np.einsum("ki,ij,kj->k", o, sigma_th, o)
    nx, ny, nz = dims
    total = np.zeros(len(obs))
    count = 0
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nx):
                if kx == ky == kz == 0:
                    continue
                q = 2 * np.pi * np.array([kx / nx, ky / ny, kz / nz])
                d = np.exp(-1j * (c @ q))
                a = d[:, None] * cmat
                if np.abs(np.linalg.eigvals(a)).max() > 1 - 1e-9:
                    continue
                qq = d[:, None] * q_noise * np.conj(d)[None, :]
                s = solve_discrete_lyapunov(a, qq)
                total += np.einsum("ki,ij,kj->k", o, s, o).real
                count += 1
    return dict(zip(obs, total / count / theory))
