"""Seeded synthetic inputs for the D3Q27 fluctuating lattice Boltzmann runs.

This module is shared by the GPU path's tests and benchmark and by the oracle
side.  It holds only input fields and tables drawn from seeded generators:
density and velocity fields (fluid at rest, transverse shear wave, Taylor-Green
vortex), standard-normal perturbation arrays, and the replica table of the
batched workload.  It contains none of the method's arithmetic (no weights,
no equilibrium, no moments): each side turns these fields into populations with
its own code.

Node order everywhere: n = x + nx*(y + ny*z); vector fields are returned as
arrays of shape (3, N).
"""
from __future__ import annotations

import numpy as np


def grid(dims):
    """Integer node coordinates (x, y, z), each of shape (N,), x fastest."""
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def rest(dims, rho0=1.0):
    """Uniform density rho0 and zero velocity."""
    n = int(np.prod(dims))
    return np.full(n, float(rho0)), np.zeros((3, n))


def shear_wave(dims, amp=0.01, rho0=1.0):
    """u_x = amp * sin(2 pi z / nz), u_y = u_z = 0, uniform density."""
    nx, ny, nz = dims
    x, y, z = grid(dims)
    rho, u = rest(dims, rho0)
    u[0] = amp * np.sin(2.0 * np.pi * z / nz)
    return rho, u


def taylor_green(dims, amp=0.01, rho0=1.0):
    """Taylor-Green vortex with one wavelength per box edge (node coordinates).

    u_x =  A sin(kx x) cos(ky y) cos(kz z)
    u_y = -A cos(kx x) sin(ky y) cos(kz z)
    u_z = 0,  k_a = 2 pi / n_a.
    """
    nx, ny, nz = dims
    sx, cx = np.sin(2 * np.pi * np.arange(nx) / nx), np.cos(2 * np.pi * np.arange(nx) / nx)
    sy, cy = np.sin(2 * np.pi * np.arange(ny) / ny), np.cos(2 * np.pi * np.arange(ny) / ny)
    cz = np.cos(2 * np.pi * np.arange(nz) / nz)
    rho, u = rest(dims, rho0)
    u[0] = (amp * sx[None, None, :] * cy[None, :, None] * cz[:, None, None]).ravel()
    u[1] = (-amp * cx[None, None, :] * sy[None, :, None] * cz[:, None, None]).ravel()
    return rho, u


def taylor_green_device(dims, amp=0.01, rho0=1.0, device="cuda"):
    """taylor_green built in device memory with torch (for large boxes).

    The same 1-D factors are multiplied in the same order in FP64, so the
    values equal those of taylor_green.  Returns (rho, u) torch tensors of
    shapes (N,) and (3, N).
    """
    import torch

    nx, ny, nz = dims
    f = lambda a: torch.as_tensor(a, dtype=torch.float64, device=device)
    sx, cx = f(np.sin(2 * np.pi * np.arange(nx) / nx)), f(np.cos(2 * np.pi * np.arange(nx) / nx))
    sy, cy = f(np.sin(2 * np.pi * np.arange(ny) / ny)), f(np.cos(2 * np.pi * np.arange(ny) / ny))
    cz = f(np.cos(2 * np.pi * np.arange(nz) / nz))
    n = nx * ny * nz
    u = torch.zeros((3, n), dtype=torch.float64, device=device)
    u[0] = (amp * sx[None, None, :] * cy[None, :, None] * cz[:, None, None]).reshape(n)
    u[1] = (-amp * cx[None, None, :] * sy[None, :, None] * cz[:, None, None]).reshape(n)
    rho = torch.full((n,), float(rho0), dtype=torch.float64, device=device)
    return rho, u


def normal_array(shape, seed):
    """Standard normal numbers from numpy's PCG64 with the given seed."""
    return np.random.default_rng(seed).standard_normal(shape)


def random_velocity(dims, seed, amp=0.02, rho_amp=0.01, rho0=1.0):
    """Smooth-free random density and velocity fields (for parity tests)."""
    n = int(np.prod(dims))
    g = np.random.default_rng(seed)
    rho = rho0 * (1.0 + rho_amp * g.uniform(-1.0, 1.0, n))
    u = amp * g.uniform(-1.0, 1.0, (3, n))
    return rho, u


def replica_table(n=64, seed=5, edges=(32, 48, 64, 96), tau=(0.55, 1.2), log_kt=(-6.0, -4.0)):
    """The batched workload: box edge, tau, kT, Philox seed and stream per replica.

    Edge uniform on ``edges``; tau (shear = bulk) uniform in ``tau``; kT
    log-uniform in 10**``log_kt``; seed 1000 + r; stream id r; ghosts at tau 1.
    """
    g = np.random.default_rng(seed)
    edge = g.choice(np.asarray(edges), size=n)
    taus = g.uniform(tau[0], tau[1], size=n)
    kts = 10.0 ** g.uniform(log_kt[0], log_kt[1], size=n)
    return [dict(dims=(int(e), int(e), int(e)), tau=float(t), kT=float(k), seed=1000 + r,
                 stream_id=r) for r, (e, t, k) in enumerate(zip(edge, taus, kts))]
