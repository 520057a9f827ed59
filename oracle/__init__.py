"""FP64 CPU oracle of the Reg-FLBM D3Q27 update (arXiv:2507.08820).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does, and this
package imports nothing from it.

The arithmetic lives in ``rflbm_oracle.c`` (plain C, FP64, dense 27x27 Hermite
matrix typed in from Table II, OpenMP over nodes).  This module only marshals
numpy arrays into it, plus the observables of Sec. III written with numpy:
moments rho, rho*u and Pi = a0^(2) + a1^(2) (Eqs. eq:rho, eq:u, and the
definition of Pi after Table III), and the shell-averaged spectrum of a
normalised FFT.

Lattice layout everywhere here: ``f[i, n]`` with ``n = x + nx*(y + ny*z)`` and
the canonical population order ``c_i = (i%3-1, (i//3)%3-1, i//9-1)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rflbm_oracle.c")
# RFLBM_ORACLE_LIBRARY names another build of the same source (the
# sanitizer build of the CPU tests); it is loaded as is, never rebuilt here.
_LIB_OVERRIDE = os.environ.get("RFLBM_ORACLE_LIBRARY")
_LIB_PATH = _LIB_OVERRIDE or os.path.join(_HERE, "liboracle.so")
_lib = None
# clang, whose AddressSanitizer runtime is the one the HIP toolchain also ships
SANITIZE_CC = "/opt/rocm/llvm/bin/clang"
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined",
                  "-shared-libsan", "-g"]

CS2 = 1.0 / 3.0


def build(verbose: bool = False, sanitize: bool = False, out: str | None = None) -> str:
    """Compile the oracle with gcc (OpenMP).  Always recompiles.  sanitize:
    AddressSanitizer and UndefinedBehaviorSanitizer build with clang into
    `out` (load it with clang's ASan runtime preloaded)."""
    out = out or os.path.join(_HERE, "liboracle.so")
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    if sanitize:
        cmd = [SANITIZE_CC, "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp", *SANITIZE_FLAGS,
               "-o", out + ".tmp", _SRC, "-lm"]
    else:
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-o", out + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    global _lib
    if out == _LIB_PATH:
        _lib = None
    return out


# Collision models: Reg-FLBM (Eq. r-flbe2), BGK-FLBM (Eq. flbe), and Reg-FLBM
# whose ghost non-equilibrium is rebuilt by the recursion of Eq. recursive_eq.
MODELS = {"reg": 0, "bgk": 1, "rec": 2}


class Params(ctypes.Structure):
    """Mirror of ``ora_params`` in rflbm_oracle.c."""

    _fields_ = [
        ("rho0", ctypes.c_double),
        ("kT", ctypes.c_double),
        ("tau_shear", ctypes.c_double),
        ("tau_bulk", ctypes.c_double),
        ("tau_ghost", ctypes.c_double * 17),
        ("seed", ctypes.c_uint64),
        ("stream_id", ctypes.c_uint32),
        ("rounds", ctypes.c_uint32),
        ("model", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


def make_params(kT=0.0, tau_shear=1.0, tau_bulk=None, tau_ghost=1.0, seed=1, stream_id=0,
                rounds=7, model="reg", rho0=1.0) -> Params:
    p = Params()
    p.rho0 = rho0
    p.kT = kT
    p.tau_shear = tau_shear
    p.tau_bulk = tau_shear if tau_bulk is None else tau_bulk
    tg = np.broadcast_to(np.asarray(tau_ghost, dtype=np.float64), (17,))
    for k in range(17):
        p.tau_ghost[k] = float(tg[k])
    p.seed = seed
    p.stream_id = stream_id
    p.rounds = rounds
    p.model = MODELS[model]
    return p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not _LIB_OVERRIDE and (not os.path.exists(_LIB_PATH)
                              or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.ora_tables.argtypes = [i32p, dp, dp, dp, dp, i32p, i32p]
    lib.ora_philox4x32.argtypes = [u32p, u32p, ctypes.c_uint32, u32p]
    lib.ora_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_uint32, ctypes.c_uint32, dp]
    lib.ora_normals.argtypes = lib.ora_uniforms.argtypes
    lib.ora_equilibrium.argtypes = [ctypes.c_double, dp, dp]
    lib.ora_collide.argtypes = [ctypes.POINTER(Params), dp, dp, dp]
    lib.ora_ghost_recursive.argtypes = [dp, dp, dp]
    lib.ora_step.argtypes = [ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_int32,
                             ctypes.c_int32, ctypes.c_uint32, dp, dp, ctypes.c_int32]
    lib.ora_step.restype = ctypes.c_int
    lib.ora_run.argtypes = [ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_int32,
                            ctypes.c_int32, ctypes.c_uint32, ctypes.c_int32, dp, dp,
                            ctypes.c_int32]
    lib.ora_run.restype = ctypes.c_int
    lib.ora_init_equilibrium.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, dp, dp,
                                         dp]
    lib.ora_init_equilibrium.restype = ctypes.c_int
    lib.ora_init_thermal.argtypes = [ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, dp, dp, dp]
    lib.ora_init_thermal.restype = ctypes.c_int
    lib.ora_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u32p(a: np.ndarray):
    assert a.dtype == np.uint32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def tables() -> dict:
    """Velocities, weights, Hermite matrix e[k, i], b_k, mu_k/(cs^2n n!), n_k, mu_k."""
    lib = _load()
    c = np.zeros((27, 3), np.int32)
    w = np.zeros(27)
    e = np.zeros((27, 27))
    b = np.zeros(27)
    hc = np.zeros(27)
    order = np.zeros(27, np.int32)
    mult = np.zeros(27, np.int32)
    i32 = ctypes.POINTER(ctypes.c_int32)
    lib.ora_tables(c.ctypes.data_as(i32), _dp(w), _dp(e), _dp(b), _dp(hc),
                   order.ctypes.data_as(i32), mult.ctypes.data_as(i32))
    return dict(c=c, w=w, e=e, b=b, hcoef=hc, order=order, mult=mult)


def philox4x32(ctr, key, rounds=10) -> np.ndarray:
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib.ora_philox4x32(_u32p(c), _u32p(k), rounds, _u32p(out))
    return out


def uniforms(seed, stream_id, rounds, node, step) -> np.ndarray:
    lib = _load()
    out = np.zeros(24)
    lib.ora_uniforms(seed, stream_id, rounds, node, step, _dp(out))
    return out


def normals(seed, stream_id, rounds, node, step) -> np.ndarray:
    """The 24 Box-Muller normals of one node and step; r_k = z[k-4], k = 4..26."""
    lib = _load()
    out = np.zeros(24)
    lib.ora_normals(seed, stream_id, rounds, node, step, _dp(out))
    return out


def equilibrium(rho: float, u) -> np.ndarray:
    lib = _load()
    uu = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(27)
    lib.ora_equilibrium(float(rho), _dp(uu), _dp(out))
    return out


def collide(params: Params, f, r) -> np.ndarray:
    """Post-collision populations of one node; r holds the 23 normals r_4..r_26."""
    lib = _load()
    ff = np.ascontiguousarray(f, dtype=np.float64)
    rr = np.zeros(24)
    rr[:23] = np.asarray(r, dtype=np.float64)[:23]
    out = np.zeros(27)
    lib.ora_collide(ctypes.byref(params), _dp(ff), _dp(rr), _dp(out))
    return out


def ghost_recursive(a2, u) -> np.ndarray:
    """Ghost non-equilibrium coefficients of modes k = 10..26 (entries 0..9 are
    0) rebuilt by Eq. recursive_eq from a2 = (xx, yy, zz, xy, xz, yz) and u."""
    lib = _load()
    aa = np.ascontiguousarray(a2, dtype=np.float64)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(27)
    lib.ora_ghost_recursive(_dp(aa), _dp(uu), _dp(out))
    return out


def init_equilibrium(dims, rho, u) -> np.ndarray:
    """f[27, N] at equilibrium for rho[N] and u[3, N] (node order x fastest)."""
    nx, ny, nz = dims
    n = nx * ny * nz
    lib = _load()
    rr = np.ascontiguousarray(np.broadcast_to(rho, (n,)), dtype=np.float64)
    uu = np.ascontiguousarray(np.reshape(u, (3, n)), dtype=np.float64)
    f = np.zeros((27, n))
    lib.ora_init_equilibrium(nx, ny, nz, _dp(rr), _dp(uu), _dp(f))
    return f


def init_thermal(params: Params, dims, rho=None, u=None) -> np.ndarray:
    """f^(0)(rho, u) plus Gaussian populations of covariance rho0 kT w_i / cs2
    (Philox at the reserved step word 0xFFFFFFFF)."""
    nx, ny, nz = dims
    n = nx * ny * nz
    lib = _load()
    rr = None if rho is None else np.ascontiguousarray(np.broadcast_to(rho, (n,)), dtype=np.float64)
    uu = None if u is None else np.ascontiguousarray(np.reshape(u, (3, n)), dtype=np.float64)
    f = np.zeros((27, n))
    lib.ora_init_thermal(ctypes.byref(params), nx, ny, nz, None if rr is None else _dp(rr),
                         None if uu is None else _dp(uu), _dp(f))
    return f


def step(params: Params, dims, f: np.ndarray, t: int, nthreads: int = 0) -> np.ndarray:
    """One collide-and-stream step of the whole lattice at step counter t."""
    nx, ny, nz = dims
    lib = _load()
    fin = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(fin)
    rc = lib.ora_step(ctypes.byref(params), nx, ny, nz, t, _dp(fin), _dp(out), nthreads)
    if rc:
        raise RuntimeError(f"ora_step failed ({rc})")
    return out


def run(params: Params, dims, f: np.ndarray, t0: int, nsteps: int, nthreads: int = 0
        ) -> np.ndarray:
    """nsteps steps from step counter t0; returns the new state (input untouched)."""
    nx, ny, nz = dims
    lib = _load()
    state = np.array(f, dtype=np.float64, order="C", copy=True)
    work = np.empty_like(state)
    rc = lib.ora_run(ctypes.byref(params), nx, ny, nz, t0, nsteps, _dp(state), _dp(work),
                     nthreads)
    if rc:
        raise RuntimeError(f"ora_run failed ({rc})")
    return state


def threads() -> int:
    return int(_load().ora_threads())


# ----------------------------------------------------------------------------
# Observables (Sec. III): moments and spectra, numpy FP64.
# ----------------------------------------------------------------------------
def velocities() -> np.ndarray:
    i = np.arange(27)
    return np.stack([i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1], axis=1)


def moments(f: np.ndarray) -> dict:
    """rho (Eq. eq:rho), j = rho u (Eq. eq:u) and Pi_ab = sum_i f_i (c_a c_b - cs2 delta_ab).

    Pi is the second-order Hermite coefficient a0^(2) + a1^(2) of the full
    population (definition below Table III).  Component order of Pi: xx, yy,
    zz, xy, xz, yz.
    """
    c = velocities().astype(np.float64)
    rho = f.sum(axis=0)
    j = c.T @ f
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    pi = np.stack([((c[:, a] * c[:, b] - (CS2 if a == b else 0.0))[:, None] * f).sum(axis=0)
                   for a, b in pairs])
    return dict(rho=rho, j=j, pi=pi)


def shell_spectrum(field: np.ndarray, dims, nshells: int | None = None):
    """Shell sums of |dm(n)|^2 with dm(n) = N^-1/2 sum_x dm(x) exp(-2 pi i n.x/L).

    field is indexed by node n = x + nx*(y + ny*z).  Shells are round(|n|) with
    n_a in (-L_a/2, L_a/2]; n = 0 is left out.  Returns (sums, counts).
    """
    nx, ny, nz = dims
    g = np.reshape(field, (nz, ny, nx))
    g = g - g.mean()
    fk = np.fft.fftn(g) / np.sqrt(g.size)
    p = np.abs(fk) ** 2
    kz = np.fft.fftfreq(nz) * nz
    ky = np.fft.fftfreq(ny) * ny
    kx = np.fft.fftfreq(nx) * nx
    # fftfreq puts -L/2 for even L; the paper's interval is (-L/2, L/2], same modulus.
    kk = np.sqrt(kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)
    shell = np.rint(kk).astype(np.int64)
    if nshells is None:
        nshells = int(shell.max()) + 1
    mask = (kk > 0) & (shell < nshells)
    sums = np.bincount(shell[mask], weights=p[mask], minlength=nshells)
    counts = np.bincount(shell[mask], minlength=nshells)
    return sums, counts
