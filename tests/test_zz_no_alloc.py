"""GPU test of rflbm_get_moments_host_noalloc, the moment readback into host
memory that allocates no device memory (fields staged through the library's
fixed per-GPU array in chunks).  Called through the C interface and compared
bit for bit with rflbm_get_moments into host memory, on two calls in a row:
first a box whose ten fields span two chunks of the array, then a smaller box
with fewer fields, so stale contents of the shared array would show."""
import ctypes

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rf():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_08820_amd as rf
    return rf


def lattice(rf, ora, dims, init_seed, **kw):
    rho, u = wl.random_velocity(dims, init_seed)
    f = ora.init_equilibrium(dims, rho, u)
    f = f + 1e-3 * ora.tables()["w"][:, None] * wl.normal_array(f.shape, init_seed + 1)
    lat = rf.Lattice(dims, **kw)
    lat.set_populations(f)
    lat.step(3)  # odd step count: the readback undoes the AA layout
    return lat


def c_abi_pair(rf, lat, mask, nf):
    lib = rf.load_library()
    ref = np.full((nf, lat.n), np.nan, dtype=np.float32)
    got = np.full((nf, lat.n), np.nan, dtype=np.float32)
    assert lib.rflbm_get_moments(lat._h, mask, ref.ctypes.data_as(ctypes.c_void_p), 1) == 0
    st = lib.rflbm_get_moments_host_noalloc(lat._h, mask, got.ctypes.data_as(ctypes.c_void_p))
    assert st == 0, lib.rflbm_last_error().decode()
    return ref, got


def test_noalloc_moments_equal_allocating_readback(rf, ora):
    print("[gpu] no-alloc moments: 72x64x48 all fields, then 20x9x7 rho", flush=True)
    big = lattice(rf, ora, (72, 64, 48), 3, kT=1e-4, tau=0.8, seed=9)
    assert 10 * big.n * 4 > 8 << 20  # more than one chunk of the array
    ref, got = c_abi_pair(rf, big, rf.M_RHO | rf.M_J | rf.M_PI, 10)
    assert np.array_equal(ref, got)
    small = lattice(rf, ora, (20, 9, 7), 4, storage="f16", kT=1e-5, tau=0.6, seed=10)
    ref2, got2 = c_abi_pair(rf, small, rf.M_RHO, 1)
    assert np.array_equal(ref2, got2)
    # the J and PI fields only, on the smaller box again
    ref3, got3 = c_abi_pair(rf, small, rf.M_J | rf.M_PI, 9)
    assert np.array_equal(ref3, got3)
    # and the binding's wrapper
    assert np.array_equal(small.moments_host_noalloc(rf.M_RHO), ref2)


def test_noalloc_rejects_bad_arguments(rf, ora):
    lib = rf.load_library()
    lat = lattice(rf, ora, (8, 8, 8), 5, kT=1e-4, seed=11)
    buf = np.zeros((10, lat.n), dtype=np.float32)
    assert lib.rflbm_get_moments_host_noalloc(lat._h, 0, buf.ctypes.data_as(ctypes.c_void_p)) == -1
    assert lib.rflbm_get_moments_host_noalloc(lat._h, 8, buf.ctypes.data_as(ctypes.c_void_p)) == -1
    assert lib.rflbm_get_moments_host_noalloc(lat._h, 1, None) == -1
    assert lib.rflbm_get_moments_host_noalloc(None, 1, buf.ctypes.data_as(ctypes.c_void_p)) == -1
