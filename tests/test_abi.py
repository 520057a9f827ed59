"""CPU checks of the C interface: the library loads, exports every function the
header declares, the ctypes structures match the C layout, and parameter
validation rejects what the model forbids (tau <= 1/2 makes the noise
amplitude of Eq. fluct_phi imaginary).  No GPU work is launched here."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2507_08820_amd as rf
from paper_2507_08820_amd import _binding

HEADER = _binding.HEADER


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rflbm_\w+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = rf.load_library()
    names = declared_functions()
    assert len(names) >= 25
    for name in names:
        assert hasattr(lib, name), name
    # and the binding declares a signature for each of them
    assert set(names) == set(_binding._SIGS)


def test_struct_layout_matches_c(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text(f"""
#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
int main(void) {{
  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(rflbm_params), offsetof(rflbm_params, rho0),
         offsetof(rflbm_params, tau_ghost), offsetof(rflbm_params, seed),
         offsetof(rflbm_params, storage_scale), sizeof(rflbm_stats), offsetof(rflbm_stats, mass_dev));
  return 0;
}}
""")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c11", str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    P, S = _binding.Params, _binding.Stats
    assert got == [ctypes.sizeof(P), P.rho0.offset, P.tau_ghost.offset, P.seed.offset,
                   P.storage_scale.offset, ctypes.sizeof(S), S.mass_dev.offset]


def required(dims, **kw):
    p = rf.make_params(dims, **kw)
    return rf.load_library().rflbm_required_bytes(ctypes.byref(p))


def test_large_boxes_are_accepted():
    # 1100 x 1000 x 1000 FP32: 119 GB, one z plane of populations 119 MB
    assert required((1100, 1000, 1000)) > 27 * 4 * 1100 * 1000 * 1000


def test_required_bytes_counts_one_lattice_copy():
    n = 512 ** 3
    b = required((512, 512, 512))
    assert 27 * 4 * n <= b < 27 * 4 * n * 1.02
    b16 = required((512, 512, 512), storage="f16", kT=1e-5)
    assert 27 * 2 * n <= b16 < 27 * 2 * n * 1.02


@pytest.mark.parametrize("kw", [
    dict(tau=0.5), dict(tau=0.4), dict(tau_bulk=0.5), dict(tau_ghost=0.5), dict(kT=-1.0),
    dict(rho0=0.0), dict(philox_rounds=8), dict(storage="f16", kT=0.0),
])
def test_invalid_parameters_are_rejected(kw):
    assert required((8, 8, 8), **kw) == 0
    p = rf.make_params((8, 8, 8), **kw)
    h = ctypes.c_void_p()
    lib = rf.load_library()
    assert lib.rflbm_create(ctypes.byref(p), None, 0, None, ctypes.byref(h)) == _binding.EINVAL
    assert lib.rflbm_last_error()


@pytest.mark.parametrize("dims", [(1, 8, 8), (8, 8, 1), (2048, 2048, 1024), (8192, 8192, 2)])
def test_invalid_boxes_are_rejected(dims):
    assert required(dims) == 0


def test_caller_buffer_too_small_is_enomem():
    p = rf.make_params((8, 8, 8))
    h = ctypes.c_void_p()
    lib = rf.load_library()
    need = lib.rflbm_required_bytes(ctypes.byref(p))
    st = lib.rflbm_create(ctypes.byref(p), ctypes.c_void_p(1 << 20), need - 1, None, ctypes.byref(h))
    assert st == _binding.ENOMEM and not h.value


def test_null_arguments():
    lib = rf.load_library()
    assert lib.rflbm_step(None, 1) == _binding.EINVAL
    assert lib.rflbm_step_count(None) == -1
    assert lib.rflbm_destroy(None) == _binding.OK
    assert lib.rflbm_set_row_blocks(None, 1) == _binding.EINVAL
    active = ctypes.c_int32(7)
    assert lib.rflbm_get_row_blocks(None, ctypes.byref(active)) == _binding.EINVAL
    assert active.value == 7


def test_batch_validation():
    lib = rf.load_library()
    arr = (_binding.Params * 3)()
    for i, d in enumerate([(8, 8, 8), (16, 4, 4), (5, 6, 7)]):
        arr[i] = rf.make_params(d, kT=1e-5)
    assert lib.rflbm_batch_required_bytes(3, arr) > 0
    arr[1] = rf.make_params((16, 4, 4), kT=1e-5, storage="f16")
    assert lib.rflbm_batch_required_bytes(3, arr) == 0  # mixed storage
    arr[1] = rf.make_params((16, 4, 4), kT=1e-5, philox_rounds=10)
    assert lib.rflbm_batch_required_bytes(3, arr) == 0  # mixed rounds
    arr[1] = rf.make_params((16, 4, 4), tau=0.5)
    assert lib.rflbm_batch_required_bytes(3, arr) == 0  # invalid replica
    assert lib.rflbm_batch_required_bytes(0, arr) == 0
    h = ctypes.c_void_p()
    assert lib.rflbm_batch_create(3, arr, None, 0, None, ctypes.byref(h)) == _binding.EINVAL
    assert b"replica 1" in lib.rflbm_last_error()


def test_fast_division_is_exact(tmp_path):
    """The magic-number division that maps a flattened node index to (x, y, z)
    in the batched kernel, checked on the host against integer division."""
    src = tmp_path / "fd.cpp"
    csrc = os.path.join(os.path.dirname(_binding.__file__), "csrc", "fastdiv.hpp")
    src.write_text(f"""
#include "{csrc}"
#include <cstdio>
#include <random>
int main() {{
  std::mt19937_64 g(1); long bad = 0;
  const uint32_t ds[] = {{2, 3, 5, 7, 31, 32, 33, 48, 64, 96, 97, 127, 128, 255, 256, 257, 1000,
                          4095, 4096, 9216, 65535, 65536, 99991, 1u << 20, (1u << 31) - 1, 1u << 31,
                          (1u << 31) + 1, 4294967295u}};
  for (uint32_t d : ds) {{
    const auto f = rflbm::make_fastdiv(d);
    for (int k = 0; k < 200000; ++k) {{
      uint32_t n = (uint32_t)g();
      if (k < 1000) n = k;
      else if (k < 2000) n = 0xffffffffu - (k - 1000);
      if (rflbm::fast_div(n, f) != n / d) ++bad;
    }}
  }}
  printf("%ld\\n", bad);
  return bad != 0;
}}
""")
    exe = tmp_path / "fd"
    subprocess.run(["g++", "-O2", "-std=c++17", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "0"


def test_params_round_trip_and_merge():
    """params_kwargs reproduces a parameter set field for field; merged_params
    changes only the keywords given (the bulk rate follows a new tau only if it
    followed the shear rate before)."""
    import numpy as np

    dims = (8, 6, 4)
    p = _binding.make_params(dims, storage="f16", model="bgk", kT=2e-5, tau=0.7,
                             tau_ghost=list(np.linspace(0.6, 1.5, 17)), rho0=1.2, seed=(5 << 32) + 3,
                             stream_id=9, philox_rounds=7, storage_scale=0.01)
    q = _binding.make_params(dims, **_binding.params_kwargs(p))
    assert bytes(p) == bytes(q)

    m = _binding.merged_params(p, dims, kT=0.0)
    assert m.kT == 0.0
    assert bytes(_binding.merged_params(m, dims, kT=2e-5)) == bytes(p)
    m = _binding.merged_params(p, dims, tau=0.9)
    assert (m.tau_shear, m.tau_bulk) == (0.9, 0.9)
    r = _binding.make_params(dims, tau=0.7, tau_bulk=1.0)
    m = _binding.merged_params(r, dims, tau=0.9)
    assert (m.tau_shear, m.tau_bulk) == (0.9, 1.0)
    m = _binding.merged_params(r, dims, tau_bulk=0.6)
    assert (m.tau_shear, m.tau_bulk) == (0.7, 0.6)


def test_field_sizes_are_checked_before_the_library_reads_them():
    """Density and velocity fields reach the library only as N and 3 N values
    in node order: a scalar density is broadcast, a box-shaped one must be
    indexed [z, y, x] (shape (nz, ny, nx)) and is flattened; any other shape,
    including the transposed box, raises before any call."""
    import numpy as np

    torch = pytest.importorskip("torch")
    dims = (4, 3, 2)
    n = 4 * 3 * 2
    assert _binding._field(1.1, "cpu", dims).shape == (n,)
    box = np.arange(n, dtype=np.float64).reshape(2, 3, 4)  # [z, y, x]
    got = _binding._field(box, "cpu", dims).numpy()
    assert got.shape == (n,)
    assert got[1 + 4 * (2 + 3 * 1)] == box[1, 2, 1]  # node n = x + nx (y + ny z) at (x, y, z) = (1, 2, 1)
    assert _binding._field(np.zeros((3, n)), "cpu", dims, rows=3).shape == (3, n)
    assert _binding._field(np.zeros((3, 2, 3, 4)), "cpu", dims, rows=3).shape == (3, n)
    for bad, rows in ((np.ones(n + 1), 1), (torch.ones(n - 1), 1), (np.zeros((3, n - 1)), 3),
                      (np.ones((4, 3, 2)), 1), (np.zeros((n, 3)), 3), (np.zeros((3, 4, 3, 2)), 3)):
        with pytest.raises(ValueError):
            _binding._field(bad, "cpu", dims, rows=rows)
    with pytest.raises(ValueError):
        _binding.copy(torch.empty(64, dtype=torch.uint8), torch.empty(32, dtype=torch.uint8), 64)
