"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU,
in a scratch directory; the GPU path is not involved), rebuilds that copy and
runs the oracle's pin tests against it: at least one pin must fail.  The
mistakes are the kind a transcription of Table II, Eq. normal_fact,
Eq. fluct_phi, Eq. r-flbe2, Eq. recursive_eq, Eq. eq:streaming, of the
Philox round or of the layout of the uniforms in its words could contain.  The unmutated
copy must pass, so a failure is the mistake's doing and not the harness's.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_TESTS = ["tests/test_oracle_tables.py", "tests/test_oracle_collide.py", "tests/test_oracle_dynamics.py",
             "tests/test_philox.py", "tests/test_oracle_recursive.py"]

# (name, text in rflbm_oracle.c, replacement)
MUTATIONS = [
    ("none", None, None),
    ("multiplicity_mu7", "{1, 1, 1, 1, 1, 1, 1, 2, 2, 2,", "{1, 1, 1, 1, 1, 1, 1, 1, 2, 2,"),
    ("table2_typo_mode13", "case 13: return x * z * z - s * x;", "case 13: return x * z * z - s * z;"),
    ("cs2_in_Hxx", "case 4: return x * x - s;", "case 4: return x * x - 0.5 * s;"),
    ("hermite_index_mode16", '"yyz",   "xyz",', '"yyz",   "xzz",'),
    ("fdt_omega_1_minus_omega", "sqrt(omega * (2.0 - omega))", "sqrt(omega * (1.0 - omega))"),
    ("ghost_noise_b_inverse", "sqrt(mu * B[k]) * fdt_factor(om_g)", "sqrt(mu / B[k]) * fdt_factor(om_g)"),
    ("ghost_relaxation_sign", "relaxed[k] = (1.0 - om_g) * ghost_neq[k];", "relaxed[k] = (om_g - 1.0) * ghost_neq[k];"),
    ("recursion_without_permutations", "for (int j = 0; j < n - 1; ++j) {", "for (int j = n - 2; j < n - 1; ++j) {"),
    ("recursion_wrong_velocity", "double r = a1_recursive(s, n - 1, a2, u) * u[last];",
     "double r = a1_recursive(s, n - 1, a2, u) * u[axis_of(s[0])];"),
    ("recursive_ghosts_from_relaxed_a2", "const double a2v[6] = {a1[4], a1[5], a1[6], a1[7], a1[8], a1[9]};",
     "const double a2v[6] = {(1.0 - om_s) * a1[4], a1[5], a1[6], a1[7], a1[8], a1[9]};"),
    ("trace_over_two", "(a1[4] + a1[5] + a1[6]) / 3.0;", "(a1[4] + a1[5] + a1[6]) / 2.0;"),
    ("bulk_shear_noise_swapped",
     "(fdt_factor(om_b) * r_mean + fdt_factor(om_s) * (r[k - 4] - r_mean))",
     "(fdt_factor(om_s) * r_mean + fdt_factor(om_b) * (r[k - 4] - r_mean))"),
    ("reference_density_in_phi", "const double mu = rho * p->kT / CS2;", "const double mu = p->rho0 * p->kT / CS2;"),
    ("streaming_direction", "const int32_t xd = (x + C[i][0] + nx) % nx;", "const int32_t xd = (x - C[i][0] + nx) % nx;"),
    ("philox_key_increment", "#define PHILOX_WEYL_A 0x9E3779B9u", "#define PHILOX_WEYL_A 0x9E3779BBu"),
    ("philox_product_word", "uint32_t n1 = (uint32_t)pb;", "uint32_t n1 = (uint32_t)pa;"),
    ("philox_key_schedule", "    if (r > 0) {\n      k0 += PHILOX_WEYL_A;", "    if (r > 1) {\n      k0 += PHILOX_WEYL_A;"),
    # the layout of the uniforms in the Philox words
    ("angle_shares_radius_bits", "{w[3] >> 16, w[3] & 0xFFFFu,", "{w[0] >> 16, w[3] & 0xFFFFu,"),
    ("radius_from_16_bits", "u[2 * m] = 1.0 - (double)(w[m] >> 9) / 8388608.0;",
     "u[2 * m] = 1.0 - (double)(w[m] >> 16) / 65536.0;"),
]


def make_copy(dst, old, new):
    os.makedirs(os.path.join(dst, "oracle"))
    for name in ("__init__.py", "rflbm_oracle.c"):
        shutil.copy(os.path.join(ROOT, "oracle", name), os.path.join(dst, "oracle", name))
    shutil.copytree(os.path.join(ROOT, "tests"), os.path.join(dst, "tests"),
                    ignore=shutil.ignore_patterns("__pycache__", "test_gpu_*", "test_oracle_mutations.py"))
    for name in ("workloads.py", "pytest.ini", "bench.py"):
        shutil.copy(os.path.join(ROOT, name), os.path.join(dst, name))
    if old is not None:
        path = os.path.join(dst, "oracle", "rflbm_oracle.c")
        with open(path) as fh:
            src = fh.read()
        assert src.count(old) == 1, old
        with open(path, "w") as fh:
            fh.write(src.replace(old, new))


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(tmp_path, name, old, new):
    dst = str(tmp_path / "copy")
    make_copy(dst, old, new)
    env = dict(os.environ)
    env.pop("RFLBM_ORACLE_LIBRARY", None)  # the copy builds and loads its own oracle
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu and not slow"] + PIN_TESTS,
                       cwd=dst, capture_output=True, text=True, timeout=900, env=env)
    tail = (r.stdout + r.stderr)[-1500:]
    if old is None:
        assert r.returncode == 0, tail
    else:
        assert r.returncode == 1, tail  # 1: tests ran and at least one failed
