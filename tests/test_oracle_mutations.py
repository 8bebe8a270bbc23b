"""The oracle's pins catch plausible mistakes (CPU).

Each case plants one mistake in a copy of the oracle's C source, builds that
copy, and runs the pin suite (tests/test_oracle.py) against it; the suite
must fail.  The mistakes are the kind a reading of Eq. (1) (Section 1) or its
chain-rule adjoint could plausibly make: a wrong constant in P_j, swapped or
transposed pixel coordinates, sin for cos, a wrong term in r^2, dropped or
flipped factors in the gradients, and a transposed upstream gradient.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, text in oracle/cgh_oracle.c, replacement)
MUTATIONS = [
    ("2pi_in_P",
     "return M_PI * pitch * pitch / (wavelength * z);",
     "return 2.0 * M_PI * pitch * pitch / (wavelength * z);"),
    ("pixel_x_y_swapped",
     "intensity_at(J->x, J->y, J->a, J->P, J->n, (double)i, (double)k);",
     "intensity_at(J->x, J->y, J->a, J->P, J->n, (double)k, (double)i);"),
    ("output_transposed",
     "J->out[(long)k * J->nx + i] =",
     "J->out[(long)i * J->ny + k] ="),
    ("sin_for_cos_forward",
     "s += a[j] * cos(P[j] * (dx * dx + dy * dy));",
     "s += a[j] * sin(P[j] * (dx * dx + dy * dy));"),
    ("r2_wrong_term",
     "s += a[j] * cos(P[j] * (dx * dx + dy * dy));",
     "s += a[j] * cos(P[j] * (dx * dx + dx * dy));"),
    ("adjoint_G_transposed",
     "double G = J->g[(long)k * J->nx + i];",
     "double G = J->g[(long)i * J->ny + k];"),
    ("adjoint_sin_for_cos",
     "Sc += G * cos(th);",
     "Sc += G * sin(th);"),
    ("adjoint_dy_for_dx",
     "Sy += G * s * dy;",
     "Sy += G * s * dx;"),
    ("gx_factor_2_dropped",
     "J->gx[t] = 2.0 * J->a[j] * Pj * Sx;",
     "J->gx[t] = J->a[j] * Pj * Sx;"),
    ("gz_sign_flipped",
     "J->gz[t] = J->a[j] * Pj / J->z[j] * Sr;",
     "J->gz[t] = -J->a[j] * Pj / J->z[j] * Sr;"),
    ("adjoint_point_by_slot",
     "double dx = (double)i - J->x[j];",
     "double dx = (double)i - J->x[t];"),
]


def _copy_tree(dst):
    """The oracle sources (not its built library), the pin suite and the seeded
    generators it uses."""
    os.makedirs(os.path.join(dst, "oracle"))
    for name in ("__init__.py", "cgh_oracle.py", "cgh_oracle.c", "brute.py"):
        shutil.copy(os.path.join(ROOT, "oracle", name), os.path.join(dst, "oracle", name))
    os.makedirs(os.path.join(dst, "paper_1002_0916_amd"))
    for name in ("__init__.py", "workloads.py"):
        shutil.copy(os.path.join(ROOT, "paper_1002_0916_amd", name),
                    os.path.join(dst, "paper_1002_0916_amd", name))
    os.makedirs(os.path.join(dst, "tests"))
    for name in ("conftest.py", "test_oracle.py"):
        shutil.copy(os.path.join(ROOT, "tests", name), os.path.join(dst, "tests", name))
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), os.path.join(dst, "tests", "golden"))


def test_mutations_are_distinct_and_apply():
    with open(os.path.join(ROOT, "oracle", "cgh_oracle.c")) as f:
        src = f.read()
    for name, old, new in MUTATIONS:
        assert src.count(old) == 1, name
        assert old != new, name


def _run_pins(dst, old=None, new=None):
    """Plants the mutation (if any) in the copy at dst and runs its pin suite."""
    _copy_tree(dst)
    if old is not None:
        path = os.path.join(dst, "oracle", "cgh_oracle.c")
        with open(path) as f:
            src = f.read()
        with open(path, "w") as f:
            f.write(src.replace(old, new, 1))
    env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "tests/test_oracle.py"], cwd=dst, env=env, capture_output=True,
                       text=True, timeout=600)
    # the copy built and loaded its own library
    assert os.path.exists(os.path.join(dst, "oracle", "libcgh_oracle.so")), r.stdout[-2000:]
    return r


def test_unmutated_copy_passes(tmp_path):
    """Control: the copied suite passes on the unchanged oracle, so a failure
    below comes from the planted mistake."""
    r = _run_pins(str(tmp_path / "copy"))
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    r = _run_pins(str(tmp_path / "copy"), old, new)
    assert r.returncode == 1 and " failed" in r.stdout, (name, r.returncode, r.stdout[-2000:])
