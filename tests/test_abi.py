"""CPU checks of the C ABI: the library loads, exports every function that
include/smre.h declares, and its host-side bound helpers agree with SciPy."""
import ctypes
import os
import re

import numpy as np
import pytest
from scipy import stats

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "smre.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smre_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["smre_dykstra_project", "smre_dykstra_incomplete", "smre_ctx_create",
              "smre_max_violation", "smre_chi2_bounds"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1503_03492_amd as m
    L = ctypes.CDLL(m.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_names_match_header():
    import paper_1503_03492_amd as m
    assert set(m.EXPORTS) <= set(declared_functions())


def test_status_strings():
    import paper_1503_03492_amd as m
    assert m.status_string(0) == "ok"
    assert "non-finite" in m.status_string(-2)


@pytest.mark.parametrize("p", [0.5, 0.9, 0.99])
def test_host_chi2_bounds_match_scipy(p):
    import paper_1503_03492_amd as m
    sides = list(range(1, 33))
    got = m.chi2_bounds(sides, p)
    ref = stats.chi2.ppf(p, np.array(sides) ** 2)
    np.testing.assert_allclose(got, ref, rtol=1e-12)


def test_host_paper_bounds():
    import paper_1503_03492_amd as m
    # q = 0: bound = mu^4 = n - 1/2
    np.testing.assert_allclose(m.paper_bounds([1, 2, 4], 0.0), [0.5, 3.5, 15.5], rtol=1e-14)


def test_header_is_plain_c_and_links(tmp_path):
    """A C program compiles against include/smre.h (C11, no C++ or HIP types
    in the signatures), links against the library and calls the host-only
    helpers (no device needed)."""
    import subprocess

    import paper_1503_03492_amd as m
    src = tmp_path / "use_abi.c"
    src.write_text(r'''
#include <stdio.h>
#include "smre.h"
int main(void) {
  int32_t sides[3] = {1, 2, 4};
  double r2[3];
  if (smre_chi2_bounds(sides, 3, 0.9, r2) != SMRE_OK) return 1;
  if (smre_paper_bounds(sides, 3, 0.0, r2) != SMRE_OK) return 2;
  if (r2[0] < 0.5 - 1e-14 || r2[0] > 0.5 + 1e-14) return 3;  /* (0.5^(1/4))^4 */
  if (smre_dykstra_project(NULL, SMRE_F32, NULL, 1, 1, 1, NULL, NULL, 0, NULL, NULL) !=
      SMRE_EINVAL) return 4;
  if (smre_admm(NULL, SMRE_F32, NULL, NULL, 1, 1, 1, NULL, NULL, NULL, NULL) != SMRE_EINVAL)
    return 5;
  printf("%s\n", smre_status_string(SMRE_ENONFINITE));
  return 0;
}
''')
    exe = tmp_path / "use_abi"
    libdir = os.path.dirname(m.LIB_PATH)
    subprocess.check_call(["gcc", "-std=c11", "-Wall", "-Werror", "-I",
                           os.path.join(ROOT, "include"), str(src), "-o", str(exe), "-L", libdir,
                           "-lsmre", f"-Wl,-rpath,{libdir}"])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, (out.returncode, out.stderr)
    assert "non-finite" in out.stdout
