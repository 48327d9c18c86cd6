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
