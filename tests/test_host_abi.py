"""Host-side checks of libdctkrylov that need no GPU.

* the shared library loads and exports every function include/dctkrylov.h declares;
* the host-built transform matrices equal the oracle's (closed forms of
  eq. dft1 and Remark 2.1, built independently on each side);
* argument validation that happens before any device call.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2103_11847_amd as dk
from oracle import tube as otube

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dctkrylov.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dctk_[a-z_T0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(dk.LIB_PATH):
        pytest.fail("libdctkrylov.so is not built; run python -m paper_2103_11847_amd.build")
    return dk.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    # and the binding wraps exactly the declared set
    assert sorted(dk.EXPORTED) == names


def test_status_strings(lib):
    for code in [0, 1, -1, -2, -3, -4, -5, -6, -7]:
        s = dk.dctk_status_string(code)
        assert s and s != "unknown status"
    assert dk.dctk_status_string(12345) == "unknown status"
    assert dk.dctk_version() >= 100


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8, 31, 32, 64])
@pytest.mark.parametrize("tb", ["th", "dct2"])
def test_library_transform_matrices_match_oracle(lib, p, tb):
    L = otube.transform_matrix(p, tb)
    Li = np.linalg.inv(L)
    ref = {dk.DCTK_MAT_L: L, dk.DCTK_MAT_LINV: Li, dk.DCTK_MAT_LINVT: Li.T, dk.DCTK_MAT_LT: L.T}
    for which, R in ref.items():
        G = np.array(dk.dctk_tube_matrix(dk.TUBES[tb], which, p))
        scale = max(1.0, np.abs(R).max())
        assert np.abs(G - R).max() <= 1e-12 * scale * p, (tb, which, p)


def test_host_validation(lib):
    buf = (ctypes.c_double * 4)()
    assert lib.dctk_tube_matrix(0, 0, 0, buf) == dk.DCTK_ESHAPE
    assert lib.dctk_tube_matrix(0, 0, 2, None) == dk.DCTK_EINVAL
    assert lib.dctk_tube_matrix(7, 0, 2, buf) == dk.DCTK_EINVAL
    assert lib.dctk_tube_matrix(0, 9, 2, buf) == dk.DCTK_EINVAL
    assert lib.dctk_create(None, 0, None) == dk.DCTK_EINVAL
    assert lib.dctk_cprod(None, None, 1.0, None, 0.0, None) == dk.DCTK_EINVAL
    assert lib.dctk_cprod_T(None, None, 1.0, None, 0.0, None) == dk.DCTK_EINVAL
    assert lib.dctk_op_create(None, 0, 0, 1, 1, 1, None, 1, None, None) == dk.DCTK_EINVAL
    assert lib.dctk_krylov_create(None, None, 0, 1, 0, None) == dk.DCTK_EINVAL
    assert lib.dctk_lsqr_tik_solve(None, None, None, None, None, None) == dk.DCTK_EINVAL
    assert lib.dctk_gmres_tik_solve(None, None, None, None, 1, None, None) == dk.DCTK_EINVAL
    assert lib.dctk_gkb_step(None, None) == dk.DCTK_EINVAL
    assert lib.dctk_destroy(None) == dk.DCTK_EINVAL
    assert lib.dctk_last_hip_error(None) == 0
