"""Host-side checks of the C interface (no GPU compute)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_1811_11720_amd as Q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "qmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(qmc_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 14
    L = C.CDLL(Q.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    L = Q.lib()
    for n in _declared():
        assert getattr(L, n).restype is not None or n == "qmc_last_error"


def test_header_constants_match_binding():
    src = open(os.path.join(ROOT, "include", "qmc.h")).read()
    for name, val in [("QMC_EINVAL", Q.QMC_EINVAL), ("QMC_ENOMEM", Q.QMC_ENOMEM), ("QMC_EDEVICE", Q.QMC_EDEVICE),
                      ("QMC_EUNSUPPORTED", Q.QMC_EUNSUPPORTED), ("QMC_DEFORM", Q.QMC_DEFORM),
                      ("QMC_EVAL_FP32", Q.QMC_EVAL_FP32), ("QMC_SPECIALISE", Q.QMC_SPECIALISE),
                      ("QMC_T_BAKER", Q.T_BAKER), ("QMC_T_SIDI", Q.T_SIDI),
                      ("QMC_NONFINITE", Q.QMC_NONFINITE), ("QMC_ERRMODE_LARGEST", Q.ERRMODE_LARGEST)]:
        m = re.search(rf"\b{name}\s*=\s*(-?\d+)", src)
        assert m and int(m.group(1)) == val, name


def test_result_struct_layout():
    # 4 doubles, u64, 2 u32, u64, 2 u32, u64, 3 doubles, 2 doubles
    assert C.sizeof(Q.Result) == 4 * 8 + 8 + 8 + 8 + 8 + 8 + 3 * 8 + 2 * 8


@pytest.mark.parametrize("seed,m,d", [(0, 1, 1), (7, 32, 6), (2 ** 63 + 5, 10, 3), (123, 64, 16)])
def test_runtime_shifts_equal_oracle_shifts(seed, m, d):
    """Two independent SplitMix64 implementations agree bit for bit."""
    assert np.array_equal(Q.shifts(seed, m, d), oracle.shifts(seed, m, d))


def test_shifts_reject_bad_arguments():
    with pytest.raises(Q.QmcError):
        Q.shifts(1, 0, 3)


def test_context_without_gpu_reports_unsupported():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    rc = Q.lib().qmc_context_create(0, None, None, 0, C.byref(h))
    assert rc == Q.QMC_EUNSUPPORTED
    assert b"device" in Q.lib().qmc_last_error()
