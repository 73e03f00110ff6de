"""The C-ABI library loads on the CPU and exports every entry point that
include/qmg.h declares; host-side argument validation works without a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "qmg.h")).read()
    return sorted(set(re.findall(r"\b(qmg_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_1607_00648_amd import qmg
    if not os.path.exists(qmg.LIB_PATH):
        pytest.fail("libqmg.so is not built (run __graft_entry__.build())")
    lib = C.CDLL(qmg.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(qmg._SIGS) == _declared()


def test_host_validation_without_device():
    from paper_1607_00648_amd import qmg
    lib = qmg.load()
    assert lib.qmg_version().decode().startswith("qmg")
    d = qmg.GridDesc(2, 6)
    o = qmg.make_opts()
    nb = C.c_size_t(0)
    assert lib.qmg_workspace_bytes(C.byref(d), C.byref(o), C.byref(nb)) == qmg.QMG_OK
    assert nb.value > 730 * 730 * 8
    bad = qmg.make_opts(omega=2.0)
    assert lib.qmg_workspace_bytes(C.byref(d), C.byref(bad), C.byref(nb)) == qmg.QMG_EINVAL
    assert b"omega" in lib.qmg_last_error(None)
    d4 = qmg.GridDesc(4, 3)
    assert lib.qmg_workspace_bytes(C.byref(d4), C.byref(o), C.byref(nb)) == qmg.QMG_EINVAL
    o2 = qmg.make_opts(coarsest_level=6)
    assert lib.qmg_workspace_bytes(C.byref(d), C.byref(o2), C.byref(nb)) == qmg.QMG_EINVAL


def test_oracle_not_imported_by_product():
    """The product package never imports the reference implementation."""
    pkg = os.path.join(ROOT, "paper_1607_00648_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


def test_adaptive_description_validation():
    """Adaptive spacetrees are linearised on the host when the workspace is
    measured; unsupported option combinations are rejected there."""
    import numpy as np
    from paper_1607_00648_amd import qmg
    lib = qmg.load()
    flags = {2: np.zeros((9, 9), bool), 3: np.zeros((27, 27), bool)}
    flags[2][3:6, 3:6] = True
    flags[3][12:15, 12:15] = True
    packed = qmg.pack_refine(2, 2, 4, flags)
    assert packed.size == 81 + 729 and packed.sum() == 18
    d = qmg.GridDesc(2, 4, 2, packed.ctypes.data_as(C.c_void_p))
    nb = C.c_size_t(0)
    ok = qmg.make_opts(transfer="galerkin")
    assert lib.qmg_workspace_bytes(C.byref(d), C.byref(ok), C.byref(nb)) == qmg.QMG_OK
    assert nb.value > 0
    assert lib.qmg_workspace_bytes(C.byref(d), C.byref(qmg.make_opts(transfer="galerkin", store="bf16")),
                                   C.byref(nb)) == qmg.QMG_OK
    for good in (qmg.make_opts(transfer="boxmg"), qmg.make_opts(transfer="boxmg", store="hier16")):
        assert lib.qmg_workspace_bytes(C.byref(d), C.byref(good), C.byref(nb)) == qmg.QMG_OK
    for bad in (qmg.make_opts(transfer="galerkin", coarsest_level=3),):
        assert lib.qmg_workspace_bytes(C.byref(d), C.byref(bad), C.byref(nb)) == qmg.QMG_EINVAL
    no_flags = qmg.GridDesc(2, 4, 2, None)
    assert lib.qmg_workspace_bytes(C.byref(no_flags), C.byref(ok), C.byref(nb)) == qmg.QMG_EINVAL
    with pytest.raises(ValueError):
        qmg.pack_refine(2, 2, 4, {2: np.zeros((8, 8), bool)})
