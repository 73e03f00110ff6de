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


def test_region_flags_match_the_generators():
    """Refinement regions evaluated by the library (host, threaded) give the
    same flags, bit for bit, as the NumPy generators: balls as in the 3D
    adaptive-balls workload, and the RFF level-set band of the band workload
    (existence tracked level by level in both)."""
    import numpy as np
    import workloads as W
    from paper_1607_00648_amd import qmg
    P = W.adaptive_balls(dim=3, base=3, level=5)
    F = qmg.region_flags(3, 5, 3, P.regions)
    assert sorted(F) == sorted(P.flags)
    for l in P.flags:
        assert np.array_equal(F[l], P.flags[l]), l
    B = W.adaptive_band(dim=3, base=2, level=5)
    F = qmg.region_flags(3, 5, 2, B.regions)
    for l in B.flags:
        assert B.flags[l].any()
        assert np.array_equal(F[l], B.flags[l]), l
    B2 = W.adaptive_band(dim=2, base=2, level=5, seed=3)
    F = qmg.region_flags(2, 5, 2, B2.regions)
    for l in B2.flags:
        assert np.array_equal(F[l], B2.flags[l]), l


def test_cell_list_regions_and_refine_bytes_combine():
    import numpy as np
    from paper_1607_00648_amd import qmg
    # level-2 cell (4,4) is refined by the bytes; level-3 cells listed: one
    # inside it (exists), one outside (does not exist: ignored), one on level 4
    # (beyond the region's level)
    flags = {2: np.zeros((9, 9), bool)}
    flags[2][4, 4] = True
    cells = [(3, 13, 12), (3, 0, 0), (4, 40, 40)]
    params = np.array([v for c in cells for v in c], dtype=np.float64)
    F = qmg.region_flags(2, 5, 2, [(qmg.REGION_CELL_LIST, 4, params)], refine=flags)
    assert F[2].sum() == 1 and F[2][4, 4]
    assert F[3][12, 13] and F[3].sum() == 1 + 1      # listed bytes are kept as given
    assert F[4].sum() == 0
    # a small ball inside one cell per level refines that cell down to its level
    ball = (qmg.REGION_BALL, 3, np.array([0.5, 0.5, 0.01]))
    G = qmg.region_flags(2, 5, 2, [ball])
    assert G[2].sum() == 1 and G[2][4, 4] and G[3].sum() == 0 and G[4].sum() == 0
    G = qmg.region_flags(2, 5, 2, [(qmg.REGION_BALL, 4, np.array([0.5, 0.5, 0.01]))])
    assert G[3].sum() == 1 and G[3][13, 13] and G[4].sum() == 0


def test_region_validation():
    import numpy as np
    from paper_1607_00648_amd import qmg
    lib = qmg.load()
    ok = qmg.make_opts(transfer="galerkin")
    nb = C.c_size_t(0)
    good = qmg.make_desc(3, 4, 2, regions=[(qmg.REGION_BALL, 4, np.array([0.5, 0.5, 0.5, 0.1]))])
    assert lib.qmg_workspace_bytes(C.byref(good), C.byref(ok), C.byref(nb)) == qmg.QMG_OK
    bad = [
        (7, 4, np.array([0.5, 0.5, 0.5, 0.1])),                  # unknown kind
        (qmg.REGION_BALL, 4, np.array([0.5, 0.5, 0.1])),          # too few values
        (qmg.REGION_BALL, 4, np.array([0.5, 0.5, 0.5, 0.0])),     # radius 0
        (qmg.REGION_BALL, 5, np.array([0.5, 0.5, 0.5, 0.1])),     # level beyond L
        (qmg.REGION_LEVELSET_BAND, 4, np.array([0.1, 1.0, 2.0, 1, 2, 3, 4, 5, 6, 0.0])),   # M = 2 needs 11
        (qmg.REGION_CELL_LIST, 4, np.array([3.0, 27.0, 0.0, 0.0])),   # index beyond 3^3
        (qmg.REGION_BALL, 4, np.array([0.5, np.nan, 0.5, 0.1])),
    ]
    for r in bad:
        d = qmg.make_desc(3, 4, 2, regions=[r])
        assert lib.qmg_workspace_bytes(C.byref(d), C.byref(ok), C.byref(nb)) == qmg.QMG_EINVAL, r
    reg = qmg.make_desc(3, 4)
    reg.n_regions = 1
    reg.regions = good.regions
    assert lib.qmg_workspace_bytes(C.byref(reg), C.byref(ok), C.byref(nb)) == qmg.QMG_EINVAL


def test_solver_option_validation():
    from paper_1607_00648_amd import qmg
    lib = qmg.load()
    d = qmg.GridDesc(2, 5)
    nb = C.c_size_t(0)
    good = [qmg.make_opts(coarse_solver="sweeps"), qmg.make_opts(eps_zero=1e-6),
            qmg.make_opts(store="hier64", iterate="fp32"), qmg.make_opts(store="bf16", iterate="fp32"),
            qmg.make_opts(store="plain64", iterate="fp64")]
    for o in good:
        assert lib.qmg_workspace_bytes(C.byref(d), C.byref(o), C.byref(nb)) == qmg.QMG_OK
    bad = [qmg.make_opts(coarse_solver=7), qmg.make_opts(eps_zero=-1.0), qmg.make_opts(eps_zero=0.5),
           qmg.make_opts(iterate=9), qmg.make_opts(store="bf16", iterate="fp64"),
           qmg.make_opts(store="plain64", iterate="fp32"), qmg.make_opts(store="bpa", iterate="fp32"),
           qmg.make_opts(store="hier64", iterate="fp32", cycle="add")]
    for o in bad:
        assert lib.qmg_workspace_bytes(C.byref(d), C.byref(o), C.byref(nb)) == qmg.QMG_EINVAL
    # FP32 iterates need the FP32 work arrays: the mixed workspace
    o64 = qmg.make_opts(store="hier64")
    o32 = qmg.make_opts(store="hier64", iterate="fp32")
    n64, n32 = C.c_size_t(0), C.c_size_t(0)
    lib.qmg_workspace_bytes(C.byref(d), C.byref(o64), C.byref(n64))
    lib.qmg_workspace_bytes(C.byref(d), C.byref(o32), C.byref(n32))
    assert n32.value != n64.value
