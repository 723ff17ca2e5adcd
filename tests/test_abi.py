"""CPU checks of the C ABI boundary: the shared library loads and exports every
function that include/fargo.h declares; parameter validation and layout
queries answer without a GPU."""
import os
import re

import numpy as np
import pytest

from paper_1602_02359_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fargo.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fargo_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import ctypes
    from paper_1602_02359_amd import fargo as F
    lib = ctypes.CDLL(F.LIB_PATH)
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(F.EXPORTED) == set(names)


def test_layout_and_validation_without_gpu():
    from paper_1602_02359_amd import fargo as F
    pr = W.disk3d_sph()
    assert F.fargo_layout(pr.params) == (1536, 518, 134)
    pr = W.disk2d_cyl()
    assert F.fargo_layout(pr.params) == (384, 134, 1)
    pr = W.random_problem("cart", nx=70, ny=5, nz=4)
    assert F.fargo_layout(pr.params) == (128, 11, 10)
    assert F.fargo_abi_version() == 1
    for bad in (dict(ny=2), dict(nz=2), dict(geometry="cyl", bc=("periodic",) * 4), dict(eos="adi", gamma=1.0)):
        with pytest.raises(F.FargoError) as e:
            F.fargo_layout(dict(pr.params, **bad))
        assert e.value.code == -1
    F.fargo_layout(dict(pr.params, nx=8192))  # long rings: the time-step pass takes them in segments
    with pytest.raises(F.FargoError) as e:
        F.fargo_layout(dict(pr.params, nx=(1 << 22) + 1))
    assert e.value.code == -6
    wsb = F.fargo_workspace_bytes(W.disk3d_sph().params)
    assert wsb > 16 * 1536 * 518 * 134 * 8


def test_fp32_bulk_layout_and_precision_check():
    import ctypes
    from paper_1602_02359_amd import fargo as F
    p64 = W.disk3d_sph().params
    p32 = dict(p64, precision="fp32")
    assert F.fargo_layout(p32) == F.fargo_layout(p64)
    w64, w32 = F.fargo_workspace_bytes(p64), F.fargo_workspace_bytes(p32)
    # the field buffers (post-source copies and two transport sets) halve;
    # geometry tables and per-ring FP64 arrays do not
    assert w32 < 0.52 * w64
    ps, keep = F.make_params(p64)
    ps.precision = 7
    n = ctypes.c_size_t()
    assert F._lib.fargo_workspace_bytes(ctypes.byref(ps), ctypes.byref(n)) == -1



def test_stream_probe_rejects_bad_arguments_without_gpu():
    """fargo_hbm_streams checks its counts, sizes and pointers before it
    launches anything."""
    import ctypes as C
    from paper_1602_02359_amd import fargo as F
    lib = F._lib
    nul = (C.c_void_p * 9)()
    for nin, nout, nx, ny, nz, march in ((0, 1, 8, 8, 8, 0), (10, 1, 8, 8, 8, 0), (2, 3, 8, 8, 8, 0),
                                         (2, 1, 0, 8, 8, 0), (2, 1, 8, 8, 0, 1), (2, 1, 8, 8, 8, 2),
                                         (2, 1, 8, 8, 8, 0)):  # the last: null field pointers
        assert lib.fargo_hbm_streams(nul, nin, nul, nout, nx, ny, nz, march, None) == -1
    assert lib.fargo_hbm_streams(None, 1, nul, 1, 8, 8, 8, 0, None) == -1
