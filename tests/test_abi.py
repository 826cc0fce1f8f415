"""CPU checks of the C ABI: the library loads, exports every function the
header declares, agrees with the oracle's DCT table bit for bit, and rejects
bad descriptors on the host before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import abcs as orc


def _declared(repo_root):
    names = set()
    inc = os.path.join(repo_root, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            text = open(os.path.join(inc, f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            for m in re.finditer(r"^\s*(?:const\s+)?[\w\s\*]+?\b((?:abcs|ida)_\w+)\s*\(", text, flags=re.M):
                names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def native():
    from paper_2001_09632_amd import _native
    return _native


def test_library_exports_declared_symbols(native, repo_root):
    L = native.lib()
    names = _declared(repo_root)
    assert {"abcs_budget", "abcs_sense", "abcs_reconstruct", "abcs_plan_create"} <= names
    for n in sorted(names):
        assert hasattr(L, n), f"{n} declared in include/ but not exported"


@pytest.mark.parametrize("B", [8, 16, 32])
def test_dct_table_matches_oracle_bitwise(native, B):
    import paper_2001_09632_amd as g
    lib_table = np.array(g.dct_basis(B))
    assert np.array_equal(lib_table, orc.dct_matrix(B))


def _err(desc):
    import paper_2001_09632_amd as g
    with pytest.raises(g.AbcsError) as e:
        g.Plan([desc])
    return e.value.status


def test_descriptor_validation(native):
    base = dict(height=256, width=256, block=16, subrate=0.25, method="bbv")
    assert _err({**base, "block": 12}) == native.ABCS_EUNSUPPORTED
    assert _err({**base, "block": 64}) == native.ABCS_EUNSUPPORTED
    assert _err({**base, "subrate": 0.0}) == native.ABCS_EDOMAIN
    assert _err({**base, "subrate": 1.5}) == native.ABCS_EDOMAIN
    assert _err({**base, "subrate": 0.6}) == native.ABCS_EDOMAIN      # BBV needs L >= 2
    assert _err({**base, "height": 8}) == native.ABCS_EDOMAIN          # no whole block
    assert _err({**base, "row_pitch": 250}) == native.ABCS_EINVAL      # pitch < width
    assert _err({**base, "row_pitch": 258}) == native.ABCS_EINVAL      # pitch not multiple of 4
    assert _err({**base, "pixel_offset": 2}) == native.ABCS_EINVAL
    assert _err({**base, "method": 7}) == native.ABCS_EINVAL
    assert _err({**base, "transform": 2}) == native.ABCS_EINVAL


def test_null_arguments(native):
    L = native.lib()
    assert L.abcs_plan_create(None, 1, ctypes.byref(ctypes.c_void_p())) == native.ABCS_EINVAL
    assert L.abcs_plan_create(None, 0, None) == native.ABCS_EINVAL
    assert L.abcs_budget(None, None, 0, None, None, None, None) == native.ABCS_EINVAL
    assert L.abcs_dct_basis(12, (ctypes.c_double * 144)()) == native.ABCS_EINVAL
    assert b"null" in L.abcs_last_error() or b"block" in L.abcs_last_error()
