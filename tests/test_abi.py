"""The C-ABI library loads (no GPU needed) and exports every symbol that
include/fe2.h declares; the ctypes descriptor matches the C layout."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2312_12771_amd", "libfe2.so")


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "fe2.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fe2_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["fe2_setup", "fe2_assemble_rve", "fe2_condense", "fe2_newton_step",
              "fe2_get_state", "fe2_destroy", "fe2_strerror"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfe2.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.fe2_abi_version.restype = ctypes.c_int
    assert lib.fe2_abi_version() == 4
    lib.fe2_strerror.restype = ctypes.c_char_p
    assert lib.fe2_strerror(0) == b"ok"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfe2.so not built")
def test_setup_rejects_bad_descriptors_without_gpu_work():
    """Validation runs before any HIP call: a wrong struct_size and a null
    descriptor fail with FE2_EINVAL."""
    from paper_2312_12771_amd import fe2
    d = fe2.fe2_problem_desc()
    d.struct_size = 3
    out = ctypes.c_void_p()
    assert fe2._lib.fe2_setup(ctypes.byref(d), None, ctypes.byref(out)) == fe2.FE2_EINVAL
    assert b"struct_size" in fe2._lib.fe2_last_error()
    assert fe2._lib.fe2_setup(None, None, ctypes.byref(out)) == fe2.FE2_EINVAL


def test_descriptor_layout_matches_header():
    """Field order of the ctypes mirror equals the C struct's field order."""
    txt = open(os.path.join(ROOT, "include", "fe2.h")).read()
    body = txt[txt.index("typedef struct fe2_problem_desc {"):txt.index("} fe2_problem_desc;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for line in body.splitlines()[1:]:
        line = line.strip().rstrip(";")
        if not line:
            continue
        decl = line.split(None, 1)[1] if not line.startswith("const") else line.split(None, 2)[2]
        for part in decl.split(","):
            fields.append(part.strip().lstrip("*").strip())
    if not os.path.exists(LIB):
        pytest.skip("libfe2.so not built")
    from paper_2312_12771_amd import fe2
    assert [f[0] for f in fe2.fe2_problem_desc._fields_] == fields


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfe2.so not built")
def test_setup_validates_the_macro_basis_without_gpu_work():
    """The RVE count must match the macro basis (n_elems * 2^dim RVEs with
    the Dirac basis, n_elems with the element basis) and the basis must be
    known; both checks run before any HIP call."""
    import workloads as W
    from paper_2312_12771_amd import fe2
    out = ctypes.c_void_p()
    pd = W.config("cfg2", macro=(2, 2), rve=6)
    pe = W.element_basis(pd)
    d, keep = fe2.make_desc(pd)
    d.macro_basis = fe2.FE2_BASIS_ELEMENT          # 16 RVEs for 4 elements
    assert fe2._lib.fe2_setup(ctypes.byref(d), None, ctypes.byref(out)) == fe2.FE2_EINVAL
    assert b"n_elems with the element basis" in fe2._lib.fe2_last_error()
    d, keep = fe2.make_desc(pe)
    d.macro_basis = fe2.FE2_BASIS_DIRAC            # 4 RVEs for 4 elements
    assert fe2._lib.fe2_setup(ctypes.byref(d), None, ctypes.byref(out)) == fe2.FE2_EINVAL
    assert b"(macro_order + 1)^dim" in fe2._lib.fe2_last_error()
    d.macro_basis = 7
    assert fe2._lib.fe2_setup(ctypes.byref(d), None, ctypes.byref(out)) == fe2.FE2_EINVAL
    assert b"macro_basis" in fe2._lib.fe2_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfe2.so not built")
def test_setup_validates_the_macro_order_without_gpu_work():
    """macro_order is 1 or 2; Q9 meshes carry 9 RVEs per element with the
    Dirac basis; quadratic hexahedra are not implemented.  All checks run
    before any HIP call."""
    import workloads as W
    from paper_2312_12771_amd import fe2
    out = ctypes.c_void_p()
    d, keep = fe2.make_desc(W.config("cfg2", macro=(2, 2), rve=6, order=2))
    assert d.macro_order == 2 and d.n_rve == 36
    d.macro_order = 3
    assert fe2._lib.fe2_setup(ctypes.byref(d), None, ctypes.byref(out)) == fe2.FE2_EINVAL
    assert b"macro_order" in fe2._lib.fe2_last_error()
    d.macro_order = 1                               # 36 RVEs for 4 elements of order 1
    assert fe2._lib.fe2_setup(ctypes.byref(d), None, ctypes.byref(out)) == fe2.FE2_EINVAL
    assert b"(macro_order + 1)^dim" in fe2._lib.fe2_last_error()
    d3, keep3 = fe2.make_desc(W.config("cfg4", macro=(1, 1, 1), rve=4))
    d3.macro_order = 2
    assert fe2._lib.fe2_setup(ctypes.byref(d3), None, ctypes.byref(out)) == fe2.FE2_ENOTSUP
    assert b"2D (Q9)" in fe2._lib.fe2_last_error()
