"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and rejects invalid descriptions before touching the device."""
import ctypes as C
import os
import re

import pytest

import paper_2402_03074_amd as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hwenou.h")).read()
    return sorted(set(re.findall(r"\b(hwenou_[a-z_]+)\s*\(", src)))


def test_header_declares_the_abi():
    assert set(_declared()) == set(H.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = C.CDLL(H.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


def test_strerror_codes():
    for code in range(7):
        assert isinstance(H.strerror(code), str) and H.strerror(code)
    assert "non-physical" in H.strerror(H.HWENOU_ENONPHYSICAL)


def _create(desc, insts):
    arr = (H.Inst * len(insts))(*insts)
    h = C.c_void_p()
    rc = H.lib().hwenou_create(C.byref(desc), len(insts), arr, None, C.byref(h))
    return rc, h


@pytest.mark.parametrize("field,value", [("dim", 3), ("eq", 7), ("precision", 2),
                                         ("weights", 5), ("gamma_low", 0.5),
                                         ("gas_gamma", 1.0), ("eps", -1.0)])
def test_create_rejects_bad_description(field, value):
    d = H.make_desc(1, "euler")
    setattr(d, field, value)
    rc, h = _create(d, [H.make_inst(10)])
    assert rc == H.HWENOU_EINVAL and not h.value


def test_create_rejects_bad_instances():
    d = H.make_desc(2, "euler")
    assert _create(d, [H.make_inst(2, 10, (0, 1, 0, 1))])[0] == H.HWENOU_EINVAL
    assert _create(d, [H.make_inst(10, 2, (0, 1, 0, 1))])[0] == H.HWENOU_EINVAL
    # overlapping instances
    a = H.make_inst(10, 10, (0, 1, 0, 1), offset=0)
    b = H.make_inst(10, 10, (0, 1, 0, 1), offset=50)
    assert _create(d, [a, b])[0] == H.HWENOU_EINVAL
    # empty domain
    assert _create(d, [H.make_inst(10, 10, (1, 1, 0, 1))])[0] == H.HWENOU_EINVAL
    # bad boundary condition
    c = H.make_inst(10, 10, (0, 1, 0, 1))
    c.bc[2] = 9
    assert _create(d, [c])[0] == H.HWENOU_EINVAL
    assert H.lib().hwenou_create(C.byref(d), 0, None, None, C.byref(C.c_void_p())) == \
        H.HWENOU_EINVAL


def test_create_rejects_reflective_scalar_law():
    """Reflective walls are defined for the Euler equations only."""
    d = H.make_desc(1, "advection")
    assert _create(d, [H.make_inst(10, 1, (0, 1), "reflective")])[0] == H.HWENOU_EINVAL
    d2 = H.make_desc(2, "burgers")
    inst = H.make_inst(10, 10, (0, 1, 0, 1), ("periodic", "periodic", "reflective"))
    assert _create(d2, [inst])[0] == H.HWENOU_EINVAL


def test_create_rejects_oversized_instance():
    """An instance of more than 2^29 cells is refused before any device call:
    the kernels address an instance with 32-bit byte offsets."""
    d = H.make_desc(2, "euler")
    assert _create(d, [H.make_inst(23171, 23171, (0, 1, 0, 1))])[0] == H.HWENOU_EUNSUPPORTED
    d1 = H.make_desc(1, "euler")
    assert _create(d1, [H.make_inst((1 << 29) + 1, 1, (0, 1))])[0] == H.HWENOU_EUNSUPPORTED


def test_calls_reject_null_handle():
    L = H.lib()
    assert L.hwenou_destroy(None) == H.HWENOU_EINVAL
    assert L.hwenou_stage(None, 0, None, None, None, None, None, None) == H.HWENOU_EINVAL
    assert L.hwenou_advance(None, None, None, 0.5, 1.0, 1, None, None) == H.HWENOU_EINVAL
    assert L.hwenou_set_launch(None, 1, 0) == H.HWENOU_EINVAL


# ---------------------------------------------------------------------------
# argument checks of the Python binding: bad tensors are rejected before the
# C-ABI is called (nothing is launched; CPU tensors stand in for the cases
# that need no device)
# ---------------------------------------------------------------------------

def _geom(dim=2, eq="euler", precision="fp64"):
    d = H.make_desc(dim, eq, precision)
    insts = [H.make_inst(8, 6 if dim == 2 else 1, (0, 1, 0, 1)),
             H.make_inst(5, 4 if dim == 2 else 1, (0, 1, 0, 1), offset=48)]
    return H.Geometry(d, insts)


def test_geometry_of_a_handle():
    g = _geom()
    assert (g.dim, g.ncomp, g.n_inst, g.plane, g.mom_dtype) == (2, 4, 2, 68, "float64")
    g = _geom(1, "advection", "mixed")
    assert (g.dim, g.ncomp, g.plane, g.mom_dtype) == (1, 1, 53, "float32")


@pytest.mark.parametrize("case", ["cpu", "dtype", "noncontig", "short", "not_tensor"])
def test_binding_rejects_bad_tensors(case):
    import torch
    g = _geom()
    need = g.dim * g.ncomp * g.plane
    t = {"cpu": torch.zeros(need, dtype=torch.float64),
         "dtype": torch.zeros(need, dtype=torch.float32),
         "noncontig": torch.zeros(2 * need, dtype=torch.float64)[::2],
         "short": torch.zeros(need - 1, dtype=torch.float64),
         "not_tensor": [0.0] * need}[case]
    with pytest.raises(H.HwenouError) as e:
        H.check_tensor(t, "hwenou_stage", "mom_in", g.mom_dtype, need,
                       require_cuda=(case == "cpu"))
    assert e.value.code == H.HWENOU_EINVAL
    assert "mom_in" in str(e.value)


def test_binding_accepts_a_matching_tensor():
    import torch
    g = _geom(precision="mixed")
    need = g.dim * g.ncomp * g.plane
    H.check_tensor(torch.zeros(need, dtype=torch.float32), "w", "mom", g.mom_dtype, need,
                   require_cuda=False)


def test_binding_rejects_unknown_handles():
    import torch
    u = torch.zeros(4)
    for call in (lambda: H.hwenou_stage(C.c_void_p(12345), 0, u, u, u, u, u, u),
                 lambda: H.hwenou_advance(C.c_void_p(12345), u, u, 0.5, 1.0, 1),
                 lambda: H.hwenou_max_wavespeed(C.c_void_p(12345), u, u)):
        with pytest.raises(H.HwenouError) as e:
            call()
        assert e.value.code == H.HWENOU_EINVAL


def test_no_alloc_step_rejects_bad_arguments_without_a_device():
    L = H.lib()
    d = H.make_desc(2, "euler")
    i = H.make_inst(10, 10, (0, 1, 0, 1))
    assert L.hwenou_step_noalloc(None, None, None, None, None, None, None, None) == \
        H.HWENOU_EINVAL
    assert L.hwenou_step_noalloc(C.byref(d), C.byref(i), None, None, None, None, None,
                                 None) == H.HWENOU_EINVAL
    bad = H.make_desc(2, "euler")
    bad.dim = 3
    one = C.c_void_p(256)  # never dereferenced: the description is rejected first
    assert L.hwenou_step_noalloc(C.byref(bad), C.byref(i), None, one, one, one, one,
                                 None) == H.HWENOU_EINVAL
    off = H.make_inst(10, 10, (0, 1, 0, 1), offset=5)  # one instance, at offset 0 only
    assert L.hwenou_step_noalloc(C.byref(d), C.byref(off), None, one, one, one, one,
                                 None) == H.HWENOU_EINVAL


def test_create_rejects_interface_bases_in_1d():
    """The per-interface projection is a 2D Euler mode."""
    d = H.make_desc(1, "euler", char_decomp="interface")
    rc, h = _create(d, [H.make_inst(10)])
    assert rc == H.HWENOU_EINVAL and not h.value
