"""CPU tests of float-channel plans: the library's channel pool and
selection (its own implementation) choose exactly the oracle's channels,
and plans reject what they cannot run."""
import pytest

from oracle import fp_config as fc

oz = pytest.importorskip("paper_2609_37693_amd")
from paper_2609_37693_amd import _lib  # noqa: E402


@pytest.mark.parametrize("fmt,gemms,k_slab", [("E4M3", 0, 2 ** 14), ("E4M3", 40, 2 ** 14),
                                              ("E2M1", 0, 2 ** 14),
                                              ("E2M1", 40, 2 ** 14), ("E2M1", 24, 2 ** 14),
                                              ("E4M3", 20, 2 ** 16), ("E2M3", 0, 2 ** 14),
                                              ("E2M3", 36, 2 ** 14), ("E2M3", 24, 2 ** 15)])
def test_library_channels_equal_oracle(fmt, gemms, k_slab):
    plan = oz.Plan(format=fmt, gemms=gemms, k_slab=k_slab)
    if gemms == 0:
        want = fc.configuration(fmt, k_slab, window_k=k_slab)
    else:
        want = fc.configuration(fmt, k_slab, q=gemms)
    assert plan.channels() == [tuple(mb) for mb in want]


def test_e2m3_plan_is_e4m3_configuration_at_2_14():
    """E2M3 and E4M3 share their usable alphabet within radius 32 at
    K_t = 2**14, so the library picks the same channels for both."""
    a = oz.Plan(format="E2M3", gemms=0, k_slab=2 ** 14)
    b = oz.Plan(format="E4M3", gemms=0, k_slab=2 ** 14)
    assert a.channels() == b.channels() and a.gemms() == 30


def test_float_plan_errors():
    with pytest.raises(_lib.OzemuError):  # slab not a multiple of 128
        oz.Plan(format="E4M3", gemms=30, k_slab=1000)
    with pytest.raises(_lib.OzemuError):
        oz.Plan(format="E4M3", gemms=30, scaling="G")
    p = oz.Plan(format="E4M3", gemms=30)
    lib = _lib.load()
    import ctypes as C
    # phase calls, cached forward and groups take INT8 plans
    st = lib.ozemu_reduce(p.handle, None, 4, 4, 4, None, 4, None, 4, None, None, None, None)
    assert st == _lib.OZEMU_ERR_UNSUPPORTED
    h = C.c_void_p()
    st = lib.ozemu_group_create(C.byref(h), 1, (C.c_void_p * 1)(p.handle.value),
                                (C.c_int64 * 1)(4), (C.c_int64 * 1)(4), (C.c_int64 * 1)(4),
                                (C.c_void_p * 1)(1), (C.c_int64 * 1)(4), (C.c_void_p * 1)(1),
                                (C.c_int64 * 1)(4), (C.c_void_p * 1)(1), (C.c_int64 * 1)(4))
    assert st == _lib.OZEMU_ERR_UNSUPPORTED
    assert p.plane_dims(5, 5, 100) == (256, 256, 128)
    p4 = oz.Plan(format="E2M1", gemms=40)
    assert p4.plane_dims(5, 5, 100) == (256, 256, 128)
    assert p4.plane_dims(5, 5, 129) == (256, 256, 256)
