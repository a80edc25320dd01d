"""Host-side logic of the library that runs without a device: the audit
decision rule of surrogate inference and the quantised normal of the
multi-scale density gate."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def sg():
    from paper_2507_01152_amd import sonosim
    sonosim.load()
    return sonosim


def test_audit_rule_per_frame_and_whole_step(sg):
    fb, whole = sg.sg_audit_decide([35.0, 29.9, 30.0, float("nan")], 30.0, 0.5)
    assert fb.tolist() == [False, True, False, True] and not whole     # 2 of 4 fail: not more than half
    fb, whole = sg.sg_audit_decide([35.0, 29.9, 10.0, float("nan")], 30.0, 0.5)
    assert fb.tolist() == [False, True, True, True] and whole
    fb, whole = sg.sg_audit_decide([], 30.0, 0.0)
    assert fb.size == 0 and not whole
    fb, whole = sg.sg_audit_decide(np.full(64, 31.0), float("inf"), 0.25)   # forced: every frame fails
    assert fb.all() and whole
    fb, whole = sg.sg_audit_decide(np.full(64, 31.0), float("-inf"), 0.0)
    assert not fb.any() and not whole


def test_audit_rule_rejects_bad_arguments(sg):
    lib = sg.load()
    import ctypes
    whole = ctypes.c_int32()
    assert lib.sg_audit_decide(-1, None, 30.0, 0.5, None, ctypes.byref(whole)) == sg.SG_EINVAL
    assert lib.sg_audit_decide(3, None, 30.0, 0.5, None, ctypes.byref(whole)) == sg.SG_EINVAL


def test_noise_quantiles_of_the_library_match_the_oracle():
    """The library's host-side quantised normal of the multi-scale gate
    (bisection on erfc, C++) equals the oracle's (scipy's ndtri), entry for
    entry: both sides then sum identical integers."""
    import oracle
    from paper_2507_01152_amd import sonosim as sg
    assert np.array_equal(sg.sg_noise_quantiles(), oracle.quantised_normal_table())
