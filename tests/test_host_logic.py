"""Host-side logic of the library that runs without a device: the audit
decision rule of surrogate inference."""
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
