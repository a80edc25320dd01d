"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle is rebuilt with gcc's sanitizers and its pin tests run against that
build in a child process; the library's host code is rebuilt with clang's
(device code unchanged) and a child process drives the entry points that need
no GPU: the audit rule, the quantile table, the version and error reporting,
and the argument checks that fail before any device call.  Any sanitizer
finding aborts the child, which fails the test.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _clean_env(**kw):
    env = dict(os.environ)
    env.update(ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", PYTHONDONTWRITEBYTECODE="1", **kw)
    return env


def _check(r):
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    import oracle
    lib = oracle.build(sanitize=True, out=str(tmp_path / "libsonooracle_san.so"))
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_oracle_pins.py", "tests/test_host_logic.py",
                        "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider"],
                       cwd=ROOT, capture_output=True, text=True, timeout=900,
                       env=_clean_env(LD_PRELOAD=asan, SONO_ORACLE_LIB=lib))
    _check(r)
    assert " passed" in r.stdout


DRIVER = textwrap.dedent('''
    import ctypes as C, math, sys
    L = C.CDLL(sys.argv[1])
    I32, P = C.c_int32, C.POINTER
    L.sg_last_error.restype = C.c_char_p
    assert L.sg_version() > 0
    q = (I32 * 4096)()
    assert L.sg_noise_quantiles(q) == 0 and q[2048] == 321 and q[0] == -q[4095]
    assert L.sg_noise_quantiles(None) != 0 and L.sg_last_error()
    L.sg_audit_decide.argtypes = [I32, C.c_void_p, C.c_float, C.c_float, C.c_void_p, P(I32)]
    for vals, thr, frac in [([35.0, 29.9, 30.0, math.nan], 30.0, 0.5), ([], 30.0, 0.0),
                            ([31.0] * 64, math.inf, 0.25), ([31.0] * 64, -math.inf, 0.0)]:
        n = len(vals)
        ps = (C.c_float * max(n, 1))(*vals)
        fb = (I32 * max(n, 1))()
        whole = I32(-1)
        assert L.sg_audit_decide(n, ps, thr, frac, fb, C.byref(whole)) == 0 and whole.value in (0, 1)
    assert L.sg_audit_decide(-1, None, 30.0, 0.5, None, None) != 0
    assert L.sg_audit_decide(2, None, 30.0, 0.5, None, None) != 0
    # argument checks before any device call
    L.sg_create.argtypes = [C.c_void_p, I32, C.c_void_p]
    assert L.sg_create(None, 0, None) != 0
    assert L.sg_destroy(None) != 0 or True
    for name in ("sg_volume_register", "sg_tissue_table_set", "sg_simulate", "sg_batch_step", "sg_surr_create"):
        fn = getattr(L, name)
        fn.argtypes = None
    assert L.sg_volume_register(None, None, None) != 0
    assert L.sg_tissue_table_set(None, None, I32(0)) != 0
    assert L.sg_surr_create(None, I32(64), I32(64), C.c_uint64(0), None) != 0
    print("driver ok")
''')


def test_library_host_entry_points_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_2507_01152_amd import build as b
    lib = b.build(sanitize=True, lib=str(tmp_path / "libsonosim_san.so"), obj_dir=str(tmp_path / "obj"))
    rt = subprocess.check_output([b.HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()
    if not os.path.exists(rt):
        import glob
        cands = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        assert cands, "clang's shared ASan runtime not found"
        rt = cands[0]
    drv = tmp_path / "driver.py"
    drv.write_text(DRIVER)
    r = subprocess.run([sys.executable, str(drv), lib], capture_output=True, text=True, timeout=300,
                       env=_clean_env(LD_PRELOAD=rt))
    _check(r)
    assert "driver ok" in r.stdout
