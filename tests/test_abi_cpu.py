"""CPU checks of the boundary: the library loads and exports every function the header declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]
LIB = os.path.join(ROOT, "paper_1107_4192_amd", "libkfmeg.so")


def declared_functions():
    text = "\n".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_][a-z_0-9]*\s*\*?\s+\*?([a-z_][a-z_0-9]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("kf_create", "kf_filter", "kf_smooth", "mne_solve", "kf_destroy"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkfmeg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkfmeg.so not built")
def test_binding_lists_the_same_symbols():
    from paper_1107_4192_amd import kfmeg
    assert sorted(kfmeg.EXPORTS) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkfmeg.so not built")
def test_plan_bytes_host_logic():
    from paper_1107_4192_amd import kfmeg
    b64 = kfmeg.kf_plan_bytes(5124, 306, 200, kfmeg.options())
    b32 = kfmeg.kf_plan_bytes(5124, 306, 200, kfmeg.options(store_fp32=True))
    ck = kfmeg.kf_plan_bytes(5124, 306, 200, kfmeg.options(checkpoint_stride=14))
    store64 = 200 * 5124 * 5136 * 8
    assert b64 > store64 and b32 < b64 and ck < b64
    assert kfmeg.kf_plan_bytes(0, 306, 200, None) == 0
    # the associative smoother's per-call allocation: T - 1 scan elements plus 8 + 16 scratch
    # matrices of N x 5136 float64, and two N-vectors
    assert kfmeg.kf_smooth_assoc_bytes(5124, 200) == (199 + 24) * 5124 * 5136 * 8 + 2 * 5124 * 8
    assert kfmeg.kf_smooth_assoc_bytes(0, 200) == 0 and kfmeg.kf_smooth_assoc_bytes(5124, 0) == 0


def test_product_path_has_no_oracle_import():
    pkg = os.path.join(ROOT, "paper_1107_4192_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkfmeg.so not built")
def test_argument_errors_before_any_launch():
    # Empty or negative sizes and null pointers are rejected on the host, before any device
    # call, with KF_EINVAL and a message; the calls below never reach the GPU.
    lib = ctypes.CDLL(LIB)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.kf_create.argtypes = [ctypes.POINTER(vp), i64, i64, i64, vp, vp, vp, vp, vp, vp, vp]
    lib.kf_create.restype = ctypes.c_int
    lib.kf_last_error.argtypes = [vp]
    lib.kf_last_error.restype = ctypes.c_char_p
    lib.mne_solve.argtypes = [i64, i64, i64, vp, vp, vp, vp, vp, vp]
    lib.mne_solve.restype = ctypes.c_int
    lib.kf_filter.argtypes = [vp, i64, vp, vp, vp]
    lib.kf_filter.restype = ctypes.c_int
    lib.kf_smooth_assoc.argtypes = [vp, vp, vp, vp]
    lib.kf_smooth_assoc.restype = ctypes.c_int
    KF_EINVAL = 1
    dummy = ctypes.c_void_p(16)          # never dereferenced: the sizes are rejected first
    plan = vp()
    for N, m, T in ((0, 3, 4), (5, 0, 4), (5, 3, 0), (-1, 3, 4)):
        st = lib.kf_create(ctypes.byref(plan), N, m, T, dummy, dummy, dummy, dummy, dummy, None, None)
        assert st == KF_EINVAL and not plan.value
        assert b"sizes" in lib.kf_last_error(None)
    st = lib.kf_create(ctypes.byref(plan), 5, 3, 4, None, dummy, dummy, dummy, dummy, None, None)
    assert st == KF_EINVAL and b"null" in lib.kf_last_error(None)
    assert lib.mne_solve(5, 3, 0, dummy, dummy, dummy, dummy, dummy, None) == KF_EINVAL
    assert lib.mne_solve(5, 3, 2, None, dummy, dummy, dummy, dummy, None) == KF_EINVAL
    assert lib.kf_filter(None, 3, dummy, dummy, None) == KF_EINVAL
    assert lib.kf_smooth_assoc(None, dummy, None, None) == KF_EINVAL
