"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/tm.h declares, and rejects bad arguments before touching a
device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tm.h")
LIB = os.path.join(ROOT, "paper_1810_00980_amd", "libtm.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tm_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libtm.so is not built: run python __graft_entry__.py")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for n in ("tm_load_graph", "tm_count_exact", "tm_estimate", "tm_free_graph", "tm_estimate_batch"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing


def test_no_library_symbol_left_undefined(lib):
    """Every function of the library's own sources is defined in it: a
    declaration whose definition went missing would otherwise only fail
    when the library is loaded lazily at the first call."""
    import subprocess
    out = subprocess.run(["nm", "-D", "--undefined-only", LIB], capture_output=True, text=True, check=True).stdout
    own = [ln.split()[-1] for ln in out.splitlines() if re.search(r"tm_|sweepdev|DevGraph|tm_graph", ln)]
    assert not own, own


def test_python_binding_covers_the_abi():
    import paper_1810_00980_amd as tm
    assert set(declared()) == set(tm.EXPORTED)


def test_strerror_and_version(lib):
    lib.tm_strerror.restype = ctypes.c_char_p
    lib.tm_version.restype = ctypes.c_char_p
    assert lib.tm_strerror(0) == b"ok"
    assert lib.tm_strerror(5).startswith(b"count overflows")
    assert b"gfx950" in lib.tm_version()


def test_argument_errors_before_device_work(lib):
    P = ctypes.c_void_p
    out = P()
    f = lib.tm_load_graph
    f.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, P]
    f.restype = ctypes.c_int32
    assert f(None, None, None, -1, 10, 0, None, ctypes.byref(out)) == 1   # m < 0
    assert f(None, None, None, 0, 0, 0, None, ctypes.byref(out)) == 1     # n <= 0
    assert f(None, None, None, 5, 10, 0, None, ctypes.byref(out)) == 1    # NULL arrays
    g = lib.tm_count_exact
    g.argtypes = [P, P, ctypes.c_int64, P, P]
    g.restype = ctypes.c_int32
    buf = (ctypes.c_uint64 * 2)()
    assert g(None, None, 5, buf, None) == 1
    e = lib.tm_estimate
    e.argtypes = [P, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, P, P, P]
    e.restype = ctypes.c_int32
    z = ctypes.c_double()
    assert e(None, None, 10, 2, 0.5, 0, ctypes.byref(z), None, None) == 1


def test_product_code_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_1810_00980_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in txt and "tm_oracle" not in txt and "orc_" not in txt, fn


def test_profile_modes_host_side(lib):
    """Timing switches: 0 off, 1 on, 2 on with each pass's kernels in series;
    anything else is rejected; a name never timed reads as zero launches."""
    assert lib.tm_profile_enable(3) == 1  # TM_EINVAL
    assert lib.tm_profile_enable(-1) == 1
    for on in (2, 1, 0):
        assert lib.tm_profile_enable(on) == 0
    assert lib.tm_profile_reset() == 0
    ms, n = ctypes.c_double(-1.0), ctypes.c_int64(-1)
    assert lib.tm_profile_read(b"crit:sweep3_tri_count", ctypes.byref(ms), ctypes.byref(n)) == 0
    assert (ms.value, n.value) == (0.0, 0)
    assert lib.tm_profile_read(None, ctypes.byref(ms), ctypes.byref(n)) == 1
