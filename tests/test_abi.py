"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and validates arguments on the host before any launch."""
import ctypes

import pytest

import paper_2604_12914_amd as lrcc


@pytest.fixture(scope="module")
def L():
    return lrcc.lib()


def test_exports_every_declared_symbol(L):
    names = lrcc.header_symbols()
    assert "lrcc_ppl_sigma" in names and "lrcc_solve" in names
    assert len(names) >= 11
    for n in names:
        assert hasattr(L, n), n


def test_status_strings(L):
    for code in range(9):
        assert L.lrcc_status_str(code)
    assert L.lrcc_status_str(0) == b"ok"
    assert L.lrcc_version().startswith(b"lrcc")


P = ctypes.c_void_p


def chk(L, o=4, v=24, nchol=64, nrhs=1, Lp=0x1000, X=0x100000, S=0x900000, dt=0, prec=0,
        cmul=0):
    return L.lrcc_check_sigma_args(o, v, nchol, nrhs, P(Lp) if Lp else None,
                                   P(X) if X else None, P(S) if S else None, dt, prec, cmul)


def test_argument_validation(L):
    assert chk(L) == lrcc.OK
    assert chk(L, o=-1) == lrcc.ERR_ARG
    assert chk(L, nchol=-2) == lrcc.ERR_ARG
    assert chk(L, X=0) == lrcc.ERR_ARG
    assert chk(L, S=0) == lrcc.ERR_ARG
    assert chk(L, Lp=0) == lrcc.ERR_ARG
    assert chk(L, dt=7) == lrcc.ERR_ARG
    assert chk(L, prec=9) == lrcc.ERR_ARG
    assert chk(L, cmul=2) == lrcc.ERR_ARG
    assert chk(L, v=5000) == lrcc.ERR_SHAPE
    assert chk(L, nchol=70000) == lrcc.ERR_SHAPE
    assert chk(L, o=8000, nrhs=1) == lrcc.ERR_SHAPE
    assert chk(L, X=0x100008) == lrcc.ERR_ARG        # complex128 needs 16-byte alignment
    assert chk(L, X=0x100008, dt=1) == lrcc.OK       # complex64 needs 8
    assert chk(L, S=0x100000 + 16) == lrcc.ERR_ARG   # sigma overlaps X
    assert b"overlaps" in L.lrcc_last_error(None)


def test_empty_extents_need_no_pointers(L):
    # no pairs (o < 2 or v < 2) or no RHS: nothing to read or write
    assert chk(L, o=1, X=0, S=0, Lp=0) == lrcc.OK
    assert chk(L, v=1, X=0, S=0, Lp=0) == lrcc.OK
    assert chk(L, nrhs=0, X=0, S=0, Lp=0) == lrcc.OK
    # no Cholesky vectors: sigma = 0, L may be NULL
    assert chk(L, nchol=0, Lp=0) == lrcc.OK


def test_create_needs_a_gfx950_device(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert L.lrcc_create(ctypes.byref(h), 0, None) == lrcc.ERR_DEVICE
    assert L.lrcc_ppl_sigma(None, 4, 24, 64, 1, None, None, None, 0, 0, 0) == lrcc.ERR_ARG


SAN_SCRIPT = r"""
import ctypes, sys
L = ctypes.CDLL(sys.argv[1])
P = ctypes.c_void_p
L.lrcc_check_sigma_args.argtypes = [ctypes.c_int] * 4 + [P] * 3 + [ctypes.c_int] * 3
L.lrcc_status_str.restype = ctypes.c_char_p
L.lrcc_last_error.restype = ctypes.c_char_p
L.lrcc_last_error.argtypes = [P]
L.lrcc_version.restype = ctypes.c_char_p
codes = []
def chk(o=4, v=24, nchol=64, nrhs=1, Lp=0x1000, X=0x100000, S=0x900000, dt=0, prec=0, cmul=0):
    codes.append(L.lrcc_check_sigma_args(o, v, nchol, nrhs, P(Lp) if Lp else None,
                                         P(X) if X else None, P(S) if S else None, dt, prec,
                                         cmul))
    L.lrcc_last_error(None)
for kw in [{}, dict(o=-1), dict(nchol=-2), dict(X=0), dict(S=0), dict(Lp=0), dict(dt=7),
           dict(prec=9), dict(cmul=2), dict(v=5000), dict(nchol=70000), dict(o=8000),
           dict(X=0x100008), dict(X=0x100008, dt=1), dict(S=0x100000 + 16), dict(o=1, X=0, S=0),
           dict(o=2**30, nrhs=2**30), dict(v=4096, nchol=65536, o=5792, nrhs=1),
           dict(o=0, v=0, nchol=0, nrhs=0, X=0, S=0, Lp=0)]:
    chk(**kw)
for s in range(-3, 12):
    L.lrcc_status_str(s)
L.lrcc_version()
h = P()
codes.append(L.lrcc_create(ctypes.byref(h), 0, None))
for fn in ("lrcc_destroy", "lrcc_set_timing", "lrcc_set_deterministic"):
    getattr(L, fn).argtypes = [P] + ([ctypes.c_int] if fn != "lrcc_destroy" else [])
    codes.append(getattr(L, fn)(None, *([1] if fn != "lrcc_destroy" else [])))
L.lrcc_last_error(None)
print("codes", codes)
"""


def test_validation_paths_under_address_and_ub_sanitizers(tmp_path):
    # the host validation and status paths of the debug library built with
    # AddressSanitizer and UndefinedBehaviorSanitizer (host code only): any
    # report aborts the child process
    import os
    import subprocess
    import sys

    from paper_2604_12914_amd import build as b
    if not (os.path.exists(b.SAN_OUT) and os.path.exists(b.SANITIZER_RUNTIME)):
        pytest.skip("sanitized debug library or sanitizer runtime not present")
    script = tmp_path / "san.py"
    script.write_text(SAN_SCRIPT)
    env = dict(os.environ, LD_PRELOAD=b.SANITIZER_RUNTIME,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, str(script), b.SAN_OUT], capture_output=True, text=True,
                       env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    codes = eval(r.stdout.split("codes", 1)[1])
    assert codes[0] == lrcc.OK and codes[1] == lrcc.ERR_ARG and codes[9] == lrcc.ERR_SHAPE
    assert codes[16] == lrcc.ERR_SHAPE          # nrhs * o(o-1)/2 far beyond 2^24, no overflow
    assert codes[-4] == lrcc.ERR_DEVICE         # no device visible
    assert codes[-3:] == [lrcc.ERR_ARG] * 3     # NULL handles
