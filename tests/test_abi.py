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
