"""The C-ABI library loads and exports every function the public header declares."""
import os
import re

import pytest

from paper_2309_06427_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "symstair.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ssp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_set():
    assert declared_functions() == sorted(_lib.SIGNATURES)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsymstair.so is not built (run __graft_entry__.build())")
    L = _lib.load()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_status_strings_without_gpu():
    L = _lib.load()
    assert L.ssp_status_str(0) == b"ok"
    assert L.ssp_status_str(1) == b"invalid argument"


def test_create_rejects_bad_sizes_without_touching_memory():
    import ctypes as C
    import numpy as np
    L = _lib.load()
    h = C.c_void_p()
    z = np.zeros(1, dtype=np.int32)
    p = z.ctypes.data_as(C.POINTER(C.c_int32))
    # nprob = 0 is rejected before any device call
    assert L.ssp_batch_create(0, p, p, p, 0, C.byref(h)) == _lib.SSP_ERR_ARG
    assert L.ssp_batch_create(1, None, p, p, 0, C.byref(h)) == _lib.SSP_ERR_ARG


def test_mlp_param_count_matches_the_layout():
    from oracle import mlp
    L = _lib.load()
    for nx, H in ((6, 128), (14, 128), (26, 128), (3, 16)):
        assert L.ssp_mlp_num_params(nx, H) == mlp.n_params(nx, H)
    assert L.ssp_mlp_num_params(0, 128) == -1


def test_mlp_create_rejects_bad_sizes():
    import ctypes as C
    L = _lib.load()
    h = C.c_void_p()
    assert L.ssp_mlp_create(0, 128, 0, C.byref(h)) == _lib.SSP_ERR_ARG
    assert L.ssp_mlp_create(6, 100, 0, C.byref(h)) == _lib.SSP_ERR_ARG
    assert L.ssp_mlp_create(6, 128, 0, None) == _lib.SSP_ERR_ARG


def test_onchip_horizon_query():
    """ssp_scaled_onchip_horizon is a pure host function.  At the bench's
    mapping (256 threads, 48 336 B of LDS), FP32 storage and the symmetric
    stair (one Horner step), the pass's LDS holds a ring of C + 3 Oh slots and
    two vector windows of C + 3 slots, plus a 16-byte spot:
      nx 6:  C = 40 knots, 43 (36 + 2 * 8) * 4 + 16 = 8 960 B, and the six
             vectors of N knots take 6 * 6 * 4 N = 144 N B: N <= 273;
      nx 14: C = 16 knots, 19 (196 + 2 * 16) * 4 + 16 = 17 344 B, 336 N B:
             N <= 92;
    nx 26 and 36 never keep their vectors in LDS, nor does scalar Jacobi
    (no scaled solve); a larger budget or block-Jacobi (no Horner window)
    holds longer horizons."""
    import ctypes as C
    from paper_2309_06427_amd import solver
    h = lambda nx, pc="sym", prec="fp32_refine64", t=256, l=48336: solver.scaled_onchip_horizon(nx, pc, prec, t, l)
    assert h(6) == 273 and h(14) == 92
    assert h(26) == 0 and h(36) == 0
    assert h(14, pc="jacobi") == 0
    assert h(14, pc="bj") > 92 and h(14, l=64000) > 92
    assert h(14, prec="fp64") < 92
    out = C.c_int32()
    assert _lib.load().ssp_scaled_onchip_horizon(14, 9, 2, 256, 48336, C.byref(out)) != _lib.SSP_OK
