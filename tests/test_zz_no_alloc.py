"""The no-allocation mixed solver (cds_dgesv_mixed_noalloc) against the
workspace entry point (cds_dgesv_mixed) through the C-ABI: the same kernels on
the same inputs, so X, the FP32 factors, the pivots and the result record must
be bitwise equal.  Two calls in a row, the second smaller, so that the second
runs on the scratch the first left behind."""
import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cds():
    import paper_1511_07174_amd as m
    m.lib()
    return m


def _run(cds, A, B, precision, noalloc):
    from paper_1511_07174_amd.cds import IR_RESULT_BYTES, decode_results
    d = torch.device("cuda", 0)
    n, nrhs = A.shape[0], B.shape[1]
    Ad = torch.from_numpy(np.asfortranarray(A)).to(d)
    Bd = torch.from_numpy(np.asfortranarray(B)).to(d)
    Ad = cds.cds.colmajor(Ad)
    Bd = cds.cds.colmajor(Bd)
    X = cds.cds.colmajor(torch.full((n, nrhs), np.nan, dtype=torch.float64, device=d))
    LU = torch.full((n * n,), np.nan, dtype=torch.float32, device=d)
    ipiv = torch.full((n,), -1, dtype=torch.int32, device=d)
    res = torch.zeros(IR_RESULT_BYTES, dtype=torch.uint8, device=d)
    h = cds.handle()
    if noalloc:
        h.gesv_mixed_noalloc(Ad, Bd, X, LU, ipiv, res, precision=precision)
    else:
        h.gesv_mixed(Ad, Bd, X, LU, ipiv, res, precision=precision)
    torch.cuda.synchronize()
    return X.cpu().numpy(), LU.cpu().numpy(), ipiv.cpu().numpy(), res.cpu().numpy(), decode_results(res)[0]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_noalloc_matches_workspace_entry_point(cds, precision):
    for n, nrhs, seed in ((1500, 3, 51), (700, 1, 52)):
        A, Xt, B = synth.uniform_system(n, nrhs, seed)
        ref = _run(cds, A, B, precision, noalloc=False)
        got = _run(cds, A, B, precision, noalloc=True)
        assert np.array_equal(got[2], ref[2]), (n, "pivots")
        assert np.array_equal(got[1], ref[1]), (n, "factors")
        assert np.array_equal(got[0], ref[0]), (n, "solution")
        assert np.array_equal(got[3], ref[3]), (n, "result record")
        assert got[4].info == 0, got[4]
        if precision == "fp32":   # BF16 factors of a uniform random matrix need more than classical refinement
            assert got[4].converged, got[4]
    assert cds.handle().device_error() == 0


def test_noalloc_rejects_what_the_scratch_cannot_hold(cds):
    L = cds.lib()
    h = cds.handle()
    d = torch.device("cuda", 0)
    t = torch.zeros(64, dtype=torch.float64, device=d)
    p = ctypes.c_void_p(t.data_ptr())
    prm = cds.default_params()
    # n = 65536 with one right-hand side needs about 138 MiB of scratch: refused before any work
    assert L.cds_dgesv_mixed_noalloc(h.h, 0, 65536, 1, p, 65536, p, 65536, p, 65536, p, p, ctypes.byref(prm), p) == 5
    fb = cds.default_params(fallback=1)
    assert L.cds_dgesv_mixed_noalloc(h.h, 0, 8, 1, p, 8, p, 8, p, 8, p, p, ctypes.byref(fb), p) == 6
    assert L.cds_dgesv_mixed_noalloc(h.h, 0, 8, 1, p, 7, p, 8, p, 8, p, p, ctypes.byref(prm), p) == 1
