"""Failure handling through the C-ABI on the GPU: argument errors are rejected
before anything is enqueued, non-finite and ill-conditioned inputs end with a
status (never a hang), the tuning table is read by the library, and repeated
runs are bitwise identical.  Every condition is forced from the host; no kernel
is made to fault or wait forever."""
import ctypes
import json
import os

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

INVALID, NOT_INIT, WS_SMALL, UNSUPPORTED, ARCH = 1, 2, 5, 6, 4


@pytest.fixture(scope="module")
def cds():
    import paper_1511_07174_amd as m
    oracle.build()
    m.lib()
    return m


def dev():
    return torch.device("cuda", 0)


def to_dev(a, dtype=torch.float64):
    return torch.from_numpy(np.asfortranarray(a)).to(dev(), dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def P(t, offset_bytes=0):
    return ctypes.c_void_p(t.data_ptr() + offset_bytes) if t is not None else ctypes.c_void_p(0)


def test_bad_arguments_are_rejected_before_any_work(cds):
    """n < 0, lda < n, null or misaligned pointers, nrhs < 0, bad options, bad refinement parameters and
    a workspace that is too small return their status; the sentinel matrices are left untouched."""
    L = cds.lib()
    h = cds.handle()
    n = 96
    A0 = synth.uniform_system(n, 1, 5)[0]
    A = to_dev(A0)
    B = to_dev(np.ones((n, 2)))
    ipiv = torch.full((n,), -7, dtype=torch.int32, device=dev())
    info = torch.full((1,), -7, dtype=torch.int32, device=dev())
    h.bind(1 << 20)
    hh = h.h
    cases = [
        (L.cds_dgetrf(hh, -1, P(A), n, P(ipiv), P(info)), INVALID),
        (L.cds_dgetrf(hh, n, P(A), n - 1, P(ipiv), P(info)), INVALID),
        (L.cds_dgetrf(hh, n, None, n, P(ipiv), P(info)), INVALID),
        (L.cds_dgetrf(hh, n, P(A), n, None, P(info)), INVALID),
        (L.cds_dgetrf(hh, n, P(A), n, P(ipiv), None), INVALID),
        (L.cds_dgetrf(hh, n, P(A, 4), n, P(ipiv), P(info)), INVALID),          # misaligned for FP64
        (L.cds_dgetrf(hh, n, P(A), n, P(ipiv, 2), P(info)), INVALID),
        (L.cds_dgetrf(None, n, P(A), n, P(ipiv), P(info)), NOT_INIT),
        (L.cds_dgetrs(hh, 0, n, -1, P(A), n, P(ipiv), P(B), n), INVALID),
        (L.cds_dgetrs(hh, 2, n, 1, P(A), n, P(ipiv), P(B), n), INVALID),        # op neither N nor T
        (L.cds_dgetrs(hh, 0, n, 2, P(A), n, P(ipiv), P(B), n - 1), INVALID),
        (L.cds_dgetrs(hh, 0, n, 1, P(A), n, None, P(B), n), INVALID),
        (L.cds_dpotrf(hh, 1, n, P(A), n, P(info)), INVALID),                   # fill other than lower
        (L.cds_dpotrf(hh, 0, n, P(A), 0, P(info)), INVALID),
        (L.cds_dpotrs(hh, 0, n, 1, P(A), n, P(B, 8), n - 2), INVALID),
        (L.cds_set_option(hh, 0, 1000), INVALID),                              # block size beyond 512
        (L.cds_set_option(hh, 99, 1), INVALID),
    ]
    bad = cds.default_params(tol=-1.0)
    res = torch.zeros(cds.cds.IR_RESULT_BYTES, dtype=torch.uint8, device=dev())
    X = torch.zeros(n, dtype=torch.float64, device=dev())
    LUlo = torch.empty(n * n, dtype=torch.float32, device=dev())
    cases.append((L.cds_dgesv_mixed(hh, 0, n, 1, P(A), n, P(B), n, P(X), n, P(LUlo), P(ipiv), ctypes.byref(bad),
                                    P(res)), INVALID))
    cases.append((L.cds_dgesv_mixed(hh, 5, n, 1, P(A), n, P(B), n, P(X), n, P(LUlo), P(ipiv), None, P(res)),
                  INVALID))                                                    # unknown precision
    cases.append((L.cds_dposv_mixed_vbatched(hh, 1, 1, 4, None, None, None, None, None, None, None, 4, None, None,
                                             P(res), None, None), UNSUPPORTED))  # BF16 batched: not offered
    cases.append((L.cds_dposv_mixed_vbatched(hh, 0, 1, 2000, None, None, None, None, None, None, None, 4, None,
                                             None, P(res), None, None), INVALID))   # nmax above 1024
    for got, want in cases:
        assert got == want, (got, want)
    # a workspace smaller than getrf needs
    ws = torch.empty(4096, dtype=torch.uint8, device=dev())
    assert L.cds_set_workspace(hh, P(ws, (256 - ws.data_ptr() % 256) % 256), 1024) == 0
    assert L.cds_dgetrf(hh, n, P(A), n, P(ipiv), P(info)) == WS_SMALL
    assert L.cds_set_workspace(hh, P(ws, 1), 1024) == INVALID                 # misaligned workspace
    assert L.cds_set_workspace(hh, None, 0) == 0
    assert L.cds_dgetrf(hh, n, P(A), n, P(ipiv), P(info)) == WS_SMALL         # no workspace at all
    h._ws = None                                                               # the next bind installs a fresh one
    h._ws_bytes = 0
    torch.cuda.synchronize()
    assert np.array_equal(host(A), A0)
    assert np.all(host(ipiv) == -7) and int(info.item()) == -7
    assert np.all(host(B) == 1.0)
    # n = 0 is a valid no-op that still writes info = 0
    h.bind(1 << 20)
    assert L.cds_dgetrf(h.h, 0, None, 1, None, P(info)) == 0
    assert int(info.item()) == 0


def test_nonfinite_inputs_end_with_a_status(cds):
    """NaN / Inf in A or b: every call returns, no bounded wait times out, the refinement reports a
    non-finite stop (reason 4) or a failed factorization (5), and the Cholesky reports the column."""
    n = 300
    A, X, B = synth.uniform_system(n, 1, 6)
    h = cds.handle()
    An = A.copy()
    An[17, 40] = np.nan
    LU, ipiv, info = cds.getrf(to_dev(An))
    torch.cuda.synchronize()
    p = host(ipiv)
    assert np.all(p >= np.arange(1, n + 1)) and np.all(p <= n)                 # a valid interchange sequence
    assert h.device_error() == 0
    Ai = A.copy()
    Ai[3, 3] = np.inf
    LU, ipiv, info = cds.getrf(to_dev(Ai))
    x = cds.getrs(LU, ipiv, to_dev(B[:, 0]))
    torch.cuda.synchronize()
    assert h.device_error() == 0
    bn = B[:, 0].copy()
    bn[5] = np.nan
    xs, res = cds.solve(to_dev(A), to_dev(bn), precision="fp32")
    assert not res[0].converged and res[0].stop_reason == 4, res[0]
    xs, res = cds.solve(to_dev(An), to_dev(B[:, 0]), precision="fp32")
    assert not res[0].converged and res[0].stop_reason in (4, 5), res[0]
    S = synth.spd_matrix(200, 9)
    S[150, 150] = np.nan
    L, info = cds.potrf(to_dev(S))
    assert int(info.item()) == 151
    assert h.device_error() == 0


def test_hilbert_fp32_does_not_converge_then_falls_back(cds):
    """Hilbert n = 12 (kappa_inf about 4e16): refinement on FP32 factors cannot converge and says so;
    with the FP64 fallback the solve ends with a backward error within the bar (the oracle's check)."""
    n = 12
    i = np.arange(n, dtype=np.float64)
    H = 1.0 / (i[:, None] + i[None, :] + 1.0)
    b = H @ np.ones(n)
    X, res = cds.solve(to_dev(H), to_dev(b), precision="fp32")
    r = res[0]
    assert not r.converged and r.stop_reason in (2, 3, 4), r
    assert not r.fell_back
    Xf, resf = cds.solve(to_dev(H), to_dev(b), precision="fp32", params=cds.default_params(fallback=1))
    rf = resf[0]
    assert rf.fell_back and rf.converged, rf
    assert oracle.eta_inf(H, host(Xf), b) <= 1e-14
    assert cds.handle().device_error() == 0


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_repeated_runs_are_bitwise_identical(cds, dtype):
    """20 runs of getrf + getrs at n = 2048 (two streams, look-ahead) give the same bits every time."""
    n = 2048
    A, X, B = synth.uniform_system(n, 1, 7)
    Ad = to_dev(A, dtype)
    bd = to_dev(B[:, 0], dtype)
    ref = None
    for rep in range(20):
        LU, ipiv, info = cds.getrf(Ad)
        x = cds.getrs(LU, ipiv, bd)
        out = (host(LU), host(ipiv), host(x))
        if ref is None:
            ref = out
            continue
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), rep
        assert np.array_equal(out[2], ref[2]), rep
    assert cds.handle().device_error() == 0


def test_cds_tune_installs_the_table(cds, tmp_path):
    """cds_tune reads the JSON table into the handle: the getrf workspace query follows the block size it
    names; a refused table leaves the installed one in place."""
    from paper_1511_07174_amd import tune
    from paper_1511_07174_amd.cds import CdsError, R_64F
    h = cds.handle()
    n = 4096

    def ws_bytes():
        return h._size("cds_getrf_bufferSize", R_64F, n, 1)
    try:
        sizes = {}
        for nb in (64, 512):
            p = tmp_path / ("t%d.json" % nb)
            p.write_text(json.dumps({"arch": "gfx950", "entries": [
                {"key": "getrf_nb", "dtype": "f64", "n_max": 1 << 20, "value": nb}]}))
            h.tune(str(p))
            sizes[nb] = ws_bytes()
        assert sizes[512] > sizes[64]
        bad = tmp_path / "bad.json"
        bad.write_text(json.dumps({"arch": "gfx942", "entries": []}))
        with pytest.raises(CdsError):
            h.tune(str(bad))
        assert ws_bytes() == sizes[512]
    finally:
        path = tune.default_table_path()
        if os.path.exists(path):
            h.tune(path)
        else:
            h.tune_clear()
