"""Autotuner for the library's tile and block sizes.

Times candidate settings on the device, keeps the fastest per size bucket and
persists a JSON table; ``load_table`` installs a table into a handle through
``cds_tune`` (the library reads the file).  Tuned quantities:

* ``getrf_nb`` (per dtype, per n bucket): block size of the blocked LU, from
  {128, 160, 192, 224, 256, 384, 512}, on the benchmark's uniform systems;
* ``potrf_nb``: same for Cholesky, from {128, 256, 384, 512}, on the seeded
  SPD matrices;
* ``vbatch_tile`` (per n bucket): block-column width of the in-workgroup
  Cholesky of the batched SPD solver, 16 or 32.

Inputs are the seeded synthetic matrices of ``synth`` at the tuned sizes.  The entry of a size
bucket applies to every n up to the bucket's size; the largest bucket's value
is repeated for all larger n.  ``handle()`` installs the table shipped with the
package (``tune_gfx950.json``) when it exists; ``CDS_TUNE_FILE`` names another
table, or ``none`` to run on the built-in defaults.

Run: ``python -m paper_1511_07174_amd.tune --out tune_gfx950.json``.
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import cds
from .cds import colmajor

KEYS = {"getrf_nb": cds.TUNE_GETRF_NB, "potrf_nb": cds.TUNE_POTRF_NB, "vbatch_tile": cds.TUNE_VBATCH_TILE}
DTYPES = {"f64": cds.R_64F, "f32": cds.R_32F}


def _timeit(fn, reps=2):
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return best


def tune_getrf(sizes=(2048, 4096, 8192, 16384), dtypes=("f64", "f32"),
                candidates=(128, 160, 192, 224, 256, 384, 512), seed=0):
    """Block size per size bucket, timed on the benchmark's workload: the seeded uniform[-1, 1]
    systems of synth.uniform_system."""
    import synth
    h = cds.handle()
    dev = torch.device("cuda", torch.cuda.current_device())
    entries, timings = [], []
    for dt in dtypes:
        tdt = torch.float64 if dt == "f64" else torch.float32
        for n in sizes:
            A = colmajor(torch.from_numpy(synth.uniform_system(n, 1, seed)[0]).to(dev, tdt))
            LU = torch.empty_like(A)
            ipiv = torch.zeros(n, dtype=torch.int32, device=dev)
            info = torch.zeros(1, dtype=torch.int32, device=dev)
            best = None
            for nb in candidates:
                h.set_option(cds.OPT_NB, nb)

                def run():
                    LU.copy_(A)
                    h.getrf_(LU, ipiv, info)
                t = _timeit(run)
                timings.append({"dtype": dt, "n": n, "nb": nb, "ms": t * 1e3})
                if best is None or t < best[1]:
                    best = (nb, t)
            h.set_option(cds.OPT_NB, 0)
            entries.append({"key": "getrf_nb", "dtype": dt, "n_max": n, "value": best[0]})
            del A, LU
        entries.append({"key": "getrf_nb", "dtype": dt, "n_max": 2 ** 31 - 1, "value": entries[-1]["value"]})
    return entries, timings


def tune_potrf(sizes=(2048, 4096, 8192, 16384), dtypes=("f64", "f32"), candidates=(128, 256, 384, 512), seed=4):
    """Block size per size bucket on the seeded SPD matrices of synth.spd_matrix."""
    import synth
    h = cds.handle()
    dev = torch.device("cuda", torch.cuda.current_device())
    entries, timings = [], []
    for dt in dtypes:
        tdt = torch.float64 if dt == "f64" else torch.float32
        for n in sizes:
            A = colmajor(torch.from_numpy(synth.spd_matrix(n, seed)).to(dev, tdt))
            L = torch.empty_like(A)
            info = torch.zeros(1, dtype=torch.int32, device=dev)
            best = None
            for nb in candidates:
                h.set_option(cds.OPT_NB, nb)

                def run():
                    L.copy_(A)
                    h.potrf_(L, info)
                t = _timeit(run)
                timings.append({"op": "potrf", "dtype": dt, "n": n, "nb": nb, "ms": t * 1e3})
                if best is None or t < best[1]:
                    best = (nb, t)
            h.set_option(cds.OPT_NB, 0)
            entries.append({"key": "potrf_nb", "dtype": dt, "n_max": n, "value": best[0]})
            del A, L
        entries.append({"key": "potrf_nb", "dtype": dt, "n_max": 2 ** 31 - 1, "value": entries[-1]["value"]})
    return entries, timings


def tune_vbatched(count=2000, nmax=1024, seed=7, thresholds=(0, 128, 256, 512, 1024)):
    """The batched SPD kernel takes 32-wide block columns for systems up to a threshold and 64-wide ones
    above it.  Time one mixed batch (count systems, n ~ U{32..nmax}, largest first) for each threshold
    and keep the fastest: the workgroups of one launch share the chip, so a bucket timed alone does
    not predict the mix."""
    import numpy as np
    h = cds.handle()
    dev = torch.device("cuda", torch.cuda.current_device())
    rng = np.random.default_rng(seed)
    sizes = rng.integers(32, nmax + 1, size=count)
    g = torch.Generator(device=dev).manual_seed(seed)
    systems = []
    for n in sizes:
        n = int(n)
        M = torch.rand(n, n, generator=g, dtype=torch.float64, device=dev) * 2 - 1
        A = M @ M.T / n + torch.eye(n, dtype=torch.float64, device=dev)
        B = torch.rand(n, 4, generator=g, dtype=torch.float64, device=dev) * 2 - 1
        systems.append((colmajor(A), colmajor(B)))
    # descriptors built once: only the launch is timed
    ordt = torch.as_tensor(np.argsort(-sizes, kind="stable"), dtype=torch.int32, device=dev)
    ns = torch.tensor([a.shape[0] for a, _ in systems], dtype=torch.int32, device=dev)
    Ap = torch.tensor([a.data_ptr() for a, _ in systems], dtype=torch.int64, device=dev)
    lda = torch.tensor([a.stride(1) for a, _ in systems], dtype=torch.int64, device=dev)
    Bp = torch.tensor([b.data_ptr() for _, b in systems], dtype=torch.int64, device=dev)
    ldb = torch.tensor([b.stride(1) for _, b in systems], dtype=torch.int64, device=dev)
    Xs = [colmajor(torch.zeros_like(b)) for _, b in systems]
    Xp = torch.tensor([x.data_ptr() for x in Xs], dtype=torch.int64, device=dev)
    ldx = torch.tensor([x.stride(1) for x in Xs], dtype=torch.int64, device=dev)
    res = torch.zeros(count * cds.IR_RESULT_BYTES, dtype=torch.uint8, device=dev)
    prm = cds.default_params(tol=1e-14, success_tol=1e-14)
    timings = []
    best = None
    for t in thresholds:
        h.tune_clear()
        h.tune_set(cds.TUNE_VBATCH_TILE, cds.R_32F, max(t, 1), 32 if t > 0 else 64)
        ms = _timeit(lambda: h.posv_mixed_vbatched(count, nmax, ns, Ap, lda, Bp, ldb, Xp, ldx, 4, res, order=ordt,
                                                   params=prm, device=dev), reps=3) * 1e3
        timings.append({"vbatch_width32_max_n": t, "systems": count, "ms": ms})
        if best is None or ms < best[1]:
            best = (t, ms)
    h.tune_clear()
    t = best[0]
    entries = [{"key": "vbatch_tile", "dtype": "f32", "n_max": t, "value": 32}] if t > 0 else []
    if t < nmax:
        entries.append({"key": "vbatch_tile", "dtype": "f32", "n_max": nmax, "value": 64})
    return entries, timings


def save_table(path, entries, timings=None):
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    table = {"arch": getattr(props, "gcnArchName", "gfx950"), "cus": props.multi_processor_count,
             "entries": entries, "timings": timings or []}
    with open(path, "w") as f:
        json.dump(table, f, indent=1)
    return path


def load_table(path, handle=None):
    """Install a saved table into a handle (default: the package's handle); the library parses the
    file (cds_tune)."""
    h = handle or cds.handle()
    h.tune(path)
    with open(path) as f:
        return json.load(f)


def default_table_path():
    return os.environ.get("CDS_TUNE_FILE", os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_gfx950.json"))


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="time the candidate block sizes and tile widths, save the table")
    ap.add_argument("--out", default=default_table_path())
    ap.add_argument("--quick", action="store_true", help="only n <= 8192")
    a = ap.parse_args(argv)
    h = cds.handle()
    h.tune_clear()
    sizes = (2048, 4096, 8192) if a.quick else (2048, 4096, 8192, 16384)
    e1, t1 = tune_getrf(sizes=sizes)
    print("getrf", e1, flush=True)
    e2, t2 = tune_potrf(sizes=sizes)
    print("potrf", e2, flush=True)
    e3, t3 = tune_vbatched()
    print("vbatched", e3, flush=True)
    save_table(a.out, e1 + e2 + e3, t1 + t2 + t3)
    print("saved", a.out, flush=True)


if __name__ == "__main__":
    main()
