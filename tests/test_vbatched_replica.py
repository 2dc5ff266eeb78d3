"""Host replica of the batched SPD kernel's scratch carving and index
arithmetic (csrc/vbatched.hip), evaluated on the CPU for every lane, wave and
loop trip: every access to the factor region W, the inverse region Winv, the
residual column sums cp and the LDS arrays stays in bounds, and every loop
ends, for nmax in {32, 64, 96}, every n <= nmax, both block widths, and the
skip path of sizes outside [1, nmax].  The expressions below restate the
kernel's; a change to one must be made to the other."""
import itertools

import numpy as np
import pytest

VNT, VNMAX, VNR, WPAD, SP = 256, 1024, 4, 32, 68


def round64(n):
    return (n + 63) // 64 * 64


def carve(nmax):
    w = round64(nmax) * (round64(nmax) + WPAD)
    inv = round64(nmax) * 64
    cpd = round64(nmax) * 16 // 2            # doubles of the residual column sums
    return w, inv, cpd, w + inv + round64(nmax) * 16


class Bounds:
    def __init__(self, nmax):
        self.w, self.inv, self.cp, self.wg = carve(nmax)
        self.hits = {}

    def chk(self, name, idx, lo, hi):
        idx = np.asarray(idx)
        if idx.size == 0:
            return
        assert idx.min() >= lo and idx.max() < hi, (name, int(idx.min()), int(idx.max()), lo, hi)
        self.hits[name] = self.hits.get(name, 0) + idx.size


def lanes():
    lane = np.arange(64)
    return lane, lane & 15, lane >> 4


def vb_potrf(B, n, JW):
    np_ = (n + JW - 1) // JW * JW
    ldw = np_ + WPAD
    RT, CT, CHR = 2, JW // 16, 128
    lane, li, lg = lanes()
    for J in range(np_ // JW):
        j0 = J * JW
        nsl = j0 // 32
        for r0 in range(j0, np_, CHR):
            for wave in range(4):
                wr0 = r0 + 32 * wave
                active = wr0 < np_
                if active and nsl > 0:
                    for s, h, rt, ct in itertools.product(range(nsl), range(2), range(RT), range(CT)):
                        a = (wr0 + 16 * rt + li) * ldw + 4 * lg + 32 * s + 16 * h
                        b = (j0 + 16 * ct + li) * ldw + 4 * lg + 32 * s + 16 * h
                        B.chk("W load (update rows)", np.concatenate([a, a + 3]), 0, B.w)
                        B.chk("W load (block rows)", np.concatenate([b, b + 3]), 0, B.w)
                        # the loads read only columns already factored
                        assert (4 * lg + 32 * s + 16 * h + 3).max() < j0
                nd = JW // 32 if r0 == j0 else 0
                if r0 == j0 and wave < nd:
                    for rt, ct, v in itertools.product(range(RT), range(CT), range(4)):
                        B.chk("LDS S row", 32 * wave + 16 * rt + 4 * lg + v, 0, 64)
                        B.chk("LDS S col", 16 * ct + li, 0, SP)
                if active and wave >= nd:
                    for rt, ct, v in itertools.product(range(RT), range(CT), range(4)):
                        row = wr0 + 16 * rt + 4 * lg + v
                        B.chk("W store (rows below)", row * ldw + j0 + 16 * ct + li, 0, B.w)
                        assert row.max() < np_
            # vb_diag (wave 0 of the diagonal chunk): Wd rows/cols < JW, Wi = Winv + J JW JW
            r = lane
            c = np.arange(JW)
            B.chk("W store (diagonal block)", ((j0 + r[r < JW])[:, None] * ldw + j0 + c[None, :]).ravel(), 0, B.w)
            B.chk("Winv store", (J * JW * JW + np.arange(JW)[:, None] * JW + c[None, :]).ravel(), 0, B.inv)
    return np_, ldw


def vb_potrs(B, np_, ldw, JW):
    tid = np.arange(VNT)
    KP, UN = VNT // JW, 16
    CQ, UB = JW // 4, 8
    RP = VNT // CQ
    nbJ = np_ // JW
    for J in range(nbJ):
        j0 = J * JW
        i, p = tid % JW, tid // JW
        m = p < VNR
        B.chk("Winv load (forward)", (J * JW * JW + i[m] * JW)[:, None] + np.arange(JW)[None, :], 0, B.inv)
        nbt = (j0 + 4 * KP * UN - 1) // (4 * KP * UN)
        for bt, u in itertools.product(range(nbt), range(UN)):
            k = 4 * p + 4 * KP * (bt * UN + u)
            ld = k < j0
            B.chk("W load (forward)", ((j0 + i) * ldw + 4 * p + 4 * KP * (bt * UN + u))[ld][:, None]
                  + np.arange(4)[None, :], 0, B.w)
            kk = np.minimum(k, np_ - 4)
            B.chk("LDS y (forward)", np.concatenate([kk, kk + 3]), 0, VNMAX)
        B.chk("LDS part (forward)", ((p * JW + i) * VNR)[:, None] + np.arange(4)[None, :], 0, 4096)
        B.chk("LDS y (block rows)", j0 + i, 0, np_)
    for J in range(nbJ - 1, -1, -1):
        j0 = J * JW
        i, p = tid % JW, tid // JW
        cq, rp = tid % CQ, tid // CQ
        nbt = (np_ - j0 - JW + RP * UB - 1) // (RP * UB)
        for bt, u in itertools.product(range(nbt), range(UB)):
            r = j0 + JW + rp + RP * (bt * UB + u)
            ld = r < np_
            base = (j0 + JW + rp + RP * (bt * UB + u)) * ldw + j0 + 4 * cq
            B.chk("W load (backward)", base[ld][:, None] + np.arange(4)[None, :], 0, B.w)
            B.chk("LDS y (backward)", np.minimum(r, np_ - 1), 0, VNMAX)
        B.chk("LDS part (backward)", ((rp * JW + 4 * cq)[:, None] + np.arange(4)[None, :]) * VNR + 3, 0, 4096)
        m = p < VNR
        B.chk("LDS part (backward read)", ((np.arange(RP)[:, None] * JW + i[m][None, :]) * VNR + p[m]).ravel(), 0, 4096)


def vb_residual(B, n, np_, lda):
    lane, _, _ = lanes()
    cc, r = lane >> 4, lane & 15
    UN = 16
    ng = (n + 3) // 4

    def nbat_c(g):
        return (n - 4 * g - 1 + 16 * UN - 1) // (16 * UN)

    for wave in range(4):
        g = wave
        while g < ng and nbat_c(g) == 0:
            g += 4
        trips = 0
        while g < ng:
            for b in range(nbat_c(g)):
                i = 4 * g + cc
                for u in range(UN):
                    c = 4 * g + 1 + r + 16 * (b * UN + u)
                    ok = (i < n) & (c > i) & (c < n)
                    B.chk("A load (column part)", (np.minimum(i, n - 1) * lda + c)[ok], 0, n * lda)
                    B.chk("LDS xs (column part)", np.minimum(c, n - 1), 0, VNMAX)
                trips += 1
                assert trips <= 4 * n + 8, "column-part pipeline does not end"
            i = 4 * g + cc
            B.chk("cp store", ((i * 8)[(r == 0) & (i < n)])[:, None] + np.arange(VNR + 1)[None, :], 0, B.cp)
            g += 4
            while g < ng and nbat_c(g) == 0:
                g += 4
    nm = (np_ + VNT - 1) // VNT
    tid = np.arange(VNT)
    for wave in range(4):
        for m in range(nm):
            wlo = VNT * m + 64 * wave
            nb = (min(n - 1, wlo + 63) + UN) // UN if wlo < n else 0
            i = VNT * m + 64 * wave + lane
            for b in range(nb):
                for u in range(UN):
                    j = b * UN + u
                    ok = (i < n) & (j <= i)
                    B.chk("A load (row part)", (i + j * lda)[ok], 0, n * lda)
                    B.chk("LDS xs (row part)", np.array([min(j, n - 1)]), 0, VNMAX)
            B.chk("cp load", ((i * 8)[i < n])[:, None] + np.arange(VNR + 1)[None, :], 0, B.cp)
            B.chk("LDS y (residual)", i[i < np_], 0, VNMAX)
    assert tid.size == VNT


def persistent_loop(sizes, nmax, grid):
    """The ticket loop with its skip path: every workgroup ends after at most batch + 1 draws."""
    batch = len(sizes)
    ticket = 0
    done = [False] * grid
    draws = [0] * grid
    handled = []
    while not all(done):
        for w in range(grid):
            if done[w]:
                continue
            t = ticket
            ticket += 1
            draws[w] += 1
            if t >= batch:
                done[w] = True
                continue
            assert draws[w] <= batch + 1
            n = sizes[t]
            handled.append((t, 1 <= n <= nmax and n <= VNMAX))
    assert sorted(t for t, _ in handled) == list(range(batch))
    return handled


@pytest.mark.parametrize("nmax", [32, 64, 96])
def test_every_access_in_bounds(nmax):
    for JW in (32, 64):
        for n in range(1, nmax + 1):
            B = Bounds(nmax)
            np_, ldw = vb_potrf(B, n, JW)
            assert np_ <= round64(nmax) and np_ <= VNMAX
            vb_potrs(B, np_, ldw, JW)
            for lda in (n, n + 3):
                vb_residual(B, n, np_, lda)
            assert B.hits, n


def test_the_skipped_case_takes_only_in_bounds_paths():
    """The sizes of the batched test kept off the GPU (50, 80, 40 with nmax = 64, grid 3): 80 is
    skipped before any of its memory is touched, the other two stay inside one workgroup's region."""
    handled = persistent_loop([50, 80, 40], 64, 3)
    assert dict(handled) == {0: True, 1: False, 2: True}
    for n in (50, 40):
        for JW in (32, 64):
            B = Bounds(64)
            np_, ldw = vb_potrf(B, n, JW)
            vb_potrs(B, np_, ldw, JW)
            vb_residual(B, n, np_, n)


@pytest.mark.parametrize("grid", [1, 3, 512])
def test_ticket_loop_ends(grid):
    for sizes in ([50, 80, 40], [0, 2000, 5, 1], list(range(1, 40))):
        persistent_loop(sizes, 64, grid)
