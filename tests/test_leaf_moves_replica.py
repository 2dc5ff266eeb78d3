"""Host replica of the LU panel's per-leaf move lists (lu.hip compose_leaf): after a leaf of wl
columns starting at c0 has chosen its pivot rows piv[0..wl), the rows that change are the
leaf's own positions c0..c1-1 and every pivot row at or beyond c1 (counted once, at the column
that first chose it); each of them receives the row whose content the leaf's interchanges bring
there, found by tracing the position back through the interchanges in reverse order.  Applied
with every source read before any write, the list must give exactly the rows that the
interchanges (rows c0 + t and piv[t] trade places, t = 0, 1, ...) give one at a time.  The
replica covers whole and partial leaves, repeated pivots and pivots inside the leaf.  No GPU
needed."""
import numpy as np
import pytest

W = 32


def sequential(m, c0, piv):
    rows = list(range(m))
    for t, p in enumerate(piv):
        rows[c0 + t], rows[p] = rows[p], rows[c0 + t]
    return rows


def compose(c0, piv, back=True):
    """The kernel's lists: lanes cc < W, pivots read four at a time in the kernel (the order of
    the reads does not matter here), entries of a partial leaf beyond wl read as -1."""
    wl = len(piv)
    c1 = c0 + wl
    pv = list(piv) + [-1] * (W - wl)
    dst, src = [], []
    others = []
    for lane in range(W):
        mypiv = pv[lane] if lane < wl else -1
        other = mypiv >= c1
        for cc in range(W):
            pc = pv[cc] if cc < wl else -1
            other = other and not (cc < lane and pc == mypiv)
        s, o = c0 + lane, mypiv
        order = range(W - 1, -1, -1) if back else range(W)
        for cc in order:
            if cc >= wl:
                continue
            a, b = c0 + cc, pv[cc]
            s = b if s == a else (a if s == b else s)
            o = b if o == a else (a if o == b else o)
        if lane < wl:
            dst.append(c0 + lane)
            src.append(s)
        if other:
            others.append((mypiv, o))
    for d, s in others:
        dst.append(d)
        src.append(s)
    return dst, src


def apply(m, dst, src):
    rows = list(range(m))
    vals = [rows[s] for s in src]          # every source read before any write
    for d, v in zip(dst, vals):
        rows[d] = v
    return rows


def random_leaf(g, m, c0, wl, repeat):
    piv = []
    for t in range(wl):
        lo = c0 + t
        if repeat and piv and g.random() < 0.3:
            cand = [p for p in piv if p >= lo]
            if cand:
                piv.append(int(g.choice(cand)))
                continue
        piv.append(int(g.integers(lo, m)))
    return piv


@pytest.mark.parametrize("wl", [32, 31, 17, 1])
@pytest.mark.parametrize("repeat", [False, True])
def test_move_lists_match_the_interchanges(wl, repeat):
    g = np.random.default_rng(wl * 7 + repeat)
    for trial in range(300):
        m = int(g.integers(wl + 1, 400))
        c0 = int(g.integers(0, m - wl + 1))
        piv = random_leaf(g, m, c0, wl, repeat)
        dst, src = compose(c0, piv)
        assert len(set(dst)) == len(dst) and sorted(dst) == sorted(src)
        assert len(dst) <= 2 * wl
        assert apply(m, dst, src) == sequential(m, c0, piv)


def test_pivots_inside_the_leaf_and_repeats():
    # column 0 takes row c0 + 5 (inside the leaf) and column 5 takes that row again; a row below
    # the leaf is chosen twice; column 2 keeps its own row
    c0, m = 10, 60
    piv = [15, 40, 12, 40, 14, 15]
    dst, src = compose(c0, piv)
    assert apply(m, dst, src) == sequential(m, c0, piv)


def test_planted_mistake_is_caught():
    # tracing the interchanges forward instead of backward breaks the lists
    g = np.random.default_rng(5)
    bad = 0
    for trial in range(50):
        m, c0, wl = 200, 30, 32
        piv = random_leaf(g, m, c0, wl, True)
        dst, src = compose(c0, piv, back=False)
        bad += apply(m, dst, src) != sequential(m, c0, piv)
    assert bad > 0
