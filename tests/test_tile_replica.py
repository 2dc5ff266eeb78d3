"""Host replica of the trailing-update GEMM's tile enumeration (gemm.hip tile_count and
tile_coords): workgroup w -> tile (tm, tn), with the XCD remap (each XCD, w % 8, takes a
contiguous range of tile ids), bands of 16 tile rows for the full mode, and the lower mode
(m >= n: the triangle of the top tile rows, then the full tile rows below it) that the
Cholesky updates use.  Every launch must cover each wanted tile exactly once and no other;
a plain enumeration of the wanted tiles is the reference.  No GPU needed."""
import math

import numpy as np
import pytest

GM = 16


def tile_count(tiles_m, tiles_n, lower):
    return tiles_n * (tiles_n + 1) // 2 + (tiles_m - tiles_n) * tiles_n if lower else tiles_m * tiles_n


def tile_coords(w, tiles_m, tiles_n, lower):
    total = tile_count(tiles_m, tiles_n, lower)
    per = total // 8
    t = (w % 8) * per + w // 8 if per > 0 and w < per * 8 else w
    if not lower:
        band, r = divmod(t, GM * tiles_n)
        rows = min(GM, tiles_m - band * GM)
        return band * GM + r % rows, r // rows
    tri = tiles_n * (tiles_n + 1) // 2
    if t < tri:
        # the kernel's float estimate of the triangle row, then its integer corrections
        r = int((math.sqrt(8.0 * t + 1.0) - 1.0) * 0.5)
        while (r + 1) * (r + 2) // 2 <= t:
            r += 1
        while r * (r + 1) // 2 > t:
            r -= 1
        return r, t - r * (r + 1) // 2
    q = t - tri
    return tiles_n + q // tiles_n, q % tiles_n


def wanted(tiles_m, tiles_n, lower):
    return {(i, j) for i in range(tiles_m) for j in range(tiles_n) if not lower or i >= j}


@pytest.mark.parametrize("lower", [False, True])
@pytest.mark.parametrize("m,n,tb", [(128, 128, 128), (16256, 16256, 128), (16256, 128, 64), (1000, 1000, 64),
                                    (5000, 192, 64), (300, 300, 128), (64, 64, 64), (900, 130, 128),
                                    (16384, 192, 128), (4096, 4096, 128)])
def test_each_tile_once(m, n, tb, lower):
    if lower and m < n:
        pytest.skip("lower mode needs m >= n")
    tm, tn = -(-m // tb), -(-n // tb)
    total = tile_count(tm, tn, lower)
    got = [tile_coords(w, tm, tn, lower) for w in range(total)]
    assert len(set(got)) == total
    assert set(got) == wanted(tm, tn, lower)


def test_lower_square_is_the_triangle():
    for t in range(1, 130):
        assert tile_count(t, t, True) == t * (t + 1) // 2


def test_planted_mistake_is_caught():
    # a rectangle part that starts one tile row too early covers a triangle tile twice
    def bad(w, tiles_m, tiles_n):
        tri = tiles_n * (tiles_n + 1) // 2
        if w < tri:
            return tile_coords(w, tiles_m, tiles_n, True)
        q = w - tri
        return tiles_n - 1 + q // tiles_n, q % tiles_n
    tm, tn = 40, 3
    got = [bad(w, tm, tn) for w in range(tile_count(tm, tn, True))]
    assert set(got) != wanted(tm, tn, True)
