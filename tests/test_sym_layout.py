"""Host checks of the tiling rules the symmetric-reuse regulariser relies on
(no GPU): for every accepted (patch, window) and a range of image sides,

  * the tiles whose regions (the tile grown by the window radius R) hold a
    pixel are the ones the combining kernel enumerates, ceil((r - R - T + 1)
    / T) <= t <= floor((r + R) / T) along each axis, with the lower bound
    computed as floor((r - R + 64 T) / T) - 64 as in the kernel;
  * regions of tiles in one residue class (t mod m along each axis, m the
    number of tiles whose regions can hold one pixel) never overlap, so the
    class planes take each region's sums without a race;
  * the tiles that hold a pixel fall in distinct classes.

Tile sizes as in the kernel: T_x = 32 - 2S columns, T_y = 16 rows (4 rows per
lane)."""
import itertools

import pytest

TH = 16


def tiles_holding(r, R, T, n):
    return [t for t in range(n) if t * T - R <= r < t * T + T + R]


def kernel_range(r, R, T, n):
    lo = max(0, (r - R + 64 * T) // T - 64)
    hi = min(n - 1, (r + R) // T)
    return list(range(lo, hi + 1))


def classes(T, R):
    return -(-(T + 2 * R) // T)


SUPPORTED = [(p, w) for p in (3, 5, 7, 9) for w in range(3, 20, 2) if not (w == 19 and p == 3)]


@pytest.mark.parametrize("patch,window", SUPPORTED)
def test_region_rules(patch, window):
    S, R = patch // 2, window // 2
    TW = 32 - 2 * S
    for T in (TW, TH):
        m = classes(T, R)
        assert m * T >= T + 2 * R
        for L in (window, 33, 64, 127):
            n = -(-L // T)
            for r in range(L):
                held = tiles_holding(r, R, T, n)
                assert kernel_range(r, R, T, n) == held
                assert len({t % m for t in held}) == len(held)
            for t1, t2 in itertools.combinations(range(n), 2):
                if t1 % m == t2 % m:   # same class: regions apart
                    assert t2 * T - R >= t1 * T + T + R or t1 * T - R >= t2 * T + T + R
