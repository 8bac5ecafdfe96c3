"""CPU replay of the forward projection's launch-order arithmetic (xcd_grouped_block and
the block decode of fp_kernel, both in csrc/forward.hip).

Checked: the XCD grouping is a permutation of [0, n) for every grid size (whole runs of
64, a partial last run, grids smaller than one run); within a whole run the 8 workgroups
that the dispatcher deals to one XCD (equal index mod 8) receive 8 consecutive
launch-order indices; and for every workload geometry and batch the decoded (row tile,
view, column tile) triples cover each tile of each view exactly once."""
import numpy as np
import pytest

import synthetic as syn

COLS, WAVES, ROWS = 64, 4, 16   # columns per block, waves per block, rows per thread


def xcd_grouped_block(b, n):
    b = np.asarray(b, dtype=np.int64)
    whole = n & ~63
    w = b & 63
    g = (b & ~63) + (w & 7) * 8 + (w >> 3)
    return np.where(b >= whole, b, g)


@pytest.mark.parametrize("n", [1, 7, 63, 64, 65, 127, 128, 200, 4096, 4100, 46080, 46081])
def test_grouping_is_a_permutation(n):
    lb = xcd_grouped_block(np.arange(n), n)
    assert np.array_equal(np.sort(lb), np.arange(n))


def test_each_xcd_gets_consecutive_indices():
    n = 64 * 5 + 17
    b = np.arange(n)
    lb = xcd_grouped_block(b, n)
    for run in range(n // 64):
        for x in range(8):
            sel = b[(b >= 64 * run) & (b < 64 * run + 64) & (b % 8 == x)]
            got = np.sort(lb[sel])
            assert np.array_equal(got, 64 * run + 8 * x + np.arange(8))


def _blocks_per_view(g, parts):
    rows = (WAVES // parts) * ROWS
    return ((g.nu + COLS - 1) // COLS) * ((g.nv + rows - 1) // rows)


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5"])
@pytest.mark.parametrize("parts", [1, 2, 4])
def test_forward_decode_covers_every_tile_once(name, parts):
    g = syn.config_geometry(name)
    B = syn.CONFIGS[name]["batch"]
    tiles_u = (g.nu + COLS - 1) // COLS
    bpv = _blocks_per_view(g, parts)
    for nb in sorted({1, B - 1, B}):
        if nb < 1:
            continue
        n = bpv * nb
        lb = xcd_grouped_block(np.arange(n), n)
        nbv = n // bpv
        rt = lb // (nbv * tiles_u)
        rem = lb - rt * nbv * tiles_u
        bi = rem // tiles_u
        tile = rt * tiles_u + (rem - bi * tiles_u)
        assert bi.min() >= 0 and bi.max() < nb
        assert tile.min() >= 0 and tile.max() < bpv
        key = bi * bpv + tile
        assert np.array_equal(np.sort(key), np.arange(n))
