"""spk_subdivide_frontier_noalloc (fixed library scratch, no allocation)
against spk_subdivide_frontier (context workspace), through the C ABI: two
rounds in a row, the second on a smaller frontier, then a round at the
maximum level; children and leaves compared as sets (output order is
unspecified), counts exactly."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _all_cells(level):
    return np.arange(8 ** level, dtype=np.int64)


def _round(spk, ctx, g, cells, level, max_level, noalloc):
    import torch
    dev = torch.device("cuda")
    n = cells.shape[0]
    c = torch.from_numpy(cells).to(dev)
    children = torch.full((8 * n,), -1, dtype=torch.int64, device=dev)
    leaves = torch.full((n,), -1, dtype=torch.int64, device=dev)
    counts = torch.full((4,), -7, dtype=torch.int64, device=dev)
    spk.subdivide_frontier(ctx, g, level, c, children, leaves, counts, max_level, "truncate", 16, noalloc=noalloc)
    ctx.sync()
    cnt = counts.cpu().numpy()
    ch = np.sort(children.cpu().numpy()[:cnt[0]])
    lv = np.sort(leaves.cpu().numpy()[:cnt[1]])
    return cnt, ch, lv


def test_noalloc_matches_workspace_round():
    import torch
    assert torch.cuda.is_available()
    from paper_2202_02444_amd import spk
    ctx = spk.Context()
    g = spk.Net.from_spec(wl.tiny_net(0))
    for level, max_level in ((4, 6), (2, 6), (3, 3)):
        cells = _all_cells(level)
        print("noalloc round: level %d, %d cells, max level %d" % (level, cells.shape[0], max_level), flush=True)
        ref = _round(spk, ctx, g, cells, level, max_level, noalloc=False)
        got = _round(spk, ctx, g, cells, level, max_level, noalloc=True)
        assert np.array_equal(ref[0], got[0]), (ref[0], got[0])
        assert ref[0][0] + ref[0][1] > 0 and ref[0][2] + ref[0][3] > 0
        # every cell is split, kept as a leaf, or counted positive / negative
        assert int(ref[0][0]) // 8 + int(ref[0][1]) + int(ref[0][2]) + int(ref[0][3]) == cells.shape[0]
        assert np.array_equal(ref[1], got[1])
        assert np.array_equal(ref[2], got[2])
    ctx.close()
