"""The batched multi-network launch (one HIP graph over per-class persistent
kernels) against single-network launches and the FP64 oracle."""
import numpy as np
import pytest

import workloads as wl
from oracle import mlp as omlp

from parity import (TOL, default_margin, endpoint_errors, gpu_classify, keep_sets_from_src, label_ambiguous,
                    oracle_labels, rigorous_vs_oracle, s_net, soundness_violations, valid_topk)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2202_02444_amd import spk
    c = spk.Context()
    yield c
    c.close()


NETS = [lambda: wl.tiny_net(0),
        lambda: wl.he_normal_mlp([3, 64, 64, 64, 1], 51, act="elu"),
        lambda: wl.siren_mlp([3, 128, 128, 1], 52, 30.0),
        lambda: wl.he_normal_mlp([3, 256, 256, 256, 1], 53, act="relu"),
        lambda: wl.tiny_net(7),
        lambda: wl.he_normal_mlp([3, 64, 64, 1], 54, act="relu")]


def _items(specs, gnets, sizes, seed):
    import torch
    dev = torch.device("cuda")
    items = []
    for i, (g, n) in enumerate(zip(gnets, sizes)):
        lo, hi = wl.boxes(n, seed + i, 1e-3, 0.25)
        items.append({"net": g, "box_lo": torch.from_numpy(lo).to(dev), "box_hi": torch.from_numpy(hi).to(dev),
                      "label": torch.empty(n, dtype=torch.uint8, device=dev),
                      "lo": torch.empty(n, device=dev), "hi": torch.empty(n, device=dev),
                      "np": (lo, hi), "spec": specs[i]})
    return items


def _single(ctx, it, policy, k):
    import torch
    from paper_2202_02444_amd import spk
    n = it["box_lo"].shape[0]
    lab = torch.empty(n, dtype=torch.uint8, device="cuda")
    lo = torch.empty(n, device="cuda")
    hi = torch.empty(n, device="cuda")
    if n:
        spk.classify_boxes(ctx, it["net"], it["box_lo"], it["box_hi"], lab, lo, hi, policy, k)
    ctx.sync()
    return lab.cpu().numpy(), lo.cpu().numpy(), hi.cpu().numpy()


def _check_equal(ctx, items, policy, k):
    for it in items:
        lab, lo, hi = _single(ctx, it, policy, k)
        assert np.array_equal(it["label"].cpu().numpy(), lab)
        assert np.array_equal(it["lo"].cpu().numpy(), lo) and np.array_equal(it["hi"].cpu().numpy(), hi)


@pytest.mark.parametrize("policy,k", [("truncate", 31), ("truncate", 12), ("fixed", 0)])
def test_batch_matches_single_launches(ctx, policy, k):
    from paper_2202_02444_amd import spk
    specs = [f() for f in NETS]
    gnets = [spk.Net.from_spec(s) for s in specs]
    items = _items(specs, gnets, [0, 1, 777, 3000, 65, 1500], 60)
    b = spk.Batch(ctx, items, policy, k)
    b.launch(ctx)
    ctx.sync()
    _check_equal(ctx, items, policy, k)
    cls = b.classes()
    assert sum(c["n_nets"] for c in cls) == len(items)
    assert len(cls) == 5   # the two tiny nets share (32, relu)
    # a new, uneven frontier: same networks, other sizes and buffers
    items2 = _items(specs, gnets, [4000, 0, 3, 129, 2048, 1], 70)
    b.update(ctx, items2)
    b.launch(ctx)
    ctx.sync()
    _check_equal(ctx, items2, policy, k)
    # the autotuner changes launch shapes only, never results
    b.tune(ctx, reps=1)
    for it in items2:
        it["label"].fill_(255)
    b.launch(ctx)
    ctx.sync()
    _check_equal(ctx, items2, policy, k)
    assert all(c["tuned_ms"] > 0 for c in b.classes() if c["groups"] > 0)
    b.close()


ORACLE_NETS = [
    lambda: wl.he_normal_mlp([3, 32, 32, 1], 81, act="relu"),
    lambda: wl.he_normal_mlp([3, 64, 64, 64, 1], 82, act="elu"),
    lambda: wl.siren_mlp([3, 128, 128, 1], 83, 30.0),
    lambda: wl.he_normal_mlp([3, 256, 256, 256, 1], 84, act="relu"),
    lambda: wl.siren_mlp([3, 64, 64, 64, 64, 1], 85, 30.0),
    lambda: wl.he_normal_mlp([3, 128, 128, 128, 1], 86, act="elu"),
    lambda: wl.he_normal_mlp([3, 256, 256, 256, 256, 1], 87, act="elu")]


@pytest.mark.parametrize("rigorous", [False, True])
def test_batch_vs_oracle(ctx, rigorous):
    """One batched launch over seven networks (every width, all three
    activations).  Each network's batched bound equals bit for bit the
    single-network launch that exports its kept sets, and the oracle replays
    those sets: in the paper's arithmetic the raw endpoints match within TOL,
    kept sets are valid top-k choices and labels are equal outside the
    ambiguity band; in the rigorous mode the bound contains the oracle's;
    every sampled f lies inside either way."""
    from paper_2202_02444_amd import spk
    specs = [f() for f in ORACLE_NETS]
    gnets = [spk.Net.from_spec(s) for s in specs]
    items = _items(specs, gnets, [700, 333, 1024, 257, 500, 64, 129], 88)
    b = spk.Batch(ctx, items, "truncate", 31, rigorous=rigorous)
    b.launch(ctx)
    ctx.sync()
    for it in items:
        net = it["spec"]
        lo, hi = it["np"]
        H = net.hidden_width()
        single = gpu_classify(ctx, it["net"], lo, hi, "truncate", 31, want_src=True, rigorous=rigorous)
        glo = it["lo"].cpu().numpy().astype(np.float64)
        ghi = it["hi"].cpu().numpy().astype(np.float64)
        lab = it["label"].cpu().numpy()
        assert np.array_equal(glo, single["lo"]) and np.array_equal(ghi, single["hi"]), net.name
        assert np.array_equal(lab, single["label"]), net.name
        rec = []
        sets = keep_sets_from_src(single["src"], 3, 31, H)
        _, _, lo_o, hi_o = omlp.bound_boxes(net, lo, hi, "truncate", 31, keep_sets=sets, record=rec)
        S = np.maximum(np.maximum(np.abs(lo_o), np.abs(hi_o)), s_net(net))
        if rigorous:
            viol, _ = rigorous_vs_oracle(single, lo_o, hi_o, S)
            assert viol.max() <= TOL, (net.name, viol.max())
        else:
            e = endpoint_errors(single["center"], single["radius"], lo_o, hi_o, S)
            assert e.max() <= TOL, (net.name, e.max())
            assert valid_topk(rec) == 0, net.name
            amb = label_ambiguous(lo_o, hi_o, S, default_margin(single))
            assert np.array_equal(lab[~amb], oracle_labels(lo_o, hi_o)[~amb]), net.name
        bad, _ = soundness_violations(net, lo, hi, glo, ghi, np.random.default_rng(9))
        assert bad == 0, net.name
    b.close()


def test_net_destroy_busy_while_held(ctx):
    """spk_net_destroy refuses (SPK_E_BUSY, nothing freed) while a batch holds
    the network, and frees it once the batch is gone."""
    import torch
    from paper_2202_02444_amd import spk
    specs = [wl.tiny_net(0), wl.he_normal_mlp([3, 64, 64, 1], 54, act="relu")]
    gnets = [spk.Net.from_spec(s) for s in specs]
    items = _items(specs, gnets, [300, 500], 90)
    b = spk.Batch(ctx, items, "truncate", 31)
    b.launch(ctx)
    ctx.sync()
    lab0 = items[0]["label"].cpu().numpy().copy()
    L = spk.lib()
    assert L.spk_net_destroy(gnets[0].handle) == spk.E_BUSY
    # the network still works
    lab, _, _ = _single(ctx, items[0], "truncate", 31)
    np.testing.assert_array_equal(lab, lab0)
    b.launch(ctx)
    ctx.sync()
    np.testing.assert_array_equal(items[0]["label"].cpu().numpy(), lab0)
    b.close()
    gnets[0].close()                             # now frees
    assert gnets[0].handle is None
    gnets[1].close()


@pytest.mark.parametrize("rigorous", [False, True])
def test_batched_octrees_equal_single_network_octrees(ctx, rigorous):
    """Frontier items: one graph launch per level classifies and compacts
    every network's frontier.  Per network and level the counts, and the
    final leaves, equal those of the single-network rounds
    (spk_subdivide_frontier), bit for bit."""
    from paper_2202_02444_amd import spk
    specs = [wl.tiny_net(0), wl.he_normal_mlp([3, 64, 64, 64, 1], 51, act="elu", bias=-0.3),
             wl.siren_mlp([3, 128, 128, 1], 52, 30.0), wl.scale_net(1), wl.tiny_net(7),
             wl.he_normal_mlp([3, 64, 64, 1], 54, act="relu")]
    gnets = [spk.Net.from_spec(s_) for s_ in specs]
    depth = 5
    levels_b, leaves_b = spk.build_octrees_batched(ctx, gnets, depth, "truncate", 31, rigorous=rigorous)
    for i, g in enumerate(gnets):
        levels_s, leaves_s = spk.build_octree(ctx, g, depth, "truncate", 31, rigorous=rigorous)
        for a, b in zip(levels_b[i], levels_s):
            assert a == b, (i, a, b)
        la = np.sort(leaves_b[i].cpu().numpy())
        lb = np.sort(leaves_s.cpu().numpy())
        assert np.array_equal(la, lb), i
    for g in gnets:
        g.close()


def test_batch_mixes_box_and_frontier_items(ctx):
    """Box items and frontier items in one batch: the boxes get the labels of
    a single classify launch, the frontier item the counts and children of a
    single subdivide round; a frontier that outgrows its capacity reports the
    required size and writes only its capacity."""
    import torch
    from paper_2202_02444_amd import spk
    specs = [wl.tiny_net(0), wl.he_normal_mlp([3, 64, 64, 1], 54, act="relu")]
    gnets = [spk.Net.from_spec(s_) for s_ in specs]
    box_items = _items(specs[:1], gnets[:1], [700], 91)
    dev = torch.device("cuda")
    cells = torch.arange(64, dtype=torch.int64, device=dev)            # all level-2 cells
    counts = torch.zeros(4, dtype=torch.int64, device=dev)
    small = torch.full((16,), -1, dtype=torch.int64, device=dev)
    fr = {"net": gnets[1], "cells": cells, "level": 2, "max_level": 6, "label": torch.empty(64, dtype=torch.uint8,
          device=dev), "counts": counts, "children": small}
    b = spk.Batch(ctx, box_items + [fr], "truncate", 31)
    b.launch(ctx)
    ctx.sync()
    lab, _, _ = _single(ctx, box_items[0], "truncate", 31)
    np.testing.assert_array_equal(box_items[0]["label"].cpu().numpy(), lab)
    ref_counts = torch.zeros(4, dtype=torch.int64, device=dev)
    big = torch.empty(8 * 64, dtype=torch.int64, device=dev)
    spk.subdivide_frontier(ctx, gnets[1], 2, cells, big, None, ref_counts, 6, "truncate", 31)
    ctx.sync(allow_nospc=True)
    c, rc = counts.cpu().numpy(), ref_counts.cpu().numpy()
    np.testing.assert_array_equal(c, rc)
    assert c[0] > 16 and np.all(small.cpu().numpy() >= 0)
    want = np.sort(big[:rc[0]].cpu().numpy())
    assert np.all(np.isin(small.cpu().numpy(), want))
    b.close()
    for g in gnets:
        g.close()
