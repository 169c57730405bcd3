"""The batched multi-network launch (one HIP graph over per-class persistent
kernels) against single-network launches and the FP64 oracle."""
import numpy as np
import pytest

import workloads as wl
from oracle import mlp as omlp

from parity import TOL, label_ambiguous, oracle_labels, s_net, soundness_violations

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


def test_batch_vs_oracle(ctx):
    """Labels equal the oracle's away from zero, and every sampled f lies in
    the batched bound."""
    from paper_2202_02444_amd import spk
    specs = [wl.he_normal_mlp([3, 64, 64, 64, 1], 55, act="relu"), wl.siren_mlp([3, 32, 32, 1], 56, 30.0)]
    gnets = [spk.Net.from_spec(s) for s in specs]
    items = _items(specs, gnets, [900, 700], 80)
    b = spk.Batch(ctx, items, "truncate", 31)
    b.launch(ctx)
    ctx.sync()
    for it in items:
        lo, hi = it["np"]
        glo = it["lo"].cpu().numpy().astype(np.float64)
        ghi = it["hi"].cpu().numpy().astype(np.float64)
        lab = it["label"].cpu().numpy()
        lo_o, hi_o = omlp.bound_boxes(it["spec"], lo, hi, "truncate", 31)[2:]
        S = np.maximum(np.maximum(np.abs(lo_o), np.abs(hi_o)), s_net(it["spec"]))
        amb = label_ambiguous(lo_o, hi_o, S, 3.9e-6 * (np.abs(lo_o) + np.abs(hi_o)))
        # free-running truncation may keep other terms on a few boxes
        assert np.mean(lab[~amb] == oracle_labels(lo_o, hi_o)[~amb]) >= 0.99
        bad, _ = soundness_violations(it["spec"], lo, hi, glo, ghi, np.random.default_rng(9))
        assert bad == 0
        assert np.all(glo <= lo_o + TOL * S) and np.all(ghi >= hi_o - TOL * S) or \
            np.mean((glo <= lo_o + TOL * S) & (ghi >= hi_o - TOL * S)) >= 0.99
    b.close()
