"""GPU parity of the bound / classify path against the FP64 oracle, through
the C ABI.  Tolerance: raw endpoints (center -/+ radius, before the rounding
inflation) within 1e-5 * S with S = max(|lo_o|, |hi_o|, RMS of f); labels
equal unless the oracle bound is within the tolerance plus the GPU's
floating-point margin of zero; the returned bound contains every sampled f."""
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


def _run(ctx, net, lo, hi, policy, k, replay=True, sound_rng=None):
    from paper_2202_02444_amd import spk
    g = spk.Net.from_spec(net)
    s = 3
    H = net.hidden_width()
    out = gpu_classify(ctx, g, lo, hi, policy, k, want_src=(policy == "truncate"))
    Snet = s_net(net)
    c_o, r_o, lo_o, hi_o = omlp.bound_boxes(net, lo, hi, policy, k)
    S = np.maximum(np.maximum(np.abs(lo_o), np.abs(hi_o)), Snet)
    free = endpoint_errors(out["center"], out["radius"], lo_o, hi_o, S)
    res = {"free": free, "out": out, "oracle": (c_o, r_o, lo_o, hi_o), "S": S}
    if policy == "truncate" and replay:
        sets = keep_sets_from_src(out["src"], s, k, H)
        rec = []
        c_r, r_r, lo_r, hi_r = omlp.bound_boxes(net, lo, hi, policy, k, keep_sets=sets, record=rec)
        res["replay"] = endpoint_errors(out["center"], out["radius"], lo_r, hi_r, S)
        res["replay_bounds"] = (lo_r, hi_r)
        res["sets"] = sets
        # the GPU's kept sets are valid top-k selections of the FP64 magnitudes
        res["topk_violations"] = valid_topk(rec)
    if sound_rng is not None:
        res["violations"], _ = soundness_violations(net, lo, hi, out["lo"], out["hi"], sound_rng)
    return res


def test_tiny_fixed(ctx):
    net = wl.tiny_net(0)
    lo, hi = wl.boxes(4096, 10, 1e-3, 0.25)
    r = _run(ctx, net, lo, hi, "fixed", 0, sound_rng=np.random.default_rng(1))
    assert r["free"].max() <= TOL, r["free"].max()
    assert r["violations"] == 0
    lo_o, hi_o = r["oracle"][2], r["oracle"][3]
    amb = label_ambiguous(lo_o, hi_o, r["S"], default_margin(r["out"]))
    lab_o = oracle_labels(lo_o, hi_o)
    assert np.array_equal(r["out"]["label"][~amb], lab_o[~amb])
    assert amb.mean() < 0.01
    # default mode: the reported widening is the tolerance margin 2^-18 (|c| + r)
    m = 3.814697265625e-06 * (np.abs(r["out"]["center"]) + r["out"]["radius"])
    assert np.allclose(r["out"]["err"], m, rtol=1e-5, atol=1e-30)


@pytest.mark.parametrize("k", [8, 16, 31])
def test_tiny_truncate(ctx, k):
    net = wl.tiny_net(0)
    lo, hi = wl.boxes(4096, 10, 1e-3, 0.25)
    r = _run(ctx, net, lo, hi, "truncate", k, sound_rng=np.random.default_rng(2))
    assert r["replay"].max() <= TOL, r["replay"].max()
    assert r["topk_violations"] == 0
    assert (r["free"] <= TOL).mean() >= 0.99
    assert r["violations"] == 0
    lo_r, hi_r = r["replay_bounds"]
    amb = label_ambiguous(lo_r, hi_r, r["S"], default_margin(r["out"]))
    assert np.array_equal(r["out"]["label"][~amb], oracle_labels(lo_r, hi_r)[~amb])


@pytest.mark.parametrize("n", [1, 7, 9, 63, 65, 1000])
def test_ragged_sizes(ctx, n):
    """Tails that do not fill a wavefront's boxes, at every width."""
    for H, seed in ((32, 3), (64, 4), (128, 5), (256, 6)):
        net = wl.he_normal_mlp([3, H, H, H, 1], seed, act="relu", bias=0.02)
        lo, hi = wl.boxes(n, 20 + n, 1e-3, 0.3)
        r = _run(ctx, net, lo, hi, "truncate", 31, sound_rng=np.random.default_rng(n))
        assert r["replay"].max() <= TOL, (H, r["replay"].max())
        assert r["topk_violations"] == 0, H
        assert r["violations"] == 0


@pytest.mark.parametrize("act,H,depth,policy,k", [
    ("elu", 64, 4, "truncate", 31), ("elu", 128, 6, "fixed", 0), ("sin", 64, 4, "truncate", 31),
    ("sin", 128, 5, "fixed", 0), ("relu", 256, 8, "truncate", 15), ("elu", 256, 5, "truncate", 31),
    ("sin", 256, 4, "truncate", 31), ("relu", 128, 7, "truncate", 31)])
def test_activation_matrix(ctx, act, H, depth, policy, k):
    widths = [3] + [H] * depth + [1]
    net = wl.siren_mlp(widths, 300 + H, 30.0) if act == "sin" else wl.he_normal_mlp(widths, 300 + H, act=act)
    lo, hi = wl.boxes(512, 31, 1e-3, 0.25)
    r = _run(ctx, net, lo, hi, policy, k, sound_rng=np.random.default_rng(3))
    key = "replay" if policy == "truncate" else "free"
    assert r[key].max() <= TOL, r[key].max()
    assert r["violations"] == 0


def test_scale_net_sample(ctx):
    """The 3 -> 256x8 -> 1 closed-blob net, truncate k = 31 and fixed: every
    box within TOL (the first hidden layer's input-axis columns are
    accumulated in FP64; in FP32 their rounding, amplified by the chord slopes
    of narrow straddling neurons, moved rare boxes past TOL)."""
    net = wl.scale_net(1)
    lo, hi = wl.boxes(1024, 11, 1e-4, 0.5)
    for policy, k in (("truncate", 31), ("fixed", 0)):
        r = _run(ctx, net, lo, hi, policy, k, sound_rng=np.random.default_rng(4))
        key = "replay" if policy == "truncate" else "free"
        print(policy, "max endpoint error %.3e" % r[key].max())
        assert r[key].max() <= TOL, (policy, np.sort(r[key])[-3:])
        assert r["violations"] == 0


def test_nonfinite_inputs(ctx):
    from paper_2202_02444_amd import spk
    net = wl.tiny_net(0)
    lo, hi = wl.boxes(64, 12, 1e-3, 0.1)
    lo[3, 1] = np.nan
    hi[5, 0] = np.inf
    lo[7, 2] = -np.inf
    g = spk.Net.from_spec(net)
    ctx.sync()                                   # clears the status word
    out = gpu_classify(ctx, g, lo, hi, "truncate", 31)
    for i in (3, 5, 7):
        assert out["label"][i] == spk.UNKNOWN
        assert out["lo"][i] == -np.inf and out["hi"][i] == np.inf
    ok = np.ones(64, bool)
    ok[[3, 5, 7]] = False
    assert np.all(np.isfinite(out["lo"][ok]))
    # the device status word counted the three boxes (gpu_classify synced once,
    # which read and cleared it); a second launch counts them again
    out = gpu_classify(ctx, g, lo, hi, "fixed", 0, rigorous=True)
    st = ctx.sync()
    assert st["nonfinite_inputs"] == 0 and not st["nospc"]
    import torch
    dev = torch.device("cuda")
    lab = torch.empty(64, dtype=torch.uint8, device=dev)
    spk.classify_boxes(ctx, g, torch.from_numpy(lo).to(dev), torch.from_numpy(hi).to(dev), lab, None, None,
                       "truncate", 31)
    spk.classify_boxes(ctx, g, torch.from_numpy(lo).to(dev), torch.from_numpy(hi).to(dev), lab, None, None,
                       "fixed", 0)
    st = ctx.sync()
    assert st["nonfinite_inputs"] == 6
    assert ctx.sync()["nonfinite_inputs"] == 0


def test_degenerate_point_boxes(ctx):
    """Zero-width boxes: the bound collapses to f(c) up to rounding."""
    net = wl.tiny_net(0)
    pts = wl.points(256, 13)
    r = _run(ctx, net, pts, pts.copy(), "truncate", 31, sound_rng=np.random.default_rng(5))
    f = omlp.forward(net, pts)
    assert r["violations"] == 0
    assert np.all(r["out"]["lo"] <= f) and np.all(r["out"]["hi"] >= f)
    assert np.all(r["out"]["hi"] - r["out"]["lo"] <= 1e-4 * np.maximum(1, np.abs(f)))


def test_general_axes_match_aabb(ctx):
    """range_bound with diagonal axes equals classify_boxes on the same AABBs;
    rotated 1-d and 2-d boxes are sound."""
    import torch
    from paper_2202_02444_amd import spk
    net = wl.tiny_net(0)
    lo, hi = wl.boxes(512, 14, 1e-3, 0.2)
    g = spk.Net.from_spec(net)
    c = ((lo.astype(np.float64) + hi) / 2).astype(np.float32)
    h = (hi - c).astype(np.float32)
    axes = np.zeros((512, 3, 3), np.float32)
    for d in range(3):
        axes[:, d, d] = h[:, d]
    dev = torch.device("cuda")
    tlo = torch.empty(512, device=dev)
    thi = torch.empty(512, device=dev)
    spk.range_bound(ctx, g, torch.from_numpy(c).to(dev), torch.from_numpy(axes).to(dev), tlo, thi, "truncate", 31)
    ctx.sync()
    lo_o, hi_o = omlp.bound_general(net, c, axes, "truncate", 31)
    S = np.maximum(np.maximum(np.abs(lo_o), np.abs(hi_o)), s_net(net))
    assert np.all(tlo.cpu().numpy() <= lo_o + TOL * S) and np.all(thi.cpu().numpy() >= hi_o - TOL * S)
    rng = np.random.default_rng(6)
    for s in (1, 2):
        ax = rng.standard_normal((256, s, 3)).astype(np.float32) * 0.05
        cc = rng.uniform(-1, 1, (256, 3)).astype(np.float32)
        tl = torch.empty(256, device=dev)
        tu = torch.empty(256, device=dev)
        spk.range_bound(ctx, g, torch.from_numpy(cc).to(dev), torch.from_numpy(ax).to(dev), tl, tu, "truncate", 31)
        ctx.sync()
        eps = rng.uniform(-1, 1, (256, 32, s))
        P = cc[:, None, :].astype(np.float64) + np.einsum("bms,bsd->bmd", eps, ax.astype(np.float64))
        f = omlp.forward(net, P.reshape(-1, 3)).reshape(256, 32)
        assert np.all(f >= tl.cpu().numpy()[:, None]) and np.all(f <= tu.cpu().numpy()[:, None])
        l2, h2 = omlp.bound_general(net, cc, ax, "truncate", 31)
        S2 = np.maximum(np.maximum(np.abs(l2), np.abs(h2)), s_net(net))
        assert np.all(tl.cpu().numpy() <= l2 + TOL * S2)


def test_eval_points(ctx):
    """Plain evaluation against the oracle's forward pass; width 256 runs 32
    points per pass (ragged counts: the pass's tail points are zeros and are
    not written)."""
    import torch
    from paper_2202_02444_amd import spk
    nets = (wl.tiny_net(0), wl.scale_net(1), wl.siren_mlp([3, 64, 64, 64, 1], 7, 30.0),
            wl.he_normal_mlp([3, 128, 128, 1], 8, act="elu"), wl.he_normal_mlp([3, 256, 256, 256, 1], 10, act="elu"),
            wl.siren_mlp([3, 256, 256, 1], 11, 30.0), wl.he_normal_mlp([3, 256, 1], 12))
    dev = torch.device("cuda")
    for net in nets:
        g = spk.Net.from_spec(net)
        for n in (1000, 1, 31, 33):
            x = wl.points(n, 9 + n)
            f = torch.full((n + 5,), 7.0, device=dev)
            spk.eval_points(ctx, g, torch.from_numpy(x).to(dev), f[:n])
            ctx.sync()
            fo = omlp.forward(net, x)
            S = max(s_net(net), 1e-30)
            out = f.cpu().numpy()
            assert np.max(np.abs(out[:n] - fo)) <= TOL * max(S, np.abs(fo).max()), (net.name, n)
            assert np.all(out[n:] == 7.0)   # nothing written past n


@pytest.mark.parametrize("act", ["relu", "elu", "sin"])
@pytest.mark.parametrize("H", [32, 64, 128, 256])
def test_rigorous_mode_every_kernel(ctx, act, H):
    """The default (rigorous) mode on every kernel instantiation (fixed,
    truncate k = 15 with 16 term slots, k = 31 with 32): every sampled f lies
    inside, the bound contains the oracle's exact bound of the same kept terms
    (to the parity tolerance) and is at most a little wider; launches are
    deterministic."""
    widths = [3] + [H] * 3 + [1]
    net = wl.siren_mlp(widths, 90 + H, 30.0) if act == "sin" else wl.he_normal_mlp(widths, 90 + H, act=act)
    lo, hi = wl.boxes(128, 91, 1e-3, 0.25)
    from paper_2202_02444_amd import spk
    g = spk.Net.from_spec(net)
    for policy, k in (("fixed", 0), ("truncate", 15), ("truncate", 31)):
        out = gpu_classify(ctx, g, lo, hi, policy, k, want_src=(policy == "truncate"), rigorous=True)
        out2 = gpu_classify(ctx, g, lo, hi, policy, k, rigorous=True)
        assert np.array_equal(out["lo"], out2["lo"]) and np.array_equal(out["hi"], out2["hi"]), (policy, k)
        bad, _ = soundness_violations(net, lo, hi, out["lo"], out["hi"], np.random.default_rng(8))
        assert bad == 0, (policy, k)
        assert np.all(np.isfinite(out["err"])) and np.all(out["err"] > 0), (policy, k)
        # the reported center is rounded to FP32: allow its half ulp
        ulp = np.spacing(np.abs(out["center"]).astype(np.float32)).astype(np.float64)
        assert np.all(out["lo"] <= out["center"] - out["radius"] + ulp)
        assert np.all(out["hi"] >= out["center"] + out["radius"] - ulp)
        if policy == "truncate":
            sets = keep_sets_from_src(out["src"], 3, k, H)
            lo_o, hi_o = omlp.bound_boxes(net, lo, hi, policy, k, keep_sets=sets)[2:]
        else:
            lo_o, hi_o = omlp.bound_boxes(net, lo, hi, policy, k)[2:]
        S = np.maximum(np.maximum(np.abs(lo_o), np.abs(hi_o)), s_net(net))
        viol, ratio = rigorous_vs_oracle(out, lo_o, hi_o, S)
        print("%s H%d %s k%d: containment %.2e, width ratio median %.4f p99 %.3g" % (
            act, H, policy, k, viol.max(), np.median(ratio), np.quantile(ratio, 0.99)))
        assert viol.max() <= TOL, (policy, k, viol.max())
        assert np.median(ratio) <= 1.5, (policy, k)


@pytest.mark.parametrize("act", ["relu", "elu", "sin"])
@pytest.mark.parametrize("depth", [1, 2, 3])
def test_every_kernel_deterministic_and_in_parity(ctx, act, depth):
    """Every kernel instantiation (width x term slots x policy) at 1-3 hidden
    layers, on enough boxes to fill many workgroups: two launches agree bit
    for bit and the raw bound matches the oracle (truncation replayed)."""
    from paper_2202_02444_amd import spk
    lo, hi = wl.boxes(1500, 65, 1e-3, 0.25)
    for H in (32, 64, 128, 256):
        widths = [3] + [H] * depth + [1]
        net = wl.siren_mlp(widths, 54, 30.0) if act == "sin" else wl.he_normal_mlp(widths, 54, act=act)
        g = spk.Net.from_spec(net)
        for policy, k in (("truncate", 31), ("truncate", 15), ("fixed", 0)):
            o1 = gpu_classify(ctx, g, lo, hi, policy, k, want_src=(policy == "truncate"))
            o2 = gpu_classify(ctx, g, lo, hi, policy, k)
            assert np.array_equal(o1["lo"], o2["lo"]) and np.array_equal(o1["hi"], o2["hi"]), (H, policy, k)
            if policy == "truncate":
                sets = keep_sets_from_src(o1["src"], 3, k, H)
                lo_o, hi_o = omlp.bound_boxes(net, lo, hi, policy, k, keep_sets=sets)[2:]
            else:
                lo_o, hi_o = omlp.bound_boxes(net, lo, hi, policy, k)[2:]
            S = np.maximum(np.maximum(np.abs(lo_o), np.abs(hi_o)), s_net(net))
            assert endpoint_errors(o1["center"], o1["radius"], lo_o, hi_o, S).max() <= TOL, (H, policy, k)
