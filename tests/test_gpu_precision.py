"""Split-BF16 and scaled split-FP16 generator products (SPK_PREC_BF16X3,
SPK_PREC_F16X3) against the FP64 oracle and the FP32 path, all with the
rounding bound folded in: the returned bound contains the oracle's exact
affine bound (same truncation choices, replayed) to the parity tolerance and
every sampled f, and is wider than FP32's by the larger split error
constants."""
import numpy as np
import pytest

import workloads as wl
from oracle import mlp as omlp

from parity import TOL, gpu_classify, keep_sets_from_src, rigorous_vs_oracle, s_net, soundness_violations

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2202_02444_amd import spk
    c = spk.Context()
    yield c
    c.close()


NETS = {"blob": lambda: wl.scale_net(1),
        "relu4": lambda: wl.he_normal_mlp([3] + [256] * 4 + [1], 61, act="relu"),
        "elu3": lambda: wl.he_normal_mlp([3] + [256] * 3 + [1], 62, act="elu"),
        "sin3": lambda: wl.siren_mlp([3] + [256] * 3 + [1], 63, 30.0)}


@pytest.mark.parametrize("prec", ["bf16x3", "f16x3", "f64"])
@pytest.mark.parametrize("name", list(NETS))
@pytest.mark.parametrize("policy,k", [("truncate", 31), ("truncate", 15), ("fixed", 0)])
def test_split_encloses_oracle(ctx, prec, name, policy, k):
    from paper_2202_02444_amd import spk
    net = NETS[name]()
    g = spk.Net.from_spec(net)
    lo, hi = wl.boxes(384, 64, 1e-4, 0.5)
    out = gpu_classify(ctx, g, lo, hi, policy, k, want_src=(policy == "truncate"), prec=prec)
    out2 = gpu_classify(ctx, g, lo, hi, policy, k, prec=prec)
    assert np.array_equal(out["lo"], out2["lo"]) and np.array_equal(out["hi"], out2["hi"])
    if policy == "truncate":
        sets = keep_sets_from_src(out["src"], 3, k, 256)
        lo_o, hi_o = omlp.bound_boxes(net, lo, hi, policy, k, keep_sets=sets)[2:]
    else:
        lo_o, hi_o = omlp.bound_boxes(net, lo, hi, policy, k)[2:]
    S = np.maximum(np.maximum(np.abs(lo_o), np.abs(hi_o)), s_net(net))
    fin = np.isfinite(out["lo"]) & np.isfinite(out["hi"])
    assert fin.mean() > 0.99
    # the enclosure contains the exact affine bound of the same kept terms
    viol, ratio = rigorous_vs_oracle(out, lo_o, hi_o, S)
    print("%s %s %s k%d: containment %.2e, width ratio median %.4f p99 %.3g" % (
        prec, name, policy, k, viol[fin].max(), np.median(ratio[fin]), np.quantile(ratio[fin], 0.99)))
    assert viol[fin].max() <= TOL
    bad, _ = soundness_violations(net, lo, hi, out["lo"], out["hi"], np.random.default_rng(65))
    assert bad == 0


def _width(o):
    return o["hi"] - o["lo"]


def test_split_bf16_vs_fp32_rigorous(ctx):
    """At equal (rigorous) soundness the split bound is at least as wide as
    FP32's (larger a-priori error constants) and centered alike."""
    from paper_2202_02444_amd import spk
    net = wl.he_normal_mlp([3] + [256] * 3 + [1], 66, act="relu")
    g = spk.Net.from_spec(net)
    lo, hi = wl.boxes(512, 67, 1e-3, 0.25)
    s = gpu_classify(ctx, g, lo, hi, "fixed", 0, prec="bf16x3")
    f = gpu_classify(ctx, g, lo, hi, "fixed", 0, rigorous=True)
    S = np.maximum(np.maximum(np.abs(f["lo"]), np.abs(f["hi"])), s_net(net))
    ratio = _width(s) / _width(f)
    assert np.median(ratio) >= 1.0 and np.mean(ratio >= 1.0 - 1e-6) >= 0.99, np.quantile(ratio, [0.01, 0.5])
    assert np.max(np.abs(s["center"] - f["center"]) / S) < 1e-3


def test_split_f16_tighter_than_bf16(ctx):
    """Scaled split FP16 carries 22 significand bits to BF16's 16: its bound
    is closer to FP32's."""
    from paper_2202_02444_amd import spk
    net = wl.he_normal_mlp([3] + [256] * 3 + [1], 66, act="relu")
    g = spk.Net.from_spec(net)
    lo, hi = wl.boxes(512, 67, 1e-3, 0.25)
    h = gpu_classify(ctx, g, lo, hi, "fixed", 0, prec="f16x3")
    b = gpu_classify(ctx, g, lo, hi, "fixed", 0, prec="bf16x3")
    f = gpu_classify(ctx, g, lo, hi, "fixed", 0, rigorous=True)
    S = np.maximum(np.maximum(np.abs(f["lo"]), np.abs(f["hi"])), s_net(net))
    rh = _width(h) / _width(f)
    rb = _width(b) / _width(f)
    assert np.median(rh) >= 1.0 - 1e-6 and np.median(rh) <= np.median(rb)
    assert np.max(np.abs(h["center"] - f["center"]) / S) < 1e-4


def test_split_f16_extreme_scales(ctx):
    """Column scaling keeps tiny boxes (generators near 1e-7) and a net with
    weights scaled by 2^-40 and 2^40 in range: bounds still enclose the oracle
    and every sampled f."""
    from paper_2202_02444_amd import spk
    base = wl.he_normal_mlp([3] + [256] * 3 + [1], 71, act="relu")
    for sc in (2.0 ** -40, 1.0, 2.0 ** 40):
        Ws = [w.copy() for w in base.weights]
        Ws[1] = (Ws[1] * sc).astype(np.float32)
        Ws[2] = (Ws[2] / sc).astype(np.float32)
        net = wl.MLPSpec(Ws, [b.copy() for b in base.biases], act="relu", omega0=1.0, name="scaled")
        g = spk.Net.from_spec(net)
        for hw in ((1e-7, 1e-6), (1e-3, 0.5)):
            lo, hi = wl.boxes(256, 72, hw[0], hw[1])
            out = gpu_classify(ctx, g, lo, hi, "truncate", 15, want_src=True, prec="f16x3")
            sets = keep_sets_from_src(out["src"], 3, 15, 256)
            lo_o, hi_o = omlp.bound_boxes(net, lo, hi, "truncate", 15, keep_sets=sets)[2:]
            S = np.maximum(np.maximum(np.abs(lo_o), np.abs(hi_o)), s_net(net))
            assert np.all(np.isfinite(out["lo"])) and np.all(np.isfinite(out["hi"]))
            viol, _ = rigorous_vs_oracle(out, lo_o, hi_o, S)
            assert viol.max() <= TOL, (sc, hw, viol.max())
            bad, _ = soundness_violations(net, lo, hi, out["lo"], out["hi"], np.random.default_rng(73))
            assert bad == 0


@pytest.mark.parametrize("prec", ["bf16x3", "f16x3", "f64"])
def test_split_unsupported_shapes(ctx, prec):
    import torch
    from paper_2202_02444_amd import spk
    g = spk.Net.from_spec(wl.he_normal_mlp([3, 64, 64, 1], 68))
    lo, hi = wl.boxes(8, 69)
    with pytest.raises(spk.SpkError) as ei:
        gpu_classify(ctx, g, lo, hi, "truncate", 31, prec=prec)
    assert ei.value.status == spk.E_UNSUPPORTED
    dev = torch.device("cuda")
    items = [{"net": spk.Net.from_spec(wl.he_normal_mlp([3, 256, 256, 1], 70)),
              "box_lo": torch.from_numpy(lo).to(dev), "box_hi": torch.from_numpy(hi).to(dev),
              "label": torch.empty(8, dtype=torch.uint8, device=dev)}]
    import ctypes
    o = spk.opts("truncate", 31, prec=prec)
    arr = (spk.BatchItem * 1)()
    arr[0] = spk.BatchItem(items[0]["net"].handle.value, 8, items[0]["box_lo"].data_ptr(),
                           items[0]["box_hi"].data_ptr(), items[0]["label"].data_ptr(), None, None)
    h = ctypes.c_void_p()
    assert spk.lib().spk_batch_create(ctx.handle, ctypes.byref(o), 1, arr, ctypes.byref(h)) == spk.E_UNSUPPORTED


def test_f64_products_tight_and_in_parity(ctx):
    """FP64 generator products on the blob sample: with the rounding bound the
    enclosure stays close to the oracle's exact bound also on the smallest
    boxes (the FP32 products' a-priori rounding dominates those), and in the
    paper's arithmetic the raw endpoints match the oracle within TOL."""
    from paper_2202_02444_amd import spk
    from parity import endpoint_errors
    net = wl.scale_net(1)
    g = spk.Net.from_spec(net)
    lo, hi = wl.boxes(1024, 11, 1e-4, 0.5)
    for rig in (True, False):
        out = gpu_classify(ctx, g, lo, hi, "truncate", 31, want_src=True, rigorous=rig, prec="f64")
        sets = keep_sets_from_src(out["src"], 3, 31, 256)
        _, _, lo_o, hi_o = omlp.bound_boxes(net, lo, hi, "truncate", 31, keep_sets=sets)
        S = np.maximum(np.maximum(np.abs(lo_o), np.abs(hi_o)), s_net(net))
        if rig:
            viol, ratio = rigorous_vs_oracle(out, lo_o, hi_o, S)
            lab_o = np.where(lo_o > 0, 1, np.where(hi_o < 0, 2, 0))
            kept = np.mean(out["label"][lab_o != 0] == lab_o[lab_o != 0])
            print("f64 rigorous blob: containment %.2e, width ratio median %.4f p90 %.3g p99 %.3g, oracle labels "
                  "kept %.3f" % (viol.max(), np.median(ratio), np.quantile(ratio, 0.9), np.quantile(ratio, 0.99), kept))
            assert viol.max() <= TOL
            assert np.median(ratio) <= 1.01 and kept >= 0.5
            bad, _ = soundness_violations(net, lo, hi, out["lo"], out["hi"], np.random.default_rng(66))
            assert bad == 0
        else:
            e = endpoint_errors(out["center"], out["radius"], lo_o, hi_o, S)
            print("f64 paper arithmetic blob: max endpoint error %.3e" % e.max())
            assert e.max() <= TOL
