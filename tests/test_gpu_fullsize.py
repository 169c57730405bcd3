"""Parity at the measured sizes, in the measured launch configuration: one
classify launch over the 1,048,576 boxes of the 8x256 blob workload (the boxes
bench.py times, seed 11), and one 512x512 ray view of the same net (bench.py's
view, seed 600).  The oracle cannot bound a million boxes in a test, so sampled
outputs are checked one by one: the GPU's kept sets of the sampled boxes are
replayed by the oracle, labels must agree outside the ambiguity band, and f
sampled in every checked box lies inside the bound."""
import numpy as np
import pytest

import workloads as wl
from oracle import mlp as omlp
from oracle import queries as oq

from parity import (TOL, default_margin, endpoint_errors, keep_sets_from_src, label_ambiguous, oracle_labels,
                    rigorous_vs_oracle, s_net, soundness_violations)

pytestmark = pytest.mark.gpu

N_FULL = 1 << 20
N_SAMPLE = 384


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2202_02444_amd import spk
    c = spk.Context()
    yield c
    c.close()


@pytest.mark.parametrize("policy,k", [("truncate", 31), ("fixed", 0)])
def test_full_size_boxes_sampled(ctx, policy, k):
    import torch
    from paper_2202_02444_amd import spk
    net = wl.scale_net(1)
    g = spk.Net.from_spec(net)
    lo, hi = wl.boxes(N_FULL, 11, 1e-4, 0.5)
    dev = torch.device("cuda")
    tl, th = torch.from_numpy(lo).to(dev), torch.from_numpy(hi).to(dev)
    lab = torch.empty(N_FULL, dtype=torch.uint8, device=dev)
    glo = torch.empty(N_FULL, device=dev)
    ghi = torch.empty(N_FULL, device=dev)
    cen = torch.empty(N_FULL, device=dev)
    rad = torch.empty(N_FULL, device=dev)
    err = torch.empty(N_FULL, device=dev)
    aux = {"center": cen, "radius": rad, "err": err}
    src = None
    if policy == "truncate":
        src = torch.full((g.n_linear - 1, N_FULL, 32), -3, dtype=torch.int16, device=dev)
        aux["slot_src"] = src
    spk.classify_boxes(ctx, g, tl, th, lab, glo, ghi, policy, k, aux=aux, rigorous=False)
    ctx.sync()
    # every box got a result
    assert bool(torch.isfinite(glo).all()) and bool(torch.isfinite(ghi).all())
    assert bool((glo <= ghi).all())
    # labels follow the bound everywhere (Procedure 1)
    lab_from_bound = torch.where(glo > 0, 1, torch.where(ghi < 0, 2, 0)).to(torch.uint8)
    assert bool((lab == lab_from_bound).all())
    # sampled boxes: the head, the tail (the last workgroup's range) and a spread
    rng = np.random.default_rng(17)
    idx = np.unique(np.concatenate([np.arange(64), np.arange(N_FULL - 64, N_FULL),
                                    rng.choice(N_FULL, N_SAMPLE - 128, replace=False)]))
    ti = torch.from_numpy(idx).to(dev)
    out = {"center": cen[ti].cpu().numpy().astype(np.float64), "radius": rad[ti].cpu().numpy().astype(np.float64),
           "lo": glo[ti].cpu().numpy().astype(np.float64), "hi": ghi[ti].cpu().numpy().astype(np.float64),
           "label": lab[ti].cpu().numpy()}
    slo, shi = lo[idx], hi[idx]
    if policy == "truncate":
        sets = keep_sets_from_src(src[:, ti, :].cpu().numpy(), 3, k, 256)
        lo_o, hi_o = omlp.bound_boxes(net, slo, shi, policy, k, keep_sets=sets)[2:]
    else:
        lo_o, hi_o = omlp.bound_boxes(net, slo, shi, policy, k)[2:]
    S = np.maximum(np.maximum(np.abs(lo_o), np.abs(hi_o)), s_net(net))
    e = endpoint_errors(out["center"], out["radius"], lo_o, hi_o, S)
    print("max endpoint error %.3e (TOL %.0e)" % (e.max(), TOL))
    assert e.max() <= TOL, np.sort(e)[-3:]
    amb = label_ambiguous(lo_o, hi_o, S, default_margin(out))
    lab_o = oracle_labels(lo_o, hi_o)
    assert np.array_equal(out["label"][~amb], lab_o[~amb])
    bad, _ = soundness_violations(net, slo, shi, out["lo"], out["hi"], np.random.default_rng(18))
    assert bad == 0


def test_full_size_rays_sampled(ctx):
    import torch
    from paper_2202_02444_amd import spk
    net = wl.scale_net(1)
    g = spk.Net.from_spec(net)
    o, d = wl.camera_rays(512, 512, 600)
    dev = torch.device("cuda")
    th = torch.empty(o.shape[0], device=dev)
    it = torch.empty(o.shape[0], dtype=torch.int32, device=dev)
    delta = 1e-3
    spk.cast_rays(ctx, g, torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev), th, it, delta=delta)
    ctx.sync()
    th = th.cpu().numpy().astype(np.float64)
    it = it.cpu().numpy()
    _, _, inside = oq.clip_to_box(o, d)
    # rays that miss the cube report no hit and no iteration
    assert np.all(np.isinf(th[~inside])) and np.all(it[~inside] == 0)
    rng = np.random.default_rng(19)
    idx = np.concatenate([rng.choice(np.flatnonzero(inside), 72, replace=False),
                          rng.choice(np.flatnonzero(~inside), 8, replace=False)])
    to, _ = oq.cast_rays(net, o[idx].astype(np.float64), d[idx].astype(np.float64), delta=delta)
    tg = th[idx]
    agree = np.isfinite(tg) == np.isfinite(to)
    assert agree.sum() >= idx.size - 2, (idx[~agree], tg[~agree], to[~agree])
    both = np.isfinite(tg) & np.isfinite(to)
    assert np.all(np.abs(tg[both] - to[both]) <= 2 * delta + 1e-4)


def test_full_size_rigorous_sampled(ctx):
    """The measured configuration in the library's default mode (every
    rounding bounded): one launch over the 1M blob boxes, truncate k = 31.
    Sampled boxes contain the oracle's exact bound of the same kept terms (to
    the parity tolerance) and every sampled f; a label is the oracle's or
    UNKNOWN outside the ambiguity band."""
    import torch
    from paper_2202_02444_amd import spk
    net = wl.scale_net(1)
    g = spk.Net.from_spec(net)
    lo, hi = wl.boxes(N_FULL, 11, 1e-4, 0.5)
    dev = torch.device("cuda")
    tl, th = torch.from_numpy(lo).to(dev), torch.from_numpy(hi).to(dev)
    lab = torch.empty(N_FULL, dtype=torch.uint8, device=dev)
    glo = torch.empty(N_FULL, device=dev)
    ghi = torch.empty(N_FULL, device=dev)
    src = torch.full((g.n_linear - 1, N_FULL, 32), -3, dtype=torch.int16, device=dev)
    spk.classify_boxes(ctx, g, tl, th, lab, glo, ghi, "truncate", 31, aux={"slot_src": src})
    ctx.sync()
    assert bool(torch.isfinite(glo).all()) and bool(torch.isfinite(ghi).all())
    lab_from_bound = torch.where(glo > 0, 1, torch.where(ghi < 0, 2, 0)).to(torch.uint8)
    assert bool((lab == lab_from_bound).all())
    rng = np.random.default_rng(23)
    idx = np.unique(np.concatenate([np.arange(64), np.arange(N_FULL - 64, N_FULL),
                                    rng.choice(N_FULL, N_SAMPLE - 128, replace=False)]))
    ti = torch.from_numpy(idx).to(dev)
    out = {"lo": glo[ti].cpu().numpy().astype(np.float64), "hi": ghi[ti].cpu().numpy().astype(np.float64)}
    g_lab = lab[ti].cpu().numpy()
    sets = keep_sets_from_src(src[:, ti, :].cpu().numpy(), 3, 31, 256)
    lo_o, hi_o = omlp.bound_boxes(net, lo[idx], hi[idx], "truncate", 31, keep_sets=sets)[2:]
    S = np.maximum(np.maximum(np.abs(lo_o), np.abs(hi_o)), s_net(net))
    viol, ratio = rigorous_vs_oracle(out, lo_o, hi_o, S)
    lab_o = oracle_labels(lo_o, hi_o)
    amb = label_ambiguous(lo_o, hi_o, S, np.zeros_like(S))
    keep = np.mean(g_lab[lab_o != 0] == lab_o[lab_o != 0])
    print("rigorous 1M blob boxes: containment %.2e, width ratio median %.4f p90 %.3g p99 %.3g, "
          "oracle labels kept %.3f" % (viol.max(), np.median(ratio), np.quantile(ratio, 0.9),
                                       np.quantile(ratio, 0.99), keep))
    assert viol.max() <= TOL
    assert np.all((g_lab[~amb] == lab_o[~amb]) | (g_lab[~amb] == spk.UNKNOWN))
    bad, _ = soundness_violations(net, lo[idx], hi[idx], out["lo"], out["hi"], np.random.default_rng(24))
    assert bad == 0


@pytest.mark.parametrize("prec", ["bf16x3", "f16x3"])
def test_full_size_split_precision_sampled(ctx, prec):
    """The precision workload at full size (same net and 1M boxes, truncate
    k = 31, split products with the rounding bound): sampled boxes contain the
    oracle's exact bound of the same kept terms and sampled f lies inside."""
    import torch
    from paper_2202_02444_amd import spk
    net = wl.scale_net(1)
    g = spk.Net.from_spec(net)
    lo, hi = wl.boxes(N_FULL, 11, 1e-4, 0.5)
    dev = torch.device("cuda")
    tl, th = torch.from_numpy(lo).to(dev), torch.from_numpy(hi).to(dev)
    lab = torch.empty(N_FULL, dtype=torch.uint8, device=dev)
    glo = torch.empty(N_FULL, device=dev)
    ghi = torch.empty(N_FULL, device=dev)
    cen = torch.empty(N_FULL, device=dev)
    rad = torch.empty(N_FULL, device=dev)
    err = torch.empty(N_FULL, device=dev)
    src = torch.full((g.n_linear - 1, N_FULL, 32), -3, dtype=torch.int16, device=dev)
    spk.classify_boxes(ctx, g, tl, th, lab, glo, ghi, "truncate", 31,
                       aux={"center": cen, "radius": rad, "err": err, "slot_src": src}, prec=prec)
    ctx.sync()
    assert bool(torch.isfinite(glo).all()) and bool(torch.isfinite(ghi).all())
    rng = np.random.default_rng(21)
    idx = np.unique(np.concatenate([np.arange(32), np.arange(N_FULL - 32, N_FULL),
                                    rng.choice(N_FULL, 192, replace=False)]))
    ti = torch.from_numpy(idx).to(dev)
    g_lo, g_hi = glo[ti].cpu().numpy().astype(np.float64), ghi[ti].cpu().numpy().astype(np.float64)
    c, r, e = (t[ti].cpu().numpy().astype(np.float64) for t in (cen, rad, err))
    sets = keep_sets_from_src(src[:, ti, :].cpu().numpy(), 3, 31, 256)
    lo_o, hi_o = omlp.bound_boxes(net, lo[idx], hi[idx], "truncate", 31, keep_sets=sets)[2:]
    S = np.maximum(np.maximum(np.abs(lo_o), np.abs(hi_o)), s_net(net))
    viol, ratio = rigorous_vs_oracle({"lo": g_lo, "hi": g_hi}, lo_o, hi_o, S)
    print("%s 1M blob boxes: containment %.2e, width ratio median %.4f p99 %.3g" % (
        prec, viol.max(), np.median(ratio), np.quantile(ratio, 0.99)))
    assert viol.max() <= TOL
    assert np.all(e > 0) and np.all(np.isfinite(c)) and np.all(r >= 0)
    bad, _ = soundness_violations(net, lo[idx], hi[idx], g_lo, g_hi, np.random.default_rng(22))
    assert bad == 0


def test_precision_soundness_1e7_points(ctx):
    """The precision workload (the 8x256 blob, 1M boxes, truncate k = 31) in
    FP32, split BF16 and split FP16, all with the rounding bound: 10 seeded
    uniform points in every box (10,485,760 points) plus the 8 corners of
    100,000 boxes, f evaluated in FP64 on the host, lie inside every
    precision's bound."""
    import time
    import torch
    from paper_2202_02444_amd import spk
    net = wl.scale_net(1)
    g = spk.Net.from_spec(net)
    lo, hi = wl.boxes(N_FULL, 11, 1e-4, 0.5)
    dev = torch.device("cuda")
    tl, th = torch.from_numpy(lo).to(dev), torch.from_numpy(hi).to(dev)
    bounds = {}
    for prec in ("f32", "bf16x3", "f16x3"):
        lab = torch.empty(N_FULL, dtype=torch.uint8, device=dev)
        glo = torch.empty(N_FULL, device=dev)
        ghi = torch.empty(N_FULL, device=dev)
        spk.classify_boxes(ctx, g, tl, th, lab, glo, ghi, "truncate", 31, prec=prec)
        ctx.sync()
        bounds[prec] = (glo.cpu().numpy().astype(np.float64), ghi.cpu().numpy().astype(np.float64))
    lo64, hi64 = lo.astype(np.float64), hi.astype(np.float64)
    rng = np.random.default_rng(2025)
    chunk = 1 << 15
    n_pts = 0
    t0 = time.perf_counter()
    for b0 in range(0, N_FULL, chunk):
        b1 = min(b0 + chunk, N_FULL)
        t = rng.uniform(0.0, 1.0, (b1 - b0, 10, 3))
        P = lo64[b0:b1, None, :] + t * (hi64[b0:b1] - lo64[b0:b1])[:, None, :]
        f = omlp.forward_torch(net, P.reshape(-1, 3)).reshape(b1 - b0, 10)
        n_pts += f.size
        for prec, (glo, ghi) in bounds.items():
            bad = (f < glo[b0:b1, None]) | (f > ghi[b0:b1, None])
            assert not bad.any(), (prec, b0 + int(np.flatnonzero(bad.any(axis=1))[0]))
        if (b0 // chunk) % 8 == 0:
            print("soundness: %d points checked (%.0f s)" % (n_pts, time.perf_counter() - t0), flush=True)
    idx = rng.choice(N_FULL, 100000, replace=False)
    corners = np.array(np.meshgrid([0, 1], [0, 1], [0, 1], indexing="ij")).reshape(3, -1).T.astype(np.float64)
    P = lo64[idx, None, :] + corners[None] * (hi64[idx] - lo64[idx])[:, None, :]
    f = omlp.forward_torch(net, P.reshape(-1, 3)).reshape(len(idx), 8)
    for prec, (glo, ghi) in bounds.items():
        assert not ((f < glo[idx, None]) | (f > ghi[idx, None])).any(), prec
    print("soundness: %d random points and %d corners inside the FP32, BF16 and FP16 bounds (%.0f s)" % (
        n_pts, f.size, time.perf_counter() - t0), flush=True)
    assert n_pts >= 10_000_000


def test_octree_depth10_sampled(ctx):
    """The bench's depth-10 octree of the 8x256 blob (paper arithmetic,
    affine-truncate(31) cells), driven round by round through the C ABI and
    checked by sampling: at every level sampled UNKNOWN and sampled classified
    cells carry the oracle's label (outside the ambiguity band), the children
    are exactly 8 per UNKNOWN cell, the POSITIVE / NEGATIVE cells of all levels
    and the depth-10 leaves tile the domain exactly, and sampled leaves are
    UNKNOWN for the oracle."""
    import torch
    from paper_2202_02444_amd import spk
    net = wl.scale_net(1)
    g = spk.Net.from_spec(net)
    S = s_net(net)
    rng = np.random.default_rng(77)
    dev = torch.device("cuda")
    depth = 10
    dom = ((-1.0,) * 3, (1.0,) * 3)
    cells = torch.zeros(1, dtype=torch.int64, device=dev)
    counts = torch.zeros(4, dtype=torch.int64, device=dev)
    volume = 0.0
    bad, checked = [], 0

    def check(codes, level, want_unknown):
        nonlocal checked
        if codes.size == 0:
            return
        lo, hi = oq.cell_bounds(codes, level, *dom)
        _, _, ly, hy = omlp.bound_boxes(net, lo, hi, "truncate", 31)
        lab_o = oracle_labels(ly, hy)
        amb = label_ambiguous(ly, hy, S, 4e-6 * (np.abs(ly) + np.abs(hy)))
        for j in range(codes.size):
            checked += 1
            ok = amb[j] or ((lab_o[j] == spk.UNKNOWN) == want_unknown)
            if not ok:
                bad.append((level, int(codes[j]), int(lab_o[j]), want_unknown))

    for level in range(depth + 1):
        n = cells.shape[0]
        at_max = level == depth
        capc = 0 if at_max else 8 * n
        children = torch.empty(max(capc, 1), dtype=torch.int64, device=dev)
        leaves = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
        spk.subdivide_frontier(ctx, g, level, cells, children[:capc] if capc else None,
                               leaves[:n] if at_max else None, counts, depth, "truncate", 31, rigorous=False)
        ctx.sync()
        c = counts.cpu().numpy()
        volume += float(c[2] + c[3]) * 8.0 ** -level
        codes = cells.cpu().numpy().astype(np.uint64)
        if at_max:
            lv = np.sort(leaves[:c[1]].cpu().numpy().astype(np.uint64))
            assert c[1] + c[2] + c[3] == n
            volume += float(c[1]) * 8.0 ** -depth
            check(lv[rng.choice(lv.size, size=min(192, lv.size), replace=False)], level, True)
            break
        kids = np.sort(children[:c[0]].cpu().numpy().astype(np.uint64))
        assert c[0] % 8 == 0 and c[0] // 8 + c[2] + c[3] == n
        parents = np.unique(kids >> np.uint64(3))
        assert parents.size == c[0] // 8
        unk = np.isin(codes, parents)
        known = np.flatnonzero(~unk)
        check(codes[rng.choice(np.flatnonzero(unk), size=min(48, int(unk.sum())), replace=False)], level, True)
        if known.size:
            check(codes[rng.choice(known, size=min(48, known.size), replace=False)], level, False)
        cells = children[:c[0]].clone()
    assert volume == 1.0, volume
    assert checked > 500
    assert not bad, bad[:5]
