"""The serving loop: requests of three kinds and uneven sizes against
resident networks give the same results alone and in a concurrent mix, and
admission never lets the requests in flight exceed the memory budget."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2202_02444_amd import spk
    specs = [wl.tiny_net(0), wl.he_normal_mlp([3, 64, 64, 64, 1], 71, act="elu"), wl.scale_net(1),
             wl.octahedron_mlp(0.55, pad_to=32)]
    nets = [spk.Net.from_spec(s) for s in specs]
    ctx = spk.Context()
    yield spk, nets, ctx
    ctx.close()


def _make_requests(seed):
    import torch
    dev = torch.device("cuda")
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(18):
        kind = ("classify", "rays", "closest")[i % 3]
        net = int(rng.integers(0, 4))
        if kind == "classify":
            n = int(rng.integers(1, 20000))
            lo, hi = wl.boxes(n, 1000 + i, 1e-3, 0.3)
            reqs.append({"type": kind, "net": net, "box_lo": torch.from_numpy(lo).to(dev),
                         "box_hi": torch.from_numpy(hi).to(dev), "label": torch.empty(n, dtype=torch.uint8, device=dev),
                         "lo": torch.empty(n, device=dev), "hi": torch.empty(n, device=dev),
                         "k": (31, 15)[i % 2]})
        elif kind == "rays":
            net = (0, 1, 3)[i % 3]   # short rays on the nets with tight bounds
            o, d = wl.camera_rays(24, 24, 1000 + i)
            n = o.shape[0]
            reqs.append({"type": kind, "net": net, "origin": torch.from_numpy(o).to(dev),
                         "dir": torch.from_numpy(d).to(dev), "t_hit": torch.empty(n, device=dev),
                         "iters": torch.empty(n, dtype=torch.int32, device=dev)})
        else:
            net = (0, 3)[i % 2]
            n = int(rng.integers(1, 600))
            q = wl.points(n, 1000 + i)
            reqs.append({"type": kind, "net": net, "q": torch.from_numpy(q).to(dev),
                         "point": torch.empty((n, 3), device=dev), "dist": torch.empty(n, device=dev),
                         "bound": torch.empty(n, device=dev), "max_level": 6})
    torch.cuda.synchronize()
    return reqs


OUT_KEYS = {"classify": ("label", "lo", "hi"), "rays": ("t_hit", "iters"), "closest": ("point", "dist", "bound")}


def _alone(spk, nets, ctx, r):
    """The same request issued directly, one at a time."""
    import torch
    outs = {k: torch.empty_like(r[k]) for k in OUT_KEYS[r["type"]]}
    g = nets[r["net"]]
    if r["type"] == "classify":
        spk.classify_boxes(ctx, g, r["box_lo"], r["box_hi"], outs["label"], outs["lo"], outs["hi"], "truncate", r["k"])
    elif r["type"] == "rays":
        spk.cast_rays(ctx, g, r["origin"], r["dir"], outs["t_hit"], outs["iters"])
    else:
        spk.closest_point(ctx, g, r["q"], outs["point"], outs["dist"], outs["bound"], max_level=r["max_level"])
    ctx.sync()
    return {k: v.cpu().numpy() for k, v in outs.items()}


def _run_server(spk, nets, reqs, budget, workers):
    srv = spk.Server(nets, budget, workers)
    ids = [srv.submit(r) for r in reqs]
    done = []
    while len(done) < len(reqs):
        done += srv.poll(64, wait=True)
    srv.close()
    return ids, done


def test_results_same_alone_and_in_the_mix(env):
    spk, nets, ctx = env
    reqs = _make_requests(5)
    ref = [_alone(spk, nets, ctx, r) for r in reqs]
    ids, done = _run_server(spk, nets, reqs, budget=1 << 30, workers=4)
    assert sorted(c["id"] for c in done) == sorted(ids)
    assert all(c["status"] == spk.OK for c in done)
    for r, want in zip(reqs, ref):
        for k, v in want.items():
            got = r[k].cpu().numpy()
            assert np.array_equal(got, v, equal_nan=True), (r["type"], k)
    # requests overlapped on the device: some start before another finishes
    spans = sorted((c["start_s"], c["done_s"]) for c in done)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    for c in done:
        assert c["submit_s"] <= c["start_s"] <= c["done_s"]


def _max_concurrent(done):
    events = sorted([(c["start_s"], 1) for c in done] + [(c["done_s"], -1) for c in done], key=lambda e: (e[0], e[1]))
    cur = best = 0
    for _, d in events:
        cur += d
        best = max(best, cur)
    return best


@pytest.mark.parametrize("fit", [1, 2])
def test_admission_respects_the_memory_budget(env, fit):
    """Every request declares B bytes and the budget is fit * B: at most fit
    requests run at once although four workers are free."""
    spk, nets, ctx = env
    reqs = _make_requests(6)[:9]
    B = 64 << 20   # closest-point requests keep their workspace within it
    for r in reqs:
        r["bytes"] = B
    ids, done = _run_server(spk, nets, reqs, budget=fit * B, workers=4)
    assert all(c["status"] == spk.OK for c in done)
    assert _max_concurrent(done) <= fit


def test_request_workspace_stays_within_declared_bytes(env):
    """A closest-point request's library workspace stays within its declared
    bytes beyond its inputs and outputs (the query chunks shrink to fit), and
    its results are those of the unconstrained call."""
    spk, nets, ctx = env
    reqs = [r for r in _make_requests(11) if r["type"] == "closest"]
    ws = 2 << 20
    for r in reqs:
        r["workspace"] = ws
    alone = [_alone(spk, nets, ctx, r) for r in reqs]
    ids, done = _run_server(spk, nets, reqs, budget=64 << 20, workers=3)
    by_id = {c["id"]: c for c in done}
    for rid, r, a in zip(ids, reqs, alone):
        c = by_id[rid]
        assert c["status"] == spk.OK
        assert 0 < c["workspace_bytes"] <= ws, (c["workspace_bytes"], ws)
        for k in OUT_KEYS["closest"]:
            np.testing.assert_array_equal(r[k].cpu().numpy(), a[k])


def test_affine_full_requests_refused(env):
    """Affine-full allocates its workspace per call, outside the admission
    budget, so the server refuses such requests at submit."""
    import torch
    spk, nets, ctx = env
    dev = torch.device("cuda")
    lo = torch.zeros((4, 3), device=dev)
    hi = torch.ones((4, 3), device=dev)
    lab = torch.empty(4, dtype=torch.uint8, device=dev)
    srv = spk.Server(nets, 1 << 30, 1)
    try:
        with pytest.raises(spk.SpkError) as e:
            srv.submit({"type": "classify", "net": 0, "box_lo": lo, "box_hi": hi, "label": lab, "policy": "full",
                        "k": 0})
        assert e.value.status == spk.E_UNSUPPORTED
    finally:
        srv.close()
