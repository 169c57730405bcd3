"""Parity helpers shared by the GPU tests: run the HIP path through the C ABI
and compare with the FP64 oracle (the HIP side never feeds the oracle except
for the explicit truncation replay, which only re-plays its kept sets)."""
import numpy as np

from oracle import mlp as omlp
from oracle import queries as oq

TOL = 1e-5   # relative parity tolerance of the bound endpoints


def s_net(net, n=4096, seed=1234):
    """RMS of f over seeded uniform points of [-1,1]^3: the scale of f."""
    rng = np.random.default_rng(seed)
    f = omlp.forward(net, rng.uniform(-1, 1, (n, 3)))
    return float(np.sqrt(np.mean(f * f)))


def gpu_classify(ctx, g, lo, hi, policy, k, want_src=False, rigorous=None, prec="f32"):
    """Classify boxes through the C ABI.  rigorous=None means the paper's
    arithmetic (SPK_FLAG_NO_ROUNDING_BOUND) for FP32 and the rounding bound for
    the split precisions, which always carry it."""
    import torch
    if rigorous is None:
        rigorous = prec != "f32"
    from paper_2202_02444_amd import spk
    dev = torch.device("cuda")
    n = lo.shape[0]
    tl = torch.from_numpy(np.ascontiguousarray(lo)).to(dev)
    th = torch.from_numpy(np.ascontiguousarray(hi)).to(dev)
    lab = torch.empty(n, dtype=torch.uint8, device=dev)
    glo = torch.empty(n, dtype=torch.float32, device=dev)
    ghi = torch.empty(n, dtype=torch.float32, device=dev)
    cen = torch.empty(n, dtype=torch.float32, device=dev)
    rad = torch.empty(n, dtype=torch.float32, device=dev)
    err = torch.empty(n, dtype=torch.float32, device=dev)
    aux = {"center": cen, "radius": rad, "err": err}
    src = None
    if want_src:
        src = torch.full((g.n_linear - 1, n, 32), -3, dtype=torch.int16, device=dev)
        aux["slot_src"] = src
    spk.classify_boxes(ctx, g, tl, th, lab, glo, ghi, policy, k, aux=aux, rigorous=rigorous, prec=prec)
    ctx.sync()
    out = {"label": lab.cpu().numpy(), "lo": glo.cpu().numpy().astype(np.float64),
           "hi": ghi.cpu().numpy().astype(np.float64), "center": cen.cpu().numpy().astype(np.float64),
           "radius": rad.cpu().numpy().astype(np.float64), "err": err.cpu().numpy().astype(np.float64)}
    if want_src:
        out["src"] = src.cpu().numpy()
    return out


def keep_sets_from_src(src, s, k, H):
    """Oracle keep masks [B, n_occ + H] per activation from the GPU's slot
    record (slot C holds oracle column C-1)."""
    sets = []
    n_occ = s
    for a in range(src.shape[0]):
        rec = src[a]
        B = rec.shape[0]
        keep = np.zeros((B, n_occ + H), dtype=bool)
        keep[:, :n_occ] = rec[:, 1:n_occ + 1] == -1
        for C in range(1, 32):
            r = rec[:, C]
            m = r >= 0
            keep[np.flatnonzero(m), n_occ + r[m]] = True
        sets.append(keep)
        n_occ = min(k, n_occ + H)
    return sets


def endpoint_errors(c_g, r_g, lo_o, hi_o, S):
    return np.maximum(np.abs((c_g - r_g) - lo_o), np.abs((c_g + r_g) - hi_o)) / S


def default_margin(out):
    """The floating-point tolerance margin the library adds in its default mode."""
    return 3.9e-6 * (np.abs(out["center"]) + out["radius"])


def label_ambiguous(lo_o, hi_o, S, err_g):
    tau = TOL * S + err_g * 1.01
    return (np.abs(lo_o) <= tau) | (np.abs(hi_o) <= tau)


def sample_points(lo, hi, rng, n_rand=8):
    """Box corners, center and random points for each box: [B, 9 + n_rand, 3]."""
    lo = lo.astype(np.float64)
    hi = hi.astype(np.float64)
    corners = np.array(np.meshgrid([0, 1], [0, 1], [0, 1], indexing="ij")).reshape(3, -1).T.astype(np.float64)
    t = np.concatenate([corners, [[0.5, 0.5, 0.5]], rng.uniform(0, 1, (n_rand, 3))])
    return lo[:, None, :] + t[None] * (hi - lo)[:, None, :]


def soundness_violations(net, lo, hi, glo, ghi, rng, n_rand=8):
    P = sample_points(lo, hi, rng, n_rand)
    B, m, _ = P.shape
    f = omlp.forward(net, P.reshape(-1, 3)).reshape(B, m)
    bad = (f < glo[:, None]) | (f > ghi[:, None])
    return int(bad.sum()), f


def oracle_labels(lo_o, hi_o):
    return oq.classify(lo_o, hi_o)


def valid_topk(record, rel=1e-5):
    """Whether each replayed kept set is a valid top-k of the FP64 candidate
    magnitudes: every kept magnitude is at least every dropped one, up to
    rel times the largest.  Returns the number of (layer, box) violations."""
    bad = 0
    for info in record:
        keep, mu = info["keep"], info["mu"]
        if keep.all():
            continue
        big = np.where(keep, mu, np.inf).min(axis=1)
        small = np.where(keep, -np.inf, mu).max(axis=1)
        bad += int(np.sum(big < small - rel * mu.max(axis=1)))
    return bad


def rigorous_vs_oracle(out, lo_o, hi_o, S):
    """A rigorous-mode bound against the oracle's exact affine bound of the same
    kept terms.  Returns (containment violation relative to S, width ratio
    g/o).  The rigorous bound widens every layer's range by the rounding
    bounds, so it contains the exact bound up to the second-order effect of
    the wider linearisation ranges (affine arithmetic is not inclusion
    monotone), which stays far below the parity tolerance."""
    viol = np.maximum(out["lo"] - lo_o, hi_o - out["hi"]) / S
    w_o = np.maximum(hi_o - lo_o, 1e-300)
    return viol, (out["hi"] - out["lo"]) / w_o


def ray_contract_violations(net, o, d, th, rays, delta, tau, h_frac=0.5, min_run=4):
    """Check GPU ray results against the delta contract of Section 4.1 in
    FP64: a reported hit t has f(p + (t + delta) r) of the other sign than f at
    the ray's start, and no region of the other sign at least ~delta long
    (min_run consecutive samples at spacing h_frac * delta) lies on the ray
    before the hit (for a miss: anywhere on its chord of [-1,1]^3).  Values
    with |f| <= tau count as either sign.  Returns a list of (ray, reason)."""
    o = np.asarray(o, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    t_in, t_out, inside = oq.clip_to_box(o, d)
    h = h_frac * delta
    bad = []
    for i in rays:
        if not inside[i]:
            if np.isfinite(th[i]):
                bad.append((int(i), "hit outside the domain"))
            continue
        start = o[i] + t_in[i] * d[i]
        f0 = omlp.forward_torch(net, start[None])[0]
        end = (t_out[i] - t_in[i]) if not np.isfinite(th[i]) else min(t_out[i] - t_in[i], th[i] - t_in[i])
        if np.isfinite(th[i]):
            fc = omlp.forward_torch(net, (start + (th[i] - t_in[i] + delta) * d[i])[None])[0]
            if not ((fc > 0) != (f0 > 0) or abs(fc) <= tau or abs(f0) <= tau):
                bad.append((int(i), "no sign change within delta of the hit"))
        if abs(f0) <= tau or end <= 0.0:
            continue
        s = np.arange(0.0, end, h)
        f = omlp.forward_torch(net, start[None, :] + s[:, None] * d[i][None, :])
        opp = ((f > 0) != (f0 > 0)) & (np.abs(f) > tau)
        run = 0
        for v in opp:
            run = run + 1 if v else 0
            if run >= min_run:
                bad.append((int(i), "skipped a region of the other sign at least delta long"))
                break
    return bad
