"""Pins of the oracle's queries (Procedures 2 and 3, Section 4.10): closed-form
ray hits, the octree's exact partition of the domain, closest points on an
exactly representable octahedron (CPU only)."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import mlp
from oracle import queries as q


def test_morton_roundtrip():
    rng = np.random.default_rng(1)
    for level in (0, 1, 5, 10, 21):
        n = 1 << level
        ix, iy, iz = (rng.integers(0, n, 100) for _ in range(3))
        code = q.morton_encode(ix, iy, iz, level)
        jx, jy, jz = q.morton_decode(code, level)
        assert np.array_equal(ix, jx) and np.array_equal(iy, jy) and np.array_equal(iz, jz)
    # children of a cell are (code << 3) | octant and tile the parent
    lo, hi = q.cell_bounds(np.array([5], dtype=np.uint64), 2, (-1, -1, -1), (1, 1, 1))
    kids = (np.uint64(5) << np.uint64(3)) | np.arange(8, dtype=np.uint64)
    klo, khi = q.cell_bounds(kids, 3, (-1, -1, -1), (1, 1, 1))
    assert np.allclose(klo.min(0), lo[0]) and np.allclose(khi.max(0), hi[0])
    assert np.isclose(np.prod(khi - klo, axis=1).sum(), np.prod(hi - lo))


def test_kd_bounds_split_widest_at_midpoint():
    lo, hi = q.kd_bounds(np.array([0b1], dtype=np.uint64), 1, (-1, -2, -1), (1, 2, 1))
    assert np.allclose(lo[0], [-1, 0, -1]) and np.allclose(hi[0], [1, 2, 1])   # y is widest
    lo, hi = q.kd_bounds(np.array([0b10], dtype=np.uint64), 2, (-1, -1, -1), (1, 1, 1))
    assert np.allclose(lo[0], [0, -1, -1]) and np.allclose(hi[0], [1, 0, 1])   # x then y


def _tree_volume(res, dom=8.0, arity=8):
    vol = 0.0
    for level, codes in res["pos"] + res["neg"]:
        vol += codes.size * dom / (arity ** level)
    L = len(res["levels"]) - 1
    vol += res["leaves"].size * dom / (arity ** L)
    return vol


@pytest.mark.parametrize("arity,depth", [(8, 5), (2, 12)])
def test_octree_partition_and_soundness(arity, depth):
    net = wl.tiny_net(0)
    res = q.octree_build(net, depth, "truncate", 16, arity=arity, keep_leaf_lists=True)
    assert _tree_volume(res, arity=arity) == 8.0          # exact: sizes are powers of two
    rng = np.random.default_rng(2)
    for (level, codes), sign in [(p, 1) for p in res["pos"]] + [(p, -1) for p in res["neg"]]:
        if codes.size == 0:
            continue
        sel = codes[rng.integers(0, codes.size, min(codes.size, 40))]
        lo, hi = (q.cell_bounds(sel, level, (-1,) * 3, (1,) * 3) if arity == 8
                  else q.kd_bounds(sel, level, (-1,) * 3, (1,) * 3))
        for b in range(sel.size):
            P = lo[b] + rng.uniform(0, 1, (64, 3)) * (hi[b] - lo[b])
            f = mlp.forward(net, P)
            assert np.all(sign * f > 0)


def test_octree_keeps_every_sampled_sign_change():
    net = wl.tiny_net(0)
    depth = 5
    res = q.octree_build(net, depth, "truncate", 31)
    leaves = set(int(c) for c in res["leaves"])
    n = 1 << depth
    rng = np.random.default_rng(3)
    ix, iy, iz = (rng.integers(0, n, 3000) for _ in range(3))
    codes = q.morton_encode(ix, iy, iz, depth)
    lo, hi = q.cell_bounds(codes, depth, (-1,) * 3, (1,) * 3)
    for b in range(codes.size):
        t = np.linspace(0, 1, 4)
        g = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
        f = mlp.forward(net, lo[b] + g * (hi[b] - lo[b]))
        if f.min() < 0 < f.max():
            assert int(codes[b]) in leaves


def _plane_net(a, b, M=16.0):
    a = np.asarray(a, dtype=np.float64)
    W1 = a[None, :].astype(np.float32)
    return wl.MLPSpec([W1, np.array([[1.0]], dtype=np.float32)],
                      [np.array([b + M], dtype=np.float32), np.array([-M], dtype=np.float32)], act="relu")


def test_cast_ray_plane_closed_form():
    a = np.array([0.5, -0.25, 0.75], dtype=np.float32).astype(np.float64)
    b = 0.125
    net = _plane_net(a, b)
    o, d = wl.camera_rays(16, 16, 4)
    o = o.astype(np.float64)
    d = d.astype(np.float64)
    delta = 1e-3
    th, it = q.cast_rays(net, o, d, delta=delta)
    t_in, t_out, inside = q.clip_to_box(o, d)
    fo = o @ a + b
    ts = -fo / (d @ a)
    exp_hit = inside & (ts >= t_in) & (ts <= t_out)
    # a start exactly on the far side of the plane has no crossing along the chord
    assert np.array_equal(np.isfinite(th), exp_hit)
    hit = exp_hit
    assert np.all(th[hit] <= ts[hit] + 1e-9) and np.all(th[hit] >= ts[hit] - delta - 1e-9)


def _octahedron_first_hit(p, r, R, T):
    """First root of g(t) = |p + t r|_1 - R on [0, T] (convex piecewise linear):
    walk the breakpoints where a coordinate changes sign."""
    bps = [0.0] + sorted(t for t in (-p / np.where(r == 0, np.inf, r)) if 0.0 < t < T) + [T]
    g = lambda t: np.abs(p + t * r).sum() - R
    for t0, t1 in zip(bps[:-1], bps[1:]):
        g0, g1 = g(t0), g(t1)
        if g0 == 0.0:
            return t0
        if (g0 > 0) != (g1 > 0):
            return t0 + g0 * (t1 - t0) / (g0 - g1)
    return math.inf


def test_cast_ray_octahedron_closed_form():
    R = 0.6
    net = wl.octahedron_mlp(R)
    o, d = wl.camera_rays(20, 20, 5, fov_deg=22.0)
    o = o.astype(np.float64)
    d = d.astype(np.float64)
    delta = 1e-3
    th, it = q.cast_rays(net, o, d, delta=delta)
    t_in, t_out, inside = q.clip_to_box(o, d)
    for i in range(o.shape[0]):
        if not inside[i]:
            assert math.isinf(th[i])
            continue
        p = o[i] + t_in[i] * d[i]
        ts = _octahedron_first_hit(p, d[i], R, t_out[i] - t_in[i])
        if math.isinf(ts):
            assert math.isinf(th[i])
        else:
            ts += t_in[i]
            assert ts - delta - 1e-9 <= th[i] <= ts + 1e-9, (i, th[i], ts)
    assert np.isfinite(th).sum() > 50


def _l1_ball_distance(x, R):
    s = np.abs(x).sum()
    if s <= R:
        return (R - s) / math.sqrt(3.0)
    u = np.sort(np.abs(x))[::-1]
    cs = np.cumsum(u)
    rho = max(j for j in range(1, 4) if u[j - 1] - (cs[j - 1] - R) / j > 0)
    theta = (cs[rho - 1] - R) / rho
    proj = np.maximum(np.abs(x) - theta, 0.0)
    return float(np.linalg.norm(np.abs(x) - proj))


def test_closest_point_octahedron():
    # a radius off the dyadic grid: with R = 0.5 the surface passes exactly
    # through cell face centers, where the sign test sees f = 0
    net = wl.octahedron_mlp(0.55)
    R = float(net.biases[1][0]) * -1.0
    rng = np.random.default_rng(6)
    L = 6
    diag = math.sqrt(3.0) * 2.0 / (1 << L)
    for _ in range(6):
        x = rng.uniform(-1, 1, 3)
        pt, dist, best = q.closest_point(net, x, max_level=L, policy="fixed")
        dstar = _l1_ball_distance(x, R)
        assert pt is not None
        assert best >= dstar - 1e-12
        assert dstar - diag / 2 - 1e-12 <= dist <= dstar + diag + 1e-12
        assert abs(np.abs(pt).sum() - R) <= math.sqrt(3.0) * diag / 2 + 1e-12


def test_valid_topk_detects_a_wrong_kept_set():
    """The top-k validity check used by the GPU tests: the oracle's own
    selection passes; keeping the smallest dropped candidate instead of the
    smallest kept one (strictly larger) fails."""
    import os
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    from parity import valid_topk
    from oracle import mlp as omlp
    net = wl.tiny_net(0)
    lo, hi = wl.boxes(64, 3, 1e-3, 0.2)
    rec = []
    omlp.bound_boxes(net, lo, hi, "truncate", 8, record=rec)
    assert valid_topk(rec) == 0
    mu = rec[0]["mu"]
    keep = rec[0]["keep"]
    b = int(np.argmax([mu[i, keep[i]].min() - mu[i, ~keep[i]].min() for i in range(len(mu))]))
    kept = np.flatnonzero(keep[b])
    dropped = np.flatnonzero(~keep[b])
    i_small = kept[np.argmin(mu[b, kept])]
    i_low = dropped[np.argmin(mu[b, dropped])]
    assert mu[b, i_low] < mu[b, i_small]
    sets = [r["keep"].copy() for r in rec]
    sets[0][b, i_small] = False
    sets[0][b, i_low] = True
    rec2 = []
    omlp.bound_boxes(net, lo, hi, "truncate", 8, keep_sets=sets, record=rec2)
    assert valid_topk(rec2) >= 1


def test_ray_contract_checker_flags_planted_mistakes():
    """The delta-contract checker used by the GPU ray tests, pinned on the
    exact octahedron |x|_1 = R: the oracle's own results pass; a miss on a ray
    through the solid, a hit moved a quarter of the chord early and a hit
    moved past the surface are each flagged."""
    from parity import ray_contract_violations
    net = wl.octahedron_mlp(0.6)
    o, d = wl.camera_rays(6, 6, 5, fov_deg=22.0)
    delta = 1e-3
    th, _ = q.cast_rays(net, o.astype(np.float64), d.astype(np.float64), delta=delta)
    rays = np.arange(o.shape[0])
    assert ray_contract_violations(net, o, d, th, rays, delta, 1e-9) == []
    hit = np.flatnonzero(np.isfinite(th))
    assert hit.size >= 4
    t_in, t_out, _ = q.clip_to_box(o, d)
    bad = th.copy()
    bad[hit[0]] = np.inf                                           # missed the solid
    bad[hit[1]] = t_in[hit[1]] + 0.25 * (th[hit[1]] - t_in[hit[1]])  # no surface there
    bad[hit[2]] = th[hit[2]] + 0.05                                 # inside, past the surface
    got = {i for i, _ in ray_contract_violations(net, o, d, bad, rays, delta, 1e-9)}
    assert got == {int(hit[0]), int(hit[1]), int(hit[2])}


def test_frustum_box_contains_the_swept_region_and_is_tight():
    """Brute force over sampled rays and distances: every point of a frustum
    between t and t + sigma lies in the oriented box, and each face of the box
    is reached by the region (up to the sampling density), including the
    forward face beyond the corner rays' front."""
    cam = wl.camera(40, 30, 9, fov_deg=70.0)
    rng = np.random.default_rng(4)
    frame = np.stack([cam["forward"], cam["right"], cam["up"]])
    for x0, x1, y0, y1 in [(0, 40, 0, 30), (3, 9, 20, 30), (17, 23, 12, 18), (39, 40, 0, 1), (0, 1, 29, 30)]:
        t, sg = 2.0, 0.7
        c, ax = q.frustum_box(cam, [x0], [x1], [y0], [y1], [t], [sg])
        # continuous tangent-plane rectangle through the extreme pixel centers
        xa, _ = q.pixel_coords(cam, x0, 0)
        xb, _ = q.pixel_coords(cam, x1 - 1, 0)
        _, ya = q.pixel_coords(cam, 0, y1 - 1)
        _, yb = q.pixel_coords(cam, 0, y0)
        n = 20000
        x = rng.uniform(min(xa, xb), max(xa, xb), n)
        y = rng.uniform(min(ya, yb), max(ya, yb), n)
        # include every combination of the x and y extremes (ends and the
        # point nearest the axis) at both distances
        cx = [xa, xb, np.clip(0.0, min(xa, xb), max(xa, xb))]
        cy = [ya, yb, np.clip(0.0, min(ya, yb), max(ya, yb))]
        ex = np.array([a for a in cx for _ in cy] * 2)
        ey = np.array([b for _ in cx for b in cy] * 2)
        es = np.repeat([t, t + sg], 9)
        s = rng.uniform(t, t + sg, n)
        x, y, s = np.concatenate([x, ex]), np.concatenate([y, ey]), np.concatenate([s, es])
        d = cam["forward"][None] + x[:, None] * cam["right"][None] + y[:, None] * cam["up"][None]
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        p = cam["eye"][None] + s[:, None] * d
        # coordinates in the box's own axes
        half = np.linalg.norm(ax[0], axis=1)
        u = ((p - c[0][None]) @ frame.T) / half[None]
        assert np.all(np.abs(u) <= 1.0 + 1e-12), np.abs(u).max()
        assert np.all(u.max(axis=0) >= 1.0 - 1e-9) and np.all(u.min(axis=0) <= -1.0 + 1e-9), (u.min(0), u.max(0))


def test_frustum_cast_octahedron_closed_form():
    """Frustum casting on the exact octahedron: every pixel's hit is the
    closed-form first intersection up to delta, and every ray through the
    solid hits (the solid is far thicker than delta)."""
    R = 0.6
    net = wl.octahedron_mlp(R)
    cam = wl.camera(32, 24, 5, fov_deg=30.0)
    delta = 1e-3
    th, steps = q.cast_frusta(net, cam, tiles=(4, 4), delta=delta)
    o, d = wl.camera_rays(32, 24, 5, fov_deg=30.0)
    n_hit = 0
    for i in range(o.shape[0]):
        p, r = o[i].astype(np.float64), q.pixel_dirs(cam, i % 32, i // 32).reshape(3)
        ts = math.inf
        bps = sorted(tt for tt in (-p / np.where(r == 0, np.inf, r)) if tt > 0.0) + [20.0]
        prev = 0.0
        g = lambda tt: np.abs(p + tt * r).sum() - R
        for t1 in bps:
            if (g(prev) > 0) != (g(t1) > 0):
                ts = prev + g(prev) * (t1 - prev) / (g(prev) - g(t1))
                break
            prev = t1
        if math.isinf(ts):
            assert math.isinf(th[i]), i
        else:
            n_hit += 1
            assert ts - delta - 1e-9 <= th[i] <= ts + 1e-9, (i, th[i], ts)
    assert n_hit > 50
    assert steps.min() >= 1


@pytest.mark.parametrize("netname", ["tiny", "elu"])
def test_frustum_cast_matches_ray_cast(netname):
    """On random networks the frustum caster and the per-ray caster return the
    same hits up to the delta contract (Section 4.1): the same hit/miss
    decision and hit distances within 2 delta, and every frustum result,
    where they differ, passes the FP64 contract check."""
    from parity import ray_contract_violations
    net = wl.tiny_net(0) if netname == "tiny" else wl.he_normal_mlp([3, 32, 32, 1], 41, act="elu", bias=-0.3)
    cam = wl.camera(24, 24, 7)
    delta = 1e-3
    th, _ = q.cast_frusta(net, cam, tiles=(4, 4), delta=delta)
    o, d = wl.camera_rays(24, 24, 7)
    tr, _ = q.cast_rays(net, o.astype(np.float64), q.pixel_dirs(cam, np.arange(576) % 24, np.arange(576) // 24),
                        delta=delta)
    agree = np.isfinite(th) == np.isfinite(tr)
    both = np.isfinite(th) & np.isfinite(tr)
    near = np.abs(np.where(both, th, 0.0) - np.where(both, tr, 0.0)) <= 2 * delta + 1e-9
    assert agree.mean() >= 0.98 and near.mean() >= 0.98
    differ = np.flatnonzero(~agree | ~near)
    dirs = q.pixel_dirs(cam, np.arange(576) % 24, np.arange(576) // 24)
    bad = ray_contract_violations(net, np.broadcast_to(cam["eye"], (576, 3)), dirs, th, differ, delta, 1e-9)
    assert not bad, bad[:5]


def _l1_range_over_box(lo, hi):
    """Exact range of |x|_1 over an axis-aligned box."""
    mx = np.maximum(np.abs(lo), np.abs(hi)).sum(axis=1)
    mn = np.where((lo <= 0) & (hi >= 0), 0.0, np.minimum(np.abs(lo), np.abs(hi))).sum(axis=1)
    return mn, mx


def test_empty_spheres_octahedron_closed_form():
    """On the exact octahedron |x|_1 = R: every returned cube lies strictly on
    one side of the surface (closed-form range of |x|_1), with the right sign;
    a point on the surface gets radius 0; radii are r0 / 2^j; the center,
    0.6 from the surface in |x|_1, gets a NEGATIVE cube of half-width at least
    0.125 (whose |x|_1 stays below 0.375)."""
    R = 0.6
    net = wl.octahedron_mlp(R)
    rng = np.random.default_rng(3)
    p = rng.uniform(-1, 1, (300, 3))
    p[0] = [R, 0.0, 0.0]                       # on the surface
    p[1] = [0.0, 0.0, 0.0]                     # the center, 0.6 from the surface
    r0, rmin = 0.5, 1e-3
    rad, lab = q.empty_spheres(net, p, r0, rmin)
    assert rad[0] == 0.0 and lab[0] == q.UNKNOWN
    ok = rad > 0
    j = np.log2(r0 / rad[ok])
    assert np.allclose(j, np.round(j))
    lo, hi = p[ok] - rad[ok, None], p[ok] + rad[ok, None]
    mn, mx = _l1_range_over_box(lo, hi)
    pos = lab[ok] == q.POSITIVE
    assert np.all(mn[pos] > R) and np.all(mx[~pos] < R)
    # the center: the cube of half-width 0.5 has |x|_1 <= 1.5 > R, so it is not
    # classified; 0.125 (|x|_1 <= 0.375) must be
    assert lab[1] == q.NEGATIVE and rad[1] >= 0.125


def _octa_at(a, R):
    """Exact ReLU network of |x - a|_1 - R (an octahedron centered at a)."""
    a = np.asarray(a, dtype=np.float32)
    W1 = np.concatenate([np.eye(3), -np.eye(3)]).astype(np.float32)
    b1 = np.concatenate([-a, a]).astype(np.float32)
    return wl.MLPSpec([W1, np.ones((1, 6), np.float32)], [b1, np.array([-R], np.float32)], act="relu")


def test_intersect_octahedra_closed_form():
    """Two L1 balls overlap iff the L1 distance of their centers is below the
    sum of their radii.  Overlapping pairs give INTERSECTION with a witness
    cell inside both (closed-form range of |x - a|_1 over the cell); a pair
    with a clear gap gives NO_INTERSECTION; touching pairs are UNDECIDED at a
    limited depth."""
    R = 0.35
    for shift, want in ((0.5, q.INTERSECTION), (0.9, q.NO_INTERSECTION), (0.7, None)):
        f = _octa_at([-shift / 2, 0.0, 0.0], R)
        g = _octa_at([shift / 2, 0.0, 0.0], R)
        res = q.intersect(f, g, 6)
        if want is not None:
            assert res["result"] == want, (shift, res)
        else:
            assert res["result"] == q.UNDECIDED and res["undecided"] > 0
        if res["result"] == q.INTERSECTION:
            lo, hi = q.cell_bounds(np.array([res["cell"]], dtype=np.uint64), res["level"], (-1,) * 3, (1,) * 3)
            for c in ([-shift / 2, 0, 0], [shift / 2, 0, 0]):
                _, mx = _l1_range_over_box(lo - np.array(c), hi - np.array(c))
                assert mx[0] < R
    # a shape against itself: inside both wherever it is inside
    f = _octa_at([0.1, 0.0, 0.0], 0.5)
    assert q.intersect(f, f, 4)["result"] == q.INTERSECTION


def test_delta_tree_octahedron():
    """The convergence test of Procedure 3 on the exact octahedron: every
    converged cell is smaller than delta / sqrt(3) in each side and contains a
    point of the surface (closed-form range of |x|_1), so it lies within
    delta of the level set; POSITIVE, NEGATIVE, converged and max-level cells
    tile the domain exactly; and a larger delta converges at a coarser level."""
    R = 0.55
    net = wl.octahedron_mlp(R)
    for delta, first in ((0.2, 5), (0.05, 7)):
        res = q.octree_build(net, 9, "fixed", 0, delta=delta)
        assert res["converged"] and res["converged"][0][0] == first
        vol = 0.0
        for lv in res["levels"]:
            vol += (lv["n_pos"] + lv["n_neg"] + lv["n_conv"]) * 8.0 ** -lv["level"]
        vol += res["leaves"].size * 8.0 ** -9
        assert vol == 1.0
        for level, codes in res["converged"]:
            lo, hi = q.cell_bounds(codes, level, (-1,) * 3, (1,) * 3)
            assert np.all(hi - lo < delta / math.sqrt(3.0))
            mn, mx = _l1_range_over_box(lo, hi)
            assert np.all(mn <= R) and np.all(mx >= R)


def _mesh_topology(tris):
    """(V, E, F, edges used by other than two triangles) of a triangle soup
    whose shared vertices are bitwise equal."""
    vid = {}
    faces = []
    for t in tris:
        ids = []
        for v in t:
            key = tuple(float(x) for x in v)
            ids.append(vid.setdefault(key, len(vid)))
        faces.append(ids)
    from collections import Counter
    ec = Counter()
    for a, b, c in faces:
        for u, w in ((a, b), (b, c), (c, a)):
            ec[(min(u, w), max(u, w))] += 1
    bad = sum(1 for k, n in ec.items() if n != 2)
    return len(vid), len(ec), len(faces), bad


def test_mc_cube_every_sign_pattern():
    """All 256 corner sign patterns of one cube: the triangles' vertices are
    exactly the crossing edges' interpolated points, every crossing edge is
    used, and the loops cut the cube consistently: the number of triangles is
    (crossing edges) - 2 (loops)."""
    rng = np.random.default_rng(5)
    p = np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], dtype=np.float64)
    for pattern in range(256):
        v = [(rng.uniform(0.1, 1.0) if (pattern >> c) & 1 else -rng.uniform(0.1, 1.0)) for c in range(8)]
        tris = q.mc_cube(v, p)
        cross = [(a, b) for a, b in q.MC_EDGES if (v[a] > 0) != (v[b] > 0)]
        pts = {tuple(p[a] + v[a] / (v[a] - v[b]) * (p[b] - p[a])) for a, b in cross}
        used = {tuple(x) for t in tris for x in t}
        assert used == pts, pattern
        if cross:
            V, E, F, bad = _mesh_topology(tris)
            # each loop of m points is a fan of m - 2 triangles
            assert V == len(cross) and (V - F) % 2 == 0 and (V - F) // 2 >= 1, pattern
            # the loops are closed polygons: their m sides are the edges used
            # once (the segments on the cube's faces), the fan diagonals twice
            assert bad == len(cross), pattern


def test_mesh_octahedron_is_closed_and_exact():
    """Leaves of the exact octahedron's octree at level 2, meshed with 3 dense
    levels (a 32^3 grid whose lines include the coordinate planes, so f is
    linear on every grid edge): every vertex lies exactly on |x|_1 = R, every
    mesh edge is shared by exactly two triangles, and the Euler
    characteristic is 2 (a sphere)."""
    R = 0.55
    net = wl.octahedron_mlp(R)
    res = q.octree_build(net, 2, "fixed", 0)
    tris, owner, cube = q.mesh_leaves(net, res["leaves"], 2, 3)
    assert tris.shape[0] > 100
    assert np.allclose(np.abs(tris).sum(axis=2), R, atol=1e-12)
    V, E, F, bad = _mesh_topology(tris)
    assert bad == 0
    assert V - E + F == 2


def test_splitmix64_reference_value():
    """The generator's first output for seed 0 is the published 0xe220a8397b1dcdaf,
    and consecutive outputs are the documented increments of the state."""
    assert int(q.splitmix64(0, np.array([0]))[0]) == 0xe220a8397b1dcdaf
    a = q.splitmix64(12345, np.arange(4))
    assert len(set(int(x) for x in a)) == 4


def test_band_sampling_and_volume_octahedron():
    """The exact octahedron |x|_1 = R: the bulk volume brackets the exact
    (4/3) R^3 and its estimate lies within 4 standard errors; the leaves of
    the band tree (r = 0.05) contain every point of the band that rejection
    sampling of the whole domain finds; band samples lie in the leaves and
    have |f| < r."""
    R = 0.55
    net = wl.octahedron_mlp(R)
    vol, lo, hi = q.bulk_volume(net, 4, 20000, 7, "fixed", 0)
    exact = 4.0 / 3.0 * R ** 3
    assert lo <= exact <= hi
    res = q.octree_build(net, 4, "fixed", 0)
    v_leaf = res["leaves"].size * 8.0 / 8.0 ** 4
    p_in = (exact - lo) / v_leaf
    se = v_leaf * math.sqrt(p_in * (1 - p_in) / 20000)
    assert abs(vol - exact) <= 4 * se + 1e-12
    r = 0.05
    bt = q.octree_build(net, 4, "fixed", 0, band=r)
    lo_c, hi_c = q.cell_bounds(bt["leaves"], 4, (-1,) * 3, (1,) * 3)

    def in_leaves(x):
        m = np.zeros(len(x), bool)
        for a, b in zip(lo_c, hi_c):
            m |= np.all((x >= a) & (x <= b), axis=1)
        return m
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, (200000, 3))
    xb = x[np.abs(np.abs(x).sum(axis=1) - R) < r]
    assert xb.shape[0] > 1000 and in_leaves(xb).all()
    pts, f, ok = q.sample_leaves(net, bt["leaves"], 4, 5000, 3, band=r)
    assert in_leaves(pts).all() and ok.sum() > 1000
    assert np.all(np.abs(np.abs(pts[ok]).sum(axis=1) - R) < r + 1e-12)
    # the band tree keeps every cell of the level-set tree
    assert np.isin(res["leaves"], bt["leaves"]).all()
