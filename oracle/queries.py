"""Geometric queries built on RangeBound (oracle; test infrastructure only).

* :func:`classify`      -- Procedure 1 steps 4-6.
* :func:`octree_build`  -- Procedure 3 run as breadth-first parallel rounds to
  a fixed depth (Section 4.5 and the fixed-depth option used for mesh
  extraction, Section 4.7), octree (arity 8) or k-d (arity 2) splits.
* :func:`cast_rays`     -- Procedure 2 with the Appendix B step safety factor.
* :func:`closest_point` -- Section 4.10 lazy best-first descent.
* :func:`cast_frusta`   -- Section 4.3 frustum ray casting (Appendix B split
  rule and spherical-front box), ending in Procedure 2 per pixel.
* :func:`empty_spheres` -- Section 4.4 empty-sphere radii by shrinking cubes.
* :func:`intersect`     -- Section 4.9 intersection test of two shapes on a
  shared octree.
* :func:`mesh_leaves`   -- Section 4.7 mesh extraction: marching cubes on the
  dense grid of each leaf cell.
* :func:`sample_leaves`, :func:`bulk_volume` -- Sections 4.6 and 4.8: uniform
  samples in leaf cells (surface band sampling) and the solid's volume.
"""
from __future__ import annotations

import heapq
import math

import numpy as np

from . import mlp

UNKNOWN, POSITIVE, NEGATIVE = 0, 1, 2


def classify(lo, hi):
    """POSITIVE if lo > 0, NEGATIVE if hi < 0, else UNKNOWN (strict)."""
    lab = np.full(np.shape(lo), UNKNOWN, dtype=np.uint8)
    lab[np.asarray(lo) > 0.0] = POSITIVE
    lab[np.asarray(hi) < 0.0] = NEGATIVE
    return lab


def range_bound(net, lo, hi, policy="truncate", k=31):
    """(lo_y, hi_y, label) for each axis-aligned box."""
    _, _, ly, hy = mlp.bound_boxes(net, lo, hi, policy, k)
    return ly, hy, classify(ly, hy)


# ---------------------------------------------------------------------------
# Cells: Morton codes (bit b of the x index at position 3b, y at 3b+1, z at
# 3b+2).  The 8 children of code c are (c << 3) | octant with octant =
# dx | dy << 1 | dz << 2.
# ---------------------------------------------------------------------------

def morton_encode(ix, iy, iz, level):
    ix = np.asarray(ix, dtype=np.uint64)
    iy = np.asarray(iy, dtype=np.uint64)
    iz = np.asarray(iz, dtype=np.uint64)
    code = np.zeros(ix.shape, dtype=np.uint64)
    for b in range(level):
        bb = np.uint64(b)
        one = np.uint64(1)
        code |= ((ix >> bb) & one) << np.uint64(3 * b)
        code |= ((iy >> bb) & one) << np.uint64(3 * b + 1)
        code |= ((iz >> bb) & one) << np.uint64(3 * b + 2)
    return code


def morton_decode(code, level):
    code = np.asarray(code, dtype=np.uint64)
    ix = np.zeros(code.shape, dtype=np.int64)
    iy = np.zeros(code.shape, dtype=np.int64)
    iz = np.zeros(code.shape, dtype=np.int64)
    one = np.uint64(1)
    for b in range(level):
        ix |= (((code >> np.uint64(3 * b)) & one).astype(np.int64)) << b
        iy |= (((code >> np.uint64(3 * b + 1)) & one).astype(np.int64)) << b
        iz |= (((code >> np.uint64(3 * b + 2)) & one).astype(np.int64)) << b
    return ix, iy, iz


def cell_bounds(code, level, dom_lo, dom_hi):
    """float64 bounds of octree cells at ``level`` over the domain box."""
    ix, iy, iz = morton_decode(code, level)
    dom_lo = np.asarray(dom_lo, dtype=np.float64)
    dom_hi = np.asarray(dom_hi, dtype=np.float64)
    size = (dom_hi - dom_lo) / float(1 << level)
    idx = np.stack([ix, iy, iz], axis=1).astype(np.float64)
    lo = dom_lo + idx * size
    hi = dom_lo + (idx + 1.0) * size
    return lo, hi


def kd_axes(depth, dom_lo, dom_hi):
    """Split axis at every k-d depth: the widest dimension of the node, the
    first one on ties (Procedure 3).  Nodes at one depth share their extents,
    so the axis sequence depends on the depth only."""
    ext = np.asarray(dom_hi, dtype=np.float64) - np.asarray(dom_lo, dtype=np.float64)
    axes = []
    for _ in range(depth):
        a = int(np.argmax(ext))
        axes.append(a)
        ext[a] /= 2.0
    return axes


def kd_bounds(code, depth, dom_lo, dom_hi):
    """Bounds of k-d nodes: ``code`` holds ``depth`` bits, the most significant
    bit being the first split; bit 1 selects the upper half (the child
    [x_l + x_s, x_u] with x_s half the width)."""
    axes = kd_axes(depth, dom_lo, dom_hi)
    code = np.asarray(code, dtype=np.uint64)
    lo = np.tile(np.asarray(dom_lo, dtype=np.float64), (code.size, 1))
    hi = np.tile(np.asarray(dom_hi, dtype=np.float64), (code.size, 1))
    for d, a in enumerate(axes):
        bit = ((code >> np.uint64(depth - 1 - d)) & np.uint64(1)).astype(bool)
        mid = (lo[:, a] + hi[:, a]) / 2.0
        lo[:, a] = np.where(bit, mid, lo[:, a])
        hi[:, a] = np.where(bit, hi[:, a], mid)
    return lo, hi


def octree_build(net, max_level, policy="truncate", k=31, dom_lo=(-1, -1, -1), dom_hi=(1, 1, 1),
                 arity=8, keep_leaf_lists=False, max_cells=None, delta=None, band=0.0):
    """Fixed-depth BuildSpatialTree in parallel rounds.

    Each round classifies every cell of the current level: POSITIVE and
    NEGATIVE cells become leaves; UNKNOWN cells below ``max_level`` are split
    (arity 8: into 8 equal octants; arity 2: the widest dimension at its
    midpoint); UNKNOWN cells at ``max_level`` form the leaf list handed to mesh
    extraction.  Returns a dict with per-level frontier sizes and counts, the
    sorted UNKNOWN leaf codes and (optionally) the POSITIVE/NEGATIVE leaves.

    With ``delta`` (octree only) the convergence test of Procedure 3 applies:
    at a level whose cells' widest side is below delta / sqrt(3), an UNKNOWN
    cell whose six face centers show both signs of f is final (within delta of
    the level set); ``converged`` then lists (level, sorted codes).  With
    ``band`` r > 0 cells are classified against the band |f| <= r (Section
    4.6): POSITIVE when f > r, NEGATIVE when f < -r.
    """
    codes = np.zeros(1, dtype=np.uint64)
    levels = []
    converged = []
    pos_leaves, neg_leaves = [], []
    unk_leaves = np.zeros(0, dtype=np.uint64)
    for level in range(max_level + 1):
        if arity == 8:
            lo, hi = cell_bounds(codes, level, dom_lo, dom_hi)
        else:
            lo, hi = kd_bounds(codes, level, dom_lo, dom_hi)
        if codes.size:
            _, _, ly, hy = mlp.bound_boxes(net, lo, hi, policy, k)
            lab = classify(ly - band, hy + band)
        else:
            lab = np.zeros(0, dtype=np.uint8)
        unk = codes[lab == UNKNOWN]
        n_conv = 0
        if delta is not None and arity == 8 and unk.size and \
                np.max(np.asarray(dom_hi, dtype=np.float64) - np.asarray(dom_lo, dtype=np.float64)) / 2.0 ** level \
                < delta / math.sqrt(3.0):
            ulo, uhi = lo[lab == UNKNOWN], hi[lab == UNKNOWN]
            pts = np.stack([face_centers(ulo[j], uhi[j]) for j in range(unk.size)])   # [m, 6, 3]
            fv = mlp.forward(net, pts.reshape(-1, 3)).reshape(unk.size, 6)
            span = np.any(fv < 0.0, axis=1) & np.any(fv > 0.0, axis=1)
            converged.append((level, np.sort(unk[span])))
            n_conv = int(span.sum())
            unk = unk[~span]
        levels.append({"level": level, "n": int(codes.size), "n_pos": int((lab == POSITIVE).sum()),
                       "n_neg": int((lab == NEGATIVE).sum()), "n_unk": int(unk.size), "n_conv": n_conv})
        if keep_leaf_lists:
            pos_leaves.append((level, codes[lab == POSITIVE]))
            neg_leaves.append((level, codes[lab == NEGATIVE]))
        if level == max_level:
            unk_leaves = np.sort(unk)
            break
        shift = np.uint64(3 if arity == 8 else 1)
        kids = [(unk << shift) | np.uint64(o) for o in range(arity)]
        codes = np.sort(np.concatenate(kids)) if unk.size else np.zeros(0, dtype=np.uint64)
        if max_cells is not None and codes.size > max_cells:
            raise RuntimeError("frontier exceeds max_cells")
    return {"levels": levels, "leaves": unk_leaves, "pos": pos_leaves, "neg": neg_leaves, "converged": converged}


# ---------------------------------------------------------------------------
# Ray casting (Procedure 2)
# ---------------------------------------------------------------------------

def clip_to_box(o, d, lo=-1.0, hi=1.0):
    """Slab test: entry/exit parameters of the rays in the box; miss flag."""
    o = np.asarray(o, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        t1 = (lo - o) * inv
        t2 = (hi - o) * inv
    tmin = np.minimum(t1, t2)
    tmax = np.maximum(t1, t2)
    # a zero direction component: inside the slab -> (-inf, inf), else empty
    zero = d == 0.0
    inside = (o >= lo) & (o <= hi)
    tmin = np.where(zero, np.where(inside, -np.inf, np.inf), tmin)
    tmax = np.where(zero, np.where(inside, np.inf, -np.inf), tmax)
    t_in = np.maximum(np.max(tmin, axis=1), 0.0)
    t_out = np.min(tmax, axis=1)
    hit = t_out > t_in
    return t_in, t_out, hit


def different_signs(a, b):
    """Sign change test: zero counts as inside (negative side)."""
    return (np.asarray(a) > 0.0) != (np.asarray(b) > 0.0)


def cast_rays(net, origin, direction, delta=1e-3, t_max=10.0, sigma0=None, eta_minus=0.5, eta_plus=1.5,
              safety=0.98, max_iters=100000, clip_to_domain=True, policy="fixed", k=31):
    """CastRay for a batch of rays, all advanced in lock-step rounds.

    Per round for each active ray: evaluate f at t + delta and return t on a
    sign change relative to f at the start; otherwise bound f on the segment
    [t, t + sigma] and either accept the step (sigma* = safety sigma, sigma
    grows by eta_plus) or reject it (sigma* = 0, sigma shrinks by eta_minus);
    then t += max(sigma*, delta).  With ``clip_to_domain`` each ray is first
    clipped to [-1,1]^3 and marched from its entry point over its chord only.

    Returns (t_hit [n] with +inf for no hit, iterations [n])."""
    o = np.asarray(origin, dtype=np.float64)
    d = np.asarray(direction, dtype=np.float64)
    n = o.shape[0]
    if sigma0 is None:
        sigma0 = t_max / 10.0
    t_hit = np.full(n, np.inf)
    iters = np.zeros(n, dtype=np.int64)
    if clip_to_domain:
        t_in, t_out, inside = clip_to_box(o, d)
        start = o + t_in[:, None] * d
        tmax_r = np.where(inside, t_out - t_in, 0.0)
        base = t_in
    else:
        start = o.copy()
        tmax_r = np.full(n, float(t_max))
        base = np.zeros(n)
        inside = np.ones(n, dtype=bool)
    t = np.zeros(n)
    sigma = np.full(n, float(sigma0))
    active = inside & (tmax_r > 0.0)
    f0 = np.zeros(n)
    if np.any(active):
        f0[active] = mlp.forward(net, start[active])
    while np.any(active):
        idx = np.flatnonzero(active)
        still = t[idx] < tmax_r[idx]
        active[idx[~still]] = False
        idx = idx[still]
        if idx.size == 0:
            break
        iters[idx] += 1
        pc = start[idx] + (t[idx] + delta)[:, None] * d[idx]
        fc = mlp.forward(net, pc)
        hit = different_signs(f0[idx], fc)
        t_hit[idx[hit]] = base[idx[hit]] + t[idx[hit]]
        active[idx[hit]] = False
        idx = idx[~hit]
        if idx.size == 0:
            continue
        ly, hy = mlp.bound_segments(net, start[idx], d[idx], t[idx], sigma[idx], policy, k)
        safe = classify(ly, hy) != UNKNOWN
        step = np.where(safe, safety * sigma[idx], 0.0)
        sigma[idx] = np.where(safe, sigma[idx] * eta_plus, sigma[idx] * eta_minus)
        t[idx] = t[idx] + np.maximum(step, delta)
        over = iters[idx] >= max_iters
        active[idx[over]] = False
    return t_hit, iters


# ---------------------------------------------------------------------------
# Closest point (Section 4.10)
# ---------------------------------------------------------------------------

def face_centers(lo, hi):
    c = (lo + hi) / 2.0
    pts = []
    for a in range(3):
        for v in (lo[a], hi[a]):
            p = c.copy()
            p[a] = v
            pts.append(p)
    return np.array(pts)


def closest_point(net, q, max_level=8, policy="fixed", k=31, dom_lo=(-1, -1, -1), dom_hi=(1, 1, 1)):
    """Lazy best-first descent of the octree for one query point q.

    Cells are visited in order of their minimum distance to q.  A cell is
    skipped when that distance is not below the best distance found, or when
    RangeBound classifies it.  A cell whose six face-center samples show both
    signs spans the level set: the best distance becomes at most the farthest
    distance from q to the cell and its center becomes the candidate.  Cells
    below ``max_level`` push their 8 children.

    Returns (point [3], distance from q to the point, best bound); point is
    None and the distances +inf if no cell spanning the surface was found."""
    q = np.asarray(q, dtype=np.float64)
    dom_lo = np.asarray(dom_lo, dtype=np.float64)
    dom_hi = np.asarray(dom_hi, dtype=np.float64)

    def mind(lo, hi):
        return float(np.linalg.norm(np.maximum(np.maximum(lo - q, q - hi), 0.0)))

    def maxd(lo, hi):
        return float(np.linalg.norm(np.maximum(np.abs(q - lo), np.abs(q - hi))))

    best = math.inf
    point = None
    heap = [(mind(dom_lo, dom_hi), 0, 0)]   # (min distance, level, code)
    while heap:
        dmin, level, code = heapq.heappop(heap)
        if dmin >= best:
            break
        lo, hi = cell_bounds(np.array([code], dtype=np.uint64), level, dom_lo, dom_hi)
        lo, hi = lo[0], hi[0]
        _, _, ly, hy = mlp.bound_boxes(net, lo[None], hi[None], policy, k)
        if classify(ly, hy)[0] != UNKNOWN:
            continue
        fv = mlp.forward(net, face_centers(lo, hi))
        if np.any(fv < 0.0) and np.any(fv > 0.0):
            dm = maxd(lo, hi)
            if dm < best:
                best = dm
                point = (lo + hi) / 2.0
        if level < max_level:
            for o in range(8):
                c2 = (code << 3) | o
                l2, h2 = cell_bounds(np.array([c2], dtype=np.uint64), level + 1, dom_lo, dom_hi)
                dm2 = mind(l2[0], h2[0])
                if dm2 < best:
                    heapq.heappush(heap, (dm2, level + 1, c2))
    if point is None:
        return None, math.inf, math.inf
    return point, float(np.linalg.norm(point - q)), best


# ---------------------------------------------------------------------------
# Frustum ray casting (Section 4.3; Appendix B)
# ---------------------------------------------------------------------------

def pixel_coords(cam, px, py):
    """Tangent-plane coordinates (x, y) of pixel centers."""
    x = (2.0 * (np.asarray(px, dtype=np.float64) + 0.5) / cam["width"] - 1.0) * cam["tan_x"]
    y = (1.0 - 2.0 * (np.asarray(py, dtype=np.float64) + 0.5) / cam["height"]) * cam["tan_y"]
    return x, y


def pixel_dirs(cam, px, py):
    """Unit directions normalize(forward + x right + y up) of pixel centers."""
    x, y = pixel_coords(cam, px, py)
    d = np.asarray(cam["forward"], dtype=np.float64)[None, :] + np.asarray(x)[..., None] * \
        np.asarray(cam["right"], dtype=np.float64)[None, :] + np.asarray(y)[..., None] * \
        np.asarray(cam["up"], dtype=np.float64)[None, :]
    return d / np.linalg.norm(d, axis=-1, keepdims=True)


def frustum_box(cam, x0, x1, y0, y1, t, sigma):
    """Oriented box (center [m, 3], axes [m, 3, 3]) bounding the part of each
    frustum between distances t and t + sigma along its rays: the points
    eye + s d with s in [t, t + sigma] and d any ray through the tangent-plane
    rectangle spanned by the centers of pixels x0..x1-1, y0..y1-1.

    The box is taken in the camera frame (forward, right, up).  A point has
    coordinates s (1, x, y) / sqrt(1 + x^2 + y^2); each coordinate is
    monotone in x (or y) with the other fixed, so its extremes lie on the
    rectangle's edges at the smallest or largest |x|, |y|.  The forward
    extent reaches (t + sigma) / sqrt(1 + x^2 + y^2) at the point of the
    rectangle nearest the axis, beyond the front face through the corner
    rays: the rays sweep a spherical front (Appendix B)."""
    x0, x1, y0, y1 = (np.asarray(v, dtype=np.int64) for v in (x0, x1, y0, y1))
    t = np.asarray(t, dtype=np.float64)
    s1 = t + np.asarray(sigma, dtype=np.float64)
    xa, _ = pixel_coords(cam, x0, 0)
    xb, _ = pixel_coords(cam, x1 - 1, 0)
    _, ya = pixel_coords(cam, 0, y1 - 1)     # y decreases down the image
    _, yb = pixel_coords(cam, 0, y0)
    xlo, xhi = np.minimum(xa, xb), np.maximum(xa, xb)
    ylo, yhi = np.minimum(ya, yb), np.maximum(ya, yb)

    def near0(lo, hi):
        return np.where((lo <= 0.0) & (hi >= 0.0), 0.0, np.minimum(np.abs(lo), np.abs(hi)))

    mx2, my2 = near0(xlo, xhi) ** 2, near0(ylo, yhi) ** 2
    Mx2, My2 = np.maximum(xlo ** 2, xhi ** 2), np.maximum(ylo ** 2, yhi ** 2)
    f_lo = t / np.sqrt(1.0 + Mx2 + My2)
    f_hi = s1 / np.sqrt(1.0 + mx2 + my2)

    def lateral(lo, hi, o_min2, o_max2):
        gmax = hi / np.sqrt(1.0 + hi ** 2 + np.where(hi >= 0.0, o_min2, o_max2))
        gmin = lo / np.sqrt(1.0 + lo ** 2 + np.where(lo <= 0.0, o_min2, o_max2))
        cmax = np.where(gmax >= 0.0, s1 * gmax, t * gmax)
        cmin = np.where(gmin <= 0.0, s1 * gmin, t * gmin)
        return cmin, cmax

    r_lo, r_hi = lateral(xlo, xhi, my2, My2)
    u_lo, u_hi = lateral(ylo, yhi, mx2, Mx2)
    frame = np.stack([np.asarray(cam["forward"], dtype=np.float64), np.asarray(cam["right"], dtype=np.float64),
                      np.asarray(cam["up"], dtype=np.float64)])
    lo = np.stack([f_lo, r_lo, u_lo], axis=-1)
    hi = np.stack([f_hi, r_hi, u_hi], axis=-1)
    mid = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo)
    center = np.asarray(cam["eye"], dtype=np.float64)[None, :] + mid @ frame
    axes = half[..., None] * frame[None, :, :]
    return center, axes


def cast_frusta(net, cam, tiles=(16, 16), delta=1e-3, sigma0=1.0, eta_minus=0.5, eta_plus=1.5, safety=0.98,
                max_iters=100000, policy="truncate", k=31):
    """Frustum ray casting of the camera's image (Section 4.3): a tiles[0] x
    tiles[1] grid of coarse frusta over the pixels marches forward in steps
    like CastRay, each step bounding f over the oriented box of the frustum
    between t and t + sigma (:func:`frustum_box`).  A step is accepted
    (t += safety sigma, sigma grows by eta_plus) when the box misses the domain
    [-1,1]^3 or f is bounded away from zero on it; otherwise sigma shrinks by
    eta_minus, and a frustum whose width along an image direction at
    distance t + sigma exceeds 2 sigma (or whose sigma fell below delta) is
    split in half along its wider direction (Appendix B).  A frustum of one
    pixel continues as that pixel's ray from t (CastRay over the ray's chord
    of the domain).  Frusta start at the distance of the domain's bounding
    sphere and stop, all their rays missing, past its far side.

    Returns (t_hit [height * width] along each pixel's unit ray, +inf for no
    hit; steps [height * width]: frustum steps plus ray iterations)."""
    W, H = cam["width"], cam["height"]
    eye = np.asarray(cam["eye"], dtype=np.float64)
    R = math.sqrt(3.0)
    t0 = max(0.0, float(np.linalg.norm(eye)) - R)
    t_far = float(np.linalg.norm(eye)) + R
    t_hit = np.full(W * H, np.inf)
    steps = np.zeros(W * H, dtype=np.int64)
    # tile boundaries: i W / tiles rounded half up
    xs = [(i * W + tiles[0] // 2) // tiles[0] for i in range(tiles[0] + 1)]
    ys = [(j * H + tiles[1] // 2) // tiles[1] for j in range(tiles[1] + 1)]
    fr = [[xs[i], xs[i + 1], ys[j], ys[j + 1], t0, float(sigma0)]
          for j in range(tiles[1]) for i in range(tiles[0]) if xs[i + 1] > xs[i] and ys[j + 1] > ys[j]]
    hand_pix, hand_t = [], []
    while fr:
        F = np.array(fr, dtype=np.float64)
        x0, x1, y0, y1 = (F[:, i].astype(np.int64) for i in range(4))
        t, sg = F[:, 4], F[:, 5]
        c, ax = frustum_box(cam, x0, x1, y0, y1, t, sg)
        lo_y, hi_y = mlp.bound_general(net, c, ax, policy, k)
        ext = np.abs(ax).sum(axis=1)
        miss = np.any((c - ext > 1.0) | (c + ext < -1.0), axis=1)
        safe = miss | (classify(lo_y, hi_y) != UNKNOWN)
        xa, _ = pixel_coords(cam, x0, 0)
        xb, _ = pixel_coords(cam, x1 - 1, 0)
        _, ya = pixel_coords(cam, 0, y1 - 1)
        _, yb = pixel_coords(cam, 0, y0)
        nxt = []
        for i in range(len(fr)):
            a0, a1, b0, b1, ti, si = fr[i]
            steps[(np.arange(b0, b1)[:, None] * W + np.arange(a0, a1)[None, :]).ravel()] += 1
            if safe[i]:
                ti += safety * si
                si *= eta_plus
                if ti < t_far:
                    nxt.append([a0, a1, b0, b1, ti, si])
                continue
            si *= eta_minus
            nx, ny = a1 - a0, b1 - b0
            if nx == 1 and ny == 1:
                hand_pix.append(b0 * W + a0)
                hand_t.append(ti)
                continue
            wx = (ti + si) * abs(xb[i] - xa[i])
            wy = (ti + si) * abs(yb[i] - ya[i])
            if max(wx, wy) > 2.0 * si or si < delta:
                if ny == 1 or (nx > 1 and wx >= wy):
                    m = (a0 + a1) // 2
                    nxt += [[a0, m, b0, b1, ti, si], [m, a1, b0, b1, ti, si]]
                else:
                    m = (b0 + b1) // 2
                    nxt += [[a0, a1, b0, m, ti, si], [a0, a1, m, b1, ti, si]]
            else:
                nxt.append([a0, a1, b0, b1, ti, si])
        fr = nxt
    if hand_pix:
        pix = np.array(hand_pix, dtype=np.int64)
        th = np.array(hand_t)
        d = pixel_dirs(cam, pix % W, pix // W)
        rel, it = cast_rays(net, eye[None, :] + th[:, None] * d, d, delta=delta, sigma0=sigma0 * 1.0,
                            eta_minus=eta_minus, eta_plus=eta_plus, safety=safety, max_iters=max_iters,
                            clip_to_domain=True, policy="fixed", k=k)
        t_hit[pix] = th + rel
        steps[pix] += it
    return t_hit, steps


# ---------------------------------------------------------------------------
# Empty spheres (Section 4.4)
# ---------------------------------------------------------------------------

def empty_spheres(net, p, r0=1.0, r_min=1e-4, policy="truncate", k=31):
    """For each point the first radius r in r0, r0/2, r0/4, ... (not below
    r_min) such that RangeBound classifies the cube [p - r, p + r]^3 as
    POSITIVE or NEGATIVE: the ball of radius r around p (inside that cube)
    then holds no point of the level set.  Returns (radius [n], 0 where no
    such r; label [n], UNKNOWN where radius is 0)."""
    p = np.asarray(p, dtype=np.float64)
    n = p.shape[0]
    radius = np.zeros(n)
    label = np.full(n, UNKNOWN, dtype=np.uint8)
    r = np.full(n, float(r0))
    act = np.arange(n)
    while act.size:
        lo = p[act] - r[act, None]
        hi = p[act] + r[act, None]
        _, _, ly, hy = mlp.bound_boxes(net, lo, hi, policy, k)
        lab = classify(ly, hy)
        done = lab != UNKNOWN
        radius[act[done]] = r[act[done]]
        label[act[done]] = lab[done]
        rest = act[~done]
        r[rest] = r[rest] * 0.5
        act = rest[r[rest] >= r_min]
    return radius, label


# ---------------------------------------------------------------------------
# Intersection of two implicit shapes (Section 4.9)
# ---------------------------------------------------------------------------

NO_INTERSECTION, INTERSECTION, UNDECIDED = 0, 1, 2


def intersect(net_f, net_g, max_level, policy="truncate", k=31, dom_lo=(-1, -1, -1), dom_hi=(1, 1, 1)):
    """Test whether the solids {f < 0} and {g < 0} overlap, subdividing an
    octree with respect to both functions in parallel rounds: a cell where
    either function is bounded POSITIVE cannot hold a common point and is
    dropped; a cell where both are bounded NEGATIVE lies inside both solids
    (an intersection; the round stops there, the witness is the smallest
    Morton code of such cells at that level); other cells split until
    max_level, where they remain undecided.

    Returns a dict: result (NO_INTERSECTION, INTERSECTION, UNDECIDED), level
    and cell of the witness, undecided (cells left at max_level) and the
    per-level frontier sizes."""
    codes = np.zeros(1, dtype=np.uint64)
    sizes = []
    for level in range(max_level + 1):
        sizes.append(int(codes.size))
        if codes.size == 0:
            return {"result": NO_INTERSECTION, "level": -1, "cell": 0, "undecided": 0, "sizes": sizes}
        lo, hi = cell_bounds(codes, level, dom_lo, dom_hi)
        _, _, lf, hf = mlp.bound_boxes(net_f, lo, hi, policy, k)
        _, _, lg, hg = mlp.bound_boxes(net_g, lo, hi, policy, k)
        a, b = classify(lf, hf), classify(lg, hg)
        both = (a == NEGATIVE) & (b == NEGATIVE)
        if np.any(both):
            return {"result": INTERSECTION, "level": level, "cell": int(codes[both].min()), "undecided": 0,
                    "sizes": sizes}
        keep = codes[(a != POSITIVE) & (b != POSITIVE)]
        if level == max_level:
            res = UNDECIDED if keep.size else NO_INTERSECTION
            return {"result": res, "level": -1, "cell": 0, "undecided": int(keep.size), "sizes": sizes}
        codes = np.sort(np.concatenate([(keep << np.uint64(3)) | np.uint64(o) for o in range(8)])) \
            if keep.size else np.zeros(0, dtype=np.uint64)
    raise AssertionError("unreachable")


# ---------------------------------------------------------------------------
# Mesh extraction in the leaf cells (Section 4.7; Appendix B dense levels)
# ---------------------------------------------------------------------------

# corner c of a cube = (c & 1, (c >> 1) & 1, (c >> 2) & 1); the 12 edges as
# corner pairs, and the 6 faces as cyclic corner lists
MC_EDGES = [(0, 1), (2, 3), (4, 5), (6, 7), (0, 2), (1, 3), (4, 6), (5, 7), (0, 4), (1, 5), (2, 6), (3, 7)]
MC_FACES = [(0, 2, 6, 4), (1, 3, 7, 5), (0, 1, 5, 4), (2, 3, 7, 6), (0, 1, 3, 2), (4, 5, 7, 6)]


def _mc_edge_index(a, b):
    return MC_EDGES.index((min(a, b), max(a, b)))


def mc_cube(v, p):
    """Marching cubes in one cube from its 8 corner values v (sign test
    v > 0, zero counts as inside) and corner positions p [8, 3].  Written
    without a case table: each face joins its crossing edges by segments (two
    crossings: one segment; four: the two corners whose sign differs from the
    face's mean are each cut off by the segment between their two edges), the
    segments close into loops over the crossing edges, and each loop, walked
    from its lowest edge toward that edge's lower-numbered neighbour, is
    triangulated as a fan.  Edge points interpolate f linearly.  Returns a
    list of triangles, each [3, 3]."""
    s = [bool(x > 0.0) for x in v]
    cross = [s[a] != s[b] for a, b in MC_EDGES]
    if not any(cross):
        return []
    pt = {}
    for e, (a, b) in enumerate(MC_EDGES):
        if cross[e]:
            t = v[a] / (v[a] - v[b])
            pt[e] = p[a] + t * (p[b] - p[a])
    nb = {e: [] for e in pt}
    for q in MC_FACES:
        edges = [_mc_edge_index(q[i], q[(i + 1) % 4]) for i in range(4)]
        ce = [e for e in edges if cross[e]]
        if len(ce) == 2:
            segs = [(ce[0], ce[1])]
        elif len(ce) == 4:
            center = (v[q[0]] + v[q[1]] + v[q[2]] + v[q[3]]) / 4.0 > 0.0
            segs = [(edges[(i - 1) % 4], edges[i]) for i in range(4) if s[q[i]] != center]
        else:
            segs = []
        for a, b in segs:
            nb[a].append(b)
            nb[b].append(a)
    tris = []
    used = set()
    for e0 in sorted(pt):
        if e0 in used:
            continue
        loop = [e0]
        used.add(e0)
        prev, cur = e0, min(nb[e0])
        while cur != e0:
            loop.append(cur)
            used.add(cur)
            a, b = nb[cur]
            prev, cur = cur, (b if a == prev else a)
        for i in range(1, len(loop) - 1):
            tris.append(np.stack([pt[loop[0]], pt[loop[i]], pt[loop[i + 1]]]))
    return tris


def mesh_leaves(net, leaves, level, dense_levels=3, dom_lo=(-1, -1, -1), dom_hi=(1, 1, 1)):
    """Triangles of the level set inside the given leaf cells (Morton codes at
    `level`): each leaf is sampled on the grid of dense_levels further
    subdivisions (Appendix B: dense evaluation of the lowest levels) and
    every grid cube is meshed by :func:`mc_cube`.  Grid points are
    dom_lo + g h with g the global index on the finest grid, so neighbouring
    leaves share their face samples.  Returns ([m, 3, 3] triangles, [m] index
    of the leaf, [m] index of the cube in the leaf, x-fastest)."""
    dom_lo = np.asarray(dom_lo, dtype=np.float64)
    dom_hi = np.asarray(dom_hi, dtype=np.float64)
    R = 1 << dense_levels
    h = (dom_hi - dom_lo) / float(1 << (level + dense_levels))
    ix, iy, iz = morton_decode(np.asarray(leaves, dtype=np.uint64), level)
    g = np.arange(R + 1)
    out, owner, cube = [], [], []
    for j in range(len(leaves)):
        base = np.array([ix[j], iy[j], iz[j]], dtype=np.int64) * R
        G = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)   # (i, j, k) x slowest
        P = dom_lo + (base + G) * h
        F = mlp.forward(net, P).reshape(R + 1, R + 1, R + 1)
        P = P.reshape(R + 1, R + 1, R + 1, 3)
        for kz in range(R):
            for ky in range(R):
                for kx in range(R):
                    cs = [(kx + (c & 1), ky + ((c >> 1) & 1), kz + ((c >> 2) & 1)) for c in range(8)]
                    v = [F[a, b, cc] for a, b, cc in cs]
                    if all(x > 0 for x in v) or all(x <= 0 for x in v):
                        continue
                    p = np.stack([P[a, b, cc] for a, b, cc in cs])
                    for t in mc_cube(v, p):
                        out.append(t)
                        owner.append(j)
                        cube.append(kx + R * (ky + R * kz))
    if not out:
        return np.zeros((0, 3, 3)), np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.stack(out), np.array(owner), np.array(cube)


# ---------------------------------------------------------------------------
# Sampling in leaf cells: surface sampling (Section 4.6) and bulk properties
# (Section 4.8)
# ---------------------------------------------------------------------------

_M64 = (1 << 64) - 1


def splitmix64(seed, k):
    """The k-th output (k = 0, 1, ...) of the splitmix64 generator (Steele,
    Lea and Flood, 2014) seeded with `seed`, for an array k (Python integers,
    exact 64-bit wrap-around)."""
    out = []
    for kk in np.asarray(k, dtype=np.uint64).ravel().tolist():
        z = (int(seed) + (int(kk) + 1) * 0x9e3779b97f4a7c15) & _M64
        z = ((z ^ (z >> 30)) * 0xbf58476d1ce4e5b9) & _M64
        z = ((z ^ (z >> 27)) * 0x94d049bb133111eb) & _M64
        out.append(z ^ (z >> 31))
    return np.array(out, dtype=np.uint64).reshape(np.shape(k))


def sample_leaves(net, leaves, level, n_samples, seed, band=math.inf, dom_lo=(-1, -1, -1), dom_hi=(1, 1, 1)):
    """Uniform samples in the union of equal-size leaf cells: sample i takes
    outputs 4i .. 4i+3 of splitmix64(seed): the leaf (first output modulo the
    leaf count) and 24-bit offsets in [0, 1) per axis.  Returns (points
    [n, 3], f [n], accepted mask |f| < band)."""
    leaves = np.asarray(leaves, dtype=np.uint64)
    i = np.arange(n_samples, dtype=np.uint64)
    leaf = (splitmix64(seed, 4 * i) % np.uint64(leaves.size)).astype(np.int64)
    lo, hi = cell_bounds(leaves[leaf], level, dom_lo, dom_hi)
    u = np.stack([(splitmix64(seed, 4 * i + np.uint64(1 + d)) >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
                  for d in range(3)], axis=1)
    pts = lo + u * (hi - lo)
    f = mlp.forward(net, pts)
    return pts, f, np.abs(f) < band


def bulk_volume(net, max_level, n_samples, seed, policy="truncate", k=31, dom_lo=(-1, -1, -1), dom_hi=(1, 1, 1)):
    """Volume of the solid {f < 0} (Section 4.8): the NEGATIVE cells of the
    fixed-depth tree count in full, the UNKNOWN leaves by the fraction of
    uniform samples in them with f < 0.  Returns (estimate, lower bound,
    upper bound): the solid holds every NEGATIVE cell and lies within the
    NEGATIVE cells and the leaves."""
    res = octree_build(net, max_level, policy, k, dom_lo, dom_hi)
    dom = float(np.prod(np.asarray(dom_hi, dtype=np.float64) - np.asarray(dom_lo, dtype=np.float64)))
    v_neg = sum(lv["n_neg"] * dom / 8.0 ** lv["level"] for lv in res["levels"])
    v_leaf = res["leaves"].size * dom / 8.0 ** max_level
    if res["leaves"].size == 0:
        return v_neg, v_neg, v_neg
    _, f, _ = sample_leaves(net, res["leaves"], max_level, n_samples, seed, math.inf, dom_lo, dom_hi)
    return v_neg + v_leaf * float(np.mean(f < 0.0)), v_neg, v_neg + v_leaf
