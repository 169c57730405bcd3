"""The C ABI library loads, exports every symbol include/spk.h declares, and
rejects invalid arguments before touching the GPU (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2202_02444_amd import spk
import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "spk.h")).read()
    return sorted(set(re.findall(r"\b(spk_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    L = spk.lib()
    names = _declared()
    assert "spk_classify_boxes" in names and "spk_cast_rays" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(spk.EXPORTS) <= set(names)


def test_status_strings_and_version():
    L = spk.lib()
    for s in range(8):
        assert L.spk_status_str(s)
    assert b"gfx950" in L.spk_version()


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced on the validation paths below


def test_net_create_rejects_bad_shapes():
    L = spk.lib()
    out = ctypes.c_void_p()
    W = [np.zeros((48, 3), np.float32), np.zeros((1, 48), np.float32)]
    b = [np.zeros(48, np.float32), np.zeros(1, np.float32)]
    wa = (ctypes.c_int32 * 3)(3, 48, 1)
    Wp = (ctypes.c_void_p * 2)(*[w.ctypes.data for w in W])
    bp = (ctypes.c_void_p * 2)(*[x.ctypes.data for x in b])
    assert L.spk_net_create(2, wa, Wp, bp, 0, 1.0, ctypes.byref(out)) == spk.E_UNSUPPORTED   # width 48
    wa2 = (ctypes.c_int32 * 3)(2, 32, 1)
    assert L.spk_net_create(2, wa2, Wp, bp, 0, 1.0, ctypes.byref(out)) == spk.E_UNSUPPORTED  # input dim 2
    wa3 = (ctypes.c_int32 * 3)(3, 32, 1)
    assert L.spk_net_create(2, wa3, Wp, bp, 7, 1.0, ctypes.byref(out)) == spk.E_INVAL        # activation
    assert L.spk_net_create(2, wa3, Wp, bp, 2, -1.0, ctypes.byref(out)) == spk.E_INVAL       # omega0
    assert L.spk_net_create(2, wa3, Wp, bp, 0, 1.0, None) == spk.E_INVAL
    assert L.spk_net_create(1, wa3, Wp, bp, 0, 1.0, ctypes.byref(out)) == spk.E_UNSUPPORTED
    Wn = [np.full((32, 3), np.nan, np.float32), np.zeros((1, 32), np.float32)]
    Wnp = (ctypes.c_void_p * 2)(*[w.ctypes.data for w in Wn])
    bn = [np.zeros(32, np.float32), np.zeros(1, np.float32)]
    bnp = (ctypes.c_void_p * 2)(*[x.ctypes.data for x in bn])
    assert L.spk_net_create(2, wa3, Wnp, bnp, 0, 1.0, ctypes.byref(out)) == spk.E_INVAL      # non-finite


def test_bound_calls_validate_before_launch():
    L = spk.lib()
    o = spk.opts("truncate", 31)
    assert L.spk_classify_boxes(None, FAKE, ctypes.byref(o), 4, FAKE, FAKE, FAKE, None, None, None) == spk.E_INVAL
    assert L.spk_classify_boxes(FAKE, FAKE, None, 4, FAKE, FAKE, FAKE, None, None, None) == spk.E_INVAL
    bad = spk.opts("truncate", 40)
    assert L.spk_classify_boxes(FAKE, FAKE, ctypes.byref(bad), 4, FAKE, FAKE, FAKE, None, None,
                                None) == spk.E_UNSUPPORTED
    full = spk.opts("full", 0, prec="f16x3")   # affine-full: FP32 products only
    assert L.spk_classify_boxes(FAKE, FAKE, ctypes.byref(full), 4, FAKE, FAKE, FAKE, None, None,
                                None) == spk.E_UNSUPPORTED
    badprec = spk.BoundOpts(1, 31, 4, 0)   # no spk_prec 4
    assert L.spk_classify_boxes(FAKE, FAKE, ctypes.byref(badprec), 4, FAKE, FAKE, FAKE, None, None,
                                None) == spk.E_UNSUPPORTED
    badflag = spk.BoundOpts(1, 31, 2, 2)   # unknown flag bit
    assert L.spk_classify_boxes(FAKE, FAKE, ctypes.byref(badflag), 4, FAKE, FAKE, FAKE, None, None,
                                None) in (spk.E_INVAL, spk.E_UNSUPPORTED)
    assert L.spk_classify_boxes(FAKE, FAKE, ctypes.byref(o), -1, FAKE, FAKE, FAKE, None, None, None) == spk.E_INVAL
    assert L.spk_classify_boxes(FAKE, FAKE, ctypes.byref(o), 0, None, None, None, None, None, None) == spk.OK
    assert L.spk_classify_boxes(FAKE, FAKE, ctypes.byref(o), 4, None, FAKE, FAKE, None, None, None) == spk.E_INVAL
    assert L.spk_range_bound(FAKE, FAKE, ctypes.byref(o), 4, 4, FAKE, FAKE, FAKE, FAKE, None) == spk.E_INVAL
    assert L.spk_range_bound(FAKE, FAKE, ctypes.byref(o), 0, 3, None, None, None, None, None) == spk.OK
    badflags = spk.BoundOpts(1, 31, 0, 8)
    assert L.spk_classify_boxes(FAKE, FAKE, ctypes.byref(badflags), 4, FAKE, FAKE, FAKE, None, None,
                                None) == spk.E_INVAL
    fx = spk.opts("fixed", 0)
    aux = spk.BoundAux(None, None, None, FAKE)
    assert L.spk_range_bound(FAKE, FAKE, ctypes.byref(fx), 4, 3, FAKE, FAKE, FAKE, FAKE,
                             ctypes.byref(aux)) == spk.E_INVAL
    assert L.spk_ctx_sync(None, None) == spk.E_INVAL
    assert L.spk_net_destroy(None) == spk.E_INVAL


def test_tree_and_ray_validation():
    L = spk.lib()
    o = spk.opts("truncate", 31)
    tp = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 6, 8)
    cnt = FAKE
    assert L.spk_subdivide_frontier(FAKE, FAKE, ctypes.byref(o), ctypes.byref(tp), 7, FAKE, 1, FAKE, 8, None, 0,
                                    cnt) == spk.E_INVAL      # level beyond max_level
    tp2 = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 6, 2)
    assert L.spk_subdivide_frontier(FAKE, FAKE, ctypes.byref(o), ctypes.byref(tp2), 0, FAKE, 1, FAKE, 8, None, 0,
                                    cnt) == spk.E_UNSUPPORTED
    tp3 = spk.TreeParams((ctypes.c_float * 3)(1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 6, 8)
    assert L.spk_subdivide_frontier(FAKE, FAKE, ctypes.byref(o), ctypes.byref(tp3), 0, FAKE, 1, FAKE, 8, None, 0,
                                    cnt) == spk.E_INVAL      # empty domain
    assert L.spk_subdivide_frontier(FAKE, FAKE, ctypes.byref(o), ctypes.byref(tp), 0, FAKE, 1, None, 8, None, 0,
                                    cnt) == spk.E_INVAL      # capacity without buffer
    # the non-allocating variant validates the same way and rejects frontiers
    # beyond its fixed scratch before any HIP call
    assert L.spk_subdivide_frontier_noalloc(FAKE, FAKE, ctypes.byref(o), ctypes.byref(tp), 7, FAKE, 1, FAKE, 8,
                                            None, 0, cnt) == spk.E_INVAL
    hdr = open(os.path.join(ROOT, "include", "spk.h")).read()
    assert int(re.search(r"#define SPK_NOALLOC_MAX_CELLS (\d+)", hdr).group(1)) == spk.NOALLOC_MAX_CELLS
    big = spk.NOALLOC_MAX_CELLS + 1
    assert L.spk_subdivide_frontier_noalloc(FAKE, FAKE, ctypes.byref(o), ctypes.byref(tp), 0, FAKE, big, FAKE,
                                            8 * big, None, 0, cnt) == spk.E_LIMIT
    assert b"fixed capacity" in L.spk_status_str(spk.E_LIMIT)
    rp = spk.ray_params()
    assert L.spk_cast_rays(FAKE, FAKE, ctypes.byref(rp), -1, FAKE, FAKE, FAKE, None) == spk.E_INVAL
    assert L.spk_cast_rays(FAKE, FAKE, ctypes.byref(rp), 0, None, None, None, None) == spk.OK
    rp_bad = spk.ray_params(delta=-1.0)
    assert L.spk_cast_rays(FAKE, FAKE, ctypes.byref(rp_bad), 4, FAKE, FAKE, FAKE, None) == spk.E_INVAL
    rp_bad2 = spk.ray_params(eta_minus=1.5)
    assert L.spk_cast_rays(FAKE, FAKE, ctypes.byref(rp_bad2), 4, FAKE, FAKE, FAKE, None) == spk.E_INVAL
    rp_bad3 = spk.ray_params()
    rp_bad3.flags = 8                          # unknown flag bit
    assert L.spk_cast_rays(FAKE, FAKE, ctypes.byref(rp_bad3), 4, FAKE, FAKE, FAKE, None) == spk.E_INVAL
    assert spk.ray_params(rigorous=False).flags == spk.FLAG_NO_ROUNDING_BOUND and spk.ray_params().flags == 0


def test_sampling_and_band_validation():
    L = spk.lib()
    tp = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 4, 8)
    na, nb = ctypes.c_int64(), ctypes.c_int64()
    f = ctypes.c_float
    call = lambda lvl, nl, lv, ns, band, pts, cap, out: L.spk_sample_leaves(FAKE, FAKE, ctypes.byref(tp), lvl, nl, lv,
                                                                            ns, 7, f(band), pts, None, cap, out,
                                                                            ctypes.byref(nb))
    assert call(3, 4, FAKE, 10, 0.1, FAKE, 10, None) == spk.E_INVAL              # no count output
    assert call(3, 4, FAKE, 10, 0.0, FAKE, 10, ctypes.byref(na)) == spk.E_INVAL  # empty band
    assert call(3, 0, None, 10, 0.1, FAKE, 10, ctypes.byref(na)) == spk.E_INVAL  # samples without leaves
    assert call(3, 4, FAKE, 10, 0.1, None, 10, ctypes.byref(na)) == spk.E_INVAL  # capacity without a buffer
    assert call(21, 4, FAKE, 10, 0.1, FAKE, 10, ctypes.byref(na)) == spk.E_INVAL
    assert call(3, 4, FAKE, 0, 0.1, None, 0, ctypes.byref(na)) == spk.OK and na.value == 0
    o = spk.opts("truncate", 31)
    cnt = FAKE
    band_delta = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 6, 8, 0.01, 0.05)
    assert L.spk_subdivide_frontier(FAKE, FAKE, ctypes.byref(o), ctypes.byref(band_delta), 0, FAKE, 1, FAKE, 8, None,
                                    0, cnt) == spk.E_INVAL
    neg = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 6, 8, 0.0, -0.5)
    assert L.spk_subdivide_frontier(FAKE, FAKE, ctypes.byref(o), ctypes.byref(neg), 0, FAKE, 1, FAKE, 8, None, 0,
                                    cnt) == spk.E_INVAL
    band = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 6, 8, 0.0, 0.05)
    r = spk.IntersectResult()
    assert L.spk_intersect(FAKE, FAKE, FAKE, ctypes.byref(o), ctypes.byref(band), ctypes.byref(r)) == spk.E_INVAL


def test_mesh_validation():
    L = spk.lib()
    tp = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 4, 8)
    m = ctypes.c_int64()
    call = lambda t, lvl, dense, n, lv, tris, cap, out: L.spk_mesh_leaves(FAKE, FAKE, ctypes.byref(t), lvl, dense, n,
                                                                         lv, tris, None, cap, out)
    assert call(tp, 3, 3, 4, FAKE, FAKE, 8, None) == spk.E_INVAL                   # no count output
    assert call(tp, 3, 5, 4, FAKE, FAKE, 8, ctypes.byref(m)) == spk.E_INVAL        # too many dense levels
    assert call(tp, 18, 3, 4, FAKE, FAKE, 8, ctypes.byref(m)) == spk.E_INVAL       # finer than level 20
    assert call(tp, 3, 3, 4, None, FAKE, 8, ctypes.byref(m)) == spk.E_INVAL        # no leaves
    assert call(tp, 3, 3, 4, FAKE, None, 8, ctypes.byref(m)) == spk.E_INVAL        # capacity without a buffer
    assert call(tp, 3, 3, 0, None, None, 0, ctypes.byref(m)) == spk.OK and m.value == 0
    kd = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 4, 2)
    assert call(kd, 3, 3, 4, FAKE, FAKE, 8, ctypes.byref(m)) == spk.E_UNSUPPORTED


def test_delta_tree_validation():
    L = spk.lib()
    o = spk.opts("truncate", 31)
    cnt = FAKE
    tp = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 6, 8, 0.01, 0)
    # the non-allocating round has no face buffers for the convergence test
    assert L.spk_subdivide_frontier_noalloc(FAKE, FAKE, ctypes.byref(o), ctypes.byref(tp), 0, FAKE, 1, FAKE, 8,
                                            None, 0, cnt) == spk.E_UNSUPPORTED
    bad = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 6, 8, -1.0, 0)
    assert L.spk_subdivide_frontier(FAKE, FAKE, ctypes.byref(o), ctypes.byref(bad), 0, FAKE, 1, FAKE, 8, None, 0,
                                    cnt) == spk.E_INVAL
    # the other tree calls take no delta
    r = spk.IntersectResult()
    assert L.spk_intersect(FAKE, FAKE, FAKE, ctypes.byref(o), ctypes.byref(tp), ctypes.byref(r)) == spk.E_INVAL
    fx = spk.opts("fixed", 0)
    assert L.spk_closest_point(FAKE, FAKE, ctypes.byref(fx), ctypes.byref(tp), 4, FAKE, FAKE, None,
                               None) == spk.E_INVAL


def test_intersect_validation():
    L = spk.lib()
    o = spk.opts("truncate", 31)
    r = spk.IntersectResult()
    tp = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 4, 8)
    assert L.spk_intersect(FAKE, FAKE, None, ctypes.byref(o), ctypes.byref(tp), ctypes.byref(r)) == spk.E_INVAL
    assert L.spk_intersect(FAKE, FAKE, FAKE, ctypes.byref(o), ctypes.byref(tp), None) == spk.E_INVAL
    kd = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 4, 2)
    assert L.spk_intersect(FAKE, FAKE, FAKE, ctypes.byref(o), ctypes.byref(kd), ctypes.byref(r)) == spk.E_UNSUPPORTED
    deep = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 21, 8)
    assert L.spk_intersect(FAKE, FAKE, FAKE, ctypes.byref(o), ctypes.byref(deep), ctypes.byref(r)) == spk.E_INVAL
    empty = spk.TreeParams((ctypes.c_float * 3)(1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 4, 8)
    assert L.spk_intersect(FAKE, FAKE, FAKE, ctypes.byref(o), ctypes.byref(empty), ctypes.byref(r)) == spk.E_INVAL


def test_empty_spheres_validation():
    L = spk.lib()
    o = spk.opts("truncate", 31)
    f = ctypes.c_float
    assert L.spk_empty_spheres(None, FAKE, ctypes.byref(o), 4, FAKE, f(1.0), f(1e-3), FAKE, FAKE) == spk.E_INVAL
    assert L.spk_empty_spheres(FAKE, FAKE, ctypes.byref(o), 4, FAKE, f(1e-3), f(1.0), FAKE, FAKE) == spk.E_INVAL
    assert L.spk_empty_spheres(FAKE, FAKE, ctypes.byref(o), 4, FAKE, f(0.0), f(0.0), FAKE, FAKE) == spk.E_INVAL
    assert L.spk_empty_spheres(FAKE, FAKE, ctypes.byref(o), 4, FAKE, f(1.0), f(1e-3), None, FAKE) == spk.E_INVAL
    assert L.spk_empty_spheres(FAKE, FAKE, ctypes.byref(o), -1, FAKE, f(1.0), f(1e-3), FAKE, FAKE) == spk.E_INVAL
    assert L.spk_empty_spheres(FAKE, FAKE, ctypes.byref(o), 0, None, f(1.0), f(1e-3), None, None) == spk.OK
    bad = spk.opts("truncate", 40)
    assert L.spk_empty_spheres(FAKE, FAKE, ctypes.byref(bad), 4, FAKE, f(1.0), f(1e-3), FAKE,
                               FAKE) == spk.E_UNSUPPORTED


def test_frustum_validation():
    L = spk.lib()
    cam = spk.camera(wl.camera(8, 6, 1))
    rp = spk.ray_params()
    o = spk.opts("fixed", 0)
    st = spk.FrustumStats()
    call = lambda r, oo, c, tx, ty, th: L.spk_cast_frusta(FAKE, FAKE, ctypes.byref(r), ctypes.byref(oo),
                                                           ctypes.byref(c), tx, ty, th, None, ctypes.byref(st))
    assert L.spk_cast_frusta(None, FAKE, ctypes.byref(rp), ctypes.byref(o), ctypes.byref(cam), 2, 2, FAKE, None,
                             None) == spk.E_INVAL
    assert call(rp, o, cam, 2, 2, None) == spk.E_INVAL                    # no output
    assert call(rp, o, cam, 0, 2, FAKE) == spk.E_INVAL                    # no tiles
    assert call(rp, o, cam, 9, 2, FAKE) == spk.E_INVAL                    # more tiles than pixels
    paper = spk.opts("fixed", 0, rigorous=False)
    assert call(rp, paper, cam, 2, 2, FAKE) == spk.E_INVAL                # arithmetic differs from the rays'
    bad = spk.camera(wl.camera(8, 6, 1))
    bad.right[0] += 1e-3                                                  # not orthonormal
    assert call(rp, o, bad, 2, 2, FAKE) == spk.E_INVAL
    bad = spk.camera(wl.camera(8, 6, 1))
    bad.tan_x = 0.0
    assert call(rp, o, bad, 2, 2, FAKE) == spk.E_INVAL
    bad = spk.camera(wl.camera(8, 6, 1))
    bad.width = 0
    assert call(rp, o, bad, 1, 1, FAKE) == spk.E_INVAL
    full = spk.opts("full", 0, prec="bf16x3")
    assert call(rp, full, cam, 2, 2, FAKE) == spk.E_UNSUPPORTED


def test_closest_point_validation():
    L = spk.lib()
    o = spk.opts("fixed", 0)
    tp = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 6, 8)
    assert L.spk_closest_point(FAKE, FAKE, ctypes.byref(o), ctypes.byref(tp), 0, None, None, None, None) == spk.OK
    assert L.spk_closest_point(FAKE, FAKE, ctypes.byref(o), ctypes.byref(tp), -1, FAKE, FAKE, None, None) == spk.E_INVAL
    assert L.spk_closest_point(FAKE, FAKE, ctypes.byref(o), ctypes.byref(tp), 4, None, FAKE, None, None) == spk.E_INVAL
    assert L.spk_closest_point(FAKE, FAKE, ctypes.byref(o), None, 4, FAKE, FAKE, None, None) == spk.E_INVAL
    tp_deep = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 21, 8)
    assert L.spk_closest_point(FAKE, FAKE, ctypes.byref(o), ctypes.byref(tp_deep), 4, FAKE, FAKE, None,
                               None) == spk.E_INVAL
    tp_kd = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 6, 2)
    assert L.spk_closest_point(FAKE, FAKE, ctypes.byref(o), ctypes.byref(tp_kd), 4, FAKE, FAKE, None,
                               None) == spk.E_UNSUPPORTED
    bad = spk.opts("truncate", 2)
    assert L.spk_closest_point(FAKE, FAKE, ctypes.byref(bad), ctypes.byref(tp), 4, FAKE, FAKE, None,
                               None) == spk.E_UNSUPPORTED   # k below 3


def test_batch_validation():
    L = spk.lib()
    o = spk.opts("truncate", 31)
    h = ctypes.c_void_p()
    items = (spk.BatchItem * 1)()
    items[0] = spk.BatchItem(None, 4, 0x1000, 0x1000, 0x1000, None, None)
    assert L.spk_batch_create(FAKE, ctypes.byref(o), 1, items, ctypes.byref(h)) == spk.E_INVAL   # null net
    assert L.spk_batch_create(FAKE, ctypes.byref(o), 0, items, ctypes.byref(h)) == spk.E_INVAL   # no items
    assert L.spk_batch_create(None, ctypes.byref(o), 1, items, ctypes.byref(h)) == spk.E_INVAL
    bad = spk.opts("truncate", 40)
    assert L.spk_batch_create(FAKE, ctypes.byref(bad), 1, items, ctypes.byref(h)) == spk.E_UNSUPPORTED
    full = spk.opts("full", 0)                                        # affine-full is not batched
    assert L.spk_batch_create(FAKE, ctypes.byref(full), 1, items, ctypes.byref(h)) == spk.E_UNSUPPORTED
    assert L.spk_batch_launch(FAKE, None) == spk.E_INVAL
    assert L.spk_batch_tune(FAKE, None, 3) == spk.E_INVAL
    assert L.spk_batch_destroy(None) == spk.E_INVAL
    n = ctypes.c_int32()
    assert L.spk_batch_classes(None, ctypes.byref(n), None, 0) == spk.E_INVAL
    # frontier items are checked before any device access
    f = spk.BatchItem()
    f.net, f.n, f.cells, f.label, f.counts, f.level = 0x1000, 4, 0x1000, 0x1000, 0x1000, 1
    f.tree = spk.TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1), 3, 2)
    items[0] = f
    assert L.spk_batch_create(FAKE, ctypes.byref(o), 1, items, ctypes.byref(h)) == spk.E_UNSUPPORTED   # k-d
    f.tree.arity = 8
    f.level = 4                                                       # beyond max_level
    items[0] = f
    assert L.spk_batch_create(FAKE, ctypes.byref(o), 1, items, ctypes.byref(h)) == spk.E_INVAL
    f.level = 1
    f.counts = None
    items[0] = f
    assert L.spk_batch_create(FAKE, ctypes.byref(o), 1, items, ctypes.byref(h)) == spk.E_INVAL   # no counts
    f.counts = 0x1000
    f.cap_children = 8                                                # capacity without a buffer
    items[0] = f
    assert L.spk_batch_create(FAKE, ctypes.byref(o), 1, items, ctypes.byref(h)) == spk.E_INVAL
    f.cap_children = 0
    f.tree.dom_hi[0] = -2.0                                           # empty domain
    items[0] = f
    assert L.spk_batch_create(FAKE, ctypes.byref(o), 1, items, ctypes.byref(h)) == spk.E_INVAL


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of every ABI struct have the C compiler's size and
    field offsets (a plain C program built against include/spk.h)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"spk_bound_opts": spk.BoundOpts, "spk_bound_aux": spk.BoundAux, "spk_tree_params": spk.TreeParams,
               "spk_ray_params": spk.RayParams, "spk_batch_item": spk.BatchItem, "spk_batch_class": spk.BatchClass,
               "spk_request": spk.Request, "spk_completion": spk.Completion,
               "spk_device_status": spk.DeviceStatus, "spk_camera": spk.Camera,
               "spk_intersect_result": spk.IntersectResult,
               "spk_frustum_stats": spk.FrustumStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "spk.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('  printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('  printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got["%s.%s" % (cname, f)]) == getattr(py, f).offset, (cname, f)


def test_server_validation():
    L = spk.lib()
    h = ctypes.c_void_p()
    assert L.spk_server_create(None, 1, 0, 4, ctypes.byref(h)) == spk.E_INVAL
    nets = (ctypes.c_void_p * 1)(0x1000)
    assert L.spk_server_create(nets, 1, 0, 0, ctypes.byref(h)) == spk.E_INVAL       # no workers
    assert L.spk_server_submit(None, None, None) == spk.E_INVAL
    n = ctypes.c_int32()
    assert L.spk_server_poll(None, None, 0, ctypes.byref(n), 0) == spk.E_INVAL
    assert L.spk_server_destroy(None) == spk.E_INVAL
