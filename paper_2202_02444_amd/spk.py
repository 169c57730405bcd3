"""Thin ctypes binding of the C ABI declared in ``include/spk.h``.

Argument marshalling only: every step of the computation runs in the HIP
library.  Device buffers are torch tensors on the GPU (torch supplies memory
and the stream); the library never sees torch types.  If ``libspk.so`` is
missing the first call raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspk.so")

OK, E_INVAL, E_NOMEM, E_NOSPC, E_DEVICE, E_UNSUPPORTED, E_BUSY, E_LIMIT = range(8)
NOALLOC_MAX_CELLS = 16777216
ACT = {"relu": 0, "elu": 1, "sin": 2}
POLICY = {"fixed": 0, "truncate": 1, "full": 2}
UNKNOWN, POSITIVE, NEGATIVE = 0, 1, 2

EXPORTS = ("spk_status_str", "spk_version", "spk_net_create", "spk_net_destroy", "spk_ctx_create",
           "spk_ctx_destroy", "spk_ctx_sync", "spk_range_bound", "spk_classify_boxes",
           "spk_subdivide_frontier", "spk_subdivide_frontier_noalloc", "spk_cast_rays", "spk_cast_frusta",
           "spk_empty_spheres", "spk_intersect", "spk_mesh_leaves", "spk_sample_leaves",
           "spk_eval_points", "spk_closest_point",
           "spk_batch_create", "spk_batch_update", "spk_batch_launch", "spk_batch_tune", "spk_batch_classes",
           "spk_batch_destroy", "spk_server_create", "spk_server_submit", "spk_server_poll",
           "spk_server_pending", "spk_server_destroy")


class BatchItem(ctypes.Structure):
    pass


class BatchClass(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("act", ctypes.c_int32), ("term_slots", ctypes.c_int32),
                ("n_nets", ctypes.c_int32), ("groups", ctypes.c_int64), ("blocks", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("tuned_ms", ctypes.c_float)]


class Request(ctypes.Structure):
    pass


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32), ("type", ctypes.c_int32),
                ("n", ctypes.c_int64), ("submit_s", ctypes.c_double), ("start_s", ctypes.c_double),
                ("done_s", ctypes.c_double), ("workspace_bytes", ctypes.c_uint64)]


class BoundOpts(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("k", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class BoundAux(ctypes.Structure):
    _fields_ = [("center", ctypes.c_void_p), ("radius", ctypes.c_void_p), ("err", ctypes.c_void_p),
                ("slot_src", ctypes.c_void_p)]


class DeviceStatus(ctypes.Structure):
    _fields_ = [("nonfinite_inputs", ctypes.c_int64), ("nospc", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("need_children", ctypes.c_int64), ("need_leaves", ctypes.c_int64)]


class Camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_float * 3), ("forward", ctypes.c_float * 3), ("right", ctypes.c_float * 3),
                ("up", ctypes.c_float * 3), ("tan_x", ctypes.c_float), ("tan_y", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class FrustumStats(ctypes.Structure):
    _fields_ = [("frustum_steps", ctypes.c_int64), ("rays_handed_off", ctypes.c_int64),
                ("ray_iterations", ctypes.c_int64), ("rounds", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class IntersectResult(ctypes.Structure):
    _fields_ = [("result", ctypes.c_int32), ("level", ctypes.c_int32), ("cell", ctypes.c_uint64),
                ("undecided", ctypes.c_int64), ("cells_bounded", ctypes.c_int64), ("rounds", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


NO_INTERSECTION, INTERSECTION, INTERSECTION_UNDECIDED = 0, 1, 2


class TreeParams(ctypes.Structure):
    _fields_ = [("dom_lo", ctypes.c_float * 3), ("dom_hi", ctypes.c_float * 3), ("max_level", ctypes.c_int32),
                ("arity", ctypes.c_int32), ("delta", ctypes.c_float), ("band", ctypes.c_float)]


class RayParams(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_float), ("t_max", ctypes.c_float), ("sigma0", ctypes.c_float),
                ("eta_minus", ctypes.c_float), ("eta_plus", ctypes.c_float), ("safety", ctypes.c_float),
                ("max_iters", ctypes.c_int32), ("clip_to_domain", ctypes.c_int32), ("flags", ctypes.c_uint32)]


BatchItem._fields_ = [("net", ctypes.c_void_p), ("n", ctypes.c_int64), ("box_lo", ctypes.c_void_p),
                      ("box_hi", ctypes.c_void_p), ("label", ctypes.c_void_p), ("lo", ctypes.c_void_p),
                      ("hi", ctypes.c_void_p), ("cells", ctypes.c_void_p), ("level", ctypes.c_int32),
                      ("reserved", ctypes.c_int32), ("tree", TreeParams), ("children", ctypes.c_void_p),
                      ("cap_children", ctypes.c_int64), ("leaves", ctypes.c_void_p), ("cap_leaves", ctypes.c_int64),
                      ("counts", ctypes.c_void_p)]

Request._fields_ = [("type", ctypes.c_int32), ("net", ctypes.c_int32), ("n", ctypes.c_int64),
                    ("a", ctypes.c_void_p), ("b", ctypes.c_void_p), ("out0", ctypes.c_void_p),
                    ("out1", ctypes.c_void_p), ("out2", ctypes.c_void_p), ("bytes", ctypes.c_size_t),
                    ("opts", BoundOpts), ("ray", RayParams), ("tree", TreeParams)]

REQ_CLASSIFY, REQ_RAYS, REQ_CLOSEST = 0, 1, 2

_lib = None


def lib():
    """Load libspk.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libspk.so is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.spk_status_str.restype = ctypes.c_char_p
        L.spk_status_str.argtypes = [ctypes.c_int]
        L.spk_version.restype = ctypes.c_char_p
        L.spk_version.argtypes = []
        L.spk_net_create.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(vp), ctypes.POINTER(vp), i32,
                                     ctypes.c_float, ctypes.POINTER(vp)]
        L.spk_net_destroy.argtypes = [vp]
        L.spk_ctx_create.argtypes = [vp, sz, ctypes.POINTER(vp)]
        L.spk_ctx_destroy.argtypes = [vp]
        L.spk_ctx_sync.argtypes = [vp, ctypes.POINTER(DeviceStatus)]
        L.spk_range_bound.argtypes = [vp, vp, ctypes.POINTER(BoundOpts), i64, i32, vp, vp, vp, vp,
                                      ctypes.POINTER(BoundAux)]
        L.spk_classify_boxes.argtypes = [vp, vp, ctypes.POINTER(BoundOpts), i64, vp, vp, vp, vp, vp,
                                         ctypes.POINTER(BoundAux)]
        L.spk_subdivide_frontier.argtypes = [vp, vp, ctypes.POINTER(BoundOpts), ctypes.POINTER(TreeParams), i32, vp,
                                             i64, vp, i64, vp, i64, vp]
        L.spk_subdivide_frontier_noalloc.argtypes = [vp, vp, ctypes.POINTER(BoundOpts), ctypes.POINTER(TreeParams), i32, vp,
                                             i64, vp, i64, vp, i64, vp]
        L.spk_cast_rays.argtypes = [vp, vp, ctypes.POINTER(RayParams), i64, vp, vp, vp, vp]
        L.spk_sample_leaves.argtypes = [vp, vp, ctypes.POINTER(TreeParams), i32, i64, vp, i64, ctypes.c_uint64,
                                        ctypes.c_float, vp, vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.spk_mesh_leaves.argtypes = [vp, vp, ctypes.POINTER(TreeParams), i32, i32, i64, vp, vp, vp, i64,
                                      ctypes.POINTER(i64)]
        L.spk_intersect.argtypes = [vp, vp, vp, ctypes.POINTER(BoundOpts), ctypes.POINTER(TreeParams),
                                    ctypes.POINTER(IntersectResult)]
        L.spk_empty_spheres.argtypes = [vp, vp, ctypes.POINTER(BoundOpts), i64, vp, ctypes.c_float,
                                        ctypes.c_float, vp, vp]
        L.spk_cast_frusta.argtypes = [vp, vp, ctypes.POINTER(RayParams), ctypes.POINTER(BoundOpts),
                                      ctypes.POINTER(Camera), i32, i32, vp, vp, ctypes.POINTER(FrustumStats)]
        L.spk_eval_points.argtypes = [vp, vp, i64, vp, vp]
        L.spk_batch_create.argtypes = [vp, ctypes.POINTER(BoundOpts), i32, ctypes.POINTER(BatchItem),
                                       ctypes.POINTER(vp)]
        L.spk_batch_update.argtypes = [vp, vp, i32, ctypes.POINTER(BatchItem)]
        L.spk_batch_launch.argtypes = [vp, vp]
        L.spk_batch_tune.argtypes = [vp, vp, i32]
        L.spk_batch_classes.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(BatchClass), i32]
        L.spk_batch_destroy.argtypes = [vp]
        L.spk_server_create.argtypes = [ctypes.POINTER(vp), i32, sz, i32, ctypes.POINTER(vp)]
        L.spk_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
        L.spk_server_poll.argtypes = [vp, ctypes.POINTER(Completion), i32, ctypes.POINTER(i32), i32]
        L.spk_server_pending.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(sz)]
        L.spk_server_destroy.argtypes = [vp]
        L.spk_closest_point.argtypes = [vp, vp, ctypes.POINTER(BoundOpts), ctypes.POINTER(TreeParams), i64, vp, vp,
                                        vp, vp]
        for name in EXPORTS:
            if name not in ("spk_status_str", "spk_version"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


class SpkError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s: %s (status %d)" % (where, lib().spk_status_str(status).decode(), status))


def _check(st, where):
    if st != OK:
        raise SpkError(st, where)


def _ptr(t, dtype=None, shape=None, name="tensor"):
    """Device pointer of a contiguous torch CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must have dtype %s" % (name, dtype))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, shape, tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


FLAG_RIGOROUS = 1
FLAG_NO_ROUNDING_BOUND = 2


PREC = {"f32": 0, "bf16x3": 1, "f16x3": 2, "f64": 3}


def opts(policy="truncate", k=31, rigorous=True, prec="f32"):
    """Bound options: rigorous=True (the library default) bounds every
    rounding; rigorous=False is the paper's arithmetic with the tolerance
    margin (SPK_FLAG_NO_ROUNDING_BOUND)."""
    return BoundOpts(POLICY[policy], int(k), PREC[prec], 0 if rigorous else FLAG_NO_ROUNDING_BOUND)


class Net:
    """A network uploaded to the current HIP device (spk_net_create)."""

    def __init__(self, weights, biases, act="relu", omega0=1.0):
        L = lib()
        Ws = [np.ascontiguousarray(np.asarray(w, dtype=np.float32)) for w in weights]
        bs = [np.ascontiguousarray(np.asarray(b, dtype=np.float32).reshape(-1)) for b in biases]
        widths = [Ws[0].shape[1]] + [w.shape[0] for w in Ws]
        n = len(Ws)
        wa = (ctypes.c_int32 * (n + 1))(*widths)
        Wp = (ctypes.c_void_p * n)(*[w.ctypes.data for w in Ws])
        bp = (ctypes.c_void_p * n)(*[b.ctypes.data for b in bs])
        h = ctypes.c_void_p()
        _check(L.spk_net_create(n, wa, Wp, bp, ACT[act], float(omega0), ctypes.byref(h)), "spk_net_create")
        self._keep = (Ws, bs)
        self.handle = h
        self.n_linear = n
        self.width = widths[1]
        self.act = act

    @classmethod
    def from_spec(cls, spec):
        return cls(spec.weights, spec.biases, spec.act, spec.omega0)

    def close(self):
        if self.handle:
            _check(lib().spk_net_destroy(self.handle), "spk_net_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A context on a HIP stream (default: torch's current stream)."""

    def __init__(self, stream=None, workspace_bytes=0):
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p()
        _check(lib().spk_ctx_create(ctypes.c_void_p(stream), workspace_bytes, ctypes.byref(h)), "spk_ctx_create")
        self.handle = h

    def sync(self, allow_nospc=False):
        """Wait for the context's stream; return the device status word since
        the previous sync as a dict.  A frontier overflow raises SpkError
        (E_NOSPC) unless allow_nospc."""
        ds = DeviceStatus()
        st = lib().spk_ctx_sync(self.handle, ctypes.byref(ds))
        if st != OK and not (st == E_NOSPC and allow_nospc):
            raise SpkError(st, "spk_ctx_sync")
        return {"nonfinite_inputs": int(ds.nonfinite_inputs), "nospc": bool(ds.nospc),
                "need_children": int(ds.need_children), "need_leaves": int(ds.need_leaves)}

    def close(self):
        if self.handle:
            _check(lib().spk_ctx_destroy(self.handle), "spk_ctx_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _aux(center=None, radius=None, err=None, slot_src=None):
    import torch
    if center is None and radius is None and err is None and slot_src is None:
        return None
    return BoundAux(_ptr(center, torch.float32, name="center"), _ptr(radius, torch.float32, name="radius"),
                    _ptr(err, torch.float32, name="err"), _ptr(slot_src, torch.int16, name="slot_src"))


def classify_boxes(ctx, net, box_lo, box_hi, label, lo=None, hi=None, policy="truncate", k=31, aux=None,
                   rigorous=True, prec="f32"):
    import torch
    n = box_lo.shape[0]
    o = opts(policy, k, rigorous, prec)
    a = _aux(**aux) if aux else None
    st = lib().spk_classify_boxes(ctx.handle, net.handle, ctypes.byref(o), n,
                                  _ptr(box_lo, torch.float32, (n, 3), "box_lo"),
                                  _ptr(box_hi, torch.float32, (n, 3), "box_hi"),
                                  _ptr(label, torch.uint8, (n,), "label"),
                                  _ptr(lo, torch.float32, (n,), "lo"), _ptr(hi, torch.float32, (n,), "hi"),
                                  ctypes.byref(a) if a is not None else None)
    _check(st, "spk_classify_boxes")


def range_bound(ctx, net, center, axes, lo, hi, policy="truncate", k=31, aux=None, rigorous=True, prec="f32"):
    import torch
    n, s = axes.shape[0], axes.shape[1]
    o = opts(policy, k, rigorous, prec)
    a = _aux(**aux) if aux else None
    st = lib().spk_range_bound(ctx.handle, net.handle, ctypes.byref(o), n, s,
                               _ptr(center, torch.float32, (n, 3), "center"),
                               _ptr(axes, torch.float32, (n, s, 3), "axes"),
                               _ptr(lo, torch.float32, (n,), "lo"), _ptr(hi, torch.float32, (n,), "hi"),
                               ctypes.byref(a) if a is not None else None)
    _check(st, "spk_range_bound")


def subdivide_frontier(ctx, net, level, cells, children, leaves, counts, max_level, policy="truncate", k=31,
                       dom_lo=(-1.0, -1.0, -1.0), dom_hi=(1.0, 1.0, 1.0), arity=8, noalloc=False, rigorous=True,
                       prec="f32", delta=0.0, band=0.0):
    """One round of Procedure 3 (spk_subdivide_frontier, or with
    noalloc=True spk_subdivide_frontier_noalloc); delta > 0 adds the
    convergence test for small cells."""
    import torch
    tp = TreeParams((ctypes.c_float * 3)(*dom_lo), (ctypes.c_float * 3)(*dom_hi), int(max_level), int(arity),
                    float(delta), float(band))
    o = opts(policy, k, rigorous, prec)
    n = cells.shape[0]
    capc = children.shape[0] if children is not None else 0
    capl = leaves.shape[0] if leaves is not None else 0
    name = "spk_subdivide_frontier_noalloc" if noalloc else "spk_subdivide_frontier"
    st = getattr(lib(), name)(ctx.handle, net.handle, ctypes.byref(o), ctypes.byref(tp), int(level),
                              _ptr(cells, torch.int64, (n,), "cells"), n,
                              _ptr(children, torch.int64, None, "children"), capc,
                              _ptr(leaves, torch.int64, None, "leaves"), capl,
                              _ptr(counts, torch.int64, (4,), "counts"))
    _check(st, name)


def ray_params(delta=1e-3, t_max=10.0, sigma0=None, eta_minus=0.5, eta_plus=1.5, safety=0.98, max_iters=100000,
               clip_to_domain=True, rigorous=True):
    """spk_ray_params; rigorous=False selects the paper's arithmetic
    (SPK_FLAG_NO_ROUNDING_BOUND) for the segment bounds."""
    if sigma0 is None:
        sigma0 = t_max / 10.0
    return RayParams(delta, t_max, sigma0, eta_minus, eta_plus, safety, int(max_iters), 1 if clip_to_domain else 0,
                     0 if rigorous else FLAG_NO_ROUNDING_BOUND)


def cast_rays(ctx, net, origin, direction, t_hit, iters=None, **params):
    import torch
    n = origin.shape[0]
    rp = ray_params(**params)
    st = lib().spk_cast_rays(ctx.handle, net.handle, ctypes.byref(rp), n,
                             _ptr(origin, torch.float32, (n, 3), "origin"),
                             _ptr(direction, torch.float32, (n, 3), "direction"),
                             _ptr(t_hit, torch.float32, (n,), "t_hit"), _ptr(iters, torch.int32, (n,), "iters"))
    _check(st, "spk_cast_rays")


def sample_leaves(ctx, net, leaves, level, n_samples, seed=0, band=math.inf, cap=None, dom_lo=(-1.0, -1.0, -1.0),
                  dom_hi=(1.0, 1.0, 1.0)):
    """spk_sample_leaves: (points [m, 3], f [m], n_below) of the accepted
    samples (|f| < band) among n_samples uniform points in the leaf cells."""
    import torch
    dev = torch.device("cuda")
    n = leaves.shape[0]
    tp = TreeParams((ctypes.c_float * 3)(*dom_lo), (ctypes.c_float * 3)(*dom_hi), int(level), 8)
    cap = int(cap if cap is not None else n_samples)
    pts = torch.empty((cap, 3), device=dev) if cap > 0 else None
    f = torch.empty(cap, device=dev) if cap > 0 else None
    na, nb = ctypes.c_int64(), ctypes.c_int64()
    st = lib().spk_sample_leaves(ctx.handle, net.handle, ctypes.byref(tp), int(level), n,
                                 _ptr(leaves, torch.int64, (n,), "leaves"), int(n_samples), int(seed) & (2 ** 64 - 1),
                                 float(band), _ptr(pts, torch.float32, None, "points"), _ptr(f, torch.float32, None, "f"),
                                 cap, ctypes.byref(na), ctypes.byref(nb))
    _check(st, "spk_sample_leaves")
    if pts is None:
        return None, None, int(nb.value)
    return pts[:na.value], f[:na.value], int(nb.value)


def bulk_volume(ctx, net, max_level, n_samples, seed=0, policy="truncate", k=31, rigorous=True, prec="f32",
                dom_lo=(-1.0,) * 3, dom_hi=(1.0,) * 3):
    """Volume of the solid {f < 0} (Section 4.8) from a fixed-depth tree:
    NEGATIVE cells in full, the UNKNOWN leaves by the fraction of uniform
    samples in them with f < 0.  Returns (estimate, lower bound, upper bound)."""
    levels, leaves = build_octree(ctx, net, max_level, policy, k, dom_lo, dom_hi, rigorous=rigorous, prec=prec)
    dom = float(np.prod(np.asarray(dom_hi, dtype=np.float64) - np.asarray(dom_lo, dtype=np.float64)))
    v_neg = sum(lv["n_neg"] * dom / 8.0 ** lv["level"] for lv in levels)
    v_leaf = leaves.shape[0] * dom / 8.0 ** max_level
    if leaves.shape[0] == 0:
        return v_neg, v_neg, v_neg
    _, _, n_below = sample_leaves(ctx, net, leaves, max_level, n_samples, seed, math.inf, cap=0,
                                  dom_lo=dom_lo, dom_hi=dom_hi)
    return v_neg + v_leaf * n_below / n_samples, v_neg, v_neg + v_leaf


def mesh_leaves(ctx, net, leaves, level, dense_levels=3, cap=None, dom_lo=(-1.0, -1.0, -1.0),
                dom_hi=(1.0, 1.0, 1.0), with_src=False):
    """spk_mesh_leaves: triangles [m, 3, 3] (GPU tensor) of the level set in
    the leaf cells (int64 Morton codes at `level`); with_src also returns the
    [m, 2] (leaf index, cube index) of each triangle.  The capacity grows and
    the call repeats once if the first guess was too small."""
    import torch
    dev = torch.device("cuda")
    n = leaves.shape[0]
    tp = TreeParams((ctypes.c_float * 3)(*dom_lo), (ctypes.c_float * 3)(*dom_hi), int(level), 8)
    cap = int(cap if cap is not None else max(1024, 4 * n * (1 << (2 * dense_levels))))
    for _ in range(2):
        tris = torch.empty((max(cap, 1), 3, 3), device=dev)
        src = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=dev) if with_src else None
        m = ctypes.c_int64()
        st = lib().spk_mesh_leaves(ctx.handle, net.handle, ctypes.byref(tp), int(level), int(dense_levels), n,
                                   _ptr(leaves, torch.int64, (n,), "leaves"), _ptr(tris, torch.float32, None, "tris"),
                                   _ptr(src, torch.int32, None, "tri_src"), cap, ctypes.byref(m))
        if st == E_NOSPC:
            cap = int(m.value)
            continue
        _check(st, "spk_mesh_leaves")
        tris = tris[:m.value]
        return (tris, src[:m.value]) if with_src else tris
    raise SpkError(E_NOSPC, "spk_mesh_leaves")


def intersect(ctx, net_f, net_g, max_level=8, policy="truncate", k=31, rigorous=True, prec="f32",
              dom_lo=(-1.0, -1.0, -1.0), dom_hi=(1.0, 1.0, 1.0)):
    """spk_intersect: whether the solids {f < 0} and {g < 0} overlap."""
    tp = TreeParams((ctypes.c_float * 3)(*dom_lo), (ctypes.c_float * 3)(*dom_hi), int(max_level), 8)
    o = opts(policy, k, rigorous, prec)
    r = IntersectResult()
    _check(lib().spk_intersect(ctx.handle, net_f.handle, net_g.handle, ctypes.byref(o), ctypes.byref(tp),
                               ctypes.byref(r)), "spk_intersect")
    return {"result": int(r.result), "level": int(r.level), "cell": int(r.cell), "undecided": int(r.undecided),
            "cells_bounded": int(r.cells_bounded), "rounds": int(r.rounds)}


def empty_spheres(ctx, net, p, radius, label, r0=1.0, r_min=1e-4, policy="truncate", k=31, rigorous=True,
                  prec="f32"):
    """spk_empty_spheres: radius [n] and label [n] for the points p [n, 3]."""
    import torch
    n = p.shape[0]
    o = opts(policy, k, rigorous, prec)
    st = lib().spk_empty_spheres(ctx.handle, net.handle, ctypes.byref(o), n, _ptr(p, torch.float32, (n, 3), "p"),
                                 float(r0), float(r_min), _ptr(radius, torch.float32, (n,), "radius"),
                                 _ptr(label, torch.uint8, (n,), "label"))
    _check(st, "spk_empty_spheres")


def camera(cam):
    """spk_camera from a dict with eye, forward, right, up, tan_x, tan_y, width,
    height (e.g. workloads.camera)."""
    f3 = ctypes.c_float * 3
    return Camera(f3(*map(float, cam["eye"])), f3(*map(float, cam["forward"])), f3(*map(float, cam["right"])),
                  f3(*map(float, cam["up"])), float(cam["tan_x"]), float(cam["tan_y"]), int(cam["width"]),
                  int(cam["height"]))


def cast_frusta(ctx, net, cam, t_hit, iters=None, tiles=(16, 16), policy="truncate", k=31, prec="f32", rigorous=True,
                **params):
    """spk_cast_frusta: t_hit [height * width] (and iters) for the camera's
    pixel rays; returns the frustum statistics as a dict."""
    import torch
    c = camera(cam)
    n = c.width * c.height
    rp = ray_params(rigorous=rigorous, **params)
    o = opts(policy, k, rigorous, prec)
    stats = FrustumStats()
    st = lib().spk_cast_frusta(ctx.handle, net.handle, ctypes.byref(rp), ctypes.byref(o), ctypes.byref(c),
                               int(tiles[0]), int(tiles[1]), _ptr(t_hit, torch.float32, (n,), "t_hit"),
                               _ptr(iters, torch.int32, (n,), "iters"), ctypes.byref(stats))
    _check(st, "spk_cast_frusta")
    return {"frustum_steps": int(stats.frustum_steps), "rays_handed_off": int(stats.rays_handed_off),
            "ray_iterations": int(stats.ray_iterations), "rounds": int(stats.rounds)}


def closest_point(ctx, net, q, point, dist=None, bound=None, max_level=8, policy="fixed", k=31,
                  dom_lo=(-1.0, -1.0, -1.0), dom_hi=(1.0, 1.0, 1.0), rigorous=True, prec="f32"):
    """spk_closest_point: point [n, 3], dist [n] and bound [n] for queries q [n, 3]."""
    import torch
    n = q.shape[0]
    tp = TreeParams((ctypes.c_float * 3)(*dom_lo), (ctypes.c_float * 3)(*dom_hi), int(max_level), 8)
    o = opts(policy, k, rigorous, prec)
    st = lib().spk_closest_point(ctx.handle, net.handle, ctypes.byref(o), ctypes.byref(tp), n,
                                 _ptr(q, torch.float32, (n, 3), "q"), _ptr(point, torch.float32, (n, 3), "point"),
                                 _ptr(dist, torch.float32, (n,), "dist"), _ptr(bound, torch.float32, (n,), "bound"))
    _check(st, "spk_closest_point")


class Batch:
    """spk_batch_*: one graph launch bounding the boxes of many networks.

    items: list of dicts with keys net (Net), box_lo, box_hi ([n, 3] float32
    device tensors), label ([n] uint8) and optionally lo, hi ([n] float32)."""

    def __init__(self, ctx, items, policy="truncate", k=31, rigorous=True):
        self.handle = None
        self._keep = None
        arr = self._items(items)
        o = opts(policy, k, rigorous)
        h = ctypes.c_void_p()
        _check(lib().spk_batch_create(ctx.handle, ctypes.byref(o), len(items), arr, ctypes.byref(h)),
               "spk_batch_create")
        self.handle = h

    def _items(self, items):
        """Box items: box_lo, box_hi, label (lo, hi optional).  Frontier items:
        cells ([n] int64 Morton codes), level, label, counts ([4] int64),
        children / leaves (capacity = their length; optional), max_level,
        dom_lo, dom_hi."""
        import torch
        arr = (BatchItem * len(items))()

        def v(p):
            return None if p is None else p.value
        for i, it in enumerate(items):
            b = BatchItem()
            b.net = it["net"].handle.value
            if it.get("cells") is not None:
                n = it["cells"].shape[0]
                b.n = n
                b.cells = v(_ptr(it["cells"], torch.int64, (n,), "cells"))
                b.level = int(it["level"])
                b.tree = TreeParams((ctypes.c_float * 3)(*it.get("dom_lo", (-1.0,) * 3)),
                                    (ctypes.c_float * 3)(*it.get("dom_hi", (1.0,) * 3)), int(it["max_level"]), 8)
                ch, lv = it.get("children"), it.get("leaves")
                b.children = v(_ptr(ch, torch.int64, None, "children")) if ch is not None and ch.numel() else None
                b.cap_children = int(ch.numel()) if ch is not None else 0
                b.leaves = v(_ptr(lv, torch.int64, None, "leaves")) if lv is not None and lv.numel() else None
                b.cap_leaves = int(lv.numel()) if lv is not None else 0
                b.counts = v(_ptr(it["counts"], torch.int64, (4,), "counts"))
            else:
                n = it["box_lo"].shape[0]
                b.n = n
                b.box_lo = v(_ptr(it["box_lo"], torch.float32, (n, 3), "box_lo"))
                b.box_hi = v(_ptr(it["box_hi"], torch.float32, (n, 3), "box_hi"))
            b.label = v(_ptr(it["label"], torch.uint8, (n,), "label"))
            b.lo = v(_ptr(it.get("lo"), torch.float32, (n,), "lo"))
            b.hi = v(_ptr(it.get("hi"), torch.float32, (n,), "hi"))
            arr[i] = b
        self._keep = list(items)   # the device buffers must outlive their use
        return arr

    def update(self, ctx, items):
        arr = self._items(items)
        _check(lib().spk_batch_update(ctx.handle, self.handle, len(items), arr), "spk_batch_update")

    def launch(self, ctx):
        _check(lib().spk_batch_launch(ctx.handle, self.handle), "spk_batch_launch")

    def tune(self, ctx, reps=3):
        _check(lib().spk_batch_tune(ctx.handle, self.handle, int(reps)), "spk_batch_tune")

    def classes(self):
        n = ctypes.c_int32()
        _check(lib().spk_batch_classes(self.handle, ctypes.byref(n), None, 0), "spk_batch_classes")
        out = (BatchClass * max(n.value, 1))()
        _check(lib().spk_batch_classes(self.handle, ctypes.byref(n), out, n.value), "spk_batch_classes")
        return [{f: getattr(out[i], f) for f, _ in BatchClass._fields_} for i in range(n.value)]

    def close(self):
        if self.handle:
            _check(lib().spk_batch_destroy(self.handle), "spk_batch_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """spk_server_*: continuous batching over resident networks.  Requests are
    dicts: {"type": "classify"|"rays"|"closest", "net": index, tensors...};
    the caller keeps every tensor alive until its completion is polled and
    must have finished writing the inputs (e.g. torch.cuda.synchronize())
    before submitting."""

    TYPES = {"classify": REQ_CLASSIFY, "rays": REQ_RAYS, "closest": REQ_CLOSEST}

    def __init__(self, nets, mem_budget, n_workers=4):
        self.handle = None
        arr = (ctypes.c_void_p * len(nets))(*[n.handle.value for n in nets])
        h = ctypes.c_void_p()
        _check(lib().spk_server_create(arr, len(nets), int(mem_budget), int(n_workers), ctypes.byref(h)),
               "spk_server_create")
        self.handle = h
        self._live = {}

    def submit(self, req):
        import torch

        def v(t):
            return None if t is None else t.data_ptr()
        r = Request()
        r.type = self.TYPES[req["type"]]
        r.net = int(req["net"])
        if req["type"] == "classify":
            r.n = req["box_lo"].shape[0]
            r.a, r.b = v(req["box_lo"]), v(req["box_hi"])
            r.out0, r.out1, r.out2 = v(req["label"]), v(req.get("lo")), v(req.get("hi"))
            r.opts = opts(req.get("policy", "truncate"), req.get("k", 31), req.get("rigorous", True))
            tensors = [req["box_lo"], req["box_hi"], req["label"], req.get("lo"), req.get("hi")]
        elif req["type"] == "rays":
            r.n = req["origin"].shape[0]
            r.a, r.b = v(req["origin"]), v(req["dir"])
            r.out0, r.out1 = v(req["t_hit"]), v(req.get("iters"))
            r.ray = ray_params(**req.get("params", {}))
            tensors = [req["origin"], req["dir"], req["t_hit"], req.get("iters")]
        else:
            r.n = req["q"].shape[0]
            r.a = v(req["q"])
            r.out0, r.out1, r.out2 = v(req["point"]), v(req.get("dist")), v(req.get("bound"))
            r.opts = opts(req.get("policy", "fixed"), req.get("k", 31), req.get("rigorous", True))
            r.tree = TreeParams((ctypes.c_float * 3)(-1, -1, -1), (ctypes.c_float * 3)(1, 1, 1),
                                int(req.get("max_level", 8)), 8)
            tensors = [req["q"], req["point"], req.get("dist"), req.get("bound")]
        io = sum(t.numel() * t.element_size() for t in tensors if t is not None)
        # default workspace: none for boxes and rays, 64 MiB for closest points
        ws = req.get("workspace", (64 << 20) if req["type"] == "closest" else 0)
        r.bytes = int(req.get("bytes", io + ws))
        rid = ctypes.c_uint64()
        _check(lib().spk_server_submit(self.handle, ctypes.byref(r), ctypes.byref(rid)), "spk_server_submit")
        self._live[rid.value] = tensors
        return rid.value

    def poll(self, max_n=64, wait=False):
        out = (Completion * max_n)()
        n = ctypes.c_int32()
        _check(lib().spk_server_poll(self.handle, out, max_n, ctypes.byref(n), 1 if wait else 0), "spk_server_poll")
        res = []
        for i in range(n.value):
            c = out[i]
            self._live.pop(c.id, None)
            res.append({"id": c.id, "status": c.status, "type": c.type, "n": c.n, "submit_s": c.submit_s,
                        "start_s": c.start_s, "done_s": c.done_s, "workspace_bytes": int(c.workspace_bytes)})
        return res

    def pending(self):
        q, r, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
        _check(lib().spk_server_pending(self.handle, ctypes.byref(q), ctypes.byref(r), ctypes.byref(b)),
               "spk_server_pending")
        return q.value, r.value, b.value

    def close(self):
        if self.handle:
            _check(lib().spk_server_destroy(self.handle), "spk_server_destroy")
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eval_points(ctx, net, x, f):
    import torch
    n = x.shape[0]
    st = lib().spk_eval_points(ctx.handle, net.handle, n, _ptr(x, torch.float32, (n, 3), "x"),
                               _ptr(f, torch.float32, (n,), "f"))
    _check(st, "spk_eval_points")


def build_delta_tree(ctx, net, delta, max_level=20, policy="truncate", k=31, rigorous=True, prec="f32",
                     dom_lo=(-1.0,) * 3, dom_hi=(1.0,) * 3):
    """BuildSpatialTree with the convergence test (Procedure 3): octree rounds
    in which, once cells are smaller than delta / sqrt(3), UNKNOWN cells whose
    face centers show both signs are final leaves (within delta of the level
    set).  Returns per-level stats and the leaves per level (a list of GPU
    tensors of Morton codes, converged cells and the cells left at
    max_level)."""
    import torch
    dev = torch.device("cuda")
    cells = torch.zeros(1, dtype=torch.int64, device=dev)
    counts = torch.zeros(4, dtype=torch.int64, device=dev)
    levels, leaves = [], []
    for level in range(max_level + 1):
        n = cells.shape[0]
        if n == 0:
            break
        at_max = level == max_level
        children = None if at_max else torch.empty(8 * n, dtype=torch.int64, device=dev)
        lv = torch.empty(n, dtype=torch.int64, device=dev)
        subdivide_frontier(ctx, net, level, cells, children, lv, counts, max_level, policy, k, dom_lo, dom_hi,
                           rigorous=rigorous, prec=prec, delta=delta)
        ctx.sync()
        c = counts.cpu().tolist()
        levels.append({"level": level, "n": n, "n_children": c[0], "n_leaves": c[1], "n_pos": c[2], "n_neg": c[3]})
        leaves.append(lv[:c[1]])
        cells = children[:c[0]] if children is not None else cells[:0]
    return levels, leaves


def build_octrees_batched(ctx, nets, max_level, policy="truncate", k=31, rigorous=True, tune=False,
                          dom_lo=(-1.0,) * 3, dom_hi=(1.0,) * 3):
    """Fixed-depth octrees of many networks at once: every level is one
    batched graph launch that classifies every network's frontier cells and
    compacts every frontier (spk_batch_* with frontier items).  Returns per
    network the per-level stats and the UNKNOWN leaf cells at max_level."""
    import torch
    dev = torch.device("cuda")
    m = len(nets)
    counts = torch.zeros((m, 4), dtype=torch.int64, device=dev)
    cells = [torch.zeros(1, dtype=torch.int64, device=dev) for _ in range(m)]
    levels = [[] for _ in range(m)]
    leaves = [torch.zeros(0, dtype=torch.int64, device=dev) for _ in range(m)]

    def items_for(level):
        at_max = level == max_level
        out = []
        for i in range(m):
            n = cells[i].shape[0]
            out.append({"net": nets[i], "cells": cells[i], "level": level, "max_level": max_level,
                        "dom_lo": dom_lo, "dom_hi": dom_hi, "label": torch.empty(n, dtype=torch.uint8, device=dev),
                        "counts": counts[i],
                        "children": None if at_max else torch.empty(8 * n, dtype=torch.int64, device=dev),
                        "leaves": torch.empty(n, dtype=torch.int64, device=dev) if at_max else None})
        return out
    its = items_for(0)
    b = Batch(ctx, its, policy, k, rigorous)
    try:
        for level in range(max_level + 1):
            if level > 0:
                its = items_for(level)
                b.update(ctx, its)
            if tune and level == max_level // 2:
                b.tune(ctx, reps=1)
            b.launch(ctx)
            ctx.sync()
            c = counts.cpu().tolist()
            for i in range(m):
                levels[i].append({"level": level, "n": int(cells[i].shape[0]), "n_children": c[i][0],
                                  "n_leaves": c[i][1], "n_pos": c[i][2], "n_neg": c[i][3]})
                if level == max_level:
                    leaves[i] = its[i]["leaves"][:c[i][1]]
                else:
                    cells[i] = its[i]["children"][:c[i][0]]
    finally:
        b.close()
    return levels, leaves


def build_octree(ctx, net, max_level, policy="truncate", k=31, dom_lo=(-1.0,) * 3, dom_hi=(1.0,) * 3,
                 cap=1 << 26, rigorous=True, prec="f32", band=0.0):
    """Fixed-depth octree by repeated spk_subdivide_frontier rounds (the
    breadth-first parallel rounds of Procedure 3).  Returns per-level stats and
    the UNKNOWN leaf cells at max_level (GPU tensor)."""
    import torch
    dev = torch.device("cuda")
    cells = torch.zeros(1, dtype=torch.int64, device=dev)
    counts = torch.zeros(4, dtype=torch.int64, device=dev)
    levels = []
    leaves = torch.zeros(0, dtype=torch.int64, device=dev)
    for level in range(max_level + 1):
        n = cells.shape[0]
        at_max = level == max_level
        capc = 0 if at_max else min(8 * n, cap)
        capl = n if at_max else 0
        children = torch.empty(max(capc, 1), dtype=torch.int64, device=dev)
        lv = torch.empty(max(capl, 1), dtype=torch.int64, device=dev)
        subdivide_frontier(ctx, net, level, cells, children[:capc] if capc else None, lv[:capl] if capl else None,
                           counts, max_level, policy, k, dom_lo, dom_hi, rigorous=rigorous, prec=prec, band=band)
        ds = ctx.sync(allow_nospc=True)
        c = counts.cpu().tolist()
        levels.append({"level": level, "n": n, "n_children": c[0], "n_leaves": c[1], "n_pos": c[2], "n_neg": c[3]})
        if at_max:
            leaves = lv[:c[1]]
            break
        if ds["nospc"] or c[0] > capc:
            raise SpkError(E_NOSPC, "build_octree")
        cells = children[:c[0]]
    return levels, leaves
