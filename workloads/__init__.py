"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws numbers: network weights, boxes, rays and query
points.  It holds none of the range-analysis arithmetic (no affine forms, no
activation bounds, no network evaluation), so that the FP64 oracle and the HIP
path can both consume the same inputs without sharing any of the method.

Every generator returns float32 numpy arrays (the precision the GPU path
consumes); the oracle widens them to float64 exactly.

Networks are described by :class:`MLPSpec`: ``weights[l]`` is row-major
``[out][in]`` and ``biases[l]`` has length ``out``.  The last layer is linear;
every other layer is followed by the activation (``relu``, ``elu`` with
alpha = 1, or ``sin`` applied as ``sin(omega0 * z)``), following the MLP
setting of the paper's Section 2 and the SIREN convention for sine networks.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math
from typing import List

import numpy as np

ACTS = ("relu", "elu", "sin")


@dataclass
class MLPSpec:
    weights: List[np.ndarray]
    biases: List[np.ndarray]
    act: str = "relu"
    omega0: float = 1.0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def widths(self) -> List[int]:
        return [self.weights[0].shape[1]] + [w.shape[0] for w in self.weights]

    @property
    def n_linear(self) -> int:
        return len(self.weights)

    def hidden_width(self) -> int:
        """Common width of the hidden layers (all configs use one width)."""
        hs = set(self.widths[1:-1])
        if len(hs) != 1:
            raise ValueError("hidden layers do not share one width: %s" % (self.widths,))
        return hs.pop()


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def he_normal_mlp(widths, seed, act="relu", bias=0.0, name=""):
    """He-normal weights W ~ N(0, 2/fan_in), constant bias (default 0)."""
    if act not in ACTS:
        raise ValueError(act)
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for n_in, n_out in zip(widths[:-1], widths[1:]):
        Ws.append(_f32(rng.standard_normal((n_out, n_in)) * math.sqrt(2.0 / n_in)))
        bs.append(_f32(np.full(n_out, bias)))
    return MLPSpec(Ws, bs, act=act, omega0=1.0, name=name or "he_%s_%s" % (act, "x".join(map(str, widths))),
                   meta={"seed": seed, "init": "he_normal"})


def siren_mlp(widths, seed, omega0=30.0, name=""):
    """SIREN initialisation: first layer U(+-1/fan_in), later layers
    U(+-sqrt(6/fan_in)/omega0), biases U(+-1/sqrt(fan_in))."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for l, (n_in, n_out) in enumerate(zip(widths[:-1], widths[1:])):
        lim = 1.0 / n_in if l == 0 else math.sqrt(6.0 / n_in) / omega0
        Ws.append(_f32(rng.uniform(-lim, lim, (n_out, n_in))))
        bl = 1.0 / math.sqrt(n_in)
        bs.append(_f32(rng.uniform(-bl, bl, n_out)))
    return MLPSpec(Ws, bs, act="sin", omega0=float(omega0), name=name or "siren_%s" % "x".join(map(str, widths)),
                   meta={"seed": seed, "init": "siren"})


# Constants of the closed-blob recipe (see blob_mlp).
BLOB_SCALE = 1.8
BLOB_L1 = 2.5
BLOB_R = 2.0


def blob_mlp(seed, width=256, n_hidden=8, scale=BLOB_SCALE, c=BLOB_L1, R=BLOB_R):
    """A random ReLU MLP 3 -> width x n_hidden -> 1 whose zero level set is a
    closed blob inside [-1,1]^3.

    It computes f(x) = scale * g(x) + c * |x|_1 - R exactly with the same
    architecture: g is a zero-bias He-normal ReLU network; six first-layer
    neurons compute relu(+x_i) and relu(-x_i); one "carrier" neuron per later
    hidden layer (neuron 0) carries their sum |x|_1 forward (ReLU is the
    identity on it); random rows never read carrier neurons; the output reads
    the carrier with weight c and has bias -R.  A zero-bias ReLU network is
    positively homogeneous, so the |x|_1 term dominates far from the origin and
    f > 0 on the cube boundary, while f(0) = -R < 0.
    """
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    # layer 1: 3 -> width
    W = rng.standard_normal((width, 3)) * math.sqrt(2.0 / 3)
    W[:6] = 0.0
    for i in range(3):
        W[2 * i, i] = 1.0
        W[2 * i + 1, i] = -1.0
    Ws.append(W)
    bs.append(np.zeros(width))
    for l in range(1, n_hidden):
        W = rng.standard_normal((width, width)) * math.sqrt(2.0 / width)
        if l == 1:
            W[:, :6] = 0.0      # random rows do not read the |x_i| neurons
            W[0, :] = 0.0
            W[0, :6] = 1.0      # carrier = sum of relu(+-x_i) = |x|_1
        else:
            W[:, 0] = 0.0       # random rows do not read the carrier
            W[0, :] = 0.0
            W[0, 0] = 1.0       # carrier copies itself
        Ws.append(W)
        bs.append(np.zeros(width))
    w = rng.standard_normal((1, width)) * math.sqrt(2.0 / width) * scale
    if n_hidden == 1:
        w[0, :6] = c
    else:
        w[0, 0] = c
    Ws.append(w)
    bs.append(np.array([-R]))
    return MLPSpec([_f32(a) for a in Ws], [_f32(b) for b in bs], act="relu", omega0=1.0,
                   name="blob_%dx%d" % (width, n_hidden),
                   meta={"seed": seed, "init": "closed_blob", "scale": scale, "c": c, "R": R})


def octahedron_mlp(R=0.5, pad_to=None):
    """The exact 3 -> 6 -> 1 ReLU network f(x) = sum_i relu(x_i) + relu(-x_i) - R
    = |x|_1 - R (an octahedron of L1 radius R).  ``pad_to`` widens the hidden
    layer with zero neurons (still exact)."""
    h = 6 if pad_to is None else pad_to
    W1 = np.zeros((h, 3))
    for i in range(3):
        W1[2 * i, i] = 1.0
        W1[2 * i + 1, i] = -1.0
    W2 = np.zeros((1, h))
    W2[0, :6] = 1.0
    return MLPSpec([_f32(W1), _f32(W2)], [_f32(np.zeros(h)), _f32([-R])], act="relu", name="octahedron",
                   meta={"R": R})


def boxes(n, seed, hw_lo=1e-3, hw_hi=0.25, dom=1.0):
    """n axis-aligned boxes: centers U[-dom, dom]^3, half-widths log-uniform in
    [hw_lo, hw_hi] drawn independently per axis.  Returns (lo, hi) as float32
    arrays of shape [n, 3]; the box is the float32 interval [lo, hi]."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-dom, dom, (n, 3))
    h = np.exp(rng.uniform(math.log(hw_lo), math.log(hw_hi), (n, 3)))
    return _f32(c - h), _f32(c + h)


def points(n, seed, dom=1.0):
    rng = np.random.default_rng(seed)
    return _f32(rng.uniform(-dom, dom, (n, 3)))


def camera(width, height, seed, radius=3.5, fov_deg=60.0):
    """A pinhole camera: eye uniform on a sphere of the given radius, looking at
    the origin, up = +z, vertical field of view fov_deg.  Returns a dict with
    the FP64 eye, orthonormal forward / right / up vectors, the tangents of the
    half fields of view (tan_x, tan_y) and the image size.  Pixel (px, py)
    (row-major from the top row) looks along normalize(forward + x right +
    y up) with x = (2 (px + 0.5) / width - 1) tan_x and
    y = (1 - 2 (py + 0.5) / height) tan_y."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(3)
    eye = radius * v / np.linalg.norm(v)
    fwd = -eye / np.linalg.norm(eye)
    up = np.array([0.0, 0.0, 1.0])
    if abs(np.dot(fwd, up)) > 0.999:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    true_up = np.cross(right, fwd)
    th = math.tan(math.radians(fov_deg) / 2.0)
    return {"eye": eye, "forward": fwd, "right": right, "up": true_up, "tan_x": th * width / height, "tan_y": th,
            "width": int(width), "height": int(height)}


def camera_rays(width, height, seed, radius=3.5, fov_deg=60.0):
    """The rays of :func:`camera`'s pixels: (origin, direction) float32
    [height*width, 3] with unit-length directions (pixel centers, row-major
    from the top row)."""
    cam = camera(width, height, seed, radius, fov_deg)
    ys = (1.0 - 2.0 * (np.arange(height) + 0.5) / height) * cam["tan_y"]
    xs = (2.0 * (np.arange(width) + 0.5) / width - 1.0) * cam["tan_x"]
    X, Y = np.meshgrid(xs, ys)
    d = cam["forward"][None, None, :] + X[..., None] * cam["right"][None, None, :] + \
        Y[..., None] * cam["up"][None, None, :]
    d = d.reshape(-1, 3)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(cam["eye"], d.shape)
    return _f32(o), _f32(d)


def tiny_net(seed=0):
    """3 -> 32 -> 32 -> 1 ReLU, He-normal, zero bias."""
    return he_normal_mlp([3, 32, 32, 1], seed, act="relu", name="tiny_relu_32x2")


def scale_net(seed=1):
    """3 -> 256 x 8 hidden -> 1 ReLU closed blob."""
    return blob_mlp(seed)


def batched_nets(n=64, base_seed=100):
    """The 64-network mix: width {64,128,256}[i mod 3], depth 4 + (i mod 5)
    hidden layers, activation {relu, elu, sin}[(i // 3) mod 3]."""
    nets = []
    for i in range(n):
        w = (64, 128, 256)[i % 3]
        depth = 4 + (i % 5)
        act = ("relu", "elu", "sin")[(i // 3) % 3]
        widths = [3] + [w] * depth + [1]
        if act == "sin":
            nets.append(siren_mlp(widths, base_seed + i, omega0=30.0))
        else:
            nets.append(he_normal_mlp(widths, base_seed + i, act=act))
    return nets


def batched_frontier_sizes(n=64, base_seed=200, lo=1e3, hi=2e5):
    out = []
    for i in range(n):
        rng = np.random.default_rng(base_seed + i)
        out.append(int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))))))
    return out
