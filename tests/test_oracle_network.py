"""Network-level pins of the oracle: soundness by brute force on tiny nets
(the fuzz protocol of Section 3.6), exactness on linear networks, interval
comparison, policy identities (CPU only)."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import affine as aa
from oracle import mlp
from oracle import queries as q


def _grid_samples(lo, hi, n=9):
    t = np.linspace(0.0, 1.0, n)
    g = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
    return lo + g * (hi - lo)


def _tiny_nets():
    nets = []
    for seed, (act, widths) in enumerate([("relu", [3, 16, 1]), ("relu", [3, 24, 24, 1]),
                                          ("elu", [3, 16, 16, 1]), ("elu", [3, 32, 32, 32, 1])]):
        nets.append(wl.he_normal_mlp(widths, 50 + seed, act=act, bias=0.05))
    nets.append(wl.siren_mlp([3, 16, 16, 1], 60, omega0=30.0))
    nets.append(wl.siren_mlp([3, 8, 8, 8, 1], 61, omega0=5.0))
    return nets


@pytest.mark.parametrize("policy,k", [("fixed", 0), ("truncate", 4), ("truncate", 11), ("full", 0)])
@pytest.mark.parametrize("net_i", range(6))
def test_soundness_bruteforce(policy, k, net_i):
    """Every point sample (a 9^3 grid including the corners, plus random points)
    lies inside the bound (Procedure 1 on many random regions)."""
    net = _tiny_nets()[net_i]
    rng = np.random.default_rng(100 + net_i)
    B = 60
    c = rng.uniform(-1, 1, (B, 3))
    h = np.exp(rng.uniform(math.log(1e-3), math.log(0.5), (B, 3)))
    lo, hi = c - h, c + h
    _, _, ly, hy = mlp.bound_boxes(net, lo, hi, policy, max(k, 3))
    for b in range(B):
        P = np.concatenate([_grid_samples(lo[b], hi[b]), lo[b] + rng.uniform(0, 1, (200, 3)) * (hi[b] - lo[b])])
        f = mlp.forward(net, P)
        tol = 1e-10 * max(1.0, np.abs(f).max())
        assert f.min() >= ly[b] - tol and f.max() <= hy[b] + tol, (b, f.min(), f.max(), ly[b], hy[b])


def test_exact_on_linear_network():
    """A ReLU net whose pre-activations stay positive over the box acts as the
    linear map J = W_L ... W_1; affine arithmetic is then exact: the bound is
    f(c) +- sum_i |J v_i|, reached at box corners."""
    rng = np.random.default_rng(12)
    net = wl.he_normal_mlp([3, 16, 16, 1], 13, act="relu", bias=0.0)
    # biases large enough that every hidden pre-activation is positive on [-2,2]^3
    W1 = net.weights[0].astype(np.float64)
    net.biases[0] = np.full(16, np.abs(W1).sum(1).max() * 2 + 1.0, dtype=np.float32)
    hmax = np.abs(W1).sum(1).max() * 2 + net.biases[0].astype(np.float64).max()
    W2 = net.weights[1].astype(np.float64)
    net.biases[1] = np.full(16, np.abs(W2).sum(1).max() * hmax + 1.0, dtype=np.float32)
    B = 40
    c = rng.uniform(-1, 1, (B, 3))
    h = rng.uniform(0.01, 0.5, (B, 3))
    lo, hi = c - h, c + h
    Ws = [np.asarray(W, dtype=np.float64) for W in net.weights]
    J = Ws[2] @ Ws[1] @ Ws[0]
    fc = mlp.forward(net, c)
    rad = np.abs(J[0][None, :] * h).sum(1)
    corners = np.array(np.meshgrid(*[[0, 1]] * 3)).reshape(3, -1).T
    for policy in ("fixed", "truncate", "full"):
        _, _, ly, hy = mlp.bound_boxes(net, lo, hi, policy, 8)
        assert np.allclose(ly, fc - rad, rtol=1e-12, atol=1e-9)
        assert np.allclose(hy, fc + rad, rtol=1e-12, atol=1e-9)
        for b in range(B):
            f = mlp.forward(net, lo[b] + corners * (hi[b] - lo[b]))
            assert f.min() == pytest.approx(ly[b], abs=1e-8) and f.max() == pytest.approx(hy[b], abs=1e-8)


def test_octahedron_net_values():
    net = wl.octahedron_mlp(0.5)
    rng = np.random.default_rng(14)
    P = rng.uniform(-1, 1, (1000, 3))
    assert np.allclose(mlp.forward(net, P), np.abs(P).sum(1) - 0.5)


def test_truncate_with_large_k_equals_full():
    net = _tiny_nets()[2]
    lo, hi = wl.boxes(64, 15, 1e-3, 0.3)
    a = mlp.bound_boxes(net, lo, hi, "truncate", 10000)
    b = mlp.bound_boxes(net, lo, hi, "full")
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_policy_tightness_order_on_average():
    """full keeps every term, so its bound is never wider than fixed's."""
    net = wl.he_normal_mlp([3, 32, 32, 1], 16, act="relu")
    lo, hi = wl.boxes(300, 17, 1e-3, 0.25)
    _, rf, _, _ = mlp.bound_boxes(net, lo, hi, "full")
    _, rx, _, _ = mlp.bound_boxes(net, lo, hi, "fixed")
    assert np.all(rf <= rx * (1 + 1e-12) + 1e-12)


def test_interval_contains_affine_first_layer_and_rate():
    """Interval-contains-affine holds exactly for linear maps (first layer of an
    axis-aligned box, where the two coincide); after nonlinear layers it is not
    a theorem, so only its rate is recorded here."""
    net = wl.tiny_net(0)
    lo, hi = wl.boxes(2000, 10, 1e-3, 0.25)
    Ws = [np.asarray(W, dtype=np.float64) for W in net.weights]
    il, iu = aa.ia_linear(lo.astype(np.float64), hi.astype(np.float64), Ws[0], net.biases[0].astype(np.float64))
    x0, X, xi = aa.from_aabb(lo, hi)
    z0, Z, zi = aa.linear(x0, X, xi, Ws[0], net.biases[0].astype(np.float64))
    al, au = aa.affine_range(z0, Z, zi)
    assert np.allclose(al, il, atol=1e-12) and np.allclose(au, iu, atol=1e-12)
    ly_i, hy_i = mlp.interval_bound_boxes(net, lo, hi)
    _, _, ly, hy = mlp.bound_boxes(net, lo, hi, "full")
    contained = (ly >= ly_i - 1e-12) & (hy <= hy_i + 1e-12)
    assert contained.mean() > 0.9


def test_interval_bound_sound():
    net = _tiny_nets()[4]
    rng = np.random.default_rng(18)
    c = rng.uniform(-1, 1, (40, 3))
    h = np.exp(rng.uniform(math.log(1e-3), math.log(0.2), (40, 3)))
    lo, hi = c - h, c + h
    il, iu = mlp.interval_bound_boxes(net, lo, hi)
    for b in range(40):
        f = mlp.forward(net, _grid_samples(lo[b], hi[b], 7))
        assert f.min() >= il[b] - 1e-12 and f.max() <= iu[b] + 1e-12


def test_segment_bound_sound_and_classify():
    net = wl.tiny_net(0)
    rng = np.random.default_rng(19)
    p = rng.uniform(-1, 1, (100, 3))
    d = rng.standard_normal((100, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    t = rng.uniform(0, 1, 100)
    s = np.exp(rng.uniform(-6, 0, 100))
    ly, hy = mlp.bound_segments(net, p, d, t, s, "fixed")
    for i in range(100):
        ts = np.linspace(t[i], t[i] + s[i], 401)
        f = mlp.forward(net, p[i] + ts[:, None] * d[i])
        assert f.min() >= ly[i] - 1e-12 and f.max() <= hy[i] + 1e-12
    lab = q.classify(ly, hy)
    assert np.array_equal(lab == q.POSITIVE, ly > 0) and np.array_equal(lab == q.NEGATIVE, hy < 0)


def test_classify_strict():
    lab = q.classify(np.array([0.0, 1e-300, -1.0, -1.0]), np.array([1.0, 1.0, 0.0, -1e-300]))
    assert list(lab) == [q.UNKNOWN, q.POSITIVE, q.UNKNOWN, q.NEGATIVE]


def _random_rotations(rng, B):
    """B random proper rotations (QR of Gaussian matrices, sign-fixed)."""
    Q, R = np.linalg.qr(rng.standard_normal((B, 3, 3)))
    Q = Q * np.sign(np.diagonal(R, axis1=1, axis2=2))[:, None, :]
    det = np.linalg.det(Q)
    Q[det < 0, :, 0] *= -1.0
    return Q


def _positive_linear_net():
    """The ReLU net of test_exact_on_linear_network: every hidden
    pre-activation is positive on [-2,2]^3, so it is the linear map J."""
    net = wl.he_normal_mlp([3, 16, 16, 1], 13, act="relu", bias=0.0)
    W1 = net.weights[0].astype(np.float64)
    net.biases[0] = np.full(16, np.abs(W1).sum(1).max() * 2 + 1.0, dtype=np.float32)
    hmax = np.abs(W1).sum(1).max() * 2 + net.biases[0].astype(np.float64).max()
    W2 = net.weights[1].astype(np.float64)
    net.biases[1] = np.full(16, np.abs(W2).sum(1).max() * hmax + 1.0, dtype=np.float32)
    return net


@pytest.mark.parametrize("s", [1, 2, 3])
def test_rotated_boxes_exact_on_linear_network(s):
    """Oriented boxes c + sum_i t_i v_i (t in [-1,1]^s, v_i orthogonal half-axes,
    Procedure 1's general region): on a network that acts as the linear map J
    the affine bound is exactly f(c) +- sum_i |J v_i|, and its ends are reached
    at the box's corners.  The axes are random rotations with unequal
    half-lengths, so a transposed axis matrix (row i = v_i read as column i)
    gives a different radius and fails."""
    rng = np.random.default_rng(70 + s)
    net = _positive_linear_net()
    B = 64
    Q = _random_rotations(rng, B)                      # columns are orthonormal directions
    h = rng.uniform(0.05, 0.6, (B, 3))
    axes = np.transpose(Q, (0, 2, 1))[:, :s, :] * h[:, :s, None]   # axes[b, i] = h_i q_i
    c = rng.uniform(-0.8, 0.8, (B, 3))
    Ws = [np.asarray(W, dtype=np.float64) for W in net.weights]
    J = (Ws[2] @ Ws[1] @ Ws[0])[0]
    fc = mlp.forward(net, c)
    rad = np.abs(np.einsum("bid,d->bi", axes, J)).sum(axis=1)
    for policy in ("fixed", "truncate", "full"):
        ly, hy = mlp.bound_general(net, c, axes, policy, 8)
        assert np.allclose(ly, fc - rad, rtol=1e-12, atol=1e-10)
        assert np.allclose(hy, fc + rad, rtol=1e-12, atol=1e-10)
    # corner brute force: the extremes of a linear map over the box
    signs = np.array(np.meshgrid(*[[-1.0, 1.0]] * s, indexing="ij")).reshape(s, -1).T
    for b in range(B):
        P = c[b] + signs @ axes[b]
        f = mlp.forward(net, P)
        assert f.min() == pytest.approx(fc[b] - rad[b], abs=1e-9)
        assert f.max() == pytest.approx(fc[b] + rad[b], abs=1e-9)
    # the transposed reading differs on these boxes (guards the pin itself)
    if s == 3:
        rad_t = np.abs(np.einsum("bdi,d->bi", axes, J)).sum(axis=1)
        assert np.max(np.abs(rad_t - rad)) > 1e-3


@pytest.mark.parametrize("net_i", [0, 2, 4])
def test_rotated_boxes_sound_on_nonlinear_nets(net_i):
    """Soundness by brute force over oriented 3-axis boxes: f at the 27
    lattice points c + sum_i t_i v_i (t_i in {-1,0,1}) and at random interior
    points lies inside the bound, for every policy."""
    net = _tiny_nets()[net_i]
    rng = np.random.default_rng(80 + net_i)
    B = 40
    Q = _random_rotations(rng, B)
    h = np.exp(rng.uniform(math.log(1e-3), math.log(0.4), (B, 3)))
    axes = np.transpose(Q, (0, 2, 1)) * h[:, :, None]
    c = rng.uniform(-1, 1, (B, 3))
    lat = np.array(np.meshgrid(*[[-1.0, 0.0, 1.0]] * 3, indexing="ij")).reshape(3, -1).T
    for policy, k in (("fixed", 3), ("truncate", 5), ("full", 3)):
        ly, hy = mlp.bound_general(net, c, axes, policy, k)
        for b in range(B):
            T = np.concatenate([lat, rng.uniform(-1, 1, (100, 3))])
            f = mlp.forward(net, c[b] + T @ axes[b])
            tol = 1e-10 * max(1.0, np.abs(f).max())
            assert f.min() >= ly[b] - tol and f.max() <= hy[b] + tol, (policy, b)


def test_rotated_box_equals_aabb_when_axes_are_diagonal():
    """With axes diag(h) the general-box form is the AABB form exactly."""
    net = _tiny_nets()[1]
    rng = np.random.default_rng(90)
    B = 30
    c = rng.uniform(-1, 1, (B, 3))
    h = np.exp(rng.uniform(math.log(1e-3), math.log(0.4), (B, 3)))
    axes = np.zeros((B, 3, 3))
    axes[:, [0, 1, 2], [0, 1, 2]] = h
    ly, hy = mlp.bound_general(net, c, axes, "truncate", 7)
    _, _, la, ha = mlp.bound_boxes(net, c - h, c + h, "truncate", 7)
    assert np.allclose(ly, la, rtol=1e-13, atol=1e-13) and np.allclose(hy, ha, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("name", ["relu", "elu", "sin", "blob"])
def test_forward_torch_equals_forward(name):
    """The PyTorch FP64 point evaluation (used for large soundness samples)
    equals the NumPy one to FP64 rounding."""
    import workloads as wl
    from oracle import mlp as omlp
    net = {"relu": lambda: wl.he_normal_mlp([3, 64, 64, 1], 5),
           "elu": lambda: wl.he_normal_mlp([3, 64, 64, 64, 1], 6, act="elu"),
           "sin": lambda: wl.siren_mlp([3, 32, 32, 1], 7, 30.0),
           "blob": lambda: wl.scale_net(1)}[name]()
    x = np.random.default_rng(3).uniform(-1.2, 1.2, (2000, 3))
    a = omlp.forward(net, x)
    b = omlp.forward_torch(net, x)
    assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.max(np.abs(a)))
