"""Pins of the oracle's arithmetic rules against closed forms, brute force and
invariants (CPU only)."""
import math
import os

import numpy as np
import pytest

from oracle import affine as aa

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "activation_params.txt")


def _golden_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            act, l, u, a, b, g = line.split()
            rows.append((act, float(l), float(u), float(a), float(b), float(g)))
    return rows


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: "%s[%g,%g]" % r[:3])
def test_activation_params_golden(row):
    act, l, u, a, b, g = row
    x0 = np.array([(l + u) / 2])
    alpha, beta, gamma = aa.act_params(act, np.array([l]), np.array([u]), x0)
    assert alpha[0] == pytest.approx(a, abs=1e-9)
    assert beta[0] == pytest.approx(b, abs=1e-9)
    assert gamma[0] == pytest.approx(g, abs=1e-9)


def _bruteforce_err(act, l, u, alpha, beta, n=20001):
    x = np.linspace(l, u, n)
    return np.max(np.abs(aa.act_fn(act, x) - (alpha * x + beta)))


@pytest.mark.parametrize("act", ["relu", "elu", "sin"])
def test_linearisation_error_is_gamma(act):
    """gamma bounds the error on a dense grid and is attained (the table's
    Chebyshev form puts beta midway between the extreme errors, both of which
    are reached inside the interval)."""
    rng = np.random.default_rng(3)
    n = 400
    c = rng.uniform(-6, 6, n)
    w = np.exp(rng.uniform(math.log(1e-3), math.log(12.0), n))
    l, u = c - w, c + w
    alpha, beta, gamma = aa.act_params(act, l, u, c)
    for i in range(n):
        err = _bruteforce_err(act, l[i], u[i], alpha[i], beta[i])
        # the grid misses an interior extremum by at most a second-order term
        h = (u[i] - l[i]) / 20000.0
        slack = 1e-12 + (h * h) * (1.0 if act != "relu" else 0.0)
        assert err <= gamma[i] + 1e-12, (act, l[i], u[i])
        assert err >= gamma[i] - slack - 1e-9 * max(1.0, abs(gamma[i])), (act, l[i], u[i], err, gamma[i])


def test_sin_params_wide_and_periodic():
    # shifting a sine interval by 2 pi shifts sin(x) - alpha x by -2 pi alpha: gamma is unchanged
    rng = np.random.default_rng(4)
    l = rng.uniform(-3, 3, 200)
    u = l + rng.uniform(0.01, 5, 200)
    a1, b1, g1 = aa.sin_params(l, u)
    a2, b2, g2 = aa.sin_params(l + 2 * math.pi, u + 2 * math.pi)
    assert np.allclose(a1, a2, atol=1e-12)
    assert np.allclose(g1, g2, atol=1e-10)
    assert np.allclose(b2, b1 - 2 * math.pi * a1, atol=1e-10)


def test_cos_range_bruteforce():
    rng = np.random.default_rng(5)
    l = rng.uniform(-20, 20, 300)
    u = l + np.exp(rng.uniform(-6, 2.5, 300))
    lo, hi = aa.cos_range(l, u)
    for i in range(300):
        x = np.linspace(l[i], u[i], 100001)
        assert lo[i] <= np.cos(x).min() + 1e-12
        assert hi[i] >= np.cos(x).max() - 1e-12
        assert lo[i] >= np.cos(x).min() - 1e-8
        assert hi[i] <= np.cos(x).max() + 1e-8


def test_elu_degenerate_interval():
    x = np.array([-0.7, 0.0, 1.3])
    a, b, g = aa.elu_params(x, x, x)
    assert np.allclose(a[0], math.exp(-0.7))
    assert np.all(g <= 1e-15) and np.all(g >= 0)
    assert np.allclose(a * x + b, aa.elu(x), atol=1e-15)


def test_dependency_problem():
    """Section 3.1: y = 2x - x.  Interval arithmetic treats the two x as
    distinct; affine arithmetic cancels them.  On [0,1] IA gives [-1,2] and AA
    the exact [0,1]; on [-1,1] IA gives [-3,3] and AA the exact [-1,1]."""
    for (l, u, ia_expect) in [(0.0, 1.0, (-1.0, 2.0)), (-1.0, 1.0, (-3.0, 3.0))]:
        # IA: t = 2x, then y = t - x with t and x as independent intervals
        tl, tu = aa.ia_linear(np.array([[l]]), np.array([[u]]), np.array([[2.0]]), np.zeros(1))
        yl, yu = aa.ia_linear(np.array([[tl[0, 0], l]]), np.array([[tu[0, 0], u]]),
                              np.array([[1.0, -1.0]]), np.zeros(1))
        assert (yl[0, 0], yu[0, 0]) == ia_expect
        # AA: the same two steps on affine forms
        x0, X, xi = aa.from_aabb(np.array([[l]]), np.array([[u]]))
        t0, T, ti = aa.matmul(x0, X, xi, np.array([[2.0], [1.0]]))   # (2x, x)
        y0, Y, yi = aa.matmul(t0, T, ti, np.array([[1.0, -1.0]]))
        lo, hi = aa.affine_range(y0, Y, yi)
        assert (lo[0, 0], hi[0, 0]) == (l, u)


def test_table2_rules_small():
    x0 = np.array([[1.0, -2.0]])
    X = np.array([[[0.5, -1.0], [0.25, 0.0]]])
    xi = np.array([[0.1, 0.2]])
    A = np.array([[2.0, -1.0], [0.0, 3.0], [-1.0, -1.0]])
    z0, Z, zi = aa.matmul(x0, X, xi, A)
    assert np.allclose(z0, [[4.0, -6.0, 1.0]])
    assert np.allclose(Z[0], [[0.75, -2.0], [0.75, 0.0], [-0.75, 1.0]])
    assert np.allclose(zi, [[0.4, 0.6, 0.3]])
    m0, M, mi = aa.mul_const(x0, X, xi, -3.0)
    assert np.allclose(m0, -3 * x0) and np.allclose(M, -3 * X) and np.allclose(mi, 3 * xi)
    a0, Aa, ai = aa.add_const(x0, X, xi, np.array([1.0, 1.0]))
    assert np.allclose(a0, x0 + 1) and np.array_equal(Aa, X) and np.array_equal(ai, xi)


def test_affine_range_contains_samples_of_linear_map():
    """Affine forms are exact under linear maps: the range read-off equals the
    brute-force extremes over the symbol corners."""
    rng = np.random.default_rng(6)
    x0 = rng.standard_normal((1, 4))
    X = rng.standard_normal((1, 4, 3))
    xi = np.zeros((1, 4))
    A = rng.standard_normal((2, 4))
    z0, Z, zi = aa.matmul(x0, X, xi, A)
    lo, hi = aa.affine_range(z0, Z, zi)
    corners = np.array(np.meshgrid(*[[-1, 1]] * 3)).reshape(3, -1).T
    vals = (A @ (x0[0][:, None] + X[0] @ corners.T)).T
    assert np.allclose(lo[0], vals.min(0))
    assert np.allclose(hi[0], vals.max(0))


def _random_state(rng, B=5, m=12, N=6):
    x0 = rng.standard_normal((B, m))
    X = rng.standard_normal((B, m, N)) * rng.uniform(0.01, 1, (B, 1, N))
    xi = np.abs(rng.standard_normal((B, m))) * 0.1
    return x0, X, xi


def test_condense_preserves_radius():
    rng = np.random.default_rng(7)
    x0, X, xi = _random_state(rng)
    gamma = np.abs(rng.standard_normal(x0.shape))
    full = np.abs(X).sum(2) + xi + gamma
    for k in (6, 9, 18):
        z0, Z, zi, keep, src = aa.condense_truncate(x0, X, xi, gamma, k)
        assert Z.shape[2] == min(k, 6 + 12)
        assert np.allclose(np.abs(Z).sum(2) + zi, full, rtol=1e-14, atol=1e-14)
    z0, Z, zi = aa.condense_fixed(x0, X, xi, gamma)
    assert np.allclose(np.abs(Z).sum(2) + zi, full)
    z0, Z, zi = aa.condense_full(x0, X, xi, gamma)
    assert np.allclose(np.abs(Z).sum(2) + zi, full)


def test_truncate_selects_top_k_with_index_ties():
    rng = np.random.default_rng(8)
    x0, X, xi = _random_state(rng, B=40, m=10, N=5)
    gamma = np.abs(rng.standard_normal(x0.shape))
    # plant exact ties: one new term equal to an old column's magnitude, and zeros
    mu_old = np.abs(X).sum(1)
    gamma[:, 3] = mu_old[:, 2]
    gamma[:, 7] = 0.0
    X[:, :, 4] = 0.0
    k = 6
    z0, Z, zi, keep, src = aa.condense_truncate(x0, X, xi, gamma, k)
    mu = np.concatenate([np.abs(X).sum(1), gamma], axis=1)
    for b in range(40):
        kept = np.flatnonzero(keep[b])
        dropped = np.flatnonzero(~keep[b])
        assert kept.size == k
        # definition: sort by (-mu, index) and take the first k
        order = sorted(range(mu.shape[1]), key=lambda i: (-mu[b, i], i))
        assert sorted(order[:k]) == list(kept)
        assert mu[b, kept].min() >= mu[b, dropped].max()


def test_truncate_slot_layout():
    """Kept old columns stay in place; kept new terms fill the freed slots in
    increasing order by increasing neuron index; a kept new term is a column
    with gamma_j on row j only."""
    rng = np.random.default_rng(9)
    x0, X, xi = _random_state(rng, B=30, m=8, N=4)
    gamma = np.abs(rng.standard_normal(x0.shape)) * 2
    k = 6
    z0, Z, zi, keep, src = aa.condense_truncate(x0, X, xi, gamma, k)
    for b in range(30):
        ko = keep[b, :4]
        kn = np.flatnonzero(keep[b, 4:])
        free = [s for s in range(k) if s >= 4 or not ko[s]]
        assert len(free) == len(kn)
        for s in range(4):
            if ko[s]:
                assert np.array_equal(Z[b, :, s], X[b, :, s]) and src[b, s] == -1
        for s, j in zip(free, kn):
            col = np.zeros(8)
            col[j] = gamma[b, j]
            assert np.array_equal(Z[b, :, s], col) and src[b, s] == j


def test_truncate_replay_reproduces():
    rng = np.random.default_rng(10)
    x0, X, xi = _random_state(rng)
    gamma = np.abs(rng.standard_normal(x0.shape))
    a = aa.condense_truncate(x0, X, xi, gamma, 7)
    b = aa.condense_truncate(x0, X, xi, gamma, 7, keep=a[3])
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_ia_contains_aa_on_linear_maps():
    """For a linear map AA is never looser than IA (triangle inequality), and
    for an axis-aligned box the two agree exactly at the first layer."""
    rng = np.random.default_rng(11)
    lo = rng.uniform(-1, 0, (50, 3))
    hi = lo + rng.uniform(0, 1, (50, 3))
    W = rng.standard_normal((16, 3))
    b = rng.standard_normal(16)
    il, iu = aa.ia_linear(lo, hi, W, b)
    x0, X, xi = aa.from_aabb(lo, hi)
    z0, Z, zi = aa.linear(x0, X, xi, W, b)
    al, au = aa.affine_range(z0, Z, zi)
    assert np.allclose(al, il, atol=1e-12) and np.allclose(au, iu, atol=1e-12)
    # second linear map on a correlated (non-box) affine form: AA within IA
    W2 = rng.standard_normal((8, 16))
    z0b, Zb, zib = aa.linear(z0, Z, zi, W2, np.zeros(8))
    al2, au2 = aa.affine_range(z0b, Zb, zib)
    il2, iu2 = aa.ia_linear(il, iu, W2, np.zeros(8))
    assert np.all(al2 >= il2 - 1e-12) and np.all(au2 <= iu2 + 1e-12)
    assert np.any(au2 - al2 < iu2 - il2 - 1e-9)
