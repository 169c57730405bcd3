"""Affine and interval arithmetic in float64 (oracle; test infrastructure only).

A batched affine form is the tuple (x0, X, xinf) of Appendix A:

* ``x0``   [B, m]     base values,
* ``X``    [B, m, N]  one column per noise symbol eps_i in [-1, 1],
* ``xinf`` [B, m]     the distinguished condensed coefficient (non-negative),
  whose symbol never cancels.

The value set it describes is x0 + X eps + xinf * eps_inf (per component).

Parity unpinned: nothing here.  Every function below is pinned by a test in
``tests/test_oracle_*.py`` against closed forms, brute force or invariants.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


# ---------------------------------------------------------------------------
# Construction and read-off (Procedure 1 step 1; Appendix A; eq. def_range)
# ---------------------------------------------------------------------------

def from_box(center, axes):
    """Affine form of a (not necessarily axis-aligned) s-dimensional box with
    center c [B, d] and s orthogonal half-axis vectors axes [B, s, d]:
    x0 = c, X = [v_1 ... v_s] (as columns), xinf = 0  (Procedure 1, Appendix A)."""
    c = np.asarray(center, dtype=np.float64)
    v = np.asarray(axes, dtype=np.float64)
    X = np.transpose(v, (0, 2, 1)).copy()
    return c.copy(), X, np.zeros_like(c)


def from_aabb(lo, hi):
    """Axis-aligned box [lo, hi]: center (lo+hi)/2 and axes diag((hi-lo)/2)
    (Procedure 3 builds exactly this: x_c = (x_l + x_u)/2, v = Diag(x_u - x_c))."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    c = (lo + hi) / 2.0
    h = hi - c
    B, d = c.shape
    axes = np.zeros((B, d, d))
    idx = np.arange(d)
    axes[:, idx, idx] = h
    return from_box(c, axes)


def from_segment(p, r, t, sigma):
    """1-d box along a ray: center p + (t + sigma/2) r, single axis (sigma/2) r
    (Procedure 2)."""
    p = np.asarray(p, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)[:, None]
    s = np.asarray(sigma, dtype=np.float64)[:, None]
    c = p + (t + s / 2.0) * r
    v = (s / 2.0) * r
    return from_box(c, v[:, None, :])


def radius(X, xinf):
    """r = sum_i |X_i| + xinf (eq. def_range, with the condensed term of
    Appendix A included)."""
    return np.abs(X).sum(axis=2) + xinf


def affine_range(x0, X, xinf):
    r = radius(X, xinf)
    return x0 - r, x0 + r


# ---------------------------------------------------------------------------
# Exact affine rules (Section 3.2; Table 2)
# ---------------------------------------------------------------------------

def add_const(x0, X, xinf, a):
    return x0 + a, X, xinf


def mul_const(x0, X, xinf, a):
    return a * x0, a * X, abs(a) * xinf


def matmul(x0, X, xinf, A):
    """z = A x: z0 = A x0, Z = A X, zinf = |A| xinf (|A| element-wise)."""
    A = np.asarray(A, dtype=np.float64)
    z0 = x0 @ A.T
    Z = np.matmul(A, X)
    zinf = xinf @ np.abs(A).T
    return z0, Z, zinf


def linear(x0, X, xinf, W, b):
    """Dense layer W x + b: matrix multiplication then constant addition."""
    z0, Z, zinf = matmul(x0, X, xinf, W)
    return add_const(z0, Z, zinf, np.asarray(b, dtype=np.float64))


# ---------------------------------------------------------------------------
# Linearisations of the activations (Table 3).  Each returns (alpha, beta,
# gamma) such that |h(x) - (alpha x + beta)| <= gamma on [l, u].
# ---------------------------------------------------------------------------

def relu_params(l, u):
    """ReLU (Table 3, Chebyshev): alpha is the chord slope, beta =
    (ReLU(l) - alpha l)/2 and the maximum error equals beta.  The two
    sign-stable cases give the exact maps (1,0,0) and (0,0,0)."""
    l = np.asarray(l, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    alpha = np.zeros_like(l)
    beta = np.zeros_like(l)
    pos = l >= 0.0
    cross = (~pos) & (u > 0.0)
    alpha[pos] = 1.0
    lc, uc = l[cross], u[cross]
    a = (np.maximum(uc, 0.0) - np.maximum(lc, 0.0)) / (uc - lc)
    alpha[cross] = a
    beta[cross] = (np.maximum(lc, 0.0) - a * lc) / 2.0
    gamma = beta.copy()
    return alpha, beta, gamma


def elu(x):
    x = np.asarray(x, dtype=np.float64)
    return np.where(x > 0.0, x, np.expm1(np.minimum(x, 0.0)))


def elu_params(l, u, x0):
    """ELU with unit scale (Table 3, Chebyshev).

    Identity when l >= 0.  Otherwise alpha is the chord slope; the upper error
    r_u is reached at the interval ends and the lower error r_l at the tangent
    point ln(alpha), where r_l = (alpha - 1) - alpha ln(alpha) (the printed r_l
    is garbled; this is the Chebyshev value the table's note names).  beta =
    (r_u + r_l)/2 and gamma = r_u - beta.

    When the interval is narrower than 1e-12 max(1, |x0|) the chord is replaced
    by the derivative at x0; r_u is then the larger of the two end errors (for
    the exact chord both ends give the same value)."""
    l = np.asarray(l, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    x0 = np.asarray(x0, dtype=np.float64)
    alpha = np.ones_like(l)
    beta = np.zeros_like(l)
    gamma = np.zeros_like(l)
    act = ~(l >= 0.0)
    if np.any(act):
        la, ua, ca = l[act], u[act], x0[act]
        w = ua - la
        small = w < 1e-12 * np.maximum(1.0, np.abs(ca))
        a = np.empty_like(la)
        ns = ~small
        a[ns] = (elu(ua[ns]) - elu(la[ns])) / w[ns]
        a[small] = np.where(ca[small] > 0.0, 1.0, np.exp(np.minimum(ca[small], 0.0)))
        r_u = np.maximum(elu(la) - a * la, elu(ua) - a * ua)
        r_l = (a - 1.0) - a * np.log(a)
        b = (r_u + r_l) / 2.0
        alpha[act] = a
        beta[act] = b
        gamma[act] = r_u - b
    return alpha, beta, gamma


def cos_range(l, u):
    """Minimum and maximum of cos on [l, u] via modular arithmetic: the end
    values, raised to 1 if some 2 pi j lies in [l, u] and lowered to -1 if some
    pi + 2 pi j does."""
    l = np.asarray(l, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    cl, cu = np.cos(l), np.cos(u)
    lo = np.minimum(cl, cu)
    hi = np.maximum(cl, cu)
    has_max = TWO_PI * np.ceil(l / TWO_PI) <= u
    has_min = TWO_PI * np.ceil((l - math.pi) / TWO_PI) + math.pi <= u
    hi = np.where(has_max, 1.0, hi)
    lo = np.where(has_min, -1.0, lo)
    return lo, hi


def sin_candidates(l, u, alpha):
    """Candidate extremal points of sin(x) - alpha x on [l, u] (Table 3): the
    two ends plus the first and last stationary point (cos x = alpha) of each
    of the two families +-e_p + 2 pi j inside the interval, clamped to it."""
    e_p = np.arccos(np.clip(alpha, -1.0, 1.0))
    e_n = -e_p
    c1 = TWO_PI * np.ceil((l + e_p) / TWO_PI) - e_p
    c2 = TWO_PI * np.ceil((l + e_n) / TWO_PI) - e_n
    c3 = TWO_PI * np.floor((u - e_p) / TWO_PI) + e_p
    c4 = TWO_PI * np.floor((u - e_n) / TWO_PI) + e_n
    cands = [l, u] + [np.clip(c, l, u) for c in (c1, c2, c3, c4)]
    return np.stack(cands, axis=0)


def sin_params(l, u):
    """sin (Table 3): alpha is the mean of the range of cos on [l, u]; r_u and
    r_l are the maximum and minimum of sin(e) - alpha e over the candidate set
    (the table prints "max" twice; the second is the minimum)."""
    l = np.asarray(l, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    s_lo, s_hi = cos_range(l, u)
    alpha = (s_lo + s_hi) / 2.0
    E = sin_candidates(l, u, alpha)
    vals = np.sin(E) - alpha[None] * E
    r_u = vals.max(axis=0)
    r_l = vals.min(axis=0)
    beta = (r_u + r_l) / 2.0
    gamma = r_u - beta
    return alpha, beta, gamma


def act_params(act, l, u, x0):
    if act == "relu":
        return relu_params(l, u)
    if act == "elu":
        return elu_params(l, u, x0)
    if act == "sin":
        return sin_params(l, u)
    raise ValueError(act)


def act_fn(act, x):
    if act == "relu":
        return np.maximum(x, 0.0)
    if act == "elu":
        return elu(x)
    if act == "sin":
        return np.sin(x)
    raise ValueError(act)


# ---------------------------------------------------------------------------
# Nonlinearity update (eq. affine_func_update; Table 2 "nonlinearities")
# ---------------------------------------------------------------------------

def apply_linearisation(x0, X, xinf, alpha, beta):
    """z0 = alpha x0 + beta, Z = diag(alpha) X, zinf = |alpha| xinf.  The new
    terms diag(gamma) are handled by the condensation policy."""
    return alpha * x0 + beta, alpha[:, :, None] * X, np.abs(alpha) * xinf


# ---------------------------------------------------------------------------
# Condensation policies (Section 3.3)
# ---------------------------------------------------------------------------

def condense_fixed(z0, Z, zinf, gamma):
    """affine-fixed: keep only the input-domain terms; every new term is
    condensed into the distinguished coefficient immediately."""
    return z0, Z, zinf + gamma


def condense_full(z0, Z, zinf, gamma):
    """affine-full: keep every term; one new column per neuron, diag(gamma)."""
    B, m, N = Z.shape
    G = np.zeros((B, m, m))
    idx = np.arange(m)
    G[:, idx, idx] = gamma
    return z0, np.concatenate([Z, G], axis=2), zinf


def truncate_select(mu, k):
    """Keep the k largest candidate magnitudes; ties go to the lower candidate
    index.  Returns a boolean keep mask [B, n_cand]."""
    B, n = mu.shape
    n_keep = min(k, n)
    order = np.argsort(-mu, axis=1, kind="stable")
    keep = np.zeros((B, n), dtype=bool)
    np.put_along_axis(keep, order[:, :n_keep], True, axis=1)
    return keep


def condense_truncate(z0, Z, zinf, gamma, k, keep=None):
    """affine-truncate(k): among the N old columns and the m new terms
    (gamma_j on neuron j) keep the k of largest magnitude and condense the rest
    (the condense operation of Section 3.3 adds their magnitudes to the
    distinguished coefficient, row by row).

    Magnitude of a term = L1 norm of its column.  Candidate order: old columns
    in their current order, then new terms by neuron index.  Layout after
    truncation: kept old columns stay in place; the kept new terms fill the
    freed positions (dropped old columns, then positions beyond the old width)
    in increasing order, by increasing neuron index.

    ``keep`` [B, N+m] replays a given selection instead of computing it.
    Returns (z0, Z', zinf', keep, src) where src[b, slot] = -1 for a kept old
    column and the neuron index for a new term.
    """
    B, m, N = Z.shape
    mu_old = np.abs(Z).sum(axis=1)
    mu = np.concatenate([mu_old, gamma], axis=1)
    if keep is None:
        keep = truncate_select(mu, k)
    keep = np.asarray(keep, dtype=bool)
    n_keep = int(keep[0].sum()) if B else min(k, N + m)
    if B and not np.all(keep.sum(axis=1) == n_keep):
        raise ValueError("kept counts differ between boxes")
    if n_keep < N:
        raise ValueError("k must be at least the number of input-domain terms")
    keep_old = keep[:, :N]
    keep_new = keep[:, N:]
    zinf = zinf + (np.abs(Z) * (~keep_old)[:, None, :]).sum(axis=2) + gamma * (~keep_new)
    width = n_keep
    Zn = np.zeros((B, m, width))
    Zn[:, :, :N] = Z * keep_old[:, None, :]
    free = np.ones((B, width), dtype=bool)
    free[:, :N] = ~keep_old
    free_order = np.argsort(~free, axis=1, kind="stable")
    new_order = np.argsort(~keep_new, axis=1, kind="stable")
    n_new = keep_new.sum(axis=1)
    src = np.full((B, width), -1, dtype=np.int64)
    bidx = np.arange(B)
    for i in range(width):
        valid = i < n_new
        if not np.any(valid):
            break
        b = bidx[valid]
        slot = free_order[valid, i]
        row = new_order[valid, i]
        Zn[b, row, slot] = gamma[b, row]
        src[b, slot] = row
    return z0, Zn, zinf, keep, src


# ---------------------------------------------------------------------------
# Interval arithmetic (Section 3.1) -- used for the interval-contains-affine
# invariant and as a comparator.
# ---------------------------------------------------------------------------

def ia_linear(l, u, W, b):
    """Interval image of W x + b as a sum of scaled intervals: each term
    W_jk [l_k, u_k] is [min, max] of its two end products."""
    W = np.asarray(W, dtype=np.float64)
    Wp = np.maximum(W, 0.0)
    Wn = np.minimum(W, 0.0)
    lo = l @ Wp.T + u @ Wn.T + b
    hi = u @ Wp.T + l @ Wn.T + b
    return lo, hi


def ia_act(act, l, u):
    if act in ("relu", "elu"):
        return act_fn(act, l), act_fn(act, u)   # monotone
    if act == "sin":
        # sin(x) = cos(x - pi/2): reuse the cos range on the shifted interval
        return cos_range(l - math.pi / 2.0, u - math.pi / 2.0)
    raise ValueError(act)
