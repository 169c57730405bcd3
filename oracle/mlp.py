"""MLP evaluation and bound propagation in float64 (oracle; test
infrastructure only).

A network is a :class:`workloads.MLPSpec`: L linear layers, the activation
after every layer but the last.  For sine networks each hidden pre-activation
is first multiplied by omega0 (Table 2 constant multiplication), then passed
through sin.
"""
from __future__ import annotations

import numpy as np

from . import affine as aa

POLICIES = ("fixed", "truncate", "full")


def _w(net):
    return [np.asarray(W, dtype=np.float64) for W in net.weights], \
           [np.asarray(b, dtype=np.float64) for b in net.biases]


def forward(net, x):
    """Plain point evaluation f(x) for x [n, d] (the scalar evaluation the
    paper compares against).  Returns [n]."""
    Ws, bs = _w(net)
    h = np.asarray(x, dtype=np.float64)
    L = len(Ws)
    for l in range(L):
        h = h @ Ws[l].T + bs[l]
        if l < L - 1:
            if net.act == "sin":
                h = net.omega0 * h
            h = aa.act_fn(net.act, h)
    return h[:, 0]


def forward_torch(net, x, threads=None):
    """The same point evaluation as :func:`forward`, with PyTorch FP64 CPU
    operations (multi-threaded matrix products and activations), for large
    sample sets.  Returns a NumPy array [n]."""
    import torch
    if threads:
        torch.set_num_threads(int(threads))
    Ws, bs = _w(net)
    h = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))
    L = len(Ws)
    for l in range(L):
        h = torch.addmm(torch.from_numpy(bs[l]), h, torch.from_numpy(Ws[l]).T)
        if l < L - 1:
            if net.act == "sin":
                h = torch.sin(net.omega0 * h)
            elif net.act == "elu":
                h = torch.where(h > 0, h, torch.expm1(torch.clamp(h, max=0.0)))
            else:
                h = torch.clamp(h, min=0.0)
    return h[:, 0].numpy()


def propagate(net, x0, X, xinf, policy="truncate", k=31, keep_sets=None, record=None):
    """Push an affine form through the network (Section 3 rules; Appendix A).

    policy: "fixed", "truncate" (k kept terms) or "full".  ``keep_sets`` is an
    optional list (one per hidden activation) of keep masks to replay a given
    truncation choice.  If ``record`` is a list, per-activation diagnostics
    (keep masks, slot sources, pre-activation ranges) are appended to it.

    Returns the output affine form (y0 [B], Y [B, N], yinf [B]).
    """
    if policy not in POLICIES:
        raise ValueError(policy)
    Ws, bs = _w(net)
    L = len(Ws)
    for l in range(L):
        x0, X, xinf = aa.linear(x0, X, xinf, Ws[l], bs[l])
        if l == L - 1:
            break
        if net.act == "sin":
            x0, X, xinf = aa.mul_const(x0, X, xinf, net.omega0)
        lo, hi = aa.affine_range(x0, X, xinf)
        alpha, beta, gamma = aa.act_params(net.act, lo, hi, x0)
        z0, Z, zinf = aa.apply_linearisation(x0, X, xinf, alpha, beta)
        info = {"lo": lo, "hi": hi, "alpha": alpha, "beta": beta, "gamma": gamma}
        if policy == "fixed":
            x0, X, xinf = aa.condense_fixed(z0, Z, zinf, gamma)
        elif policy == "full":
            x0, X, xinf = aa.condense_full(z0, Z, zinf, gamma)
        else:
            keep = None if keep_sets is None else keep_sets[l]
            x0, X, xinf, keep, src = aa.condense_truncate(z0, Z, zinf, gamma, k, keep=keep)
            info["keep"] = keep
            info["src"] = src
            # candidate magnitudes (old columns, then new terms) for top-k checks
            info["mu"] = np.concatenate([np.abs(Z).sum(axis=1), gamma], axis=1)
        if record is not None:
            record.append(info)
    return x0[:, 0], X[:, 0, :], xinf[:, 0]


def bound_boxes(net, lo, hi, policy="truncate", k=31, keep_sets=None, record=None):
    """Range bound [lo_y, hi_y] of f over each axis-aligned box [lo, hi]
    (Procedure 1 steps 1-3).  Returns (center, radius, lo_y, hi_y)."""
    x0, X, xinf = aa.from_aabb(lo, hi)
    y0, Y, yinf = propagate(net, x0, X, xinf, policy, k, keep_sets, record)
    r = np.abs(Y).sum(axis=1) + yinf
    return y0, r, y0 - r, y0 + r


def bound_general(net, center, axes, policy="truncate", k=31):
    x0, X, xinf = aa.from_box(center, axes)
    y0, Y, yinf = propagate(net, x0, X, xinf, policy, k)
    r = np.abs(Y).sum(axis=1) + yinf
    return y0 - r, y0 + r


def bound_segments(net, p, r, t, sigma, policy="fixed", k=31):
    x0, X, xinf = aa.from_segment(p, r, t, sigma)
    y0, Y, yinf = propagate(net, x0, X, xinf, policy, k)
    rad = np.abs(Y).sum(axis=1) + yinf
    return y0 - rad, y0 + rad


def interval_bound_boxes(net, lo, hi):
    """Plain interval arithmetic through the network (Section 3.1)."""
    Ws, bs = _w(net)
    l = np.asarray(lo, dtype=np.float64)
    u = np.asarray(hi, dtype=np.float64)
    L = len(Ws)
    for i in range(L):
        l, u = aa.ia_linear(l, u, Ws[i], bs[i])
        if i == L - 1:
            break
        if net.act == "sin":
            l, u = net.omega0 * l, net.omega0 * u   # omega0 > 0
        l, u = aa.ia_act(net.act, l, u)
    return l[:, 0], u[:, 0]
