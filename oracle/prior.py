"""Regularisers phi(D x) on one tile support (FP64).

D is the forward finite-difference operator (Section IV-A).  At the last
row/column the difference is 0 (Neumann, the default reading) or wraps to the
first row/column (the paper's circular D).

* Smoothed total variation: phi = sum_l ( sqrt(g_h^2 + g_v^2 + eps^2) - eps ).
  The -eps makes phi(constant) = 0 and does not move the minimiser.
* Huber (Section IV-A), applied per pixel to the isotropic gradient norm:
  phi = sum_l H_delta(|g(l)|) with H_delta(t) = t^2/2 for t <= delta and
  delta (t - delta/2) otherwise.  delta -> infinity gives (1/2)||D x||^2.
"""
from __future__ import annotations

import numpy as np


def forward_diff(x, bc="neumann"):
    """(g_h, g_v): horizontal and vertical forward differences of x."""
    gh = np.zeros_like(x)
    gv = np.zeros_like(x)
    gh[:, :-1] = x[:, 1:] - x[:, :-1]
    gv[:-1, :] = x[1:, :] - x[:-1, :]
    if bc == "circular":
        gh[:, -1] = x[:, 0] - x[:, -1]
        gv[-1, :] = x[0, :] - x[-1, :]
    elif bc != "neumann":
        raise ValueError(bc)
    return gh, gv


def forward_diff_adjoint(ph, pv, bc="neumann"):
    """D^T (ph, pv), the exact transpose of :func:`forward_diff`."""
    out = np.zeros_like(ph)
    if bc == "neumann":
        out[:, :-1] -= ph[:, :-1]
        out[:, 1:] += ph[:, :-1]
        out[:-1, :] -= pv[:-1, :]
        out[1:, :] += pv[:-1, :]
    else:
        out -= ph
        out += np.roll(ph, 1, axis=1)
        out -= pv
        out += np.roll(pv, 1, axis=0)
    return out


def value(x, kind, param, bc="neumann"):
    """phi(D x) for kind 'tv' (param = eps) or 'huber' (param = delta)."""
    gh, gv = forward_diff(x, bc)
    n2 = gh * gh + gv * gv
    if kind == "tv":
        return float(np.sum(np.sqrt(n2 + param * param) - param))
    if kind == "huber":
        n = np.sqrt(n2)
        return float(np.sum(np.where(n <= param, 0.5 * n2, param * (n - 0.5 * param))))
    raise ValueError(kind)


def gradient(x, kind, param, bc="neumann"):
    """grad_x phi(D x) = D^T (d phi / d g)."""
    gh, gv = forward_diff(x, bc)
    n2 = gh * gh + gv * gv
    if kind == "tv":
        s = 1.0 / np.sqrt(n2 + param * param)
    elif kind == "huber":
        n = np.sqrt(n2)
        s = param / np.maximum(n, param)
    else:
        raise ValueError(kind)
    return forward_diff_adjoint(s * gh, s * gv, bc)


def lipschitz(kind, param):
    """Bound on the Lipschitz constant of grad phi: ||D||^2 <= 8 times the
    curvature bound of the scalar penalty (1/eps for TV, 1 for Huber)."""
    if kind == "tv":
        return 8.0 / param
    if kind == "huber":
        return 8.0
    raise ValueError(kind)


def value_change(x, dx, kind, param, bc="neumann"):
    """phi(D (x + dx)) - phi(D x), summed per pixel in a form without
    cancellation: with a = D x and b = D (x + dx) = a + D dx,
    |b|^2 - |a|^2 = <D dx, a + b>, and
      smoothed TV: sqrt(|b|^2 + eps^2) - sqrt(|a|^2 + eps^2)
                   = (|b|^2 - |a|^2) / (sqrt(|b|^2 + eps^2) + sqrt(|a|^2 + eps^2));
      Huber: (|b|^2 - |a|^2) / 2 where both norms are <= delta,
             delta (|b|^2 - |a|^2) / (|b| + |a|) where both exceed it,
             the plain difference of the two pieces otherwise."""
    ah, av = forward_diff(x, bc)
    dh, dv = forward_diff(dx, bc)
    bh, bv = ah + dh, av + dv
    na2, nb2 = ah * ah + av * av, bh * bh + bv * bv
    diff = dh * (ah + bh) + dv * (av + bv)
    if kind == "tv":
        return float(np.sum(diff / (np.sqrt(nb2 + param * param) + np.sqrt(na2 + param * param))))
    if kind == "huber":
        na, nb = np.sqrt(na2), np.sqrt(nb2)
        ha = np.where(na <= param, 0.5 * na2, param * (na - 0.5 * param))
        hb = np.where(nb <= param, 0.5 * nb2, param * (nb - 0.5 * param))
        both_in = (na <= param) & (nb <= param)
        both_out = (na > param) & (nb > param)
        out = np.where(both_in, 0.5 * diff, hb - ha)
        out = np.where(both_out, param * diff / np.where(both_out, na + nb, 1.0), out)
        return float(np.sum(out))
    raise ValueError(kind)

