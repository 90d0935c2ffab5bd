"""Differentiable unrolled l2 PDHG: forward recursion and reverse recursion.

TEST INFRASTRUCTURE ONLY (see the package docstring).

K steps of the preconditioned PDHG of "Preconditioned PDHG for simple
regularizers" with g = lambda ||x||^2/2, where the per-step sizes sigma_k,
tau_k, theta_k and lambda are free (learnable) real parameters:

  ax_k      = A xbar_k
  u_{k+1}   = (u_k + sigma_k p (ax_k - y)) / (1 + sigma_k p)
  ahu_k     = A^H u_{k+1}
  x_{k+1}   = (x_k - tau_k ahu_k) / (1 + tau_k lambda)
  xbar_{k+1}= x_{k+1} + theta_k (x_{k+1} - x_k)

with x_0 = xbar_0 = x0 (zeros by default) and u_0 = 0.  Loss
L = 1/2 ||x_K - x_gt||^2.

Gradient convention (PyTorch's, for a real loss of complex tensors):
grad z = dL/dRe z + i dL/dIm z.  For a complex-linear map v = M z the
vector-Jacobian product is M^H g_v; for a real parameter s multiplying w,
dL/ds = Re <g_v, dv/ds> = Re sum conj(g_v) dv/ds.

The reverse recursion below is derived by hand from the five lines above,
step by step in reverse order; it is pinned against float64 central finite
differences (tests/test_oracle_solver.py).
"""
from __future__ import annotations

import numpy as np


def _re(a, b):
    return float(np.vdot(a, b).real)


def forward(fwd, adj, y, p, sigma, tau, theta, lam, shape, x0=None, keep=True):
    """Run K steps; returns x_K and the per-step record for the reverse pass."""
    K = len(sigma)
    y = np.asarray(y, np.complex128)
    P = np.broadcast_to(np.asarray(p, np.float64), y.shape)
    x = np.zeros(shape, np.complex128) if x0 is None else np.array(x0, np.complex128)
    xbar = x.copy()
    u = np.zeros(y.shape, np.complex128)
    rec = []
    for k in range(K):
        ax = fwd(xbar)
        u_new = (u + sigma[k] * P * (ax - y)) / (1.0 + sigma[k] * P)
        ahu = adj(u_new)
        x_new = (x - tau[k] * ahu) / (1.0 + tau[k] * lam)
        xbar_new = x_new + theta[k] * (x_new - x)
        if keep:
            rec.append({"x": x, "u": u, "ax": ax, "u_new": u_new, "ahu": ahu, "x_new": x_new})
        x, xbar, u = x_new, xbar_new, u_new
    return x, rec


def loss(x, x_gt):
    r = x - x_gt
    return 0.5 * float(np.vdot(r, r).real)


def backward(fwd, adj, y, p, sigma, tau, theta, lam, rec, g_xK):
    """Reverse recursion. Returns dict of gradients (sigma, tau, theta, lam, y, x0)."""
    K = len(sigma)
    y = np.asarray(y, np.complex128)
    P = np.broadcast_to(np.asarray(p, np.float64), y.shape)
    gs = np.zeros(K)
    gt = np.zeros(K)
    gth = np.zeros(K)
    glam = 0.0
    gy = np.zeros(y.shape, np.complex128)
    gx = np.array(g_xK, np.complex128)          # grad wrt x_{k+1}
    gxb = np.zeros_like(gx)                     # grad wrt xbar_{k+1}
    gu = np.zeros(y.shape, np.complex128)       # grad wrt u_{k+1}
    for k in range(K - 1, -1, -1):
        r = rec[k]
        x, x_new, ahu, ax, u_new = r["x"], r["x_new"], r["ahu"], r["ax"], r["u_new"]
        # xbar_{k+1} = (1 + theta) x_{k+1} - theta x_k
        gth[k] = _re(gxb, x_new - x)
        gxt = gx + (1.0 + theta[k]) * gxb
        gx_prev = -theta[k] * gxb
        # x_{k+1} = (x_k - tau ahu) / (1 + tau lam)
        dd = 1.0 + tau[k] * lam
        gx_prev = gx_prev + gxt / dd
        g_ahu = -tau[k] * gxt / dd
        gt[k] = _re(gxt, (-ahu - lam * x_new) / dd)
        glam += _re(gxt, -tau[k] * x_new / dd)
        # ahu = A^H u_{k+1}
        gut = gu + fwd(g_ahu)
        # u_{k+1} = (u_k + sigma p (ax - y)) / (1 + sigma p)
        e = 1.0 + sigma[k] * P
        gu_prev = gut / e
        g_ax = sigma[k] * P * gut / e
        gy = gy - g_ax
        gs[k] = _re(gut, P * (ax - y - u_new) / e)
        # ax = A xbar_k
        gxb_prev = adj(g_ax)
        gx, gxb, gu = gx_prev, gxb_prev, gu_prev
    # x_0 = xbar_0 = x0
    gx0 = gx + gxb
    return {"sigma": gs, "tau": gt, "theta": gth, "lam": glam, "y": gy, "x0": gx0}
