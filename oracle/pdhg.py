"""Power method, step schedule and diagonally preconditioned PDHG (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Operators are passed as a pair of callables (fwd, adj) acting on an image of
the problem's shape and on coil-major k-space of shape (C, M), so the same
solver runs with the exact NDFT or the gridding NUFFT.

Objective (Problem Setup, Eq. obj):  1/2 ||A x - y||^2 + g(x), with
  g = lambda ||x||^2 / 2              (l2)
  g = lambda ||W x||_1                (l1-wavelet, W unitary)

PDHG for simple g ("Preconditioned PDHG for simple regularizers"), one
iteration k:
  u     <- (I + sigma P)^{-1} (u + sigma P (A xbar - y))
  x_new <- prox_{tau g}(x - tau A^H u)
  xbar  <- x_new + theta (x_new - x)
with sigma_0 = 1, tau_0 = 1/lambda_max(P A A^H) and, for the accelerated
schedule, theta_k = 1 / (1 + 2 sigma_k min_i p_i), sigma_{k+1} = theta_k
sigma_k, tau_{k+1} = tau_k / theta_k (printed without a square root; read as
printed).  theta_k is evaluated with the sigma of the same iteration, after
the dual and primal updates of that iteration.  Constant steps (theta = 1)
are available as accel=False.  Initial values (unstated in the paper):
x = xbar = 0 and u = 0 unless given.

lambda_max(P A A^H) equals lambda_max(A^H P A) (same non-zero spectrum), and
is estimated with the power method on A^H P A for 30 iterations (Experiments
section): v_0 = ones / ||ones||, w = A^H P A v_k, lambda_k = ||w||,
v_{k+1} = w / lambda_k; the estimate is the last lambda_k.

Dual objective (Supporting Materials, convex dual), in the sign convention of
the PDHG iterate u (which tends to A x* - y):
  D(u) = -1/2 ||u||^2 - Re<u, y> - g*(-A^H u),   g* = ||.||^2/(2 lambda) for l2.
The Supporting Materials write x = A^H u / lambda for their dual variable;
with the PDHG sign, u* = A x* - y and x* = -A^H u* / lambda.

l2 dual solver (Supporting Materials, connection to Trzasko et al.): the dual
optimum of the l2 problem solves (A A^H + lambda I) u = lambda y and gives
x = A^H u / lambda; `l2_dual_pcg` solves it by conjugate gradients with the
k-space preconditioner P as M^-1.  (The Supplement's u is the negative of the
PDHG iterate u; its printed relation A x = u + y reads A x = y - u in its own
sign, which is what x = A^H u / lambda and the optimality condition give.)

Pins: power method vs eigvalsh of the dense A^H P A; l2 PDHG converges to the
CG solution of (A^H A + lambda I) x = A^H y; duality gap -> 0; the unitary
special case (single coil, full Cartesian, p = 1) matches the closed-form
proximal solutions; preconditioned runs end below the unpreconditioned run;
the dual PCG reaches the primal CG solution with and without P, and P cuts
the iterations it needs (tests/test_oracle_solver.py).
"""
from __future__ import annotations

import math

import numpy as np

from . import wavelet


def power_method(fwd, adj, p, shape, iters: int = 30):
    v = np.ones(shape, dtype=np.complex128)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        k = fwd(v)
        if p is not None:
            k = p * k
        w = adj(k)
        lam = float(np.linalg.norm(w))
        v = w / lam
    return lam


def schedule(lmax: float, pmin: float, iters: int, sigma0: float = 1.0, accel: bool = True):
    """(sigma_k, tau_k, theta_k) for k = 0..iters-1."""
    sig = np.empty(iters)
    tau = np.empty(iters)
    th = np.empty(iters)
    s, t = float(sigma0), 1.0 / (float(sigma0) * float(lmax))
    for k in range(iters):
        sig[k], tau[k] = s, t
        th[k] = 1.0 / (1.0 + 2.0 * s * pmin) if accel else 1.0
        s, t = th[k] * s, t / th[k]
    return sig, tau, th


def prox_l2(z, t, lam):
    return z / (1.0 + t * lam)


def prox_l1wav(z, t, lam, levels=4):
    return wavelet.inverse(wavelet.soft(wavelet.forward(z, levels), t * lam), levels)


def make_prox(reg: str, lam: float, levels: int = 4):
    if reg == "l2":
        return lambda z, t: prox_l2(z, t, lam)
    if reg == "l1wav":
        return lambda z, t: prox_l1wav(z, t, lam, levels)
    raise ValueError(reg)


def regulariser(reg, lam, x, levels=4):
    if reg == "l2":
        return 0.5 * lam * float(np.vdot(x, x).real)
    if reg == "l1wav":
        return lam * float(np.sum(np.abs(wavelet.forward(x, levels))))
    raise ValueError(reg)


def objective(fwd, y, x, reg, lam, levels=4):
    r = fwd(x) - y
    return 0.5 * float(np.vdot(r, r).real) + regulariser(reg, lam, x, levels)


def dual_objective_l2(adj, y, u, lam):
    ahu = adj(u)
    return (-0.5 * float(np.vdot(u, u).real) - float(np.vdot(u, y).real)
            - float(np.vdot(ahu, ahu).real) / (2.0 * lam))


def pdhg(fwd, adj, y, p, shape, reg, lam, iters, lmax=None, power_iters=30,
         sigma0=1.0, accel=True, levels=4, x0=None, u0=None, history=None):
    """Run the preconditioned PDHG; returns (x, u, info)."""
    y = np.asarray(y, dtype=np.complex128)
    P = np.ones(y.shape) if p is None else np.broadcast_to(np.asarray(p, np.float64), y.shape)
    if lmax is None:
        lmax = power_method(fwd, adj, None if p is None else P, shape, power_iters)
    pmin = float(P.min())
    sig, tau, th = schedule(lmax, pmin, iters, sigma0, accel)
    prox = make_prox(reg, lam, levels)
    x = np.zeros(shape, np.complex128) if x0 is None else np.array(x0, np.complex128).reshape(shape)
    xbar = x.copy()
    u = np.zeros(y.shape, np.complex128) if u0 is None else np.array(u0, np.complex128)
    if history is not None:
        history.append(objective(fwd, y, x, reg, lam, levels))
    for k in range(iters):
        u = (u + sig[k] * P * (fwd(xbar) - y)) / (1.0 + sig[k] * P)
        x_new = prox(x - tau[k] * adj(u), tau[k])
        xbar = x_new + th[k] * (x_new - x)
        x = x_new
        if history is not None:
            history.append(objective(fwd, y, x, reg, lam, levels))
    return x, u, {"lmax": lmax, "pmin": pmin, "sigma": sig, "tau": tau, "theta": th}


def cg_l2(fwd, adj, y, shape, lam, tol=1e-13, maxiter=5000):
    """x* of (A^H A + lam I) x = A^H y by scipy's conjugate gradient."""
    from scipy.sparse.linalg import LinearOperator, cg
    N = int(np.prod(shape))

    def mv(v):
        v = v.reshape(shape)
        return (adj(fwd(v)) + lam * v).ravel()

    op = LinearOperator((N, N), matvec=mv, dtype=np.complex128)
    b = adj(np.asarray(y, np.complex128)).ravel()
    x, info = cg(op, b, rtol=tol, atol=0.0, maxiter=maxiter)
    return x.reshape(shape), info


def l2_dual_pcg(fwd, adj, y, p, shape, lam, iters, history=None):
    """l2-regularised reconstruction through its dual (Supporting Materials,
    connection to Trzasko et al.): the dual optimum solves
    (A A^H + lam I) u = lam y, and x = A^H u / lam.  Solved with conjugate
    gradients preconditioned by the diagonal k-space preconditioner P
    (M^-1 = P; P = I when p is None), u_0 = 0.  Returns (x, u); `history`
    receives the relative residual ||r_k|| / ||r_0|| before every iteration
    and after the last."""
    y = np.asarray(y, dtype=np.complex128)
    P = np.ones(y.shape) if p is None else np.broadcast_to(np.asarray(p, np.float64), y.shape)
    H = lambda v: fwd(adj(v)) + lam * v
    u = np.zeros(y.shape, np.complex128)
    r = lam * y
    z = P * r
    d = z.copy()
    rz = float(np.vdot(r, z).real)
    r0 = float(np.linalg.norm(r))
    for _ in range(iters):
        if history is not None:
            history.append(float(np.linalg.norm(r)) / r0)
        q = H(d)
        alpha = rz / float(np.vdot(d, q).real)
        u = u + alpha * d
        r = r - alpha * q
        z = P * r
        rz_new = float(np.vdot(r, z).real)
        d = z + (rz_new / rz) * d
        rz = rz_new
    if history is not None:
        history.append(float(np.linalg.norm(r)) / r0)
    return adj(u) / lam, u
