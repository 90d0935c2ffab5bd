"""Total-variation regularised PDHG (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "Preconditioned PDHG for simple regularizers composed with linear
operators": g(x) = h(G x) with G the finite-difference operator and
h = lambda ||.||_1, solved with a second dual variable v for G x:

  u     <- (I + sigma P)^{-1} (u + sigma P (A xbar - y))
  v     <- prox_{sigma h*}(v + sigma G xbar)
  x_new <- x - tau (A^H u + G^H v)
  xbar  <- x_new + theta (x_new - x)

with constant steps sigma = theta = 1 and
tau = 1 / (lambda_max(P A A^H) + lambda_max(G G^H)).

Readings (the paper is silent or garbled on these):
  * G: periodic forward differences along every image axis, stacked over the
    axes, (G x)_a[n] = x[n + e_a] - x[n]; G^H v = sum_a v_a[n - e_a] - v_a[n].
  * h = lambda sum |.| over every component of G x (anisotropic TV, complex
    modulus per component).
  * The printed dual step reads prox_{tau h}; the dual update of PDHG takes
    the prox of sigma h*, the conjugate, which for h = lambda ||.||_1 is the
    projection onto {|v_i| <= lambda} (independent of sigma).
  * lambda_max(G G^H) = sum_a max_k 2 (1 - cos(2 pi k / N_a)), which is 4 d
    when every N_a is even.
  * Initial values x = xbar = 0, u = 0, v = 0.

Pins (tests/test_oracle_solver.py): G^H is the adjoint of G (dot test);
G kills constants and matches a loop-by-loop difference on a tiny array;
lambda_max(G^H G) of the dense matrix equals the closed form; after many
iterations the iterates satisfy the optimality conditions of
min 1/2 ||A x - y||^2 + lambda ||G x||_1 (stationarity, |v| <= lambda and
Re <v, G x> = lambda ||G x||_1).
"""
import numpy as np

from . import pdhg as _pdhg


def grad(x):
    """Periodic forward differences, shape (d, *x.shape)."""
    x = np.asarray(x)
    return np.stack([np.roll(x, -1, axis=a) - x for a in range(x.ndim)])


def grad_adj(v):
    """Adjoint of grad: sum_a v_a[n - e_a] - v_a[n]."""
    v = np.asarray(v)
    return sum(np.roll(v[a], 1, axis=a) - v[a] for a in range(v.shape[0]))


def lmax_gg(shape):
    """lambda_max(G G^H) in closed form."""
    tot = 0.0
    for n in shape:
        k = np.arange(n)
        tot += float(np.max(2.0 * (1.0 - np.cos(2.0 * np.pi * k / n))))
    return tot


def project(v, lam):
    """prox of sigma h* for h = lam ||.||_1: projection onto |v_i| <= lam."""
    mag = np.abs(v)
    return v / np.maximum(1.0, mag / lam)


def tv(x, lam):
    return lam * float(np.sum(np.abs(grad(x))))


def objective(fwd, y, x, lam):
    r = fwd(x) - y
    return 0.5 * float(np.vdot(r, r).real) + tv(x, lam)


def tv_pdhg(fwd, adj, y, p, shape, lam, iters, lmax=None, power_iters=30, history=None):
    """Run the TV PDHG; returns (x, u, v, info)."""
    y = np.asarray(y, dtype=np.complex128)
    P = np.ones(y.shape) if p is None else np.broadcast_to(np.asarray(p, np.float64), y.shape)
    if lmax is None:
        lmax = _pdhg.power_method(fwd, adj, None if p is None else P, shape, power_iters)
    sigma, theta = 1.0, 1.0
    tau = 1.0 / (lmax + lmax_gg(shape))
    x = np.zeros(shape, np.complex128)
    xbar = x.copy()
    u = np.zeros(y.shape, np.complex128)
    v = np.zeros((len(shape),) + tuple(shape), np.complex128)
    if history is not None:
        history.append(objective(fwd, y, x, lam))
    for _ in range(iters):
        u = (u + sigma * P * (fwd(xbar) - y)) / (1.0 + sigma * P)
        v = project(v + sigma * grad(xbar), lam)
        x_new = x - tau * (adj(u) + grad_adj(v))
        xbar = x_new + theta * (x_new - x)
        x = x_new
        if history is not None:
            history.append(objective(fwd, y, x, lam))
    return x, u, v, {"lmax": lmax, "tau": tau}


def kkt_residuals(fwd, adj, y, x, v, lam):
    """Relative violations of the optimality conditions at (x, v)."""
    g = grad(x)
    stat = adj(fwd(x) - np.asarray(y)) + grad_adj(v)
    ref = np.linalg.norm(adj(np.asarray(y)))
    feas = max(0.0, float(np.max(np.abs(v))) / lam - 1.0)
    tvx = lam * float(np.sum(np.abs(g)))
    comp = abs(float(np.vdot(v, g).real) - tvx) / max(tvx, 1e-300)
    return float(np.linalg.norm(stat) / ref), feas, comp


__all__ = ["grad", "grad_adj", "lmax_gg", "project", "tv", "objective", "tv_pdhg", "kkt_residuals"]
