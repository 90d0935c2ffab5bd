"""l2-optimised diagonal k-space preconditioners (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "l2 optimized diagonal k-space preconditioners" and Appendix A:
p = argmin || diag(p) A A^H - I ||_F^2 gives, for every row a_i of A,

    p[i]^{-1} = sum_j |a_i^H a_j|^2 / ||a_i||^2.                  (definition)

Single channel (Eq. sc_precond), rows a_i[n] = e^{-i omega_i.n}/sqrt(N):
    p[i]^{-1} = sum_j prod_a D_{N_a}(f_ia - f_ja),
    D_N(f) = | sin(pi f) / (N sin(pi f / N)) |^2,  D_N(0) = 1,
with f = omega N / (2 pi) in cycles.  The printed prefactor 1/N is read as
1/N^2: only that value agrees with the general definition, with Eq.
mc_precond at C = 1, s = 1, and with the stated p = 1 for Cartesian sampling.

Multi channel (Eq. mc_precond), rows a_ci[n] = s_c[n] e^{-i omega_i.n}/sqrt(N):
    p_c[i]^{-1} = 1/(||s_c||^2 N) sum_j sum_d |sum_n s_c s_d^* e^{-i(omega_i-omega_j).n}|^2

Efficient build ("Efficient computation of the multi-channel preconditioner",
Fig. 2), in the paper's order:
  1. q_cd = s_c s_d^*;  r_cd[k] = sum_{m-n=k} conj(q_cd[n]) q_cd[m], computed
     as the inverse FFT of |FFT_{2N}(zero-padded q_cd)|^2.
  2. h[k] = N^{-1/2} sum_j e^{+i omega_j.k} (point-spread function).
  3. p_c[i]^{-1} = 1/(||s_c||^2 sqrt(N)) sum_k sum_d r_cd[k] h[k] e^{-i omega_i.k}.
  4. p = 1 / Re(p^{-1})  (the value is real up to rounding).
The lags k live on the centred 2N image (k_a in [-N_a, N_a)); the -N_a lag
of r is zero.  Steps 2 and 3 are sums over the trajectory: `efficient_exact`
evaluates them exactly (NDFT on the 2N image), `efficient_nufft` with the
gridding NUFFT on the 2N image using the plan's alpha and W.  SC is the same
build with C = 1 and s = 1, where r is the separable triangle prod(N_a - |k_a|).

Pipe-Menon density compensation (Experiments: the first of the three k-space
preconditioners compared with PDHG, from Pipe and Menon's gridding work):
the fixed-point iteration w <- w / |(C * C * w)(x_i)| from w = 1, where the
convolution with the gridding kernel C is evaluated by spreading w onto the
oversampled grid and interpolating back at the samples (the NUFFT's own
kernel, alpha and W), `pipe_menon_dcf`.  Readings (the paper gives no
details): 30 iterations, the plan's kernel and grid, one weight per sample
shared by every coil.  The raw weights have an arbitrary scale, and with the
dual step fixed (sigma0 = 1) the primal step tau = 1/lambda_max(P A A^H)
carries it into the proximal threshold; `dcf_preconditioner` therefore scales
them so that lambda_max(P A A^H) = 1 (power method, 30 iterations), the value
the l2-optimised preconditioners are designed to approach.

Pins: definition vs efficient_exact (1e-10); SC closed form vs definition;
Cartesian full sampling gives p = 1 (SC, and MC with unit sum-of-squares
maps); MC at C = 1, s = 1 equals SC; p > 0 and invariance to a global map
phase; efficient_nufft vs definition within the NUFFT error
(tests/test_oracle_solver.py).  DCF: duplicating every sample halves every
weight; a single sample's weight is 1 / prod_a sum_t C(u_at)^2 of the kernel
taps; the weights of a fully sampled Cartesian grid on the grid points are
equal; on a 2D radial trajectory they grow like |k| (log-log slope 1) in the
mid range.
"""
from __future__ import annotations

import math

import numpy as np

from . import ndft
from .nufft import Nufft


def definition(maps, coords, shape):
    """p from the dense Gram matrix (tiny problems). Shape (C, M)."""
    A = ndft.matrix(maps, coords, shape)          # (CM, N)
    gram = A @ A.conj().T                          # a_i^H a_j up to conjugation
    num = np.sum(np.abs(gram) ** 2, axis=1)
    den = np.sum(np.abs(A) ** 2, axis=1)
    C = 1 if maps is None else np.asarray(maps).shape[0]
    return (den / num).reshape(C, -1)


def sc_closed_form(coords, shape):
    """Single-channel p from the squared Dirichlet kernel. Shape (M,)."""
    k = np.asarray(coords, dtype=np.float64)
    M = k.shape[0]
    inv = np.ones((M, M))
    for a, n in enumerate(shape):
        f = k[:, a] * n / (2 * math.pi)
        df = f[:, None] - f[None, :]
        num = np.sin(math.pi * df)
        den = n * np.sin(math.pi * df / n)
        with np.errstate(invalid="ignore", divide="ignore"):
            D = np.where(np.abs(den) > 1e-300, (num / den) ** 2, 1.0)
        # the ratio tends to 1 where f_i - f_j is a multiple of N
        D = np.where(np.isclose(den, 0.0, atol=1e-14), 1.0, D)
        inv = inv * D
    return 1.0 / inv.sum(axis=1)


def autocorrelations(maps, shape):
    """r_c = sum_d r_cd on the centred 2N lag image, for every coil c."""
    shape = tuple(shape)
    d = len(shape)
    L = tuple(2 * n for n in shape)
    S = np.ones((1,) + shape, dtype=np.complex128) if maps is None else np.asarray(maps, np.complex128)
    C = S.shape[0]
    R = np.zeros((C,) + L)
    for c in range(C):
        for dd in range(C):
            q = S[c] * np.conj(S[dd])
            Q = np.fft.fftn(q, s=L, axes=tuple(range(d)))
            R[c] += np.abs(Q) ** 2
    r = np.stack([np.fft.ifftn(R[c]) for c in range(C)])   # circular lags k mod 2N
    # move lag k to centred index k + N
    for a in range(d):
        r = np.roll(r, shape[a], axis=a + 1)
    return r                                                # (C, *L), lag -N is ~0


def _norms(maps, shape):
    if maps is None:
        return np.array([float(np.prod(shape))])
    S = np.asarray(maps, np.complex128)
    return np.sum(np.abs(S.reshape(S.shape[0], -1)) ** 2, axis=1)


def efficient_exact(maps, coords, shape):
    """Efficient build with exact sums over the trajectory. Shape (C, M)."""
    shape = tuple(shape)
    d = len(shape)
    N = int(np.prod(shape))
    L = tuple(2 * n for n in shape)
    NL = int(np.prod(L))
    r = autocorrelations(maps, shape)
    M = np.asarray(coords).shape[0]
    # h[k] = N^{-1/2} sum_j e^{+i omega_j.k}; the NDFT adjoint on the 2N image
    # carries the factor NL^{-1/2}
    h = ndft.adjoint(np.ones((1, M)), None, coords, L) * math.sqrt(NL) / math.sqrt(N)
    nrm = _norms(maps, shape)
    out = []
    for c in range(r.shape[0]):
        v = r[c] * h
        s = ndft.forward(v, None, coords, L)[0] * math.sqrt(NL)   # sum_k v[k] e^{-i omega.k}
        out.append(np.real(s) / (nrm[c] * math.sqrt(N)))
    return 1.0 / np.stack(out)


def efficient_nufft(maps, coords, shape, alpha, width):
    """Efficient build with the gridding NUFFT on the 2N image. Shape (C, M)."""
    shape = tuple(shape)
    d = len(shape)
    L = tuple(2 * n for n in shape)
    r = autocorrelations(maps, shape)
    op = Nufft(coords, L, None, alpha, width)
    M = op.M
    h = op.adjoint(np.ones((1, M))) * math.sqrt(2.0 ** d)
    nrm = _norms(maps, shape)
    out = []
    for c in range(r.shape[0]):
        v = r[c] * h
        s = op.forward(v)[0] * math.sqrt(2.0 ** d)
        out.append(np.real(s) / nrm[c])
    return 1.0 / np.stack(out)


def pipe_menon_dcf(coords, shape, alpha, width, iters=30, op=None):
    """Pipe-Menon density compensation weights, shape (M,): w <- w / |G G^T w|
    with G the gridding interpolation (kernel taps onto the oversampled grid),
    `iters` times from w = 1.  `op`: an oracle Nufft already built on the same
    coordinates, shape, alpha and width (its taps are reused; maps play no
    part).  The weights are real, so spreading and interpolation run on real
    arrays."""
    if op is None:
        op = Nufft(coords, shape, None, alpha, width)
    size = int(np.prod(op.G))
    w = np.ones(op.M)
    for _ in range(iters):
        grid = np.zeros(size)
        for flat, t in op._taps:
            grid += np.bincount(flat, weights=t * w, minlength=size)
        v = np.zeros(op.M)
        for flat, t in op._taps:
            v += t * grid[flat]
        w = w / np.abs(v)
    return w


def dcf_preconditioner(coords, shape, maps, alpha, width, iters=30, power_iters=30):
    """Pipe-Menon weights scaled to lambda_max(P A A^H) = 1, shape (M,)."""
    from .pdhg import power_method
    w = pipe_menon_dcf(coords, shape, alpha, width, iters)
    op = Nufft(coords, shape, maps, alpha, width)
    return w / power_method(op.forward, op.adjoint, w, shape, power_iters)
