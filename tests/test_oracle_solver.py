"""Pins for the oracle's preconditioner, wavelet, PDHG and unrolled gradient."""
import math
import os

import numpy as np
import pytest

import synth
from oracle import ndft, nufft, pdhg, precond, unrolled, wavelet


def _rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _cartesian(shape):
    g = np.meshgrid(*[np.arange(n) - n // 2 for n in shape], indexing="ij")
    return np.stack([2 * math.pi * gi.ravel() / n for gi, n in zip(g, shape)], axis=1).astype(np.float32)


# ---------------------------------------------------------- preconditioner
@pytest.mark.parametrize("shape,C", [((6, 8), 3), ((4, 4, 6), 2)])
def test_precond_efficient_equals_definition(shape, C):
    rng = np.random.default_rng(0)
    k = synth.random_coords(60, len(shape), rng)
    maps = synth.coil_maps(shape, C, rng)
    pd = precond.definition(maps, k, shape)
    pe = precond.efficient_exact(maps, k, shape)
    np.testing.assert_allclose(pe, pd, rtol=1e-10)
    assert np.all(pd > 0)


def test_precond_sc_closed_form_equals_definition():
    rng = np.random.default_rng(1)
    shape = (8, 10)
    k = synth.random_coords(80, 2, rng)
    np.testing.assert_allclose(precond.sc_closed_form(k, shape), precond.definition(None, k, shape)[0], rtol=1e-8)
    np.testing.assert_allclose(precond.efficient_exact(None, k, shape)[0], precond.definition(None, k, shape)[0], rtol=1e-10)


def test_precond_cartesian_is_one():
    """Cartesian sampling: p = 1 for SC, and for MC with unit-SoS maps."""
    shape = (6, 8)
    k = _cartesian(shape)
    np.testing.assert_allclose(precond.sc_closed_form(k, shape), 1.0, rtol=1e-6)
    maps = synth.coil_maps(shape, 3, np.random.default_rng(2))
    np.testing.assert_allclose(precond.efficient_exact(maps, k, shape), 1.0, rtol=1e-5)


def test_precond_mc_single_unit_coil_equals_sc():
    rng = np.random.default_rng(3)
    shape = (8, 8)
    k = synth.random_coords(50, 2, rng)
    ones = np.ones((1,) + shape, np.complex128)
    np.testing.assert_allclose(precond.efficient_exact(ones, k, shape), precond.efficient_exact(None, k, shape), rtol=1e-12)


def test_precond_global_phase_invariance():
    rng = np.random.default_rng(4)
    shape = (6, 6)
    k = synth.random_coords(40, 2, rng)
    maps = synth.coil_maps(shape, 2, rng)
    p1 = precond.efficient_exact(maps, k, shape)
    p2 = precond.efficient_exact(maps * np.exp(1j * 0.7), k, shape)
    np.testing.assert_allclose(p1, p2, rtol=1e-12)


def test_precond_nufft_build_within_nufft_error():
    rng = np.random.default_rng(5)
    shape = (8, 10)
    k = synth.random_coords(120, 2, rng)
    maps = synth.coil_maps(shape, 3, rng)
    pd = precond.definition(maps, k, shape)
    pn = precond.efficient_nufft(maps, k, shape, 2.0, 6)
    assert np.max(np.abs(pn - pd) / pd) < 1e-3
    pn4 = precond.efficient_nufft(maps, k, shape, 1.25, 4)
    assert np.max(np.abs(pn4 - pd) / pd) < 5e-2


def test_dcf_duplicated_samples_halve():
    rng = np.random.default_rng(8)
    k = synth.random_coords(200, 2, rng)
    w1 = precond.pipe_menon_dcf(k, (12, 16), 1.25, 4)
    w2 = precond.pipe_menon_dcf(np.concatenate([k, k]), (12, 16), 1.25, 4)
    np.testing.assert_allclose(2 * w2[:200], w1, rtol=1e-12)
    np.testing.assert_allclose(2 * w2[200:], w1, rtol=1e-12)


@pytest.mark.parametrize("kk", [(0.3, -1.1), (-math.pi, 2.0), (1.7, 0.0, -0.4)])
def test_dcf_single_sample_from_kernel_taps(kk):
    from oracle import kb as okb
    k = np.array([kk], np.float32)
    shape = (16,) * len(kk)
    alpha, W = 1.25, 4
    G = nufft.grid_shape(shape, alpha)
    g = nufft.canonical_coords(k, G)[0].astype(np.float64)
    beta = okb.kb_beta(alpha, W)
    v = 1.0
    for a in range(len(kk)):
        j = np.floor(g[a]) - W // 2 + 1 + np.arange(W)
        v *= float(np.sum(okb.kb_kernel(g[a] - j, W, beta) ** 2))
    w = precond.pipe_menon_dcf(k, shape, alpha, W)
    np.testing.assert_allclose(w, [1.0 / v], rtol=1e-12)


def test_dcf_preconditioner_has_unit_lambda_max():
    from oracle import pdhg as opdhg
    rng = np.random.default_rng(9)
    shape = (12, 16)
    k = synth.random_coords(400, 2, rng)
    maps = synth.coil_maps(shape, 3, rng)
    p = precond.dcf_preconditioner(k, shape, maps, 1.25, 4)
    A = ndft.matrix(maps, k, shape)                       # dense (CM, N)
    Pb = np.tile(p, 3)                                    # one weight per sample, every coil
    lam = np.linalg.eigvalsh((A.conj().T * Pb) @ A).max()  # lambda_max(A^H P A) = lambda_max(P A A^H)
    # the power method on the gridding NUFFT: within its error of the exact A
    assert abs(lam - 1.0) < 2e-2, lam
    op = nufft.Nufft(k, shape, maps, 1.25, 4)
    assert abs(opdhg.power_method(op.forward, op.adjoint, p, shape, 30) - 1.0) < 1e-6


def test_dcf_equal_on_a_cartesian_grid():
    shape = (16, 16)
    w = precond.pipe_menon_dcf(_cartesian(shape), shape, 2.0, 4)   # samples on grid points
    assert (w.max() - w.min()) / w.mean() < 1e-2


def test_dcf_radial_grows_like_radius():
    k = synth.radial_2d(256, 128)
    w = precond.pipe_menon_dcf(k, (64, 64), 1.25, 4)
    r = np.linalg.norm(k.astype(np.float64), axis=1)
    m = (r > 0.25 * math.pi) & (r < 0.75 * math.pi)
    slope = np.polyfit(np.log(r[m]), np.log(w[m]), 1)[0]
    assert abs(slope - 1.0) < 0.05, slope
    # converged: the gridding kernel's self-convolution of w is ~1 at the samples
    op = nufft.Nufft(k, (64, 64), None, 1.25, 4)
    v = np.abs(op.interp(op.spread(w.astype(np.complex128))))
    assert np.median(np.abs(v - 1.0)) < 1e-2


# ---------------------------------------------------------------- wavelet
def test_db4_defining_identity():
    h = wavelet.db4_filter()
    assert len(h) == 8
    xi = np.random.default_rng(0).uniform(-math.pi, math.pi, 50)
    H = np.array([np.sum(h * np.exp(-1j * x * np.arange(8))) for x in xi])
    y = np.sin(xi / 2) ** 2
    P = 1 + 4 * y + 10 * y ** 2 + 20 * y ** 3
    np.testing.assert_allclose(np.abs(H) ** 2, 2 * np.cos(xi / 2) ** 8 * P, rtol=1e-12, atol=1e-14)
    assert abs(h[0]) > abs(h[-1])                       # minimum phase: energy first


def test_db4_orthonormal_and_vanishing_moments():
    h = wavelet.db4_filter()
    g = wavelet.highpass(h)
    for s in range(4):
        v = np.sum(h[2 * s:] * h[:8 - 2 * s])
        assert abs(v - (1.0 if s == 0 else 0.0)) < 1e-14
    t = np.arange(8)
    for m in range(4):
        assert abs(np.sum(g * t ** m)) < 1e-9 * max(1, 8 ** m)
    assert abs(np.sum(h) - math.sqrt(2)) < 1e-15


def test_db4_matches_published_table():
    """The derived filter equals Daubechies' printed N = 4 coefficients (16 decimals)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "db4_lowpass_daubechies.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    ref = np.array([float(v) for _, v in rows])
    assert [int(i) for i, _ in rows] == list(range(8))
    np.testing.assert_allclose(wavelet.db4_filter(), ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("shape,levels", [((16,), 2), ((16, 8), 2), ((8, 8, 16), 2)])
def test_wavelet_is_orthogonal(shape, levels):
    n = int(np.prod(shape))
    Wm = np.stack([wavelet.forward(np.eye(n)[i].reshape(shape), levels).ravel() for i in range(n)], axis=1)
    np.testing.assert_allclose(Wm.T @ Wm, np.eye(n), atol=1e-13)
    c = np.random.default_rng(1).standard_normal(shape)
    np.testing.assert_allclose(wavelet.inverse(c, levels).ravel(), Wm.T @ c.ravel(), atol=1e-13)


def test_wavelet_polynomial_has_zero_details():
    """A cubic signal gives zero detail coefficients away from the wrap."""
    x = (np.arange(64) / 64.0) ** 3
    c = wavelet.forward(x, 1)
    d = c[32:]
    assert np.max(np.abs(d[:28])) < 1e-12


def _band_mask(shape, levels):
    """True on the coarsest approximation block, False on every detail band."""
    m = np.zeros(shape, bool)
    m[tuple(slice(0, n >> levels) for n in shape)] = True
    return m


@pytest.mark.parametrize("shape,levels", [((64,), 4), ((32, 16), 2), ((32, 16), 3), ((16, 16, 32), 3),
                                          ((16, 16, 16), 4)])
def test_wavelet_constant_multilevel(shape, levels):
    """A constant c: every detail band of every level is zero (the filter has
    vanishing moments and the constant is periodic), and the coarsest
    approximation equals c 2^(d L / 2) (each level and axis multiplies it by
    sum h = sqrt 2).  Transforming anything but the approximation block at a
    level breaks both."""
    c = 0.7 - 0.3j
    out = wavelet.forward(np.full(shape, c), levels)
    m = _band_mask(shape, levels)
    np.testing.assert_allclose(out[m], c * 2.0 ** (len(shape) * levels / 2), rtol=1e-13)
    assert np.max(np.abs(out[~m])) < 1e-12
    np.testing.assert_allclose(wavelet.inverse(out, levels), np.full(shape, c), atol=1e-13)


def test_wavelet_cubic_details_zero_at_every_level():
    """A cubic along a 1D signal: away from the periodic wrap, the details of
    every level vanish (the approximation of a cubic is a cubic on the half
    grid, and db4 has four vanishing moments)."""
    n, levels = 256, 4
    x = (np.arange(n) / n - 0.3) ** 3 + 0.2 * (np.arange(n) / n)
    out = wavelet.forward(x, levels)
    L = n
    for lev in range(levels):
        half = L // 2
        d = out[half:L]
        # outputs whose 8-tap window wraps, or reaches an input the wrap has
        # already touched: the last 3, 5, 6, 6 of levels 1-4; 7 are skipped
        keep = half - 7
        assert keep > 8 and np.max(np.abs(d[:keep])) < 1e-12, lev
        L = half


def _dense_level(n, h):
    """One periodised analysis level as an n x n matrix, rows a[k] then d[k]."""
    g = wavelet.highpass(h)
    A = np.zeros((n, n))
    for k in range(n // 2):
        for t in range(len(h)):
            A[k, (2 * k + t) % n] += h[t]
            A[n // 2 + k, (2 * k + t) % n] += g[t]
    return A


@pytest.mark.parametrize("shape,levels", [((32,), 3), ((16, 8), 2), ((8, 8, 16), 2), ((16, 16), 3)])
def test_wavelet_multilevel_equals_dense_pyramid(shape, levels):
    """The multi-level transform built independently as a product of dense
    matrices: level l acts as the Kronecker product of the one-level matrices
    on the approximation block of level l - 1 (leading n/2^l entries of every
    axis) and as the identity on everything else."""
    h = wavelet.db4_filter()
    n = int(np.prod(shape))
    idx = np.arange(n).reshape(shape)
    Wt = np.eye(n)
    for lev in range(levels):
        sub = tuple(s >> lev for s in shape)
        K = np.ones((1, 1))
        for s in sub:
            K = np.kron(K, _dense_level(s, h))
        sel = idx[tuple(slice(0, s) for s in sub)].ravel()
        Ml = np.eye(n)
        Ml[np.ix_(sel, sel)] = K
        Wt = Ml @ Wt
    x = np.random.default_rng(3).standard_normal(shape) + 1j * np.random.default_rng(4).standard_normal(shape)
    np.testing.assert_allclose(wavelet.forward(x, levels).ravel(), Wt @ x.ravel(), atol=1e-12)
    np.testing.assert_allclose(wavelet.inverse(x, levels).ravel(), Wt.T @ x.ravel(), atol=1e-12)


def test_wavelet_level_recursion():
    """Level l equals the one-level transform of the level l - 1
    approximation block, with the detail bands of earlier levels untouched."""
    rng = np.random.default_rng(5)
    shape = (32, 16, 16)
    x = rng.standard_normal(shape)
    for levels in (2, 3, 4):
        full = wavelet.forward(x, levels)
        prev = wavelet.forward(x, levels - 1)
        blk = tuple(slice(0, s >> (levels - 1)) for s in shape)
        want = prev.copy()
        want[blk] = wavelet.forward(prev[blk], 1)
        np.testing.assert_allclose(full, want, atol=1e-13)


def test_soft_threshold_cases():
    v = np.array([0.0, 3 + 4j, 0.5j, -2.0])
    out = wavelet.soft(v, 1.0)
    np.testing.assert_allclose(out, [0.0, (3 + 4j) * 0.8, 0.0, -1.0])


# ------------------------------------------------------------------- PDHG
def _small_problem(C=3, seed=0, shape=(16, 16)):
    rng = np.random.default_rng(seed)
    k = synth.radial_2d(24, 32)
    maps = synth.coil_maps(shape, C, rng)
    x = synth.phantom(shape, rng)
    op = nufft.Nufft(k, shape, maps, 2.0, 4)
    y = op.forward(x) + synth.noise((C, k.shape[0]), 1e-3, rng)
    return op, y, k, maps, x


def test_power_method_matches_eigvalsh():
    rng = np.random.default_rng(1)
    shape = (6, 6)
    k = synth.random_coords(40, 2, rng)
    maps = synth.coil_maps(shape, 2, rng)
    A = ndft.matrix(maps, k, shape)
    p = precond.definition(maps, k, shape)
    M = A.conj().T @ (p.ravel()[:, None] * A)
    lam = np.linalg.eigvalsh(M)[-1]
    f = lambda v: ndft.forward(v, maps, k, shape)
    a = lambda u: ndft.adjoint(u, maps, k, shape)
    est = pdhg.power_method(f, a, p, shape, 300)
    assert abs(est - lam) < 1e-8 * lam
    est30 = pdhg.power_method(f, a, p, shape, 30)
    assert est30 <= lam * (1 + 1e-12) and est30 > 0.5 * lam
    lam_i = np.linalg.eigvalsh(A.conj().T @ A)[-1]
    assert abs(pdhg.power_method(f, a, None, shape, 300) - lam_i) < 1e-8 * lam_i
    assert abs(lam_i - np.linalg.norm(A, 2) ** 2) < 1e-10 * lam_i


def test_schedule_closed_form():
    """The accelerated schedule (theta_k = 1/(1 + 2 sigma_k gamma), sigma_{k+1}
    = theta_k sigma_k, tau_{k+1} = tau_k / theta_k, gamma = min p) solved in
    closed form: 1/sigma_{k+1} = 1/sigma_k + 2 gamma, so sigma_k =
    sigma_0 / (1 + 2 k gamma sigma_0), tau_k = tau_0 (1 + 2 k gamma sigma_0)
    and sigma_k tau_k stays sigma_0 tau_0 = 1 / lambda_max."""
    lam_max, gam, K = 4.0, 0.25, 7
    s, t, th = pdhg.schedule(lam_max, gam, K)
    k = np.arange(len(s))
    np.testing.assert_allclose(s, 1.0 / (1.0 + 2.0 * k * gam), rtol=1e-14)
    np.testing.assert_allclose(t, (1.0 + 2.0 * k * gam) / lam_max, rtol=1e-14)
    kk = np.arange(len(th))
    np.testing.assert_allclose(th, (1.0 + 2.0 * kk * gam) / (1.0 + 2.0 * (kk + 1) * gam), rtol=1e-14)
    np.testing.assert_allclose(s * t, 1.0 / lam_max, rtol=1e-14)


def test_pdhg_l2_converges_to_cg_and_gap_closes():
    op, y, k, maps, _ = _small_problem()
    lam = 1e-3
    shape = op.shape
    xs, info = pdhg.cg_l2(op.forward, op.adjoint, y, shape, lam)
    assert info == 0
    # the fixed-point relation x* = -A^H (A x* - y) / lam (sign-corrected Supplement)
    u_star = op.forward(xs) - y
    np.testing.assert_allclose(xs, -op.adjoint(u_star) / lam, rtol=0, atol=1e-6 * np.abs(xs).max())
    p = precond.efficient_nufft(maps, k, shape, 2.0, 4)
    gaps = []
    for iters in (50, 1500):
        x, u, _ = pdhg.pdhg(op.forward, op.adjoint, y, p, shape, "l2", lam, iters)
        gaps.append(pdhg.objective(op.forward, y, x, "l2", lam) - pdhg.dual_objective_l2(op.adjoint, y, u, lam))
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-4
    fx = pdhg.objective(op.forward, y, x, "l2", lam)
    assert 0 <= gaps[1] < 1e-4 * fx and gaps[1] < 0.05 * gaps[0]


def test_pdhg_preconditioning_beats_identity():
    op, y, k, maps, _ = _small_problem(seed=1)
    lam = 1e-3
    shape = op.shape
    xs, _ = pdhg.cg_l2(op.forward, op.adjoint, y, shape, lam)
    fstar = pdhg.objective(op.forward, y, xs, "l2", lam)
    res = {}
    for name, p in [("I", None), ("SC", precond.efficient_nufft(None, k, shape, 2.0, 4)[0]),
                    ("MC", precond.efficient_nufft(maps, k, shape, 2.0, 4))]:
        h = []
        pdhg.pdhg(op.forward, op.adjoint, y, p, shape, "l2", lam, 30, history=h)
        res[name] = h[-1] - fstar
        assert h[-1] < h[0]
    assert res["SC"] < 0.1 * res["I"] and res["MC"] < 0.1 * res["I"]


def test_pdhg_unitary_special_cases():
    """One coil, full Cartesian, p = 1: closed-form minimisers."""
    shape = (16, 16)
    rng = np.random.default_rng(2)
    k = _cartesian(shape)
    y = _rand_c(rng, (1, 256))
    f = lambda v: ndft.forward(v, None, k, shape)
    a = lambda u: ndft.adjoint(u, None, k, shape)
    ahy = a(y)
    lam = 0.3
    # float32 coordinates leave A unitary to ~1e-7, hence the 5e-6 bound
    x, _, info = pdhg.pdhg(f, a, y, None, shape, "l2", lam, 100, accel=False)
    np.testing.assert_allclose(x, ahy / (1 + lam), atol=5e-6)
    xa, _, info = pdhg.pdhg(f, a, y, None, shape, "l2", lam, 1600)   # O(1/k^2) schedule
    np.testing.assert_allclose(xa, ahy / (1 + lam), atol=2e-5)
    lam1 = 0.05
    x1, _, _ = pdhg.pdhg(f, a, y, None, shape, "l1wav", lam1, 200, levels=2, accel=False)
    want = wavelet.inverse(wavelet.soft(wavelet.forward(ahy, 2), lam1), 2)
    np.testing.assert_allclose(x1, want, atol=5e-6)


# ------------------------------------------------------ unrolled gradients
def test_unrolled_gradient_matches_finite_differences():
    op, y, k, maps, xgt = _small_problem(C=2, seed=3, shape=(8, 8))
    p = precond.efficient_nufft(maps, k, op.shape, 2.0, 4)
    K = 4
    sig = np.array([1.0, 0.8, 0.7, 0.6])
    lmax = pdhg.power_method(op.forward, op.adjoint, p, op.shape, 30)
    tau = np.array([0.5, 0.6, 0.7, 0.8]) / lmax
    th = np.array([0.9, 0.8, 0.85, 0.7])
    lam = 0.01
    x0 = 0.1 * _rand_c(np.random.default_rng(9), op.shape)

    def L(s, t, h, l, yy=y, xx=x0):
        xK, _ = unrolled.forward(op.forward, op.adjoint, yy, p, s, t, h, l, op.shape, x0=xx, keep=False)
        return unrolled.loss(xK, xgt)

    xK, rec = unrolled.forward(op.forward, op.adjoint, y, p, sig, tau, th, lam, op.shape, x0=x0)
    g = unrolled.backward(op.forward, op.adjoint, y, p, sig, tau, th, lam, rec, xK - xgt)
    eps = 1e-6
    for i in range(K):
        e = np.zeros(K)
        e[i] = eps
        for name, base, fn in [("sigma", sig, lambda v: L(v, tau, th, lam)),
                               ("tau", tau, lambda v: L(sig, v, th, lam)),
                               ("theta", th, lambda v: L(sig, tau, v, lam))]:
            h = eps * max(abs(base[i]), 1e-3)
            ee = np.zeros(K)
            ee[i] = h
            fd = (fn(base + ee) - fn(base - ee)) / (2 * h)
            assert abs(fd - g[name][i]) <= 1e-6 * max(1.0, abs(fd)), (name, i, fd, g[name][i])
    h = eps * lam
    fd = (L(sig, tau, th, lam + h) - L(sig, tau, th, lam - h)) / (2 * h)
    assert abs(fd - g["lam"]) <= 1e-5 * max(1.0, abs(fd))
    # complex inputs: directional derivatives along random directions
    rng = np.random.default_rng(10)
    for name, base, grad in [("y", y, g["y"]), ("x0", x0, g["x0"])]:
        dv = _rand_c(rng, base.shape)
        hh = 1e-6
        if name == "y":
            fd = (L(sig, tau, th, lam, yy=y + hh * dv) - L(sig, tau, th, lam, yy=y - hh * dv)) / (2 * hh)
        else:
            fd = (L(sig, tau, th, lam, xx=x0 + hh * dv) - L(sig, tau, th, lam, xx=x0 - hh * dv)) / (2 * hh)
        an = float(np.vdot(grad, dv).real)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, fd, an)


# ------------------------------------------------------------------- TV
from oracle import tv as otv  # noqa: E402


def test_tv_grad_is_adjoint_pair_and_kills_constants():
    rng = np.random.default_rng(40)
    for shape in [(6, 8), (4, 6, 10)]:
        x = _rand_c(rng, shape)
        v = _rand_c(rng, (len(shape),) + shape)
        lhs = np.vdot(otv.grad(x), v)
        rhs = np.vdot(x, otv.grad_adj(v))
        assert abs(lhs - rhs) < 1e-12 * abs(rhs)
        assert np.abs(otv.grad(np.full(shape, 2.0 - 1.0j))).max() == 0.0
    # loop by loop on a tiny array (periodic forward differences)
    x = _rand_c(rng, (3, 4))
    g = otv.grad(x)
    for i in range(3):
        for j in range(4):
            assert g[0, i, j] == x[(i + 1) % 3, j] - x[i, j]
            assert g[1, i, j] == x[i, (j + 1) % 4] - x[i, j]


def test_tv_lmax_matches_dense_spectrum():
    for shape in [(4, 6), (2, 4, 6), (5, 6)]:
        N = int(np.prod(shape))
        M = np.zeros((N, N), complex)
        for i in range(N):
            e = np.zeros(N, complex)
            e[i] = 1.0
            M[:, i] = otv.grad_adj(otv.grad(e.reshape(shape))).ravel()
        lam = float(np.linalg.eigvalsh(M).max())
        assert abs(lam - otv.lmax_gg(shape)) < 1e-10
        if all(n % 2 == 0 for n in shape):
            assert abs(lam - 4 * len(shape)) < 1e-10


def test_tv_pdhg_reaches_optimality():
    """Exact NDFT, one coil: after 3000 iterations the iterates satisfy the
    optimality conditions of 1/2||Ax - y||^2 + lam ||G x||_1, and the
    SC-preconditioned run finds the same minimiser."""
    shape = (8, 10)
    rng = np.random.default_rng(41)
    k = synth.random_coords(160, 2, rng, specials=False)
    f = lambda v: ndft.forward(v, None, k, shape)
    a = lambda u: ndft.adjoint(u, None, k, shape)
    y = f(synth.phantom(shape, rng)) + synth.noise((1, 160), 1e-2, rng)
    lam = 0.02
    hist = []
    x, _, v, _ = otv.tv_pdhg(f, a, y, None, shape, lam, 3000, history=hist)
    stat, feas, comp = otv.kkt_residuals(f, a, y, x, v, lam)
    assert stat < 1e-7 and feas <= 1e-12 and comp < 1e-6
    assert hist[-1] < hist[0]
    p = precond.sc_closed_form(k, shape)
    xp, _, vp, _ = otv.tv_pdhg(f, a, y, p, shape, lam, 3000)
    assert max(otv.kkt_residuals(f, a, y, xp, vp, lam)) < 1e-6
    assert np.linalg.norm(xp - x) < 1e-6 * np.linalg.norm(x)


def test_l2_dual_pcg_reaches_primal_solution():
    """The dual route gives the primal CG minimiser of (A^H A + lam I) x = A^H y
    (a different linear system), with and without the k-space preconditioner."""
    shape = (12, 14)
    rng = np.random.default_rng(51)
    C = 3
    k = synth.spiral_2d(6, 120, 2.0)
    maps = synth.coil_maps(shape, C, rng)
    f = lambda v: ndft.forward(v, maps, k, shape)
    a = lambda u: ndft.adjoint(u, maps, k, shape)
    y = f(synth.phantom(shape, rng)) + synth.noise((C, k.shape[0]), 1e-3, rng)
    lam = 0.1
    xc, _ = pdhg.cg_l2(f, a, y, shape, lam)
    for p in (None, precond.efficient_exact(None, k, shape)[0], precond.efficient_exact(maps, k, shape)):
        hist = []
        x, u = pdhg.l2_dual_pcg(f, a, y, p, shape, lam, 300, history=hist)
        assert np.linalg.norm(x - xc) < 1e-8 * np.linalg.norm(xc)
        # the dual optimality condition itself
        res = f(a(u)) + lam * u - lam * y
        assert np.linalg.norm(res) < 1e-8 * np.linalg.norm(lam * y)
        assert hist[0] == 1.0 and hist[-1] < 1e-8
