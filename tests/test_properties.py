"""Property tests (hypothesis) over random problem shapes, trajectories with
awkward samples and random coil maps.

CPU (oracle): linearity and adjointness of the gridding NUFFT, its closeness
to the exact NDFT, and positivity / coil-phase invariance of the
preconditioner.  GPU: the library's forward and adjoint against the oracle
within 1e-4, its adjoint identity, and its bit-exact sort, on the same random
problems (fewer examples: each builds a plan)."""
import math

import numpy as np
import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import HealthCheck, given, settings  # noqa: E402
from hypothesis import strategies as st  # noqa: E402

import synth  # noqa: E402
from oracle import ndft, nufft, precond  # noqa: E402

EVEN = [4, 6, 8, 10, 12, 16, 20]


@st.composite
def problems(draw, max_m=300, dims=(2, 3)):
    d = draw(st.sampled_from(dims))
    shape = tuple(draw(st.sampled_from(EVEN if d == 2 else EVEN[:5])) for _ in range(d))
    C = draw(st.integers(1, 3))
    M = draw(st.integers(8 * d, max_m))
    alpha = draw(st.sampled_from([1.25, 2.0]))
    W = draw(st.sampled_from([2, 4, 6]))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.default_rng(seed)
    k = synth.random_coords(M, d, rng)                       # k = 0, -pi, just below pi, on grid lines
    axis = draw(st.booleans())
    if axis:                                                   # a few samples on the axes (integer grid coords)
        k[8 * d: 8 * d + 4, 1:] = 0.0
    maps = synth.coil_maps(shape, C, rng) if C > 1 else None
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    y = rng.standard_normal((C, M)) + 1j * rng.standard_normal((C, M))
    return shape, k, maps, alpha, W, x, y, rng


SET = settings(max_examples=25, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])


@SET
@given(problems())
def test_oracle_nufft_linear_and_adjoint(pb):
    shape, k, maps, alpha, W, x, y, rng = pb
    op = nufft.Nufft(k, shape, maps, alpha, W)
    x2 = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    a, b = 0.3 - 1.1j, 2.0 + 0.5j
    lhs = op.forward(a * x + b * x2)
    rhs = a * op.forward(x) + b * op.forward(x2)
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(rhs)
    p1 = np.vdot(op.forward(x), y)
    p2 = np.vdot(x, op.adjoint(y))
    assert abs(p1 - p2) <= 1e-12 * max(abs(p1), 1e-300)


@SET
@given(problems(dims=(2,)))
def test_oracle_nufft_close_to_ndft(pb):
    shape, k, maps, alpha, W, x, y, rng = pb
    if W == 2:      # a two-tap kernel is no approximation worth a bound
        return
    ye = ndft.forward(x, maps, k, shape)
    yn = nufft.Nufft(k, shape, maps, alpha, W).forward(x)
    # the gridding error of each (alpha, W) on random 2D problems is about
    # 7e-3 / 7e-4 (W 4) and 5e-4 / 3e-5 (W 6) for alpha 1.25 / 2, at most
    # 9.5e-3 / 1.4e-3 and 9.6e-4 / 1.1e-5 over 400 random problems; the
    # bounds leave room for the spread of small sample counts
    bound = {(1.25, 4): 0.04, (2.0, 4): 5e-3, (1.25, 6): 4e-3, (2.0, 6): 3e-4}
    assert np.linalg.norm(yn - ye) <= bound[(alpha, W)] * np.linalg.norm(ye)


@settings(max_examples=15, deadline=None, derandomize=True)
@given(st.integers(0, 2 ** 31 - 1), st.sampled_from([(6, 8), (8, 8), (4, 4, 6)]), st.integers(1, 3),
       st.floats(0.0, 2 * math.pi))
def test_oracle_precond_positive_and_phase_invariant(seed, shape, C, phi):
    rng = np.random.default_rng(seed)
    k = synth.random_coords(40, len(shape), rng)
    maps = synth.coil_maps(shape, C, rng) if C > 1 else None
    p = precond.efficient_exact(maps, k, shape)
    assert np.all(np.isfinite(p)) and np.all(p > 0)
    if maps is not None:
        q = precond.efficient_exact(maps * np.exp(1j * phi), k, shape)
        np.testing.assert_allclose(p, q, rtol=1e-10)


# ------------------------------------------------------------------- GPU
def _kp():
    import paper_1902_09657_amd as kp
    return kp


def _dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


GSET = settings(max_examples=12, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])


@pytest.mark.gpu
@GSET
@given(problems(max_m=3000))
def test_gpu_nufft_matches_oracle(pb):
    import torch
    kp = _kp()
    shape, k, maps, alpha, W, x, y, rng = pb
    C = 1 if maps is None else maps.shape[0]
    print("property case", shape, C, k.shape[0], alpha, W, flush=True)
    op = nufft.Nufft(k, shape, maps, alpha, W)
    plan = kp.nufft_plan(_dev(k, torch.float32), shape, None if maps is None else _dev(maps, torch.complex64),
                         oversamp=alpha, kb_width=W)
    xt, yt = _dev(x, torch.complex64), _dev(y, torch.complex64)
    yg = kp.nufft_forward(plan, xt)
    xg = kp.nufft_adjoint(plan, yt)
    yo, xo = op.forward(x), op.adjoint(y)
    assert np.linalg.norm(yg.cpu().numpy() - yo) <= 1e-4 * np.linalg.norm(yo)
    assert np.linalg.norm(xg.cpu().numpy() - xo) <= 1e-4 * np.linalg.norm(xo)
    # adjoint identity of the library's own pair (float32 arithmetic)
    lhs = torch.vdot(yg.flatten().to(torch.complex128), yt.flatten().to(torch.complex128)).item()
    rhs = torch.vdot(xt.flatten().to(torch.complex128), xg.flatten().to(torch.complex128)).item()
    assert abs(lhs - rhs) <= 1e-5 * abs(rhs)
    # the sort is bit-exact
    info = plan.info()
    g = nufft.canonical_coords(k, nufft.grid_shape(shape, alpha))
    perm_o, off_o = nufft.sort_by_bin(g, info["grid"], info["bin_size"])
    perm, boff, _, _ = [t.cpu().numpy() for t in plan.sort()]
    assert np.array_equal(perm, perm_o) and np.array_equal(boff, off_o)
    plan.close()
