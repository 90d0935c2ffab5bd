"""GPU parity of the plan, forward and adjoint NUFFT against the FP64 oracle.

Bars: the sort (permutation, bin offsets, tile touch lists) and the float32
canonical grid coordinates are bit-exact; floating-point outputs match within
1e-4 relative L2 (typically ~1e-6).
"""
import math

import numpy as np
import pytest

import synth
from oracle import nufft as onufft

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _kp():
    import paper_1902_09657_amd as kp
    return kp


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def case(shape, C, M, seed, alpha, W, specials=True):
    rng = np.random.default_rng(seed)
    d = len(shape)
    k = synth.random_coords(M, d, rng, specials=specials)
    maps = synth.coil_maps(shape, C, rng) if C > 1 else None
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    y = rng.standard_normal((C, M)) + 1j * rng.standard_normal((C, M))
    return k, maps, x, y


CASES = [
    # shape, C, M, alpha, W
    ((40, 48), 3, 3000, 1.25, 4),
    ((32, 32), 1, 1500, 2.0, 4),
    ((30, 22), 2, 777, 2.0, 6),
    ((16, 20, 24), 2, 4000, 1.25, 4),
    ((12, 10, 8), 4, 1000, 2.0, 2),
    ((24, 24), 8, 2049, 1.25, 8),
    # grids of the specialised FFT lengths (160, 200, 256, 400)
    ((160, 128), 8, 20000, 1.25, 4),
    ((128, 200), 1, 20000, 2.0, 4),
    ((128, 128, 160), 2, 30000, 1.25, 4),
    # register-resident passes along axes 0 and 1 (lengths 200, 240, 256)
    ((24, 160, 24), 2, 8000, 1.25, 4),
    ((192, 24, 24), 2, 8000, 1.25, 4),
    ((128, 24, 40), 2, 8000, 2.0, 4),
    # and along the coil-map axis (fused coil multiply / coil sum), C = 8, 4, 1
    ((16, 16, 128), 8, 4000, 1.25, 4),
    ((16, 24, 192), 4, 4000, 1.25, 4),
    ((24, 16, 160), 1, 3000, 1.25, 4),
    # 3D, coils in groups of four (the tap-lane interpolation)
    ((24, 32, 40), 4, 6000, 1.25, 4),
    ((40, 36, 44), 8, 30000, 1.25, 4),
    # three and four coil groups per piece (blocks dealt to (piece, group) pairs)
    ((24, 24, 32), 12, 5000, 1.25, 4),
    ((16, 24, 24), 16, 3000, 1.25, 4),
]


def _plan(kp, k, shape, maps, alpha, W, **kw):
    m = None if maps is None else dev(maps, torch.complex64)
    return kp.nufft_plan(dev(k, torch.float32), shape, m, oversamp=alpha, kb_width=W, **kw)


@pytest.mark.parametrize("shape,C,M,alpha,W", CASES)
def test_grid_coords_and_sort_bit_exact(shape, C, M, alpha, W):
    kp = _kp()
    k, maps, _, _ = case(shape, C, M, 11, alpha, W)
    print("case", shape, C, M, alpha, W, flush=True)
    plan = _plan(kp, k, shape, maps, alpha, W)
    info = plan.info()
    G = onufft.grid_shape(shape, alpha)
    assert tuple(info["grid"]) == G
    g_or = onufft.canonical_coords(k, G)
    g_gpu = plan.grid_coords().cpu().numpy()
    assert np.array_equal(g_gpu.view(np.uint32), g_or.view(np.uint32))
    B = info["bin_size"]
    perm_o, off_o = onufft.sort_by_bin(g_or, G, B)
    perm, boff, toff, touch = [t.cpu().numpy() for t in plan.sort()]
    assert np.array_equal(perm, perm_o)
    assert np.array_equal(boff, off_o)
    toff_o, touch_o = onufft.tile_touch_lists(g_or[perm_o], G, info["spread_bin_size"], W)
    assert np.array_equal(toff, toff_o)
    assert np.array_equal(touch, touch_o)
    plan.close()


@pytest.mark.parametrize("where", ["centre", "corner", "two", "one"])
def test_sort_offsets_degenerate_trajectories(where):
    """Bin and tile offsets when every sample falls in one or two bins
    (long runs of equal keys, empty leading and trailing bins): bit-exact."""
    kp = _kp()
    shape = (24, 40, 32)
    M = {"centre": 3000, "corner": 2000, "two": 2500, "one": 1}[where]
    k = np.zeros((M, 3), np.float32)
    if where == "corner":
        k[:] = np.float32(-np.pi)
    elif where == "two":
        k[M // 2:] = np.float32(2.5)
    print("degenerate sort", where, flush=True)
    plan = _plan(kp, k, shape, None, 1.25, 4)
    info = plan.info()
    G = onufft.grid_shape(shape, 1.25)
    g_or = onufft.canonical_coords(k, G)
    perm_o, off_o = onufft.sort_by_bin(g_or, G, info["bin_size"])
    perm, boff, toff, touch = [t.cpu().numpy() for t in plan.sort()]
    assert np.array_equal(perm, perm_o)
    assert np.array_equal(boff, off_o)
    toff_o, touch_o = onufft.tile_touch_lists(g_or[perm_o], G, info["spread_bin_size"], 4)
    assert np.array_equal(toff, toff_o)
    assert np.array_equal(touch, touch_o)
    plan.close()


NSPECIAL = 8   # synth.random_coords puts its special points first


@pytest.mark.parametrize("shape,C,M,alpha,W", CASES)
def test_forward_adjoint_parity(shape, C, M, alpha, W):
    kp = _kp()
    k, maps, x, y = case(shape, C, M, 12, alpha, W)
    print("case", shape, C, M, alpha, W, flush=True)
    op = onufft.Nufft(k, shape, maps, alpha, W)
    plan = _plan(kp, k, shape, maps, alpha, W)
    yg = kp.nufft_forward(plan, dev(x, torch.complex64)).cpu().numpy()
    yo = op.forward(x)
    assert rel(yg, yo) < 1e-4
    # the special samples one by one (k = 0, -pi, just below pi, exactly on
    # grid lines), where an edge tap of the wrong weight would be diluted in
    # the global figure: each sample's coil vector within 1e-4 of the oracle's
    for i in range(NSPECIAL):
        e = np.linalg.norm(yg[:, i] - yo[:, i]) / max(np.linalg.norm(yo[:, i]), 1e-2 * np.sqrt(np.mean(np.abs(yo) ** 2)))
        assert e < 1e-4, (i, k[i], e)
    xg = kp.nufft_adjoint(plan, dev(y, torch.complex64)).cpu().numpy()
    assert rel(xg, op.adjoint(y)) < 1e-4
    # adjoint of each special sample alone (a unit value in coil 0): its
    # spreading weights decide the whole image
    for i in range(NSPECIAL):
        yi = np.zeros((C, M), np.complex128)
        yi[0, i] = 1.0
        xi = kp.nufft_adjoint(plan, dev(yi, torch.complex64)).cpu().numpy()
        e = rel(xi, op.adjoint(yi))
        assert e < 1e-4, (i, k[i], e)
    plan.close()


def test_heavy_tiles_split_path():
    """Tiny chunks force every busy tile through the split path (partial
    tiles added in slot order)."""
    kp = _kp()
    shape, C = (24, 28), 3
    k, maps, x, y = case(shape, C, 2500, 13, 1.25, 4)
    k[100:900] = 0.0                     # a dense centre
    op = onufft.Nufft(k, shape, maps, 1.25, 4)
    for chunk, bins in ((7, (5, 6)), (64, (5, 6)), (64, (5, 4))):
        plan = _plan(kp, k, shape, maps, 1.25, 4, max_chunk=chunk, bin_size=bins)
        assert plan.info()["heavy_tiles"] > 0
        xg = kp.nufft_adjoint(plan, dev(y, torch.complex64)).cpu().numpy()
        assert rel(xg, op.adjoint(y)) < 1e-4
        yg = kp.nufft_forward(plan, dev(x, torch.complex64)).cpu().numpy()
        assert rel(yg, op.forward(x)) < 1e-4
        plan.close()


@pytest.mark.parametrize("chunk", [0, 8192])
def test_work_items_beyond_interleave_limit(chunk):
    """5000 samples at k = 0: with max_chunk 8192 the centre tiles form work
    items of more than 4096 entries, which keep their chunks of consecutive
    entries; the default splits them into interleaved items."""
    kp = _kp()
    shape, C = (32, 32), 4
    k, maps, x, y = case(shape, C, 9000, 17, 1.25, 4)
    k[:5000] = 0.0
    op = onufft.Nufft(k, shape, maps, 1.25, 4)
    plan = _plan(kp, k, shape, maps, 1.25, 4, max_chunk=chunk)
    if chunk:
        assert plan.info()["heavy_tiles"] == 0
    xg = kp.nufft_adjoint(plan, dev(y, torch.complex64)).cpu().numpy()
    assert rel(xg, op.adjoint(y)) < 1e-4
    yg = kp.nufft_forward(plan, dev(x, torch.complex64)).cpu().numpy()
    assert rel(yg, op.forward(x)) < 1e-4
    plan.close()


@pytest.mark.parametrize("C,bins", [(8, None), (4, (5, 10, 5)), (12, (8, 10, 6)), (4, (8, 10, 3))])
def test_dense_centre_3d(C, bins):
    """Thousands of samples in one tile: interpolation pieces and weight
    batches split, spreading tiles split; odd tile shapes."""
    kp = _kp()
    shape = (32, 40, 24)
    k, maps, x, y = case(shape, C, 12000, 15, 1.25, 4)
    k[200:3400] = 0.0
    k[5000:5300] = np.float32(-np.pi)
    print("dense 3d", C, bins, flush=True)
    op = onufft.Nufft(k, shape, maps, 1.25, 4)
    kw = {} if bins is None else dict(bin_size=bins)
    plan = _plan(kp, k, shape, maps, 1.25, 4, **kw)
    yg = kp.nufft_forward(plan, dev(x, torch.complex64)).cpu().numpy()
    assert rel(yg, op.forward(x)) < 1e-4
    xg = kp.nufft_adjoint(plan, dev(y, torch.complex64)).cpu().numpy()
    assert rel(xg, op.adjoint(y)) < 1e-4
    plan.close()


@pytest.mark.parametrize("shape,sbins,chunk", [
    ((32, 32, 32), (8, 8, 4), 0),      # grid 40^3 in the default 3D spreading tiles
    ((32, 32, 32), (8, 8, 2), 0),      # shallower tiles
    ((32, 64, 24), (4, 16, 3), 0),     # 64 lines as 4 x 16, 3 cells deep
    ((32, 32, 32), (8, 8, 4), 128),    # every busy tile split: partial tiles added in slot order
])
def test_spread_eight_coils_two_threads_per_line(shape, sbins, chunk):
    """8 coils and 64 lines per spreading tile: two threads per line, each
    with every coil, the entries of a line split between them."""
    kp = _kp()
    C, M = 8, 12000
    k, maps, x, y = case(shape, C, M, 21, 1.25, 4)
    k[300:1500] = 0.0                    # a dense centre
    print("spread 8 coils", shape, sbins, chunk, flush=True)
    op = onufft.Nufft(k, shape, maps, 1.25, 4)
    plan = _plan(kp, k, shape, maps, 1.25, 4, spread_bin_size=sbins, max_chunk=chunk)
    info = plan.info()
    assert info["spread_bin_size"] == sbins
    if chunk:
        assert info["heavy_tiles"] > 0
    xg = kp.nufft_adjoint(plan, dev(y, torch.complex64)).cpu().numpy()
    assert rel(xg, op.adjoint(y)) < 1e-4
    for i in range(NSPECIAL):
        yi = np.zeros((C, M), np.complex128)
        yi[i % C, i] = 1.0
        e = rel(kp.nufft_adjoint(plan, dev(yi, torch.complex64)).cpu().numpy(), op.adjoint(yi))
        assert e < 1e-4, (i, k[i], e)
    plan.close()


def test_adjoint_identity_on_gpu():
    kp = _kp()
    shape, C = (20, 24, 16), 3
    k, maps, x, y = case(shape, C, 5000, 14, 1.25, 4)
    plan = _plan(kp, k, shape, maps, 1.25, 4)
    xt, yt = dev(x, torch.complex64), dev(y, torch.complex64)
    ax = kp.nufft_forward(plan, xt)
    ahy = kp.nufft_adjoint(plan, yt)
    lhs = torch.vdot(ax.flatten().to(torch.complex128), yt.flatten().to(torch.complex128)).item()
    rhs = torch.vdot(xt.flatten().to(torch.complex128), ahy.flatten().to(torch.complex128)).item()
    assert abs(lhs - rhs) <= 1e-5 * abs(rhs)
    plan.close()


def test_config1_radial_parity():
    """128^2 single coil, 64 x 256 radial, alpha 2, W 4 (axis-aligned spokes, -pi)."""
    kp = _kp()
    cfg = synth.config(1)
    x, maps, k, _ = cfg.inputs(1)
    op = onufft.Nufft(k, cfg.shape, None, cfg.alpha, cfg.width)
    plan = _plan(kp, k, cfg.shape, None, cfg.alpha, cfg.width)
    yg = kp.nufft_forward(plan, dev(x, torch.complex64)).cpu().numpy()
    assert rel(yg, op.forward(x)) < 1e-4
    yy = op.forward(x)
    xg = kp.nufft_adjoint(plan, dev(yy, torch.complex64)).cpu().numpy()
    assert rel(xg, op.adjoint(yy)) < 1e-4
    perm, boff, _, _ = [t.cpu().numpy() for t in plan.sort()]
    G = onufft.grid_shape(cfg.shape, cfg.alpha)
    perm_o, off_o = onufft.sort_by_bin(onufft.canonical_coords(k, G), G, plan.info()["bin_size"])
    assert np.array_equal(perm, perm_o) and np.array_equal(boff, off_o)
    plan.close()


def test_edge_cases():
    kp = _kp()
    # a single sample
    shape = (8, 8)
    k = np.zeros((1, 2), np.float32)
    plan = _plan(kp, k, shape, None, 2.0, 4)
    x = np.random.default_rng(0).standard_normal(shape) + 0j
    op = onufft.Nufft(k, shape, None, 2.0, 4)
    assert rel(kp.nufft_forward(plan, dev(x, torch.complex64)).cpu().numpy(), op.forward(x)) < 1e-4
    plan.close()
    # out-of-range and NaN coordinates are rejected
    for bad in (np.array([[10.0, 0.0]], np.float32), np.array([[np.nan, 0.0]], np.float32)):
        with pytest.raises(kp.KpError) as ei:
            _plan(kp, bad, shape, None, 2.0, 4)
        assert ei.value.code == -1
    # 3D spreading tiles too long on axis 1 for the per-entry weight offset
    k3 = np.zeros((4, 3), np.float32)
    with pytest.raises(kp.KpError) as ei:
        _plan(kp, k3, (16, 64, 16), None, 2.0, 2, spread_bin_size=(1, 64, 4))
    assert ei.value.code == -2
    # coordinates slightly beyond pi wrap periodically
    k2 = np.array([[math.pi + 0.3, -math.pi - 0.2], [0.1, 0.2]], np.float32)
    plan = _plan(kp, k2, shape, None, 2.0, 4)
    op = onufft.Nufft(k2, shape, None, 2.0, 4)
    assert rel(kp.nufft_forward(plan, dev(x, torch.complex64)).cpu().numpy(), op.forward(x)) < 1e-4
    plan.close()


def test_profiling_stages():
    """Every profiling stage runs on a 3D plan (the prox stage with 3 levels:
    24 = 3 x 8); an unknown stage is refused."""
    kp = _kp()
    from paper_1902_09657_amd import _lib
    L = _lib.load()
    s = torch.cuda.current_stream()
    sp = __import__("ctypes").c_void_p(s.cuda_stream)
    k, maps, _, _ = case((16, 24, 32), 4, 3000, 5, 1.25, 4)
    plan = _plan(kp, k, (16, 24, 32), maps, 1.25, 4)
    for st in range(_lib.KP_STAGE_PROX + 1):
        print("stage", st, flush=True)
        _lib.check(L.nufft_stage(plan.handle, st, 2, sp))
    torch.cuda.synchronize()
    assert L.nufft_stage(plan.handle, _lib.KP_STAGE_PROX + 1, 1, sp) == -1
    plan.close()


def test_wrong_sized_buffers_refused():
    """Buffers whose size differs from the plan's are refused on the host,
    before any launch (the C-ABI only sees bare pointers)."""
    kp = _kp()
    rng = np.random.default_rng(7)
    shape, C, M = (16, 16), 2, 300
    k = rng.uniform(-math.pi, math.pi, (M, 2)).astype(np.float32)
    maps = rng.standard_normal((C,) + shape) + 1j * rng.standard_normal((C,) + shape)
    plan = _plan(kp, k, shape, maps, 1.25, 4)
    x_bad = dev(np.zeros((16, 15)), torch.complex64)
    y_bad = dev(np.zeros((C, M - 1)), torch.complex64)
    y = dev(np.zeros((C, M)), torch.complex64)
    p_bad = dev(np.ones(M + 1), torch.float32)
    for call in (lambda: kp.nufft_forward(plan, x_bad),
                 lambda: kp.nufft_adjoint(plan, y_bad),
                 lambda: kp.pdhg_solve(plan, y_bad, iters=1, lambda_max=1.0),
                 lambda: kp.pdhg_solve(plan, y, p_bad, iters=1, lambda_max=1.0),
                 lambda: kp.pdhg_solve(plan, y, iters=1, lambda_max=1.0, x0=x_bad),
                 lambda: kp.pdhg_lambda_max(plan, p_bad),
                 lambda: kp.l2_dual_cg(plan, y, p_bad, iters=1)):
        with pytest.raises(ValueError):
            call()
    # lambda_max_out is written in place through its pointer: a host tensor,
    # a wrong dtype or an empty tensor is refused before the solve starts
    for bad, exc in ((torch.zeros(1, dtype=torch.float32), TypeError),
                     (torch.zeros(1, dtype=torch.float64, device="cuda"), TypeError),
                     (torch.zeros(0, dtype=torch.float32, device="cuda"), ValueError)):
        with pytest.raises(exc):
            kp.pdhg_solve(plan, y, iters=1, lambda_max_out=bad)
    lm = torch.zeros(1, dtype=torch.float32, device="cuda")
    kp.pdhg_solve(plan, y, iters=1, lambda_max=1.5, lambda_max_out=lm)
    assert float(lm.item()) == 1.5
    torch.cuda.synchronize()
    plan.close()
