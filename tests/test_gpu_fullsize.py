"""GPU parity at the full sizes of the benchmark workloads.

* 2D radial 128^2 (1 coil, SC, l2, 20 iterations) and 2D spiral 256^2 (8 coils,
  MC, l1-db4, 30 iterations): the whole solve against the oracle; the spiral
  workload also with the TV regulariser and, for l2, through its dual (10
  MC-preconditioned CG iterations).
* 3D UTE 160^3, 8 coils, 2.56 M samples/coil (the timed workload, same plan as
  the benchmark): the canonical coordinates, sort and touch lists bit for bit;
  the full forward and adjoint against the oracle, the adjoint identity, and
  the first two PDHG iterations against the oracle (P = I and a fixed
  lambda_max keep the oracle's cost to four NUFFTs per iteration).  With two
  of the eight coils on the full image and trajectory: the MC preconditioner
  built at 2N, lambda_max with that p, and two l1-db4 iterations with that p
  and the library's own power method.
* Slices of the 64-slice batched workload, solved as one batch, against the
  oracle slice by slice.
* The differentiable workload's slice size (256^2, 12 coils, 24 x 2048 spiral):
  unrolled forward and gradients against the oracle's reverse recursion.
"""
import numpy as np
import pytest

import synth
from oracle import nufft as onufft
from oracle import pdhg as opdhg
from oracle import precond as oprecond
from oracle import unrolled as ounrolled

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")


def _kp():
    import paper_1902_09657_amd as kp
    return kp


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _plan(kp, k, shape, maps, alpha, W):
    m = None if maps is None else dev(maps, torch.complex64)
    return kp.nufft_plan(dev(k, torch.float32), shape, m, oversamp=alpha, kb_width=W)


@pytest.mark.parametrize("cfg_id", [1, 2])
def test_2d_workload_full_solve(cfg_id):
    kp = _kp()
    cfg = synth.config(cfg_id)
    print("full solve", cfg.name, flush=True)
    x, maps, k, w = cfg.inputs(seed=cfg_id)
    op = onufft.Nufft(k, cfg.shape, maps, cfg.alpha, cfg.width)
    y = op.forward(x) + w
    if cfg.precond == "sc":
        p = oprecond.efficient_nufft(None, k, cfg.shape, cfg.alpha, cfg.width)[0]
    else:
        p = oprecond.efficient_nufft(maps, k, cfg.shape, cfg.alpha, cfg.width)
    hist = []
    xo, _, _ = opdhg.pdhg(op.forward, op.adjoint, y, p, cfg.shape, cfg.reg, cfg.lam, cfg.iters, levels=4,
                          history=hist)
    plan = _plan(kp, k, cfg.shape, maps, cfg.alpha, cfg.width)
    pg = kp.precond_build(plan, kp.KP_PRECOND_SC if cfg.precond == "sc" else kp.KP_PRECOND_MC).cpu().numpy()
    assert rel(pg, p) < 1e-4
    xg, hg = kp.pdhg_solve(plan, dev(y, torch.complex64), dev(p, torch.float32), reg=cfg.reg, lam=cfg.lam,
                           iters=cfg.iters, wavelet_levels=4, objective=True)
    print("x rel", rel(xg.cpu().numpy(), xo), flush=True)
    assert rel(xg.cpu().numpy(), xo) < 1e-4
    np.testing.assert_allclose(hg, hist, rtol=1e-4)
    assert hg[-1] < hg[0]
    plan.close()


def test_2d_spiral_workload_tv_solve():
    """The 2D spiral workload (256^2, 8 coils, MC) with the TV regulariser."""
    from oracle import tv as otv
    kp = _kp()
    cfg = synth.config(2)
    x, maps, k, w = cfg.inputs(seed=2)
    op = onufft.Nufft(k, cfg.shape, maps, cfg.alpha, cfg.width)
    y = op.forward(x) + w
    p = oprecond.efficient_nufft(maps, k, cfg.shape, cfg.alpha, cfg.width)
    hist = []
    xo, _, _, _ = otv.tv_pdhg(op.forward, op.adjoint, y, p, cfg.shape, cfg.lam, cfg.iters, history=hist)
    plan = _plan(kp, k, cfg.shape, maps, cfg.alpha, cfg.width)
    xg, hg = kp.pdhg_solve(plan, dev(y, torch.complex64), dev(p, torch.float32), reg="tv", lam=cfg.lam,
                           iters=cfg.iters, objective=True)
    assert rel(xg.cpu().numpy(), xo) < 1e-4
    np.testing.assert_allclose(hg, hist, rtol=1e-4)
    plan.close()


def test_2d_spiral_workload_l2_dual_cg():
    """The 2D spiral workload's data (256^2, 8 coils) solved for l2 through its
    dual: MC-preconditioned CG, 10 iterations, x, u and the residual history."""
    kp = _kp()
    cfg = synth.config(2)
    x, maps, k, w = cfg.inputs(seed=2)
    op = onufft.Nufft(k, cfg.shape, maps, cfg.alpha, cfg.width)
    y = op.forward(x) + w
    p = oprecond.efficient_nufft(maps, k, cfg.shape, cfg.alpha, cfg.width)
    ho = []
    xo, uo = opdhg.l2_dual_pcg(op.forward, op.adjoint, y, p, cfg.shape, 1e-2, 10, history=ho)
    plan = _plan(kp, k, cfg.shape, maps, cfg.alpha, cfg.width)
    xg, ug, hg = kp.l2_dual_cg(plan, dev(y, torch.complex64), dev(p, torch.float32), lam=1e-2, iters=10,
                               want_u=True, residuals=True)
    print("dual cg x rel", rel(xg.cpu().numpy(), xo), flush=True)
    assert rel(xg.cpu().numpy(), xo) < 1e-4
    assert rel(ug.cpu().numpy(), uo) < 1e-4
    np.testing.assert_allclose(hg, ho, rtol=1e-3, atol=1e-5)
    plan.close()


def test_3d_ute_support_pruned_two_coils():
    """128^3 (grid 160^3), 2 coils, UTE: the axis-0 FFT passes store / load
    only each column's support range and spreading skips the empty corner
    tiles; a forward first leaves other data in the grid buffers."""
    kp = _kp()
    shape, C = (128, 128, 128), 2
    rng = np.random.default_rng(23)
    k = synth.ute_3d(2000, 128)
    maps = synth.coil_maps(shape, C, rng)
    x = synth.phantom(shape, rng)
    op = onufft.Nufft(k, shape, maps, 1.25, 4)
    plan = _plan(kp, k, shape, maps, 1.25, 4)
    yg = kp.nufft_forward(plan, dev(x, torch.complex64)).cpu().numpy()
    assert rel(yg, op.forward(x)) < 1e-4
    y = (rng.standard_normal(yg.shape) + 1j * rng.standard_normal(yg.shape)) / np.sqrt(2.0)
    xg = kp.nufft_adjoint(plan, dev(y, torch.complex64)).cpu().numpy()
    assert rel(xg, op.adjoint(y)) < 1e-4
    plan.close()


@pytest.fixture(scope="module")
def ute():
    """The timed 3D workload: inputs, the oracle operator and the GPU plan."""
    kp = _kp()
    cfg = synth.config(3)
    x, maps, k, w = cfg.inputs(seed=3)
    print("3D UTE: oracle taps", flush=True)
    op = onufft.Nufft(k, cfg.shape, maps, cfg.alpha, cfg.width)
    plan = _plan(kp, k, cfg.shape, maps, cfg.alpha, cfg.width)
    yield kp, cfg, x, maps, k, w, op, plan
    plan.close()


def test_3d_ute_forward_adjoint_full(ute):
    kp, cfg, x, maps, k, w, op, plan = ute
    print("3D UTE forward", flush=True)
    yg = kp.nufft_forward(plan, dev(x, torch.complex64)).cpu().numpy()
    yo = op.forward(x)
    assert rel(yg, yo) < 1e-4
    print("3D UTE adjoint", flush=True)
    rng = np.random.default_rng(31)
    y = (rng.standard_normal(yo.shape) + 1j * rng.standard_normal(yo.shape)) / np.sqrt(2.0)
    xg = kp.nufft_adjoint(plan, dev(y, torch.complex64)).cpu().numpy()
    assert rel(xg, op.adjoint(y)) < 1e-4


def test_3d_ute_adjoint_identity(ute):
    kp, cfg, x, maps, k, w, op, plan = ute
    rng = np.random.default_rng(32)
    xt = dev(x, torch.complex64)
    yt = dev(rng.standard_normal(w.shape) + 1j * rng.standard_normal(w.shape), torch.complex64)
    ax = kp.nufft_forward(plan, xt)
    ahy = kp.nufft_adjoint(plan, yt)
    lhs = torch.vdot(ax.flatten().to(torch.complex128), yt.flatten().to(torch.complex128)).item()
    rhs = torch.vdot(xt.flatten().to(torch.complex128), ahy.flatten().to(torch.complex128)).item()
    assert abs(lhs - rhs) <= 1e-5 * abs(rhs)


def test_3d_ute_sort_bit_exact(ute):
    """The timed plan's canonical coordinates, sort and spreading touch lists
    at full size (2.56 M samples, 8.4 M touch entries), bit for bit."""
    kp, cfg, x, maps, k, w, op, plan = ute
    info = plan.info()
    G = onufft.grid_shape(cfg.shape, cfg.alpha)
    assert tuple(info["grid"]) == G
    print("3D UTE sort", info["bin_size"], info["spread_bin_size"], flush=True)
    g_or = onufft.canonical_coords(k, G)
    assert np.array_equal(plan.grid_coords().cpu().numpy().view(np.uint32), g_or.view(np.uint32))
    perm_o, off_o = onufft.sort_by_bin(g_or, G, info["bin_size"])
    perm, boff, toff, touch = [t.cpu().numpy() for t in plan.sort()]
    assert np.array_equal(perm, perm_o)
    assert np.array_equal(boff, off_o)
    toff_o, touch_o = onufft.tile_touch_lists(g_or[perm_o], G, info["spread_bin_size"], cfg.width)
    assert np.array_equal(toff, toff_o)
    assert np.array_equal(touch, touch_o)


@pytest.fixture(scope="module")
def ute2(ute):
    """Two of the eight coils of the timed workload on the full 160^3 image and
    trajectory, with the oracle's multi-channel preconditioner (built at 2N:
    320^3 lags, 400^3 grid) and its power-method lambda_max (3 iterations:
    the oracle needs about 14 s per NUFFT pair at this size)."""
    kp, cfg, x, maps, k, w, op, plan = ute
    m2 = maps[:2]
    op2 = op.with_maps(m2)
    plan2 = _plan(kp, k, cfg.shape, m2, cfg.alpha, cfg.width)
    print("3D UTE two coils: oracle MC preconditioner at 2N", flush=True)
    p_o = oprecond.efficient_nufft(m2, k, cfg.shape, cfg.alpha, cfg.width)
    print("3D UTE two coils: oracle lambda_max", flush=True)
    lmax_o = opdhg.power_method(op2.forward, op2.adjoint, p_o, cfg.shape, 3)
    yield kp, cfg, x, m2, k, w[:2], op2, plan2, p_o, lmax_o
    plan2.close()


def test_3d_ute_dcf_full(ute):
    """The Pipe-Menon weights of the timed plan (2.56 M samples, 30 fixed-point
    iterations): the GPU's scaled weights are the oracle's raw weights times
    one constant (1 / lambda_max), sample by sample."""
    kp, cfg, x, maps, k, w, op, plan = ute
    print("3D UTE DCF", flush=True)
    p = kp.precond_build(plan, kp.KP_PRECOND_DCF).cpu().numpy().astype(np.float64)
    wo = oprecond.pipe_menon_dcf(k, cfg.shape, cfg.alpha, cfg.width, op=op)
    ratio = p / wo
    c = float(np.median(ratio))
    print("3D UTE DCF scale", c, "max dev", float(np.max(np.abs(ratio / c - 1.0))), flush=True)
    assert np.all(p > 0)
    assert rel(p / c, wo) < 1e-4
    assert np.max(np.abs(ratio / c - 1.0)) < 1e-3


def test_3d_ute_mc_precond_full(ute2):
    kp, cfg, x, m2, k, w, op2, plan2, p_o, lmax_o = ute2
    p_g = kp.precond_build(plan2, kp.KP_PRECOND_MC).cpu().numpy()
    r = rel(p_g, p_o)
    print("3D UTE MC precond rel", r, flush=True)
    assert np.all(p_g > 0)
    assert r < 1e-4


def test_3d_ute_lambda_max_mc(ute2):
    kp, cfg, x, m2, k, w, op2, plan2, p_o, lmax_o = ute2
    lg = float(kp.pdhg_lambda_max(plan2, dev(p_o, torch.float32), 3).item())
    print("3D UTE lambda_max", lg, lmax_o, flush=True)
    assert abs(lg - lmax_o) <= 1e-5 * lmax_o


def test_3d_ute_pdhg_mc_power_method(ute2):
    """Two l1-db4 PDHG iterations with the oracle's MC p; the library runs its
    own power method inside pdhg_solve (lambda_max <= 0), the oracle uses its
    own estimate (equal within 1e-5 by the test above)."""
    kp, cfg, x, m2, k, w, op2, plan2, p_o, lmax_o = ute2
    y = op2.forward(x) + w
    xo, uo, _ = opdhg.pdhg(op2.forward, op2.adjoint, y, p_o, cfg.shape, "l1wav", cfg.lam, 2, lmax=lmax_o, levels=4)
    xg, ug = kp.pdhg_solve(plan2, dev(y, torch.complex64), dev(p_o, torch.float32), reg="l1wav", lam=cfg.lam,
                           iters=2, wavelet_levels=4, lambda_max=0.0, power_iters=3, want_u=True)
    rx, ru = rel(xg.cpu().numpy(), xo), rel(ug.cpu().numpy(), uo)
    print("3D UTE MC PDHG rel x", rx, "u", ru, flush=True)
    assert rx < 1e-4 and ru < 1e-4


def test_3d_ute_pdhg_first_iterations(ute):
    kp, cfg, x, maps, k, w, op, plan = ute
    print("3D UTE two PDHG iterations", flush=True)
    y = op.forward(x) + w
    lmax = 2.0
    xo, uo, _ = opdhg.pdhg(op.forward, op.adjoint, y, None, cfg.shape, "l1wav", cfg.lam, 2, lmax=lmax, levels=4)
    xg, ug = kp.pdhg_solve(plan, dev(y, torch.complex64), None, reg="l1wav", lam=cfg.lam, iters=2,
                           wavelet_levels=4, lambda_max=lmax, want_u=True)
    assert rel(xg.cpu().numpy(), xo) < 1e-4
    assert rel(ug.cpu().numpy(), uo) < 1e-4


def test_batched_workload_slices():
    """Three slices of the 64-slice set (the two first of size 128 and the
    first of size 192), 12 coils, SC preconditioner, l2, 20 iterations."""
    kp = _kp()
    sl = synth.slice_config4(64, seed=4, ncoils=12)
    pick = [i for i, (s, _) in enumerate(sl) if s[0] == 128][:2] + [i for i, (s, _) in enumerate(sl) if s[0] == 192][:1]
    coords, maps_l, ys, ps, ops = [], [], [], [], []
    for i in pick:
        shape, k = sl[i]
        rp, rm, _, rn = synth.streams(4000 + i)
        x = synth.phantom(shape, rp)
        m = synth.coil_maps(shape, 12, rm)
        op = onufft.Nufft(k, shape, m, 1.25, 4)
        ys.append(op.forward(x) + synth.noise((12, k.shape[0]), 1e-3, rn))
        ps.append(oprecond.efficient_nufft(None, k, shape, 1.25, 4)[0])
        coords.append(dev(k, torch.float32))
        maps_l.append(dev(m, torch.complex64))
        ops.append(op)
    print("batched slices", pick, [sl[i][0] for i in pick], flush=True)
    b = kp.nufft_plan_batch(coords, [sl[i][0] for i in pick], maps_l, oversamp=1.25, kb_width=4, tune=True)
    assert all(kp.nufft_batch_info(b, j)["fast"] for j in range(len(pick)))
    lm = [1.5] * len(pick)
    xb = kp.pdhg_solve_batch(b, [dev(y, torch.complex64) for y in ys], [dev(p, torch.float32) for p in ps],
                             lam=1e-3, iters=20, lambda_max=lm)
    for j, i in enumerate(pick):
        xo, _, _ = opdhg.pdhg(ops[j].forward, ops[j].adjoint, ys[j], ps[j], sl[i][0], "l2", 1e-3, 20, lmax=lm[j])
        r = rel(xb[j].cpu().numpy(), xo)
        print("slice", i, sl[i][0], "rel", r, flush=True)
        assert r < 1e-4
    b.close()



def test_batched_workload_all_64_slices():
    """The whole 64-slice batch as the benchmark times it: phantom data, the
    multi-channel preconditioner and each slice's own power-method lambda_max
    (30 iterations), one pdhg_solve_batch.  Every slice equals the plain
    per-slice solve on a plan with the batch's tiles within 1e-6; two
    sampled slices (one of size 128, one of size 192) take their data, MC
    preconditioner and lambda_max from the oracle side only and equal the
    FP64 oracle within 1e-4 (their GPU lambda_max within 1e-5 of the
    oracle's)."""
    kp = _kp()
    C, K, lam = 12, 20, 1e-3
    sl = synth.slice_config4(64, seed=4, ncoils=C)
    pick = [[i for i, (s, _) in enumerate(sl) if s[0] == n][0] for n in (128, 192)]
    coords, maps_l, ys, ps, lms, ops = [], [], [], [], [], {}
    print("batched 64 slices, oracle-sampled", pick, flush=True)
    for i, (shape, k) in enumerate(sl):
        rp, rm, _, rn = synth.streams(4000 + i)
        x = synth.phantom(shape, rp)
        m = synth.coil_maps(shape, C, rm)
        kt, mt = dev(k, torch.float32), dev(m, torch.complex64)
        pl = _plan(kp, k, shape, m, 1.25, 4)
        if i in pick:
            op = onufft.Nufft(k, shape, m, 1.25, 4)
            y = op.forward(x) + synth.noise((C, k.shape[0]), 1e-3, rn)
            p = oprecond.efficient_nufft(m, k, shape, 1.25, 4)
            lm = opdhg.power_method(op.forward, op.adjoint, p, shape, 30)
            lg = float(kp.pdhg_lambda_max(pl, dev(p, torch.float32), 30).item())
            print("slice", i, shape, "lambda_max gpu", lg, "oracle", lm, flush=True)
            assert abs(lg - lm) <= 1e-5 * lm
            ops[i] = (op, y, p, lm)
            yt, pt = dev(y, torch.complex64), dev(p, torch.float32)
        else:
            yt = kp.nufft_forward(pl, dev(x, torch.complex64)) + dev(synth.noise((C, k.shape[0]), 1e-3, rn),
                                                                     torch.complex64)
            pt = kp.precond_build(pl, kp.KP_PRECOND_MC)
            lm = float(kp.pdhg_lambda_max(pl, pt, 30).item())
        pl.close()
        coords.append(kt)
        maps_l.append(mt)
        ys.append(yt)
        ps.append(pt)
        lms.append(lm)
    b = kp.nufft_plan_batch(coords, [s for s, _ in sl], maps_l, oversamp=1.25, kb_width=4, tune=True)
    assert all(kp.nufft_batch_info(b, j)["fast"] for j in range(len(sl)))
    with pytest.raises(ValueError):   # mixed preconditioner kinds are refused
        kp.pdhg_solve_batch(b, ys, ps[:1] + [p[0].contiguous() for p in ps[1:]], lam=lam, iters=K, lambda_max=lms)
    xb = kp.pdhg_solve_batch(b, ys, ps, lam=lam, iters=K, lambda_max=lms)
    worst = 0.0
    for i, (shape, k) in enumerate(sl):
        inf = kp.nufft_batch_info(b, i)
        pl = kp.nufft_plan(coords[i], shape, maps_l[i], oversamp=1.25, kb_width=4, bin_size=inf["bin_size"],
                           max_chunk=inf["max_chunk"], spread_bin_size=inf["spread_bin_size"])
        xp = kp.pdhg_solve(pl, ys[i], ps[i], reg="l2", lam=lam, iters=K, lambda_max=lms[i])
        worst = max(worst, rel(xb[i].cpu().numpy(), xp.cpu().numpy()))
        pl.close()
    print("batch vs plain (same tiles), worst rel", worst, flush=True)
    assert worst < 1e-6
    for i in pick:
        op, y, p, lm = ops[i]
        xo, _, _ = opdhg.pdhg(op.forward, op.adjoint, y, p, sl[i][0], "l2", lam, K, lmax=lm)
        r = rel(xb[i].cpu().numpy(), xo)
        print("slice", i, sl[i][0], "rel vs oracle", r, flush=True)
        assert r < 1e-4
    b.close()


def test_differentiable_workload_slice():
    from paper_1902_09657_amd.autograd import UnrolledPdhg, schedule_params
    kp = _kp()
    cfg = synth.config(5)
    x, maps, k, w = cfg.inputs(seed=5000)
    print("unrolled", cfg.name, flush=True)
    op = onufft.Nufft(k, cfg.shape, maps, cfg.alpha, cfg.width)
    y = op.forward(x) + w
    p = oprecond.efficient_nufft(maps, k, cfg.shape, cfg.alpha, cfg.width)
    K, lmax = cfg.iters, 1.8
    sig, tau, th = opdhg.schedule(lmax, float(p.min()), K)
    xK, rec = ounrolled.forward(op.forward, op.adjoint, y, p, sig, tau, th, cfg.lam, cfg.shape)
    g = ounrolled.backward(op.forward, op.adjoint, y, p, sig, tau, th, cfg.lam, rec, xK - x)
    plan = _plan(kp, k, cfg.shape, maps, cfg.alpha, cfg.width)
    pt = dev(p, torch.float32)
    params = schedule_params(plan, pt, K, lam=cfg.lam, lambda_max=lmax).requires_grad_(True)
    xg = UnrolledPdhg.apply(dev(y, torch.complex64), params, plan, pt, K, 4, None)
    assert rel(xg.detach().cpu().numpy(), xK) < 1e-4
    r = xg - dev(x, torch.complex64)
    (0.5 * (r.real ** 2 + r.imag ** 2).sum()).backward()
    want = np.concatenate([g["sigma"], g["tau"], g["theta"], [g["lam"]]])
    assert rel(params.grad.cpu().numpy(), want) < 1e-3
    plan.close()
