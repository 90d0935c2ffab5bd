"""GPU parity of the batched solve: every slice of a batch against the plain
per-slice solve (same kernels, same tiles) and against the oracle; graph
replays checked against the first launch with eager work in between."""
import numpy as np
import pytest

import synth
from oracle import nufft as onufft
from oracle import pdhg as opdhg
from oracle import precond as oprecond

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


def slices(sizes, spokes, C, seed):
    """Radial slices (N, S spokes of 2N samples), seeded maps and random data."""
    rng = np.random.default_rng(seed)
    out = []
    for n, s in zip(sizes, spokes):
        k = synth.radial_2d(s, 2 * n)
        maps = synth.coil_maps((n, n), C, rng) if C > 1 else None
        y = (rng.standard_normal((C, k.shape[0])) + 1j * rng.standard_normal((C, k.shape[0]))).astype(np.complex64)
        out.append(((n, n), k, maps, y))
    return out


def make_batch(kp, sl, tune, alpha=1.25, W=4):
    coords = [dev(k, torch.float32) for _, k, _, _ in sl]
    maps = None if sl[0][2] is None else [dev(m, torch.complex64) for _, _, m, _ in sl]
    return kp.nufft_plan_batch(coords, [s for s, _, _, _ in sl], maps, oversamp=alpha, kb_width=W, tune=tune)


def plain_solve(kp, sh, k, maps, y, p, alpha, W, bin_size=None, max_chunk=0, spread_bin_size=None, **kw):
    plan = kp.nufft_plan(dev(k, torch.float32), sh, None if maps is None else dev(maps, torch.complex64),
                         oversamp=alpha, kb_width=W, bin_size=bin_size, max_chunk=max_chunk,
                         spread_bin_size=spread_bin_size)
    x = kp.pdhg_solve(plan, dev(y, torch.complex64), p, reg="l2", **kw)
    plan.close()
    return x


# grid lengths 160, 200, 240: the one-launch-per-phase path
FAST = dict(sizes=[128, 160, 192, 128], spokes=[40, 24, 33, 64])
# grid lengths 320 and 400 (the narrower column blocks of the long lengths)
LONG = dict(sizes=[256, 320, 128], spokes=[20, 16, 30])


@pytest.mark.parametrize("C,sizes", [(4, "FAST"), (8, "FAST"), (12, "FAST"), (16, "FAST"), (8, "LONG"), (12, "LONG")])
def test_batch_fast_equals_plain(C, sizes):
    kp = _kp()
    print("batch fast C", C, sizes, flush=True)
    cfg = FAST if sizes == "FAST" else LONG
    sl = slices(cfg["sizes"], cfg["spokes"], C, 11)
    b = make_batch(kp, sl, tune=False)
    assert all(kp.nufft_batch_info(b, i)["fast"] for i in range(len(b)))
    ps = []
    for sh, k, maps, y in sl:
        plan = kp.nufft_plan(dev(k, torch.float32), sh, dev(maps, torch.complex64))
        ps.append(kp.precond_build(plan, kp.KP_PRECOND_MC))
        plan.close()
    xb = kp.pdhg_solve_batch(b, [dev(y, torch.complex64) for *_, y in sl], ps, lam=1e-3, iters=12)
    for i, (sh, k, maps, y) in enumerate(sl):
        xp = plain_solve(kp, sh, k, maps, y, ps[i], 1.25, 4, lam=1e-3, iters=12)
        r = rel(xb[i].cpu().numpy(), xp.cpu().numpy())
        print("slice", i, sh, "rel", r, flush=True)
        assert r < 1e-6
    b.close()


def test_batch_tuned_equals_plain_same_tiles():
    kp = _kp()
    print("batch tuned", flush=True)
    sl = slices([128, 192, 160], [48, 20, 60], 4, 12)
    b = make_batch(kp, sl, tune=True)
    # per-slice lambda_max given by the caller
    lm = [3.0 + i for i in range(len(sl))]
    xb = kp.pdhg_solve_batch(b, [dev(y, torch.complex64) for *_, y in sl], None, lam=1e-2, iters=8, lambda_max=lm)
    for i, (sh, k, maps, y) in enumerate(sl):
        inf = kp.nufft_batch_info(b, i)
        assert inf["fast"]
        # the plain plan takes the tuned tiles and split size, so both sides
        # sum in the same order
        xp = plain_solve(kp, sh, k, maps, y, None, 1.25, 4, bin_size=inf["bin_size"], max_chunk=inf["max_chunk"],
                         spread_bin_size=inf["spread_bin_size"], lam=1e-2, iters=8, lambda_max=lm[i])
        r = rel(xb[i].cpu().numpy(), xp.cpu().numpy())
        print("slice", i, sh, inf["bin_size"], inf["spread_bin_size"], inf["max_chunk"], "rel", r, flush=True)
        assert r < 1e-6
    b.close()


@pytest.mark.parametrize("fast", [True, False])
def test_batch_oracle(fast):
    kp = _kp()
    print("batch oracle fast", fast, flush=True)
    rng = np.random.default_rng(13)
    if fast:
        sizes, spokes, C = [128, 160], [24, 16], 4
    else:
        sizes, spokes, C = [32, 40, 24], [20, 30, 12], 3
    sl = []
    ys, ps, ops = [], [], []
    for n, s in zip(sizes, spokes):
        k = synth.radial_2d(s, 2 * n)
        maps = synth.coil_maps((n, n), C, rng)
        x = synth.phantom((n, n), rng)
        op = onufft.Nufft(k, (n, n), maps, 1.25, 4)
        y = op.forward(x) + synth.noise((C, k.shape[0]), 1e-3, rng)
        sl.append(((n, n), k, maps, y))
        ys.append(y)
        ps.append(oprecond.efficient_nufft(maps, k, (n, n), 1.25, 4))
        ops.append(op)
    b = make_batch(kp, sl, tune=fast)
    assert kp.nufft_batch_info(b, 0)["fast"] == fast
    xb = kp.pdhg_solve_batch(b, [dev(y, torch.complex64) for y in ys], [dev(p, torch.float32) for p in ps],
                             lam=1e-3, iters=10)
    for i, (sh, *_rest) in enumerate(sl):
        xo, _, _ = opdhg.pdhg(ops[i].forward, ops[i].adjoint, ys[i], ps[i], sh, "l2", 1e-3, 10)
        r = rel(xb[i].cpu().numpy(), xo)
        print("slice", i, sh, "rel", r, flush=True)
        assert r < 1e-4
    b.close()


def test_batch_graph_replays():
    kp = _kp()
    print("batch replays", flush=True)
    sl = slices([160, 128, 192], [30, 50, 18], 4, 14)
    b = make_batch(kp, sl, tune=False)
    ys = [dev(y, torch.complex64) for *_, y in sl]
    ref = [x.cpu().numpy() for x in kp.pdhg_solve_batch(b, ys, None, lam=1e-3, iters=6)]
    plan = kp.nufft_plan(dev(sl[0][1], torch.float32), sl[0][0], dev(sl[0][2], torch.complex64))
    for rep in range(4):
        # eager work and synchronisations between replays
        junk = kp.nufft_adjoint(plan, ys[0])
        torch.cuda.synchronize()
        (junk.abs() * 2).sum().item()
        xs = kp.pdhg_solve_batch(b, ys, None, lam=1e-3, iters=6)
        for i in range(len(sl)):
            assert np.array_equal(xs[i].cpu().numpy(), ref[i]), (rep, i)
    # a different iteration count recaptures; back to 6 replays the same result
    x4 = kp.pdhg_solve_batch(b, ys, None, lam=1e-3, iters=4)
    assert rel(x4[0].cpu().numpy(), ref[0]) > 0
    xs = kp.pdhg_solve_batch(b, ys, None, lam=1e-3, iters=6)
    for i in range(len(sl)):
        assert np.array_equal(xs[i].cpu().numpy(), ref[i])
    plan.close()
    b.close()


def test_batch_autotune_cached_and_valid():
    kp = _kp()
    print("autotune", flush=True)
    k = synth.radial_2d(40, 256)
    rng = np.random.default_rng(15)
    maps = synth.coil_maps((128, 128), 12, rng)
    t1 = kp.nufft_autotune(dev(k, torch.float32), (128, 128), dev(maps, torch.complex64))
    t2 = kp.nufft_autotune(dev(k, torch.float32), (128, 128), dev(maps, torch.complex64))
    assert t1 == t2
    assert 160 % t1["bin_size"][0] == 0 and t1["bin_size"][0] * 3 <= 256
    assert t1["max_chunk"] in (512, 1024, 2048)
    # spreading tiles: the sort tile's lines, 4 or 2 cells deep
    assert t1["spread_bin_size"][0] == t1["bin_size"][0] and t1["spread_bin_size"][1] in (2, 4)


def test_batch_invalid():
    kp = _kp()
    sl = slices([128, 128], [8, 8], 4, 16)
    b = make_batch(kp, sl, tune=False)
    ys = [dev(y, torch.complex64) for *_, y in sl]
    with pytest.raises(kp.KpError) as ei:
        kp.pdhg_solve_batch(b, ys, None, iters=0)
    assert ei.value.code == kp._lib.KP_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        kp.pdhg_solve_batch(b, ys[:1], None)
    b.close()
