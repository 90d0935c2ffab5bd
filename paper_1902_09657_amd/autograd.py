"""torch.autograd.Function wrappers over the library's differentiable calls.

Gradient convention is PyTorch's for complex tensors (grad = dL/dRe + i dL/dIm),
under which the vector-Jacobian product of a complex-linear map is its
conjugate transpose: A's backward is A^H and A^H's backward is A.  Every
computation (NUFFT, unrolled PDHG, its reverse recursion) runs in the HIP
library; these classes only marshal tensors.
"""
from __future__ import annotations

import math

import torch

from . import _lib
from . import Plan, PdhgOpts, nufft_adjoint, nufft_forward, _p_kind, _ptr, _stream, _dev, _numel, _p_numel, _nimg


class SenseNufft(torch.autograd.Function):
    """y = A x (multi-coil SENSE NUFFT); backward applies A^H."""

    @staticmethod
    def forward(ctx, x, plan: Plan):
        ctx.plan = plan
        return nufft_forward(plan, x)

    @staticmethod
    def backward(ctx, gy):
        return nufft_adjoint(ctx.plan, gy.contiguous()), None


class SenseNufftAdjoint(torch.autograd.Function):
    """x = A^H y; backward applies A."""

    @staticmethod
    def forward(ctx, y, plan: Plan):
        ctx.plan = plan
        return nufft_adjoint(plan, y)

    @staticmethod
    def backward(ctx, gx):
        return nufft_forward(ctx.plan, gx.contiguous()), None


def pack_params(sigma, tau, theta, lam):
    """Learnable step sizes as one float32 vector [3K+1] (sigma, tau, theta, lambda)."""
    return torch.cat([sigma.reshape(-1), tau.reshape(-1), theta.reshape(-1), lam.reshape(1)]).float().contiguous()


class UnrolledPdhg(torch.autograd.Function):
    """x_K of K unrolled l2 PDHG steps with learnable per-step sizes and lambda.

    forward(y, params, plan, p, K, ckpt_every, x0=None) -> x_K
      y      complex64 [C][M] data (differentiable)
      params float32 [3K+1] = sigma[K], tau[K], theta[K], lambda (differentiable)
      p      None, float32 [M] (single-channel) or [C][M] (multi-channel)
      x0     None or complex64 image (differentiable)
    Iterates are checkpointed every `ckpt_every` steps; the backward pass
    recomputes each segment from its checkpoint.
    """

    @staticmethod
    def forward(ctx, y, params, plan: Plan, p, K: int, ckpt_every: int, x0=None):
        L = _lib.load()
        y = _numel(_dev(y, torch.complex64, "y"), plan.ncoils * plan.nsamples, "y")
        params = _dev(params, torch.float32, "params")
        if params.numel() != 3 * K + 1:
            raise ValueError("params must hold 3K+1 values")
        if p is not None:
            p = _p_numel(_dev(p, torch.float32, "p"), plan.ncoils, plan.nsamples)
        if x0 is not None:
            x0 = _numel(_dev(x0, torch.complex64, "x0"), _nimg(plan.shape), "x0")
        nbytes = L.pdhg_unrolled_ckpt_bytes(plan.handle, int(K), int(ckpt_every))
        if nbytes <= 0:
            raise ValueError("invalid K / ckpt_every")
        ckpt = torch.empty(nbytes, dtype=torch.uint8, device=y.device)
        x = torch.empty(plan.shape, dtype=torch.complex64, device=y.device)
        _lib.check(L.pdhg_unrolled_forward(plan.handle, _ptr(y), _ptr(p), _p_kind(p), _ptr(params), int(K),
                                           int(ckpt_every), _ptr(x0), _ptr(x), _ptr(ckpt), _stream()))
        ctx.plan, ctx.K, ctx.S = plan, int(K), int(ckpt_every)
        ctx.has_p = p is not None
        ctx.has_x0 = x0 is not None
        extra = ([p] if p is not None else []) + ([x0] if x0 is not None else [])
        ctx.save_for_backward(y, params, ckpt, *extra)
        return x

    @staticmethod
    def backward(ctx, gx):
        L = _lib.load()
        saved = list(ctx.saved_tensors)
        y, params, ckpt = saved[:3]
        rest = saved[3:]
        p = rest.pop(0) if ctx.has_p else None
        x0 = rest.pop(0) if ctx.has_x0 else None
        gx = _numel(gx.contiguous().to(torch.complex64), _nimg(ctx.plan.shape), "grad of x")
        g_params = torch.empty_like(params)
        g_y = torch.empty_like(y)
        g_x0 = torch.empty(ctx.plan.shape, dtype=torch.complex64, device=y.device) if ctx.has_x0 else None
        _lib.check(L.pdhg_unrolled_backward(ctx.plan.handle, _ptr(y), _ptr(p), _p_kind(p), _ptr(params), ctx.K, ctx.S,
                                            _ptr(x0), _ptr(ckpt), _ptr(gx), _ptr(g_params), _ptr(g_y), _ptr(g_x0),
                                            _stream()))
        return g_y, g_params, None, None, None, None, g_x0


_SIDE_STREAMS = {}


def _side_streams(n, device):
    """Up to `n` (at most 4: the hardware queues a process gets by default)
    side streams of default priority, created once per device."""
    key = (device.index if device.index is not None else torch.cuda.current_device())
    have = _SIDE_STREAMS.setdefault(key, [])
    while len(have) < min(n, 4):
        have.append(torch.cuda.Stream(device=device))
    return have[: min(n, 4)]


def _check_slice(plan, y, params, p, K):
    y = _numel(_dev(y, torch.complex64, "y"), plan.ncoils * plan.nsamples, "y")
    params = _dev(params, torch.float32, "params")
    if params.numel() != 3 * K + 1:
        raise ValueError("params must hold 3K+1 values")
    if p is not None:
        p = _p_numel(_dev(p, torch.float32, "p"), plan.ncoils, plan.nsamples)
    return y, params, p


class UnrolledPdhgBatch(torch.autograd.Function):
    """x_K of every slice of a batch of independent problems: K unrolled l2
    PDHG steps per slice, each with its own plan, data y_i, preconditioner p_i
    and learnable parameters params_i (as UnrolledPdhg).  The slices are small
    (one 2D slice fills a fraction of the GPU), so they run concurrently, each
    on one of up to four side streams, in the forward and in the backward
    pass; the current stream waits for all of them.

    apply(K, ckpt_every, plans, ps, y_0 .. y_{n-1}, params_0 .. params_{n-1})
    returns the tuple (x_0, .., x_{n-1})."""

    @staticmethod
    def forward(ctx, K, S, plans, ps, *tensors):
        L = _lib.load()
        n = len(plans)
        if len(tensors) != 2 * n or len(ps) != n:
            raise ValueError("one y, one params and one p (or None) per plan")
        ys, prms, pp = [], [], []
        for i in range(n):
            y, params, p = _check_slice(plans[i], tensors[i], tensors[n + i], ps[i], K)
            ys.append(y)
            prms.append(params)
            pp.append(p)
        cur = torch.cuda.current_stream()
        dev = ys[0].device
        xs, cks = [], []
        for i, plan in enumerate(plans):  # outputs and checkpoints on the current stream
            nbytes = L.pdhg_unrolled_ckpt_bytes(plan.handle, int(K), int(S))
            if nbytes <= 0:
                raise ValueError("invalid K / ckpt_every")
            cks.append(torch.empty(nbytes, dtype=torch.uint8, device=dev))
            xs.append(torch.empty(plan.shape, dtype=torch.complex64, device=dev))
        streams = _side_streams(n, dev)
        for st in streams:
            st.wait_stream(cur)
        for i, plan in enumerate(plans):
            with torch.cuda.stream(streams[i % len(streams)]):
                _lib.check(L.pdhg_unrolled_forward(plan.handle, _ptr(ys[i]), _ptr(pp[i]), _p_kind(pp[i]),
                                                   _ptr(prms[i]), int(K), int(S), None, _ptr(xs[i]), _ptr(cks[i]),
                                                   _stream()))
        for st in streams:
            cur.wait_stream(st)
        ctx.plans, ctx.ps, ctx.K, ctx.S, ctx.n = plans, pp, int(K), int(S), n
        ctx.save_for_backward(*ys, *prms, *cks)
        return tuple(xs)

    @staticmethod
    def backward(ctx, *gxs):
        L = _lib.load()
        n = ctx.n
        saved = ctx.saved_tensors
        ys, prms, cks = saved[:n], saved[n:2 * n], saved[2 * n:]
        cur = torch.cuda.current_stream()
        dev = ys[0].device
        g_ys = [torch.empty_like(y) for y in ys]
        g_ps = [torch.empty_like(p) for p in prms]
        gx = []
        for i, plan in enumerate(ctx.plans):
            g = gxs[i]
            g = torch.zeros(plan.shape, dtype=torch.complex64, device=dev) if g is None else \
                _numel(g.contiguous().to(torch.complex64), _nimg(plan.shape), "grad of x")
            gx.append(g)
        streams = _side_streams(n, dev)
        for st in streams:
            st.wait_stream(cur)
        for i, plan in enumerate(ctx.plans):
            with torch.cuda.stream(streams[i % len(streams)]):
                p = ctx.ps[i]
                _lib.check(L.pdhg_unrolled_backward(plan.handle, _ptr(ys[i]), _ptr(p), _p_kind(p), _ptr(prms[i]),
                                                    ctx.K, ctx.S, None, _ptr(cks[i]), _ptr(gx[i]), _ptr(g_ps[i]),
                                                    _ptr(g_ys[i]), None, _stream()))
        for st in streams:
            cur.wait_stream(st)
        return (None, None, None, None, *g_ys, *g_ps)


def unrolled_pdhg_batch(ys, params, plans, ps=None, K=10, ckpt_every=None):
    """Functional form of UnrolledPdhgBatch: lists of per-slice y, params,
    plans and p (or None); returns the list of x_K."""
    if ckpt_every is None:
        ckpt_every = max(1, math.ceil(math.sqrt(K)))
    n = len(plans)
    ps = [None] * n if ps is None else list(ps)
    return list(UnrolledPdhgBatch.apply(int(K), int(ckpt_every), list(plans), ps, *ys, *params))


def unrolled_pdhg(y, params, plan, p=None, K=10, ckpt_every=None, x0=None):
    """Functional form of UnrolledPdhg; ckpt_every defaults to ceil(sqrt(K))."""
    if ckpt_every is None:
        ckpt_every = max(1, math.ceil(math.sqrt(K)))
    return UnrolledPdhg.apply(y, params, plan, p, int(K), int(ckpt_every), x0)


def schedule_params(plan: Plan, p=None, K=10, lam=1e-3, lambda_max=0.0, sigma0=1.0, accel=True, power_iters=30):
    """float32 [3K+1]: the step sizes pdhg_solve would take (and lambda), as
    the initial value of learnable unrolled parameters."""
    import ctypes
    if p is not None:
        p = _p_numel(_dev(p, torch.float32, "p"), plan.ncoils, plan.nsamples)
    o = PdhgOpts()
    o.reg = _lib.KP_REG_L2
    o.lam = float(lam)
    o.iters = int(K)
    o.lambda_max = float(lambda_max)
    o.power_iters = int(power_iters)
    o.sigma0 = float(sigma0)
    o.accel = 1 if accel else 0
    params = torch.empty(3 * int(K) + 1, dtype=torch.float32, device=plan.device)
    _lib.check(_lib.load().pdhg_schedule_params(plan.handle, _ptr(p), _p_kind(p), ctypes.byref(o), _ptr(params),
                                                _stream()))
    return params
