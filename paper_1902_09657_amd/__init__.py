"""MI355X-native hot path of k-space-preconditioned PDHG (Ong, Uecker, Lustig).

Python binding over the C ABI of libkpdhg (include/kpdhg.h), with the same
function names.  Tensors are torch tensors on the GPU (complex64 / float32);
each call runs on torch's current HIP stream.  The binding only marshals
arguments; every computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (KP_PRECOND_DCF, KP_PRECOND_MC, KP_PRECOND_NONE, KP_PRECOND_SC, KP_REG_L1_WAVELET, KP_REG_L2, KP_REG_TV,
                   KpError, PdhgOpts, PlanInfo, Tuning)

__all__ = [
    "Plan", "nufft_plan", "nufft_forward", "nufft_forward_noalloc", "nufft_adjoint", "precond_build", "pdhg_lambda_max",
    "pdhg_solve", "l2_dual_cg", "nufft_destroy", "nufft_autotune", "Batch", "nufft_plan_batch", "nufft_batch_info",
    "pdhg_solve_batch", "nufft_batch_destroy", "KpError", "KP_PRECOND_NONE", "KP_PRECOND_SC", "KP_PRECOND_MC", "KP_PRECOND_DCF",
    "KP_REG_L2", "KP_REG_L1_WAVELET", "KP_REG_TV",
]


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s" % (name, dtype))
    return t.contiguous()


def _out(t, dtype, n, name):
    """An output buffer the library writes through its pointer: a contiguous
    device tensor of the right dtype and size, used as given (never a copy)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s" % (name, dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return _numel(t, n, name)


def _numel(t, n, name):
    """Refuse a buffer whose size differs from what the library will read or
    write through its pointer (the C-ABI takes bare pointers)."""
    if t is not None and t.numel() != n:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), n))
    return t


def _p_numel(p, ncoils, nsamples):
    """p is [M] (single-channel) or [C, M] (multi-channel)."""
    if p is not None:
        _numel(p, nsamples if p.dim() == 1 else ncoils * nsamples, "p")
    return p


def _nimg(shape):
    n = 1
    for v in shape:
        n *= int(v)
    return n


class Plan:
    """A NUFFT plan (owns the library handle); see nufft_plan."""

    def __init__(self, handle, shape, ncoils, nsamples, device):
        self.handle = handle
        self.shape = tuple(shape)
        self.ncoils = int(ncoils)
        self.nsamples = int(nsamples)
        self.device = device

    def info(self) -> dict:
        inf = PlanInfo()
        _lib.check(_lib.load().nufft_plan_info(self.handle, ctypes.byref(inf)))
        d = inf.ndim
        return {
            "ndim": d, "shape": tuple(inf.shape[:d]), "grid": tuple(inf.grid[:d]),
            "ncoils": inf.ncoils, "nsamples": inf.nsamples, "kb_width": inf.kb_width,
            "oversamp": inf.oversamp, "kb_beta": inf.kb_beta, "bin_size": tuple(inf.bin_size[:d]),
            "nbins": inf.nbins, "ntouch": inf.ntouch, "nwork": inf.nwork,
            "heavy_tiles": inf.heavy_tiles, "workspace_bytes": inf.workspace_bytes,
            "spread_bin_size": tuple(inf.spread_bin_size[:d]), "nspread_tiles": inf.nspread_tiles,
            "max_chunk": inf.max_chunk,
        }

    def sort(self):
        """(perm, bin_offsets, touch_offsets, touch) as int32 device tensors."""
        inf = self.info()
        dev = self.device
        perm = torch.empty(self.nsamples, dtype=torch.int32, device=dev)
        boff = torch.empty(inf["nbins"] + 1, dtype=torch.int32, device=dev)
        toff = torch.empty(inf["nspread_tiles"] + 1, dtype=torch.int32, device=dev)
        touch = torch.empty(max(inf["ntouch"], 1), dtype=torch.int32, device=dev)
        _lib.check(_lib.load().nufft_plan_sort(self.handle, _ptr(perm), _ptr(boff), _ptr(toff), _ptr(touch), _stream()))
        return perm, boff, toff, touch[: inf["ntouch"]]

    def grid_coords(self):
        g = torch.empty((self.nsamples, len(self.shape)), dtype=torch.float32, device=self.device)
        _lib.check(_lib.load().nufft_plan_grid_coords(self.handle, _ptr(g), _stream()))
        return g

    def close(self):
        if self.handle:
            _lib.load().nufft_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nufft_plan(coords, shape, maps=None, oversamp=1.25, kb_width=4, bin_size=None, max_chunk=0,
               spread_bin_size=None) -> Plan:
    """Plan for coordinates [M][d] (float32, rad/pixel) and maps [C][*shape] (complex64).

    bin_size: sort / interpolation tiles; spread_bin_size: spreading tiles
    (default: bin_size when that is given, else the built-in choice)."""
    L = _lib.load()
    coords = _dev(coords, torch.float32, "coords")
    shape = tuple(int(n) for n in shape)
    d = len(shape)
    if coords.dim() != 2 or coords.shape[1] != d:
        raise ValueError("coords must have shape [M, %d]" % d)
    C = 1
    if maps is not None:
        maps = _dev(maps, torch.complex64, "maps")
        C = maps.shape[0]
        if tuple(maps.shape[1:]) != shape:
            raise ValueError("maps must have shape [C, *shape]")
    tun = None
    if bin_size is not None or max_chunk or spread_bin_size is not None:
        tun = Tuning()
        for a in range(3):
            tun.bin_size[a] = int(bin_size[a]) if bin_size is not None and a < d else 0
            tun.spread_bin_size[a] = int(spread_bin_size[a]) if spread_bin_size is not None and a < d else 0
        tun.max_chunk = int(max_chunk)
    h = ctypes.c_void_p()
    shp = (ctypes.c_int64 * d)(*shape)
    _lib.check(L.nufft_plan(ctypes.byref(h), d, shp, C, coords.shape[0], _ptr(coords), _ptr(maps),
                            float(oversamp), int(kb_width), ctypes.byref(tun) if tun is not None else None,
                            _stream()))
    return Plan(h, shape, C, coords.shape[0], coords.device)


def nufft_forward(plan: Plan, x, out=None):
    x = _numel(_dev(x, torch.complex64, "x"), _nimg(plan.shape), "x")
    if out is None:
        out = torch.empty((plan.ncoils, plan.nsamples), dtype=torch.complex64, device=plan.device)
    _out(out, torch.complex64, plan.ncoils * plan.nsamples, "out")
    _lib.check(_lib.load().nufft_forward(plan.handle, _ptr(x), _ptr(out), _stream()))
    return out


def nufft_forward_noalloc(plan: Plan, x, out):
    """nufft_forward with the FFT grids in the library's static per-device
    array: no device allocation in the library, `out` supplied by the caller."""
    x = _numel(_dev(x, torch.complex64, "x"), _nimg(plan.shape), "x")
    _out(out, torch.complex64, plan.ncoils * plan.nsamples, "out")
    _lib.check(_lib.load().nufft_forward_noalloc(plan.handle, _ptr(x), _ptr(out), _stream()))
    return out


def nufft_adjoint(plan: Plan, y, out=None):
    y = _numel(_dev(y, torch.complex64, "y"), plan.ncoils * plan.nsamples, "y")
    if out is None:
        out = torch.empty(plan.shape, dtype=torch.complex64, device=plan.device)
    _out(out, torch.complex64, _nimg(plan.shape), "out")
    _lib.check(_lib.load().nufft_adjoint(plan.handle, _ptr(y), _ptr(out), _stream()))
    return out


def precond_build(plan: Plan, kind):
    """p for kind SC or DCF: float32 [M]; MC: [C, M] (caller sample order)."""
    n = (plan.nsamples,) if kind in (KP_PRECOND_SC, KP_PRECOND_DCF) else (plan.ncoils, plan.nsamples)
    p = torch.empty(n, dtype=torch.float32, device=plan.device)
    _lib.check(_lib.load().precond_build(plan.handle, int(kind), _ptr(p), _stream()))
    return p


def _p_kind(p):
    if p is None:
        return KP_PRECOND_NONE
    return KP_PRECOND_SC if p.dim() == 1 else KP_PRECOND_MC


def pdhg_lambda_max(plan: Plan, p=None, iters=30):
    out = torch.empty(1, dtype=torch.float32, device=plan.device)
    if p is not None:
        p = _p_numel(_dev(p, torch.float32, "p"), plan.ncoils, plan.nsamples)
    _lib.check(_lib.load().pdhg_lambda_max(plan.handle, _ptr(p), _p_kind(p), int(iters), _ptr(out), _stream()))
    return out


def pdhg_solve(plan: Plan, y, p=None, reg="l2", lam=1e-3, iters=20, wavelet_levels=4, lambda_max=0.0,
               power_iters=30, sigma0=1.0, accel=True, x0=None, u0=None, objective=False, want_u=False,
               lambda_max_out=None):
    """Run the preconditioned PDHG (reg "l2", "l1wav" or "tv").  Returns x (and u,
    objective history when asked)."""
    y = _numel(_dev(y, torch.complex64, "y"), plan.ncoils * plan.nsamples, "y")
    if p is not None:
        p = _p_numel(_dev(p, torch.float32, "p"), plan.ncoils, plan.nsamples)
    o = PdhgOpts()
    regs = {"l2": KP_REG_L2, "l1wav": KP_REG_L1_WAVELET, "tv": KP_REG_TV}
    if reg not in regs:
        raise ValueError("reg must be one of %s" % sorted(regs))
    o.reg = regs[reg]
    o.lam = float(lam)
    o.iters = int(iters)
    o.wavelet_levels = int(wavelet_levels)
    o.lambda_max = float(lambda_max)
    o.power_iters = int(power_iters)
    o.sigma0 = float(sigma0)
    o.accel = 1 if accel else 0
    if x0 is not None:
        x0 = _numel(_dev(x0, torch.complex64, "x0"), _nimg(plan.shape), "x0")
    if u0 is not None:
        u0 = _numel(_dev(u0, torch.complex64, "u0"), plan.ncoils * plan.nsamples, "u0")
    o.x0 = _ptr(x0).value
    o.u0 = _ptr(u0).value
    hist = None
    if objective:
        hist = (ctypes.c_double * (iters + 1))()
        o.objective_host = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
    if lambda_max_out is not None:
        # written in place through its pointer: a device float32 tensor of at
        # least one element, used as given (not a contiguous copy)
        if not isinstance(lambda_max_out, torch.Tensor) or not lambda_max_out.is_cuda:
            raise TypeError("lambda_max_out must be a CUDA (HIP) tensor")
        if lambda_max_out.dtype != torch.float32:
            raise TypeError("lambda_max_out must be torch.float32")
        if lambda_max_out.numel() < 1:
            raise ValueError("lambda_max_out must hold at least one element")
        o.lambda_max_out = lambda_max_out.data_ptr()
    x = torch.empty(plan.shape, dtype=torch.complex64, device=plan.device)
    u = torch.empty((plan.ncoils, plan.nsamples), dtype=torch.complex64, device=plan.device) if want_u else None
    _lib.check(_lib.load().pdhg_solve(plan.handle, _ptr(y), _ptr(p), _p_kind(p), ctypes.byref(o), _ptr(x), _ptr(u),
                                      _stream()))
    out = [x]
    if want_u:
        out.append(u)
    if objective:
        out.append([hist[i] for i in range(iters + 1)])
    return out[0] if len(out) == 1 else tuple(out)


def l2_dual_cg(plan: Plan, y, p=None, lam=1e-3, iters=50, want_u=False, residuals=False):
    """l2 reconstruction through its dual: preconditioned CG on (A A^H + lam I) u = lam y,
    x = A^H u / lam.  Returns x (and u, relative residual history when asked)."""
    y = _numel(_dev(y, torch.complex64, "y"), plan.ncoils * plan.nsamples, "y")
    if p is not None:
        p = _p_numel(_dev(p, torch.float32, "p"), plan.ncoils, plan.nsamples)
    x = torch.empty(plan.shape, dtype=torch.complex64, device=plan.device)
    u = torch.empty((plan.ncoils, plan.nsamples), dtype=torch.complex64, device=plan.device) if want_u else None
    hist = (ctypes.c_double * (int(iters) + 1))() if residuals else None
    _lib.check(_lib.load().l2_dual_cg(plan.handle, _ptr(y), _ptr(p), _p_kind(p), float(lam), int(iters), _ptr(x),
                                      _ptr(u), hist, _stream()))
    out = [x]
    if want_u:
        out.append(u)
    if residuals:
        out.append([hist[i] for i in range(int(iters) + 1)])
    return out[0] if len(out) == 1 else tuple(out)


def nufft_destroy(plan: Plan):
    plan.close()


def nufft_autotune(coords, shape, maps=None, oversamp=1.25, kb_width=4) -> dict:
    """Tile shape picked by timing candidate tilings (cached per problem class)."""
    coords = _dev(coords, torch.float32, "coords")
    shape = tuple(int(n) for n in shape)
    d = len(shape)
    C = 1
    if maps is not None:
        maps = _dev(maps, torch.complex64, "maps")
        C = maps.shape[0]
    best = Tuning()
    shp = (ctypes.c_int64 * d)(*shape)
    _lib.check(_lib.load().nufft_autotune(d, shp, C, coords.shape[0], _ptr(coords), _ptr(maps), float(oversamp),
                                          int(kb_width), ctypes.byref(best), _stream()))
    return {"bin_size": tuple(best.bin_size[:d]), "max_chunk": best.max_chunk,
            "spread_bin_size": tuple(best.spread_bin_size[:d])}


class Batch:
    """Plans of many independent 2D slices (owns the library handle)."""

    def __init__(self, handle, shapes, ncoils, nsamples, device, keep):
        self.handle = handle
        self.shapes = [tuple(s) for s in shapes]
        self.ncoils = int(ncoils)
        self.nsamples = [int(m) for m in nsamples]
        self.device = device
        self._keep = keep

    def __len__(self):
        return len(self.shapes)

    def close(self):
        if self.handle:
            _lib.load().nufft_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr_array(ts):
    return (ctypes.c_void_p * len(ts))(*[0 if t is None else t.data_ptr() for t in ts])


def nufft_plan_batch(coords, shapes, maps=None, oversamp=1.25, kb_width=4, tune=True) -> Batch:
    """coords: list of float32 [M_i, 2]; shapes: list of (N0, N1); maps: list of [C, N0, N1] or None."""
    n = len(coords)
    if len(shapes) != n or (maps is not None and len(maps) != n):
        raise ValueError("coords, shapes and maps must have one entry per slice")
    coords = [_dev(c, torch.float32, "coords") for c in coords]
    shapes = [tuple(int(v) for v in s) for s in shapes]
    for c, s in zip(coords, shapes):
        if len(s) != 2 or c.dim() != 2 or c.shape[1] != 2:
            raise ValueError("batched slices are 2D: coords [M, 2], shape (N0, N1)")
    C = 1
    if maps is not None:
        maps = [_dev(m, torch.complex64, "maps") for m in maps]
        C = maps[0].shape[0]
        for m, s in zip(maps, shapes):
            if m.shape[0] != C or tuple(m.shape[1:]) != s:
                raise ValueError("maps must be [C, *shape] with one C for all slices")
    shp = (ctypes.c_int64 * (2 * n))(*[v for s in shapes for v in s])
    ms = (ctypes.c_int64 * n)(*[c.shape[0] for c in coords])
    h = ctypes.c_void_p()
    _lib.check(_lib.load().nufft_plan_batch(ctypes.byref(h), n, shp, ms, C, _ptr_array(coords),
                                            _ptr_array(maps) if maps is not None else None, float(oversamp),
                                            int(kb_width), 1 if tune else 0, _stream()))
    return Batch(h, shapes, C, [c.shape[0] for c in coords], coords[0].device, (coords, maps))


def nufft_batch_info(batch: Batch, slice_index: int) -> dict:
    inf = PlanInfo()
    fast = ctypes.c_int(0)
    _lib.check(_lib.load().nufft_batch_info(batch.handle, int(slice_index), ctypes.byref(inf), ctypes.byref(fast)))
    d = inf.ndim
    return {
        "shape": tuple(inf.shape[:d]), "grid": tuple(inf.grid[:d]), "bin_size": tuple(inf.bin_size[:d]),
        "nwork": inf.nwork, "heavy_tiles": inf.heavy_tiles, "fast": bool(fast.value),
        "spread_bin_size": tuple(inf.spread_bin_size[:d]), "max_chunk": inf.max_chunk,
    }


def pdhg_solve_batch(batch: Batch, y, p=None, lam=1e-3, iters=20, lambda_max=0.0, power_iters=30, sigma0=1.0,
                     accel=True):
    """l2 PDHG on every slice; y: list of [C, M_i]; p: None or list of [M_i] / [C, M_i].

    lambda_max: 0 (power method per slice), one float for every slice, or a
    list with one value per slice."""
    n = len(batch)
    if len(y) != n or (p is not None and len(p) != n):
        raise ValueError("y and p must have one entry per slice")
    y = [_numel(_dev(t, torch.complex64, "y"), batch.ncoils * m, "y[%d]" % i)
         for i, (t, m) in enumerate(zip(y, batch.nsamples))]
    kind = KP_PRECOND_NONE
    if p is not None:
        p = [_dev(t, torch.float32, "p") for t in p]
        kind = _p_kind(p[0])
        # one preconditioner kind for the whole batch: every p must be [M_i]
        # (single-channel) or every p [C, M_i] (multi-channel)
        for i, (t, m) in enumerate(zip(p, batch.nsamples)):
            want = (m,) if kind == KP_PRECOND_SC else (batch.ncoils, m)
            if tuple(t.shape) != want:
                raise ValueError("p[%d] has shape %s, expected %s (all slices need the same preconditioner kind)"
                                 % (i, tuple(t.shape), want))
    o = PdhgOpts()
    o.reg = KP_REG_L2
    o.lam = float(lam)
    o.iters = int(iters)
    o.wavelet_levels = 4
    lm = None
    if isinstance(lambda_max, (list, tuple)):
        if len(lambda_max) != n:
            raise ValueError("lambda_max must have one entry per slice")
        lm = (ctypes.c_float * n)(*[float(v) for v in lambda_max])
        o.lambda_max = 0.0
    else:
        o.lambda_max = float(lambda_max)
    o.power_iters = int(power_iters)
    o.sigma0 = float(sigma0)
    o.accel = 1 if accel else 0
    xs = [torch.empty(s, dtype=torch.complex64, device=batch.device) for s in batch.shapes]
    _lib.check(_lib.load().pdhg_solve_batch(batch.handle, _ptr_array(y), _ptr_array(p) if p is not None else None,
                                            kind, ctypes.byref(o), lm, _ptr_array(xs), _stream()))
    return xs


def nufft_batch_destroy(batch: Batch):
    batch.close()
