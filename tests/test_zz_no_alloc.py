"""nufft_forward_noalloc (the forward NUFFT with its FFT grids in the
library's static per-device array) against nufft_forward, called through the
C ABI: two calls in a row, the second with a smaller plan and input, on 2D
and 3D plans; a plan whose grid exceeds the static array is refused."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _abi_noalloc(kp, plan, x, y):
    """Call the entry point through the C ABI directly (ctypes)."""
    from paper_1902_09657_amd import _lib
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return _lib.load().nufft_forward_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()),
                                             ctypes.c_void_p(y.data_ptr()), s)


def _case(shape, C, M, seed):
    rng = np.random.default_rng(seed)
    k = synth.random_coords(M, len(shape), rng)
    maps = synth.coil_maps(shape, C, rng)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return k, maps, x


@pytest.mark.parametrize("first,second", [
    (((96, 80), 8, 9000), ((40, 48), 3, 2000)),            # 2D: 120 x 100 grid, then 50 x 60
    (((48, 40, 32), 4, 20000), ((24, 16, 32), 2, 3000)),   # 3D (support-pruned axis-0 passes)
])
def test_noalloc_forward_equals_forward(first, second):
    import paper_1902_09657_amd as kp
    for n, (shape, C, M) in enumerate((first, second)):
        print("noalloc call", n, shape, C, M, flush=True)
        k, maps, x = _case(shape, C, M, 40 + n)
        plan = kp.nufft_plan(_dev(k, torch.float32), shape, _dev(maps, torch.complex64), oversamp=1.25, kb_width=4)
        xt = _dev(x, torch.complex64)
        want = kp.nufft_forward(plan, xt)
        got = torch.full((C, M), float("nan"), dtype=torch.complex64, device="cuda")
        assert _abi_noalloc(kp, plan, xt, got) == 0
        torch.cuda.synchronize()
        # the same kernels on the same inputs: identical results
        assert torch.equal(got, want), float((got - want).abs().max())
        # the binding's wrapper of the same entry point
        got2 = torch.empty_like(got)
        kp.nufft_forward_noalloc(plan, xt, got2)
        assert torch.equal(got2, want)
        plan.close()


def test_noalloc_refuses_large_grid():
    import paper_1902_09657_amd as kp
    # 2D 256^2 image, alpha 2: 512^2 grid x 9 coils x 8 B = 18.9 MB > 16 MiB
    k, maps, x = _case((256, 256), 9, 1000, 50)
    plan = kp.nufft_plan(_dev(k, torch.float32), (256, 256), _dev(maps, torch.complex64), oversamp=2.0,
                         kb_width=4)
    y = torch.empty((9, 1000), dtype=torch.complex64, device="cuda")
    with pytest.raises(kp.KpError) as ei:
        kp.nufft_forward_noalloc(plan, _dev(x, torch.complex64), y)
    assert ei.value.code == -2 and "16777216" in str(ei.value)
    plan.close()
