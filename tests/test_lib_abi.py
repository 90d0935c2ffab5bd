"""The C-ABI library loads, exports every declared symbol, and validates
arguments on the host (no device work)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1902_09657_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libkpdhg.so not built")
    return L


def _declared():
    src = open(os.path.join(ROOT, "include", "kpdhg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_and_binding_agree():
    L = _lib()
    assert _declared() == sorted(L.EXPORTS)


def test_every_symbol_exported():
    L = _lib()
    lib = L.load()
    for name in _declared():
        assert hasattr(lib, name), name


def _validate(**kw):
    L = _lib()
    lib = L.load()
    args = dict(ndim=2, shape=(16, 16), ncoils=1, nsamples=10, coords=1, maps=None, oversamp=1.25, kb_width=4,
                tuning=None)
    args.update(kw)
    shp = (ctypes.c_int64 * max(1, len(args["shape"])))(*args["shape"])
    tun = args["tuning"]
    return lib.nufft_plan_validate(args["ndim"], shp, args["ncoils"], args["nsamples"],
                                   ctypes.c_void_p(args["coords"]), ctypes.c_void_p(args["maps"]),
                                   args["oversamp"], args["kb_width"],
                                   ctypes.byref(tun) if tun is not None else None)


def test_validation_error_paths():
    L = _lib()
    assert _validate() == 0
    assert _validate(ndim=4, shape=(4, 4, 4, 4)) == L.KP_ERR_INVALID_ARG
    assert _validate(shape=(15, 16)) == L.KP_ERR_INVALID_ARG          # odd N
    assert _validate(ncoils=0) == L.KP_ERR_INVALID_ARG
    assert _validate(nsamples=0) == L.KP_ERR_INVALID_ARG
    assert _validate(coords=None) == L.KP_ERR_INVALID_ARG
    assert _validate(ncoils=4, maps=None) == L.KP_ERR_INVALID_ARG     # maps required
    assert _validate(oversamp=1.1) == L.KP_ERR_INVALID_ARG
    assert _validate(kb_width=5) == L.KP_ERR_INVALID_ARG
    assert _validate(ncoils=32, maps=8) == L.KP_ERR_UNSUPPORTED
    t = L.Tuning()
    t.bin_size[0] = 7                                                  # 7 does not divide 20
    assert _validate(tuning=t) == L.KP_ERR_INVALID_ARG
    msg = L.load().kp_last_error().decode()
    assert "bin_size" in msg


def test_library_db4_matches_oracle():
    """The library derives its own db4 filter; it must equal the oracle's."""
    L = _lib()
    from oracle import wavelet
    h = (ctypes.c_double * 8)()
    assert L.load().kp_db4_filter(h) == 0
    np.testing.assert_allclose(np.array(h[:]), wavelet.db4_filter(), rtol=0, atol=1e-13)


def test_binding_size_checks():
    """The binding's size checks (host only: CPU tensors)."""
    import torch
    from paper_1902_09657_amd import _numel, _p_numel, _nimg
    assert _nimg((4, 5, 6)) == 120
    t = torch.zeros(3, 7)
    assert _numel(t, 21, "t") is t
    with pytest.raises(ValueError):
        _numel(t, 20, "t")
    assert _p_numel(torch.zeros(7), 3, 7) is not None          # single-channel [M]
    assert _p_numel(torch.zeros(3, 7), 3, 7) is not None       # multi-channel [C, M]
    with pytest.raises(ValueError):
        _p_numel(torch.zeros(21), 3, 7)                        # flat [C*M] read as [M]
    with pytest.raises(ValueError):
        _p_numel(torch.zeros(2, 7), 3, 7)


def test_missing_library_fails_loudly():
    """No fallback: a missing shared library is an error, not a slower path."""
    import subprocess
    import sys
    code = ("from paper_1902_09657_amd import _lib\n"
            "try:\n    _lib.load('/nonexistent/libkpdhg.so')\nexcept ImportError:\n    print('raised')\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert out.stdout.strip() == "raised", out.stderr


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1902_09657_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", src, flags=re.M), f
