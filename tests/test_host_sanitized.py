"""The C ABI's host-side error paths under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; the device code is built as
usual): every translation unit of the library is compiled with the host
sanitizers, linked with tests/host/error_paths.cpp, and run.  Every call the
driver makes returns before any device work, so no GPU is needed."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1902_09657_amd", "csrc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    pytest.skip("hipcc not found")


@pytest.mark.timeout(900)
def test_error_paths_under_host_sanitizers(tmp_path):
    from paper_1902_09657_amd import build as B
    hipcc = _hipcc()

    def comp(src):
        obj = str(tmp_path / src.replace(".hip", ".o"))
        cmd = [hipcc, *B.FLAGS, *B.PER_FILE.get(src, []), *SAN, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(comp, B.SOURCES))
    drv = str(tmp_path / "error_paths.o")
    cmd = [hipcc, "-x", "c++", "-std=c++17", *SAN, "-c", os.path.join(ROOT, "tests", "host", "error_paths.cpp"),
           "-o", drv]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "error_paths")
    cmd = [hipcc, "--offload-arch=gfx950", *SAN, drv, *objs, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="-1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "OK: 0 failed checks" in r.stdout, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
