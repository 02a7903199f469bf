"""AddressSanitizer + UndefinedBehaviorSanitizer runs of the CPU-side code: the oracle (every
entry point on small sketches) and the host-only paths of the C ABI (validation, error
texts, the tuning cache file).  Host code only: the device code of the library is built
without sanitizers, and nothing here touches a GPU."""
import os
import subprocess

import pytest

from conftest import ROOT

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/lib/llvm/bin/clang++"
CSRC = os.path.join(ROOT, "paper_1805_09246_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")

pytestmark = pytest.mark.slow


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
          "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
          os.path.join(ROOT, "oracle", "sps_oracle.c"),
          os.path.join(ROOT, "tests", "csrc", "oracle_sanitize.c"), "-o", exe, "-lm",
          "-lpthread"])
    assert "oracle sanitizer run ok" in _run([exe], env=ENV)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_abi_host_paths_under_asan_ubsan(tmp_path):
    t = str(tmp_path)
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer"]
    common = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include")]
    objs = []
    for src in ("sps_api.hip", "sps_kernels.hip", "sps_mlp.hip"):
        o = os.path.join(t, src + ".o")
        _run(common + host_san + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    drv = os.path.join(t, "drv.o")
    _run([CLANGXX, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
          "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-c",
          os.path.join(ROOT, "tests", "csrc", "abi_host_sanitize.cpp"), "-o", drv])
    exe = os.path.join(t, "abi_san")
    _run([HIPCC, "--offload-arch=gfx950"] + host_san[:4] + [drv] + objs + ["-o", exe])
    assert "host ABI sanitizer run ok" in _run([exe, t], env=ENV)
