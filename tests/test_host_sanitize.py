"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU, no GPU): gempic.hip and denoise.hip compiled with the sanitizers on the
host side only (the device code is built as usual and never runs), linked
with tests/host_checks.c, which drives every configuration the C ABI must
reject, the NULL-argument paths, the error strings and the clean-up of a
handle whose device allocation fails.  Any sanitizer report aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
FLAGS = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


@pytest.mark.slow
@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_code_under_sanitizers(tmp_path):
    srcs = [os.path.join(ROOT, "paper_2509_16793_amd", "csrc", f) for f in ("gempic.hip", "denoise.hip")]
    objs, procs = [], []
    for src in srcs:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        procs.append(subprocess.Popen([HIPCC] + FLAGS + HOST_SAN + ["-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    drv = str(tmp_path / "host_checks.o")
    procs.append(subprocess.Popen([HIPCC] + FLAGS + HOST_SAN + ["-x", "c++", "-c",
                                  os.path.join(ROOT, "tests", "host_checks.c"), "-o", drv],
                                  stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for p in procs:
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, out.decode(errors="replace")[-2000:]
    exe = str(tmp_path / "host_checks")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950"] + HOST_SAN + [drv] + objs + ["-o", exe],
                       capture_output=True, timeout=300)
    assert r.returncode == 0, r.stderr.decode(errors="replace")[-2000:]
    env = dict(os.environ)
    # the HIP runtime's own allocations at load are not the library's
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["HIP_VISIBLE_DEVICES"] = ""
    r = subprocess.run([exe], capture_output=True, timeout=120, env=env)
    out = r.stdout.decode(errors="replace") + r.stderr.decode(errors="replace")
    assert r.returncode == 0 and "host checks ok" in out, out[-3000:]
