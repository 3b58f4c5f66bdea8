"""The host side of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer,
on the CPU (no GPU needed).

The library's sources are compiled with the sanitizers on their host code only
(each -fsanitize flag behind -Xarch_host; device code is built as usual) and
linked with tests/asan/host_check.c into one executable, which exercises every
entry point's argument checks with NULL handles and pointers, context and server
creation on devices that do not exist, and the factors-file header parser on a
valid header, every truncation and every single-byte corruption.  A sanitizer
report aborts the run.  Objects are kept under tests/asan/_build and rebuilt when
their source or a header changes.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2407_20356_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(ROOT, "tests", "asan", "_build")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined"]
DEVICE = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _newest_header():
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    hs += [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE)]
    return max(os.path.getmtime(h) for h in hs)


def _compile(src, hdr_time):
    obj = os.path.join(OUT, os.path.basename(src) + ".o")
    if os.path.exists(obj) and os.path.getmtime(obj) > max(os.path.getmtime(src), hdr_time):
        return obj
    cmd = [HIPCC, "-O1", "-g", "-fPIC", "-std=c++17", "--offload-arch=gfx950", "-fno-omit-frame-pointer",
           *SAN_HOST, *DEVICE, "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"compile failed: {src}\n{r.stderr[-3000:]}")
    return obj


def _build():
    import concurrent.futures as cf
    os.makedirs(OUT, exist_ok=True)
    hdr = _newest_header()
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(lambda s: _compile(s, hdr), srcs))
    drv = os.path.join(ROOT, "tests", "asan", "host_check.c")
    dobj = os.path.join(OUT, "host_check.o")
    r = subprocess.run([CLANG, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                        "-I", INCLUDE, "-c", drv, "-o", dobj], capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(r.stderr[-3000:])
    exe = os.path.join(OUT, "host_check")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", *SAN_HOST, *objs, dobj, "-o", exe],
                       capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(r.stderr[-3000:])
    return exe


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not found")
@pytest.mark.timeout(900)
def test_host_side_under_address_and_ub_sanitizers(tmp_path):
    exe = _build()
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["HIP_VISIBLE_DEVICES"] = ""          # the host paths only, also on a machine with a GPU
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=300)
    sys.stdout.write(r.stdout)
    sys.stderr.write(r.stderr[-5000:])
    assert r.returncode == 0, r.stderr[-3000:]
    assert "host checks passed" in r.stdout
