"""Host-only checks of the C ABI: the library loads, exports every function that
include/xpcs.h declares, and the ctypes structures match the C layout."""

import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from tests.conftest import ROOT

INCLUDE = os.path.join(ROOT, "include")
HEADER = os.path.join(INCLUDE, "xpcs.h")


def _declared_functions(path=HEADER):
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:xpcs_status|void|const char \*|size_t|int32_t|int64_t)\s*\**\s*(\w+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def _all_declared():
    names = []
    for h in sorted(os.listdir(INCLUDE)):
        if h.endswith(".h"):
            names += _declared_functions(os.path.join(INCLUDE, h))
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2407_20356_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2407_20356_amd import build
        build.build_library()
    return _lib.load()


def test_header_declares_the_three_paper_calls():
    names = _declared_functions()
    for n in ("compress_frames", "correlate_two_time", "g2_from_two_time", "correlate_two_time_raw",
              "xpcs_create", "xpcs_destroy", "xpcs_sync", "xpcs_set_stream", "xpcs_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2407_20356_amd import _lib
    names = _declared_functions()
    for n in names:
        assert hasattr(lib, n), f"{n} declared in xpcs.h but not exported"
    # the binding declares exactly the header's functions
    assert sorted(_lib.SIGNATURES) == names
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    for n in _all_declared():
        assert n in exported, f"{n} declared in include/ but not exported"
    # and every exported C entry point is declared in include/
    ours = {n for n in exported if n.startswith("xpcs_") or n in ("compress_frames", "correlate_two_time",
                                                                  "correlate_two_time_raw", "g2_from_two_time")}
    assert ours <= set(_all_declared()), ours - set(_all_declared())


def test_struct_layout_matches_header():
    from paper_2407_20356_amd import _lib
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "xpcs.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(xpcs_factors), offsetof(xpcs_factors, k),
         offsetof(xpcs_factors, n_roi), offsetof(xpcs_factors, U), offsetof(xpcs_factors, sigma),
         offsetof(xpcs_factors, V), offsetof(xpcs_factors, roi_npix), offsetof(xpcs_factors, roi_sum),
         offsetof(xpcs_factors, roi_gram));
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(xpcs_compress_opts), offsetof(xpcs_compress_opts, oversample),
         offsetof(xpcs_compress_opts, power_iters), offsetof(xpcs_compress_opts, precision),
         offsetof(xpcs_compress_opts, seed), offsetof(xpcs_compress_opts, basis));
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(xpcs_stream_desc), offsetof(xpcs_stream_desc, dtype),
         offsetof(xpcs_stream_desc, n_roi), offsetof(xpcs_stream_desc, k), offsetof(xpcs_stream_desc, roi_label),
         offsetof(xpcs_stream_desc, basis), offsetof(xpcs_stream_desc, window), offsetof(xpcs_stream_desc, max_block));
  printf("%d %d %d %d %d %d\n", XPCS_U8, XPCS_U16, XPCS_F32, XPCS_F64, XPCS_ALL_ROIS, XPCS_PREC_BF16);
  printf("%d %d %d %d %d\n", XPCS_EQUEUED, XPCS_STREAM_QUEUED, XPCS_STREAM_ADMITTED, XPCS_STREAM_FAILED,
         XPCS_PREC_FP8);
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    F, O = _lib.XpcsFactors, _lib.XpcsCompressOpts
    want_f = [ctypes.sizeof(F), F.k.offset, F.n_roi.offset, F.U.offset, F.sigma.offset, F.V.offset,
              F.roi_npix.offset, F.roi_sum.offset, F.roi_gram.offset]
    assert [int(x) for x in lines[0].split()] == want_f
    want_o = [ctypes.sizeof(O), O.oversample.offset, O.power_iters.offset, O.precision.offset, O.seed.offset,
              O.basis.offset]
    assert [int(x) for x in lines[1].split()] == want_o
    D = _lib.XpcsStreamDesc
    want_d = [ctypes.sizeof(D), D.dtype.offset, D.n_roi.offset, D.k.offset, D.roi_label.offset, D.basis.offset,
              D.window.offset, D.max_block.offset]
    assert [int(x) for x in lines[2].split()] == want_d
    assert [int(x) for x in lines[3].split()] == [_lib.XPCS_U8, _lib.XPCS_U16, _lib.XPCS_F32, _lib.XPCS_F64,
                                                   _lib.XPCS_ALL_ROIS, _lib.XPCS_PREC_BF16]
    assert [int(x) for x in lines[4].split()] == [_lib.XPCS_EQUEUED, _lib.XPCS_STREAM_QUEUED,
                                                   _lib.XPCS_STREAM_ADMITTED, _lib.XPCS_STREAM_FAILED,
                                                   _lib.XPCS_PREC_FP8]


def test_null_context_is_rejected_without_a_gpu(lib):
    # Entry points check their arguments before touching the device.
    assert lib.compress_frames(None, None, 1, 1, 1, None, 1, None, None) == -1
    assert lib.correlate_two_time(None, None, 0, 0, 1, None, 10, 1, None, None) == -1
    assert lib.correlate_two_time_raw(None, None, 1, 1, 1, None, 1, 0, 0, 1, None, 10, 1, None, None, None) == -1
    assert lib.g2_from_two_time(None, None, 10, 1, 1, None, None) == -1
    assert lib.g2_from_factors(None, None, 0, 0, 1, None, None) == -1
    assert lib.fit_relaxation(None, None, None, 1, 1, 0, 1, None, 10, None, None) == -1
    assert lib.two_time_stats(None, None, 0, 0, 1, None, None, None) == -1
    assert lib.xpcs_sync(None) == -1
    assert lib.xpcs_last_error(None) == b""
    assert lib.xpcs_stream_open(None, None, None) == -1
    assert lib.xpcs_stream_push(None, None, 1, None, 10) == -1
    assert lib.xpcs_stream_g2(None, None, None) == -1
    assert lib.xpcs_stream_frames(None) == 0
    lib.xpcs_stream_close(None)
    lib.xpcs_destroy(None)
    assert lib.xpcs_server_create(0, 0, 1, 1, None) == -1
    assert lib.xpcs_server_open(None, None, None, None) == -1
    assert lib.xpcs_server_state(None, 1, None) == -1
    assert lib.xpcs_server_push(None, 1, None, 1, None, 10, None) == -1
    assert lib.xpcs_server_poll(None, 1, 1, None, None, None) == -1
    assert lib.xpcs_server_g2(None, 1, None, None) == -1
    assert lib.xpcs_server_wait(None, 0) == -1
    assert lib.xpcs_server_close(None, 1) == -1
    assert lib.xpcs_server_stats(None, None, None, None) == -1
    assert lib.xpcs_server_last_error(None) == b"NULL server"
    lib.xpcs_server_destroy(None)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2407_20356_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _lib.load()
