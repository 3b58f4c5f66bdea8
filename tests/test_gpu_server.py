"""Serving (xpcs_server_*): many online streams on one GPU, through the C ABI.

A stream served in a mix -- detectors of different sizes, ROI maps, windows and
count types, blocks interleaved across lanes that run concurrently -- must give
exactly what the same stream gives alone (xpcs_stream_*): the same kernels on the
same data in the same order, so band rows and g2 sums are compared bit for bit.
Admission is checked on both limits: slots (max_streams) and the HBM budget.
"""

import functools

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import say, to_dev, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


def _spec(side_h, side_w, n_roi, k, window, dtype, blocks, seed):
    labels = synth.annular_labels(side_h, side_w, n_roi, r_in=2.0)
    M = side_h * side_w
    F = synth.speckle_frames_numpy(M, sum(blocks) + 200, 0.4, 0.2, 25.0, dtype, seed=seed)
    U, _, _ = O.exact_basis(F[:200], k)
    return dict(labels=labels, n_roi=n_roi, F=F[200:], U=U, window=window, blocks=blocks, dtype=dtype)


@functools.lru_cache(maxsize=None)
def _specs():
    return [
        _spec(48, 48, 3, 16, 200, "u8", [100, 64, 128, 37], 21),
        _spec(40, 64, 5, 24, 90, "u16", [50, 50, 50, 21], 22),
        _spec(32, 32, 2, 8, 300, "u8", [256, 44], 23),
    ]


def _dev(sp):
    import torch
    F = sp["F"]
    Fd = to_dev(F.view(np.int16)).view(torch.uint16) if F.dtype == np.uint16 else to_dev(F)
    Ud = to_dev(np.ascontiguousarray(sp["U"].T.astype(np.float32)))
    Ld = to_dev(sp["labels"].astype(np.int32))
    return Fd, Ud, Ld


def _alone(sp):
    """The stream by itself on a fresh context (xpcs_stream_*)."""
    import torch
    from paper_2407_20356_amd import api
    Fd, Ud, Ld = _dev(sp)
    ctx = api.Context(0)
    s = api.Stream(ctx, Ld, sp["n_roi"], Ud, window=sp["window"], max_block=max(sp["blocks"]),
                   dtype=torch.uint16 if sp["dtype"] == "u16" else torch.uint8)
    bands, t = [], 0
    for b in sp["blocks"]:
        bands.append(s.push(Fd[t:t + b]))
        t += b
    g2, npairs = s.g2()
    ctx.sync()
    out = [to_np(x) for x in bands], to_np(g2), to_np(npairs)
    s.close()
    ctx.close()
    return out


def _same(a, b):
    np.testing.assert_array_equal(np.nan_to_num(a, nan=-7.0), np.nan_to_num(b, nan=-7.0))


def test_streams_in_a_mix_equal_streams_alone():
    import torch
    from paper_2407_20356_amd import api
    SPECS = _specs()
    srv = api.Server(0, lanes=2, max_streams=8)
    devs = [_dev(sp) for sp in SPECS]
    ids = []
    for sp, (Fd, Ud, Ld) in zip(SPECS, devs):
        sid, state = srv.open(Ld, sp["n_roi"], Ud, sp["window"], max(sp["blocks"]),
                              dtype=torch.uint16 if sp["dtype"] == "u16" else torch.uint8)
        assert state == api.L.XPCS_STREAM_ADMITTED
        ids.append(sid)
    bands = [[] for _ in SPECS]
    pos = [0] * len(SPECS)
    for step in range(max(len(sp["blocks"]) for sp in SPECS)):          # blocks interleaved across streams
        for i, sp in enumerate(SPECS):
            if step < len(sp["blocks"]):
                b = sp["blocks"][step]
                say(f"server push stream {i} block {step} ({b} frames)")
                bands[i].append(srv.push(ids[i], devs[i][0][pos[i]:pos[i] + b]))
                pos[i] += b
    g2s = [srv.g2(sid) for sid in ids]
    srv.wait()
    for i, sp in enumerate(SPECS):
        done = srv.poll(ids[i])
        assert [f for _, f in done] == sp["blocks"]
        assert all(lat > 0 for lat, _ in done)
    used, admitted, queued = srv.stats()
    assert admitted == 3 and queued == 0 and used > 0
    for i, sp in enumerate(SPECS):
        say(f"stream {i} alone")
        ab, ag2, anp = _alone(sp)
        for x, y in zip(bands[i], ab):
            _same(to_np(x), y)
        _same(to_np(g2s[i][0]), ag2)
        np.testing.assert_array_equal(to_np(g2s[i][1]), anp)
        srv.close(ids[i])
    assert srv.stats()[1] == 0
    srv.destroy()


def test_admission_by_slots_and_by_budget():
    import torch
    from paper_2407_20356_amd import api
    sp = _specs()[0]
    Fd, Ud, Ld = _dev(sp)
    mb = max(sp["blocks"])

    # slots: the third request waits until a stream closes
    srv = api.Server(0, lanes=2, max_streams=2)
    a, sa = srv.open(Ld, sp["n_roi"], Ud, sp["window"], mb)
    b, sb = srv.open(Ld, sp["n_roi"], Ud, sp["window"], mb)
    c, sc = srv.open(Ld, sp["n_roi"], Ud, sp["window"], mb)
    assert (sa, sb, sc) == (api.L.XPCS_STREAM_ADMITTED, api.L.XPCS_STREAM_ADMITTED, api.L.XPCS_STREAM_QUEUED)
    assert srv.stats()[1:] == (2, 1)
    with pytest.raises(api.XpcsError, match="EQUEUED"):
        srv.push(c, Fd[:10])
    srv.close(a)
    assert srv.state(c) == api.L.XPCS_STREAM_ADMITTED
    srv.destroy()

    # budget: learn one stream's state bytes, then allow one stream and half of another
    probe = api.Server(0, lanes=1, max_streams=4)
    probe.open(Ld, sp["n_roi"], Ud, sp["window"], mb)
    one = probe.stats()[0]
    probe.open(Ld, sp["n_roi"], Ud, sp["window"], mb)
    state_bytes = probe.stats()[0] - one
    probe.destroy()
    assert state_bytes > 0
    srv = api.Server(0, hbm_budget_bytes=one + state_bytes // 2, lanes=1, max_streams=4)
    a, sa = srv.open(Ld, sp["n_roi"], Ud, sp["window"], mb)
    b, sb = srv.open(Ld, sp["n_roi"], Ud, sp["window"], mb)
    assert (sa, sb) == (api.L.XPCS_STREAM_ADMITTED, api.L.XPCS_STREAM_QUEUED)
    say("budget: push to the admitted stream, then close it to admit the waiting one")
    srv.push(a, Fd[:mb])
    srv.close(a)
    assert srv.state(b) == api.L.XPCS_STREAM_ADMITTED
    bands, t = [], 0
    for blk in sp["blocks"]:
        bands.append(srv.push(b, Fd[t:t + blk]))
        t += blk
    g2, npairs = srv.g2(b)
    srv.wait(b)
    ab, ag2, anp = _alone(sp)
    for x, y in zip(bands, ab):
        _same(to_np(x), y)
    _same(to_np(g2), ag2)
    np.testing.assert_array_equal(to_np(npairs), anp)
    srv.destroy()

    # a stream that cannot fit even alone is refused
    tiny = api.Server(0, hbm_budget_bytes=1 << 16, lanes=1, max_streams=4)
    with pytest.raises(api.XpcsError, match="EBUDGET"):
        tiny.open(Ld, sp["n_roi"], Ud, sp["window"], mb)
    tiny.destroy()
