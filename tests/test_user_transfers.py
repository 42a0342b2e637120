"""User transfer specialisations (Sec. VII-B: user implementations of
transfers between layouts, with a priority that falls back to more general
ones).  The registry's order and fallback are checked on the host: the
callbacks here enqueue nothing, so rl_convert / rl_transfer never reach the
device.  A GPU test runs a real user transfer against the oracle."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2511_04853_amd as P
import workloads as W
from tests import rlhelp as H


def fake_views(sp, n, src_kind=("aos", 0), dst_kind=("soa", 0), src_space="device"):
    """Views over host arrays standing in for device buffers (validation
    reads only their addresses)."""
    sl = sp.layout(*src_kind, space=src_space)
    dl = sp.layout(*dst_kind)
    sb = [np.zeros(max(1, b), np.uint8) for b in sl.lib.buffer_bytes(n)]
    db = [np.zeros(max(1, b), np.uint8) for b in dl.lib.buffer_bytes(n)]
    return sl, dl, P.View(sl.lib, n, sb), P.View(dl.lib, n, db)


class Recorder:
    def __init__(self, name, status, log):
        self.name, self.status, self.log = name, status, log

    def __call__(self, src, dst, n, stream, user):
        self.log.append((self.name, n, src.contents.layout, dst.contents.layout))
        return self.status


def test_priority_order_and_fallback():
    sp = H.SchemaPair(W.PLAIN8)
    sl, dl, sv, dv = fake_views(sp, 100)
    log = []
    ids = []
    try:
        i1, k1 = P.register_transfer(sl.lib, dl.lib, 10, Recorder("low", P.RL_OK, log))
        ids.append(i1)
        assert P.lib().rl_convert(sv.ref(), dv.ref(), 100, None) == P.RL_OK
        assert [e[0] for e in log] == ["low"] and log[0][1] == 100
        assert log[0][2] == sl.lib.handle.value and log[0][3] == dl.lib.handle.value
        i2, k2 = P.register_transfer(sl.lib, dl.lib, 20, Recorder("declines", P.RL_EUNSUPPORTED, log))
        ids.append(i2)
        log.clear()
        assert P.lib().rl_convert(sv.ref(), dv.ref(), 100, None) == P.RL_OK
        assert [e[0] for e in log] == ["declines", "low"]
        i3, k3 = P.register_transfer(sl.lib, None, 30, Recorder("fails", P.RL_EINVAL, log))
        ids.append(i3)
        log.clear()
        assert P.lib().rl_convert(sv.ref(), dv.ref(), 100, None) == P.RL_EINVAL
        assert [e[0] for e in log] == ["fails"]
        assert "user transfer" in P.rl_last_error()
        P.unregister_transfer(i3)
        ids.remove(i3)
        log.clear()
        assert P.lib().rl_convert(sv.ref(), dv.ref(), 100, None) == P.RL_OK
        assert [e[0] for e in log] == ["declines", "low"]
        # equal priorities: registration order
        i4, k4 = P.register_transfer(sl.lib, dl.lib, 20, Recorder("second20", P.RL_OK, log))
        ids.append(i4)
        log.clear()
        assert P.lib().rl_convert(sv.ref(), dv.ref(), 100, None) == P.RL_OK
        assert [e[0] for e in log] == ["declines", "second20"]
    finally:
        for i in ids:
            P.unregister_transfer(i)


def test_wildcards_and_non_matching_pairs():
    sp = H.SchemaPair(W.PLAIN8)
    sl, dl, sv, dv = fake_views(sp, 64, dst_kind=("aosoa", 16))
    other = sp.layout("soa")
    log = []
    i_any_dst, k1 = P.register_transfer(sl.lib, None, 5, Recorder("src-any", P.RL_OK, log))
    i_other, k2 = P.register_transfer(other.lib, dl.lib, 50, Recorder("other-pair", P.RL_OK, log))
    try:
        assert P.lib().rl_convert(sv.ref(), dv.ref(), 64, None) == P.RL_OK
        assert [e[0] for e in log] == ["src-any"]
        # a layout of another schema never matches
        sp2 = H.SchemaPair(W.CELL)
        sl2, dl2, sv2, dv2 = fake_views(sp2, 8)
        i_dst_any, k3 = P.register_transfer(None, dl2.lib, 1, Recorder("cell-dst", P.RL_OK, log))
        log.clear()
        assert P.lib().rl_convert(sv.ref(), dv.ref(), 64, None) == P.RL_OK
        assert [e[0] for e in log] == ["src-any"]
        P.unregister_transfer(i_dst_any)
    finally:
        P.unregister_transfer(i_any_dst)
        P.unregister_transfer(i_other)


def test_rl_transfer_consults_the_registry():
    sp = H.SchemaPair(W.PLAIN8)
    sl, dl, sv, dv = fake_views(sp, 10, src_space="pinned")
    log = []
    i, k = P.register_transfer(sl.lib, dl.lib, 0, Recorder("h2d", P.RL_OK, log))
    try:
        o = P.rl_xfer_opts(0)
        assert P.lib().rl_transfer(sv.ref(), dv.ref(), 10, None, ctypes.byref(o)) == P.RL_OK
        assert [e[0] for e in log] == ["h2d"]
    finally:
        P.unregister_transfer(i)


def test_registration_errors():
    sp = H.SchemaPair(W.PLAIN8)
    a = sp.layout("aos")
    c = H.SchemaPair(W.CELL).layout("soa")
    cb = P.TRANSFER_FN(lambda *args: 0)
    i = ctypes.c_uint64()
    assert P.lib().rl_register_transfer(a.lib.handle, None, 0, P.TRANSFER_FN(), None, ctypes.byref(i)) == P.RL_EINVAL
    assert P.lib().rl_register_transfer(None, None, 0, cb, None, ctypes.byref(i)) == P.RL_EINVAL
    assert P.lib().rl_register_transfer(a.lib.handle, c.lib.handle, 0, cb, None, ctypes.byref(i)) == P.RL_EINVAL
    assert P.lib().rl_unregister_transfer(10 ** 12) == P.RL_EINVAL


@pytest.mark.gpu
def test_user_transfer_on_the_device_matches_the_oracle():
    """A user implementation of records -> columns for the plain schema
    (torch slicing of the record bytes) registered above the library's own:
    its output equals the oracle's conversion, and declining hands the call
    to the library's kernels with the same result."""
    torch = pytest.importorskip("torch")
    sp = H.SchemaPair(W.PLAIN8)
    aos, soa = sp.layout("aos"), sp.layout("soa")
    n = 10_000
    v = W.plain_values(n, seed=3)
    sb = oracle.pack(sp.orc, v, aos.orc)
    st, want, _ = oracle.convert(aos.orc, sb, soa.orc, n)
    dsrc = H.to_device(sb)
    ddst = H.alloc_device(soa.lib.buffer_bytes(n))
    offs, stride = aos.lib.slot_offsets, aos.lib.stride
    sizes = [W.TYPE_SIZE[f.type] for f in W.PLAIN8.fields]
    calls = []
    decline = [False]

    def user(src, dst, cnt, stream, u):
        calls.append(cnt)
        if decline[0]:
            return P.RL_EUNSUPPORTED
        assert src.contents.buffers[0] == dsrc[0].data_ptr()
        rec = dsrc[0][:cnt * stride].view(cnt, stride)
        for c, (o, s) in enumerate(zip(offs, sizes)):
            ddst[c][:cnt * s].view(cnt, s).copy_(rec[:, o:o + s])
        return P.RL_OK

    i, keep = P.register_transfer(aos.lib, soa.lib, 100, user)
    try:
        P.convert(P.View(aos.lib, n, dsrc), P.View(soa.lib, n, ddst), n)
        torch.cuda.synchronize()
        assert calls == [n]
        H.assert_same_bytes(H.to_numpy(ddst), want, "user transfer")
        ddst2 = H.alloc_device(soa.lib.buffer_bytes(n))
        decline[0] = True
        P.convert(P.View(aos.lib, n, dsrc), P.View(soa.lib, n, ddst2), n)
        assert P.sync() == 0
        assert calls == [n, n]
        H.assert_same_bytes(H.to_numpy(ddst2), want, "declined: library kernels")
    finally:
        P.unregister_transfer(i)


@pytest.mark.gpu
def test_a_user_transfer_can_wrap_the_library_transfer():
    """A specialisation that calls rl_convert itself (for instance to do
    work around the default conversion) reaches the library's own kernels:
    it runs once, does not recurse, and the result is the oracle's."""
    pytest.importorskip("torch")
    sp = H.SchemaPair(W.CELL)
    aos, soa = sp.layout("aos"), sp.layout("soa", storage=H.narrowed_storage(W.CELL))
    n = 50_001
    v = W.cell_values(n, seed=8)
    sb = oracle.pack(sp.orc, v, aos.orc)
    st, want, _ = oracle.convert(aos.orc, sb, soa.orc, n)
    assert st == 0
    dsrc = H.to_device(sb)
    ddst = H.alloc_device(soa.lib.buffer_bytes(n))
    calls, nested = [], []

    def wrapper(src, dst, cnt, stream, u):
        calls.append(cnt)
        r = P.lib().rl_convert(src, dst, cnt, ctypes.c_void_p(stream))
        nested.append(r)
        return r

    i, keep = P.register_transfer(aos.lib, soa.lib, 5, wrapper)
    try:
        P.convert(P.View(aos.lib, n, dsrc), P.View(soa.lib, n, ddst), n)
        assert P.sync() == 0, P.rl_last_error()
        assert calls == [n] and nested == [P.RL_OK]
        H.assert_same_bytes(H.to_numpy(ddst), want, "wrapped library transfer")
    finally:
        P.unregister_transfer(i)
