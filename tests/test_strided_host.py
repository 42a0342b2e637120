"""Host-side behaviour of strided layouts (a user's index-to-address map,
Sec. VII-B) that needs no GPU: layout validation, buffer sizes against the
oracle's, and the checks every entry point makes before any device work."""
import ctypes

import pytest

import oracle
import paper_2511_04853_amd as P
import workloads as W


def test_layout_validation():
    s = P.Schema(W.PLAIN8)
    P.Layout(s, "strided")
    P.Layout(s, "strided", leaf_strides=[8, 4, 12, 400, 16, 2, 1, 4], indexed=True)
    for bad in ([0, 4, 4, 4, 8, 2, 1, 4],        # zero
                [6, 4, 4, 4, 8, 2, 1, 4],        # not a multiple of 4
                [4, 4, 4, 4, 12, 2, 1, 4],       # f64 leaf: 12 is not a multiple of 8
                [4, 4, 4, 4, 8, 2, 1, 1 << 31]):  # too large
        with pytest.raises(P.RelayoutError) as e:
            P.Layout(s, "strided", leaf_strides=bad)
        assert e.value.status == P.RL_EINVAL, bad
    with pytest.raises(P.RelayoutError) as e:
        P.Layout(P.Schema(W.CLUSTER), "strided")
    assert e.value.status == P.RL_EUNSUPPORTED
    d = P.rl_layout_desc()      # a kind past RL_STRIDED
    d.kind = 4
    h = ctypes.c_void_p()
    assert P.lib().rl_layout_create(s.handle, ctypes.byref(d), ctypes.byref(h)) == P.RL_EINVAL


@pytest.mark.parametrize("decl", [W.PLAIN8, W.CELL, W.SENSOR], ids=lambda d: d.name)
@pytest.mark.parametrize("indexed", [False, True])
@pytest.mark.parametrize("n", [0, 1, 1037])
def test_buffer_sizes_match_oracle(decl, indexed, n):
    S = oracle.Schema(decl)
    strides = [W.TYPE_SIZE[t] * (1 + c % 3) for c, t in enumerate(S.leaf_types())]
    lib = P.Layout(P.Schema(decl), "strided", leaf_strides=strides, indexed=indexed)
    orc = oracle.make_layout(S, "strided", leaf_strides=strides, indexed=indexed)
    assert lib.buffer_bytes(n) == oracle.buffer_sizes(orc, n)


def _view(layout, n, ptrs):
    return P.View(layout, n, ptrs)


def test_checks_before_device_work():
    s = P.Schema(W.PLAIN8)
    st = P.Layout(s, "strided", leaf_strides=[32, 32, 32, 32, 32, 32, 32, 32])
    soa = P.Layout(s, "soa")
    base = 1 << 40
    offs = [0, 4, 8, 12, 16, 24, 26, 28]
    rec = _view(st, 100, [base + o for o in offs])          # fields of one record array
    cols = _view(soa, 100, [(1 << 41) + k * (1 << 24) for k in range(8)])
    s0 = ctypes.c_void_p(0)
    rc = P.lib().rl_convert
    # the destination's leaves may share memory, but not the source's
    over = _view(soa, 100, [base + 64] + [(1 << 41) + k * (1 << 24) for k in range(1, 8)])
    assert rc(rec.ref(), over.ref(), 10, s0) == P.RL_EOVERLAP
    assert rc(cols.ref(), rec.ref(), 0, s0) == P.RL_OK
    mis = _view(st, 100, [base + o + (1 if k == 0 else 0) for k, o in enumerate(offs)])
    assert rc(cols.ref(), mis.ref(), 10, s0) == P.RL_EALIGN
    # indexed: the index table is the last buffer and must be 8-byte aligned
    ist = P.Layout(s, "strided", indexed=True)
    bad_idx = _view(ist, 100, [(1 << 42) + k * (1 << 24) for k in range(8)] + [(1 << 43) + 4])
    assert rc(cols.ref(), bad_idx.ref(), 10, s0) == P.RL_EALIGN
    # entry points that do not take strided layouts
    h = ctypes.c_void_p()
    assert P.lib().rl_batch_create(None, ctypes.byref(h)) == P.RL_OK
    assert P.lib().rl_batch_add(h, cols.ref(), rec.ref(), 10) == P.RL_EUNSUPPORTED
    P.lib().rl_batch_destroy(h)
    assert P.lib().rl_erase(rec.ref(), 10, 0, 1, s0) == P.RL_EUNSUPPORTED
    assert P.lib().rl_insert(rec.ref(), 10, 0, cols.ref(), 1, s0) == P.RL_EUNSUPPORTED
    hst = P.Layout(s, "strided", space="pinned")
    hrec = _view(hst, 100, [base + o for o in offs])
    o = P.rl_xfer_opts(0)
    assert P.lib().rl_transfer(hrec.ref(), cols.ref(), 10, s0, ctypes.byref(o)) == P.RL_EUNSUPPORTED
    assert P.lib().rl_transfer_noalloc(hrec.ref(), cols.ref(), 10, s0, ctypes.byref(o)) == P.RL_EUNSUPPORTED
    c = ctypes.c_void_p()
    assert P.lib().rl_collection_create(st.handle, 10, None, s0, ctypes.byref(c)) == P.RL_EUNSUPPORTED
