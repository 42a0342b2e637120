"""rl_transfer_noalloc: the transfer entry point that allocates nothing
(staging in the library's fixed device array) gives the same bytes as
rl_transfer and as the oracle, on two calls in a row on one stream (the
second smaller, so it reuses the array the first one left behind), and
refuses a staged transfer beyond its limit without enqueuing anything."""
import numpy as np
import pytest

import oracle
import paper_2511_04853_amd as P
import workloads as W
from tests import rlhelp as H

pytestmark = pytest.mark.gpu


def _pinned_from(bufs):
    out = H.alloc_pinned([len(b) for b in bufs])
    for t, b in zip(out, bufs):
        if t is not None:
            t.numpy()[:] = b
    return out


def _pageable_from(bufs):
    import torch
    return [None if len(b) == 0 else torch.from_numpy(np.array(b, copy=True)) for b in bufs]


@pytest.mark.parametrize("space", ["pinned", "host"])
@pytest.mark.parametrize("dst", [("soa", 0), ("aosoa", 64)], ids=str)
def test_h2d_two_calls_match_rl_transfer(space, dst):
    import torch
    sp = H.SchemaPair(W.CELL)
    aos = sp.layout("aos", space=space)
    dl = sp.layout(*dst, storage=H.narrowed_storage(W.CELL))
    stream = torch.cuda.current_stream()
    runs = []
    for n, seed in ((190_000, 1001), (70_001, 77)):
        v = W.cell_values(n, seed=seed)
        sbytes = oracle.pack(sp.orc, v, aos.orc)
        st, want, _ = H.oracle_convert(aos, sbytes, dl, n, [], [])
        assert st == 0
        hsrc = _pinned_from(sbytes) if space == "pinned" else _pageable_from(sbytes)
        got = H.alloc_device(dl.lib.buffer_bytes(n))
        ref = H.alloc_device(dl.lib.buffer_bytes(n))
        runs.append((n, hsrc, got, ref, want))
    # both no-allocation calls back to back on one stream, then the same
    # transfers through rl_transfer
    for n, hsrc, got, ref, want in runs:
        P.transfer_noalloc(P.View(aos.lib, n, hsrc), P.View(dl.lib, n, got), n, stream, mode="staged")
    for n, hsrc, got, ref, want in runs:
        P.transfer(P.View(aos.lib, n, hsrc), P.View(dl.lib, n, ref), n, stream, mode="staged")
    assert P.sync(stream) == 0, P.rl_last_error()
    for n, hsrc, got, ref, want in runs:
        g = H.to_numpy(got)
        H.assert_same_bytes(g, H.to_numpy(ref), f"noalloc vs rl_transfer n={n}")
        H.assert_same_bytes(g, want, f"noalloc vs oracle n={n}")


def test_d2h_two_calls_match_rl_transfer():
    import torch
    sp = H.SchemaPair(W.CELL)
    soa = sp.layout("soa", storage=H.narrowed_storage(W.CELL))
    aos = sp.layout("aos", space="pinned")
    stream = torch.cuda.current_stream()
    runs = []
    for n, seed in ((100_003, 4), (999, 5)):
        v = W.cell_values(n, seed=seed)
        sbytes = oracle.pack(sp.orc, v, soa.orc)
        st, want, _ = H.oracle_convert(soa, sbytes, aos, n, [], [])
        assert st == 0
        dsrc = H.to_device(sbytes)
        runs.append((n, dsrc, H.alloc_pinned(aos.lib.buffer_bytes(n)), H.alloc_pinned(aos.lib.buffer_bytes(n)),
                     want))
    for n, dsrc, got, ref, want in runs:
        P.transfer_noalloc(P.View(soa.lib, n, dsrc), P.View(aos.lib, n, got), n, stream, mode="staged")
    for n, dsrc, got, ref, want in runs:
        P.transfer(P.View(soa.lib, n, dsrc), P.View(aos.lib, n, ref), n, stream, mode="staged")
    assert P.sync(stream) == 0, P.rl_last_error()
    for n, dsrc, got, ref, want in runs:
        g = H.to_numpy(got)
        H.assert_same_bytes(g, H.to_numpy(ref), f"d2h noalloc vs rl_transfer n={n}")
        H.assert_same_bytes(g, want, f"d2h noalloc vs oracle n={n}")


def test_jagged_round_trip_two_calls():
    """Jagged collections take the staged path: records and a shuffled pool
    in, SoA with offsets out, and back into a canonical pool."""
    import torch
    sp = H.SchemaPair(W.CLUSTER)
    aos_h = sp.layout("aos", space="pinned")
    soa = sp.layout("soa")
    stream = torch.cuda.current_stream()
    runs = []
    for n, seed in ((20_000, 11), (5_001, 12)):
        v = W.cluster_values(n, seed=seed)
        tot = H.totals(v)
        sbytes = oracle.pack(sp.orc, v, aos_h.orc, pool_order=True)
        st, want, _ = H.oracle_convert(aos_h, sbytes, soa, n, tot, tot)
        assert st == 0
        canon = oracle.pack(sp.orc, v, aos_h.orc, pool_order=False)
        runs.append(dict(n=n, tot=tot, hsrc=_pinned_from(sbytes), want=want, canon=canon,
                         got=H.alloc_device(soa.lib.buffer_bytes(n, tot)),
                         ref=H.alloc_device(soa.lib.buffer_bytes(n, tot)),
                         back=H.alloc_pinned(aos_h.lib.buffer_bytes(n, tot)),
                         back_ref=H.alloc_pinned(aos_h.lib.buffer_bytes(n, tot))))
    for r in runs:
        n, tot = r["n"], r["tot"]
        P.transfer_noalloc(P.View(aos_h.lib, n, r["hsrc"], tot), P.View(soa.lib, n, r["got"], tot), n, stream)
        P.transfer_noalloc(P.View(soa.lib, n, r["got"], tot), P.View(aos_h.lib, n, r["back"], tot), n, stream)
    for r in runs:
        n, tot = r["n"], r["tot"]
        P.transfer(P.View(aos_h.lib, n, r["hsrc"], tot), P.View(soa.lib, n, r["ref"], tot), n, stream)
        P.transfer(P.View(soa.lib, n, r["ref"], tot), P.View(aos_h.lib, n, r["back_ref"], tot), n, stream)
    assert P.sync(stream) == 0, P.rl_last_error()
    for r in runs:
        g = H.to_numpy(r["got"])
        H.assert_same_bytes(g, H.to_numpy(r["ref"]), f"jagged h2d noalloc vs rl_transfer n={r['n']}")
        H.assert_same_bytes(g, r["want"], f"jagged h2d noalloc vs oracle n={r['n']}")
        b = H.to_numpy(r["back"])
        H.assert_same_bytes(b, H.to_numpy(r["back_ref"]), f"jagged d2h noalloc vs rl_transfer n={r['n']}")
        H.assert_same_bytes(b, r["canon"], f"jagged d2h noalloc vs canonical n={r['n']}")


def test_staged_transfer_beyond_the_limit_is_refused():
    import torch
    sp = H.SchemaPair(W.CELL)
    aos = sp.layout("aos", space="pinned")
    soa = sp.layout("soa")
    n = P.TRANSFER_NOALLOC_LIMIT // 32 + 1_000
    assert aos.lib.buffer_bytes(n)[0] > P.TRANSFER_NOALLOC_LIMIT
    hsrc = H.alloc_pinned(aos.lib.buffer_bytes(n), fill=0)
    ddst = H.alloc_device(soa.lib.buffer_bytes(n))
    o = P.rl_xfer_opts(P.XFER_MODES["staged"])
    import ctypes
    st = P.lib().rl_transfer_noalloc(P.View(aos.lib, n, hsrc).ref(), P.View(soa.lib, n, ddst).ref(), n,
                                     P.stream_ptr(None), ctypes.byref(o))
    assert st == P.RL_ELIMIT, P.STATUS_NAMES.get(st, st)
    assert "at most" in P.rl_last_error()
    torch.cuda.synchronize()
    # nothing was enqueued: the destination keeps its fill
    for t in ddst:
        assert int((t != H.SENTINEL).sum().item()) == 0
    # zero-copy needs no staging: the same transfer goes through
    P.transfer_noalloc(P.View(aos.lib, n, hsrc), P.View(soa.lib, n, ddst), n, mode="zero_copy")
    assert P.sync() == 0, P.rl_last_error()
    for t in ddst:
        assert int((t != 0).sum().item()) == 0
