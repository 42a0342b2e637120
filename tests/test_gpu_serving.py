"""Serving on the GPU: events admitted under a device-memory budget, their
collections converted concurrently on several streams, results resident
until released.  Each event's result must be the same bytes alone and in
the mix (and the oracle's); the budget is never exceeded; an event larger
than the budget is refused; a stalled consumer blocks admission; queued
events can be cancelled."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2511_04853_amd as P
import workloads as W
from tests import rlhelp as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_hip = None


def d2h(ptr, nbytes):
    """Copy nbytes of device memory at ptr to a numpy array."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
    out = np.empty(nbytes, dtype=np.uint8)
    if nbytes:
        torch.cuda.synchronize()
        assert _hip.hipMemcpy(ctypes.c_void_p(out.ctypes.data), ctypes.c_void_p(ptr),
                              ctypes.c_size_t(nbytes), 2) == 0   # hipMemcpyDeviceToHost
    return out


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


DECLS = [W.PLAIN8, W.CELL, W.CLUSTER]


class Events:
    """Pinned host sources for a set of events and the oracle's results."""

    def __init__(self, n_events, scale=10, seed=1004):
        self.sp = [H.SchemaPair(d) for d in DECLS]
        self.src = [sp.layout("aos", space="pinned") for sp in self.sp]
        self.dst = [sp.layout("soa", storage=H.narrowed_storage(sp.decl) if sp.decl is W.CELL else None)
                    for sp in self.sp]
        sizes = W.serving_events(n_events, seed=seed) // scale + 1
        self.events = []
        for e, row in enumerate(sizes):
            items = []
            for j, (sp, decl) in enumerate(zip(self.sp, DECLS)):
                n = int(row[j])
                if decl is W.CELL:
                    v = W.cell_values(n, seed=seed + 17 * e)
                elif decl is W.CLUSTER:
                    v = W.cluster_values(n, seed=seed + 17 * e + 1)
                else:
                    v = W.plain_values(n, seed=seed + 17 * e + 2)
                sbytes = oracle.pack(sp.orc, v, self.src[j].orc, pool_order=True)
                mem = [len(sbytes[1]) // self.src[j].orc.member_stride[0]] if decl.offset_types else []
                st, want, tot = oracle.convert(self.src[j].orc, sbytes, self.dst[j].orc, n, mem, mem)
                assert st == 0
                pinned = H.alloc_pinned([len(b) for b in sbytes])
                for t, b in zip(pinned, sbytes):
                    if t is not None:
                        t.numpy()[:] = b
                view = P.View(self.src[j].lib, n, pinned, mem)
                sizes_dst = self.dst[j].lib.buffer_bytes(n, mem)
                items.append(dict(view=view, n=n, want=want, sizes=sizes_dst, tot=tot))
            self.events.append(items)

    def submit(self, server, e):
        return server.submit([(it["view"], self.dst[j].lib, it["n"]) for j, it in enumerate(self.events[e])])

    def check(self, e, res):
        for j, it in enumerate(self.events[e]):
            got = []
            for b, (ptr, size) in enumerate(zip(res["buffers"][j], it["sizes"])):
                want_len = len(it["want"][b])
                got.append(d2h(ptr, want_len) if size else np.zeros(0, np.uint8))
            H.assert_same_bytes(got, it["want"], f"event {e} item {j}")


def test_results_alone_and_in_the_mix_are_identical():
    ev = Events(24)
    # alone: one event at a time
    srv = P.Server(1 << 30, max_in_flight=1, n_streams=1)
    for e in range(len(ev.events)):
        t = ev.submit(srv, e)
        res = srv.wait(t)
        assert res["status"] == 0
        ev.check(e, res)
        srv.release(t)
    srv.close()
    # in the mix: all submitted at once, 8 in flight over 4 streams
    srv = P.Server(1 << 30, max_in_flight=8, n_streams=4)
    tickets = [ev.submit(srv, e) for e in range(len(ev.events))]
    for e, t in enumerate(tickets):
        res = srv.wait(t)
        assert res["status"] == 0
        ev.check(e, res)
    st = srv.stats()
    assert st["completed"] == len(tickets) and st["submitted"] == len(tickets)
    assert st["p50_ms"] > 0 and st["p99_ms"] >= st["p50_ms"]
    for t in tickets:
        srv.release(t)
    srv.close()


def test_budget_is_never_exceeded_and_a_stalled_consumer_blocks():
    ev = Events(10, scale=20)
    need = max(sum(sum((b + 255) // 256 * 256 for b in it["sizes"]) for it in items) for items in ev.events)
    budget = 3 * need
    srv = P.Server(budget, max_in_flight=8, n_streams=2)
    tickets = [ev.submit(srv, e) for e in range(len(ev.events))]
    # only what fits the budget completes while nothing is released
    done = [t for t in tickets[:2] if srv.wait(t, timeout_ms=20_000) is not None]
    assert len(done) == 2
    assert srv.wait(tickets[-1], timeout_ms=300) is None     # blocked behind the budget
    assert srv.stats()["peak_bytes"] <= budget
    # releasing in order lets every event through
    for e, t in enumerate(tickets):
        res = srv.wait(t, timeout_ms=20_000)
        assert res is not None, f"event {e} never admitted"
        ev.check(e, res)
        srv.release(t)
        assert srv.stats()["peak_bytes"] <= budget
    srv.close()


def test_event_larger_than_budget_is_refused():
    ev = Events(1, scale=10)
    srv = P.Server(4096, max_in_flight=2, n_streams=1)
    with pytest.raises(P.RelayoutError) as e:
        ev.submit(srv, 0)
    assert e.value.status == P.RL_EBUDGET
    srv.close()


def test_each_event_reports_its_own_device_status():
    """One event whose jagged source has a member block past the end of its
    pool (the kernels' bounds check rejects it, nothing is read out of
    bounds): that event alone reports RL_EBOUNDS, every other event's
    result is the oracle's."""
    from tests import npref
    ev = Events(12, scale=10, seed=2024)
    bad_e = 5
    item = ev.events[bad_e][2]                       # the cluster collection
    rec = item["view"].tensors[0].numpy().view(npref.record_dtype(W.CLUSTER))
    i = int(np.nonzero(rec["len0"])[0][0])
    rec["ptr0"][i] = item["view"].tensors[1].numel() - 8
    srv = P.Server(1 << 30, max_in_flight=8, n_streams=4)
    tickets = [ev.submit(srv, e) for e in range(len(ev.events))]
    for e, t in enumerate(tickets):
        res = srv.wait(t)
        if e == bad_e:
            assert res["status"] == P.RL_EBOUNDS
        else:
            assert res["status"] == 0, (e, res["status"])
            ev.check(e, res)
    for t in tickets:
        srv.release(t)
    srv.close()


def test_zero_object_items_take_no_pool_block():
    """An event whose collections hold no objects fits a budget of its
    (zero) result bytes and completes."""
    ev = Events(1, scale=10)
    srv = P.Server(1 << 20, max_in_flight=2, n_streams=1)
    items = [(it["view"], ev.dst[j].lib, 0) for j, it in enumerate(ev.events[0])]
    t = srv.submit(items)
    res = srv.wait(t, timeout_ms=20_000)
    assert res is not None and res["status"] == 0
    srv.release(t)
    srv.close()


def test_queued_events_can_be_cancelled():
    """The largest event fills the budget and is held; events queued behind
    it can be cancelled (never converted, tickets forgotten), the admitted
    one cannot; after its release the remaining events complete with the
    oracle's bytes."""
    ev = Events(6, scale=20, seed=77)
    needs = [sum(sum((b + 255) // 256 * 256 for b in it["sizes"]) for it in items) for items in ev.events]
    big = int(np.argmax(needs))
    order = [big] + [e for e in range(len(ev.events)) if e != big]
    srv = P.Server(needs[big] + (256 << 10), max_in_flight=8, n_streams=1)   # + the look-back region
    tickets = {e: ev.submit(srv, e) for e in order}
    res = srv.wait(tickets[big], timeout_ms=20_000)
    assert res is not None and res["status"] == 0
    ev.check(big, res)
    assert srv.cancel(tickets[big]) == P.RL_EBUSY
    gone = order[1::2]
    for e in gone:
        assert srv.cancel(tickets[e]) == P.RL_OK
        assert srv.cancel(tickets[e]) == P.RL_EINVAL
    srv.release(tickets[big])
    for e in order[2::2]:
        res = srv.wait(tickets[e], timeout_ms=20_000)
        assert res is not None and res["status"] == 0
        ev.check(e, res)
        srv.release(tickets[e])
    st = srv.stats()
    assert st["submitted"] == len(order) and st["completed"] == len(order) - len(gone)
    srv.close()
