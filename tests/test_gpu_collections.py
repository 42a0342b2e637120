"""Collections owning their memory in a memory context, and re-homing them
(Sec. VII-A: allocate with the new context information, copy from the old
memory, free it), for device, pinned host and pageable host contexts with a
layout change on the way; every step against the oracle's conversion."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2511_04853_amd as P
import workloads as W
from tests import rlhelp as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


def read(coll, space):
    """The collection's buffers as numpy bytes (through rl_memcopy for
    device memory)."""
    v, ptrs, sizes = coll.view()
    out = []
    for p, sz in zip(ptrs, sizes):
        if space == "device":
            a = np.zeros(sz, np.uint8)
            if sz:
                P.memcopy(a, "host", p, "device", sz)
            out.append(a)
        else:
            out.append(np.frombuffer(ctypes.string_at(p, sz), np.uint8).copy() if sz else np.zeros(0, np.uint8))
    torch.cuda.synchronize()
    return out


def fill(coll, bufs, space):
    v, ptrs, sizes = coll.view()
    for p, b in zip(ptrs, bufs):
        if len(b):
            if space == "device":
                P.memcopy(p, "device", np.ascontiguousarray(b), "host", len(b))
            else:
                ctypes.memmove(p, np.ascontiguousarray(b).ctypes.data, len(b))
    torch.cuda.synchronize()


def footprint(got, want, layout_orc, n, members, what):
    sizes = oracle.buffer_sizes(layout_orc, n, members)
    for k, sz in enumerate(sizes):
        assert np.array_equal(got[k][:sz], np.asarray(want[k]).view(np.uint8)[:sz]), f"{what}: buffer {k}"


@pytest.mark.parametrize("decl", [W.CELL, W.SENSOR, W.CLUSTER], ids=lambda d: d.name)
def test_rehome_through_every_memory_context(decl):
    sp = H.SchemaPair(decl)
    n, cap = 5_003, 6_000
    v = W.cluster_values(n, seed=3, mean_len=5.0) if decl is W.CLUSTER else W.generic_values(decl, n, seed=3)
    jag = bool(decl.offset_types)
    tot = v.total(0) if jag else 0
    mem = [tot + 100] if jag else []
    steps = [("soa", 0, "device"), ("aos", 0, "pinned"), ("aosoa", 64, "host"), ("aosoa", 32, "device"),
             ("soa", 0, "host"), ("soa", 0, "device")]
    if jag:   # records only between offsets layouts
        steps = [("soa", 0, "device"), ("aos", 0, "pinned"), ("aosoa", 64, "host"), ("soa", 0, "device"),
                 ("aos", 0, "host"), ("aosoa", 32, "device")]
    kind, w, space = steps[0]
    L = sp.layout(kind, w, space=space)
    coll = P.Collection(L.lib, cap, mem)
    assert all(not np.any(b) for b in read(coll, space)), "created zero-filled"
    cur = oracle.pack(sp.orc, v, L.orc)
    fill(coll, cur, space)
    cur_orc = L.orc
    layouts = [L]
    for kind, w, space in steps[1:]:
        NL = sp.layout(kind, w, space=space)
        layouts.append(NL)
        st, want, _ = oracle.convert(cur_orc, cur, NL.orc, n, [tot] if jag else [], [tot] if jag else [])
        assert st == 0
        coll.rehome(NL.lib, n)
        assert P.sync() == 0, P.rl_last_error()
        got = read(coll, space)
        footprint(got, want, NL.orc, n, [tot] if jag else [], f"rehome to {kind}{w} {space}")
        cur, cur_orc = want, NL.orc
    coll.close()


def test_collection_errors():
    sp = H.SchemaPair(W.CELL)
    L = sp.layout("soa")
    coll = P.Collection(L.lib, 100)
    other = H.SchemaPair(W.PLAIN8).layout("soa")
    assert P.lib().rl_collection_rehome(coll.h, other.lib.handle, 10, None) == P.RL_EINVAL
    assert P.lib().rl_collection_rehome(coll.h, L.lib.handle, 101, None) == P.RL_EINVAL
    # the collection is unchanged and still usable
    coll.rehome(sp.layout("aos", space="pinned").lib, 100)
    coll.close()
