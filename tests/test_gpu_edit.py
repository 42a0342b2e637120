"""GPU parity of insertion, deletion and compaction (Sec. VII-B: insert and
erase on a collection's arrays; compaction after a filter): rl_select,
rl_erase and rl_insert against the oracle's gathers, byte for byte over the
result's footprint, for every layout kind, narrowing storage, jagged groups
(compaction between any kinds, appends between offsets layouts), AoSoA
shifts larger than one scratch band, and the device-side statuses."""
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


def values(decl, n, seed):
    if decl is W.CLUSTER:
        return W.cluster_values(n, seed=seed, mean_len=6.0)
    if decl is W.CELL:
        return W.cell_values(n, seed=seed)
    return W.generic_values(decl, n, seed=seed, mean_len=3.0)


def footprint_equal(got, want_bufs, layout, n, members, what):
    sizes = oracle.buffer_sizes(layout.orc, n, members)
    assert len(got) >= len(sizes)
    for k, sz in enumerate(sizes):
        g = got[k][:sz]
        w = np.asarray(want_bufs[k]).view(np.uint8)[:sz]
        if not np.array_equal(g, w):
            bad = np.nonzero(g != w)[0]
            raise AssertionError(f"{what}: buffer {k} differs at {bad.size} of {sz} bytes, first {bad[:6]}")


KINDS = [("aos", 0), ("soa", 0), ("aosoa", 32), ("aosoa", 3)]


@pytest.mark.parametrize("decl", [W.PLAIN8, W.CELL, W.SENSOR], ids=lambda d: d.name)
@pytest.mark.parametrize("sk,dk", [(("aos", 0), ("soa", 0)), (("soa", 0), ("aosoa", 32)),
                                   (("aosoa", 64), ("aos", 0)), (("aos", 0), ("aos", 0)),
                                   (("aosoa", 3), ("aosoa", 5))], ids=str)
@pytest.mark.parametrize("n,rule", [(1, "all"), (1000, "none"), (4097, "random"), (70_001, "random")])
def test_select_dense(decl, sk, dk, n, rule):
    sp = H.SchemaPair(decl)
    storage = H.narrowed_storage(decl) if decl is W.CELL and dk[0] != "aos" else None
    src, dst = sp.layout(*sk), sp.layout(*dk, storage=storage)
    v = values(decl, n, seed=n + 3)
    sb = oracle.pack(sp.orc, v, src.orc)
    keep = {"all": np.ones(n, np.uint8), "none": np.zeros(n, np.uint8),
            "random": (np.random.default_rng(n).random(n) < 0.4).astype(np.uint8)}[rule]
    st, want, count, _ = oracle.select(src.orc, sb, dst.orc, n, keep)
    assert st == 0
    dsrc = H.to_device(sb)
    ddst = H.alloc_device(dst.lib.buffer_bytes(n))
    kept = torch.zeros(1, dtype=torch.int64, device="cuda")
    P.select(P.View(src.lib, n, dsrc), P.View(dst.lib, n, ddst), n, torch.from_numpy(keep).cuda(), kept)
    assert P.sync() == 0, P.rl_last_error()
    assert int(kept.item()) == count
    footprint_equal(H.to_numpy(ddst), want, dst, count, [], f"select {rule} {sk}->{dk} n={n}")


@pytest.mark.parametrize("decl", [W.CLUSTER, W.PARTICLE], ids=lambda d: d.name)
@pytest.mark.parametrize("sk,dk", [(("aos", 0), ("soa", 0)), (("soa", 0), ("aos", 0)),
                                   (("aosoa", 16), ("soa", 0)), (("soa", 0), ("aosoa", 8))], ids=str)
@pytest.mark.parametrize("n", [1, 3001, 50_000])
def test_select_jagged(decl, sk, dk, n):
    sp = H.SchemaPair(decl)
    src, dst = sp.layout(*sk), sp.layout(*dk)
    v = values(decl, n, seed=n + 7)
    sb = oracle.pack(sp.orc, v, src.orc, pool_order=True)
    tot = v.total(0)
    smem = [len(sb[1]) // src.orc.member_stride[0]] if sk[0] == "aos" else [tot]
    keep = (np.random.default_rng(n + 1).random(n) < 0.5).astype(np.uint8)
    st, want, count, tots = oracle.select(src.orc, sb, dst.orc, n, keep, smem)
    assert st == 0
    ddst = H.alloc_device(dst.lib.buffer_bytes(n, [tot]))
    kept = torch.zeros(1, dtype=torch.int64, device="cuda")
    P.select(P.View(src.lib, n, H.to_device(sb), smem), P.View(dst.lib, n, ddst, [tot]), n,
             torch.from_numpy(keep).cuda(), kept)
    assert P.sync() == 0, P.rl_last_error()
    assert int(kept.item()) == count
    footprint_equal(H.to_numpy(ddst), want, dst, count, tots, f"jagged select {sk}->{dk} n={n}")


def test_select_member_capacity_too_small():
    sp = H.SchemaPair(W.CLUSTER)
    soa = sp.layout("soa")
    n = 2000
    v = values(W.CLUSTER, n, 11)
    sb = oracle.pack(sp.orc, v, soa.orc)
    tot = v.total(0)
    keep = np.ones(n, np.uint8)
    cap = tot - 5
    st, _, _, _ = oracle.select(soa.orc, sb, soa.orc, n, keep, [tot])
    assert st == 0
    sizes = soa.lib.buffer_bytes(n, [cap])
    ddst = H.alloc_device([x + 64 for x in sizes])
    P.select(P.View(soa.lib, n, H.to_device(sb), [tot]), P.View(soa.lib, n, ddst, [cap]), n,
             torch.from_numpy(keep).cuda())
    assert P.sync() == P.RL_ECAPACITY
    got = H.to_numpy(ddst)
    for k in (7, 8):   # member columns untouched past the capacity
        assert np.all(got[k][sizes[k]:] == H.SENTINEL)


@pytest.mark.parametrize("decl", [W.PLAIN8, W.CELL, W.SENSOR], ids=lambda d: d.name)
@pytest.mark.parametrize("kind", KINDS, ids=str)
@pytest.mark.parametrize("n,at,count", [(5000, 0, 10), (5000, 100, 4000), (5000, 4990, 10), (5000, 2500, 1),
                                        (77, 0, 77)])
def test_erase_dense(decl, kind, n, at, count):
    sp = H.SchemaPair(decl)
    L = sp.layout(*kind)
    v = values(decl, n, seed=at + count)
    bufs = oracle.pack(sp.orc, v, L.orc)
    st, want, _ = oracle.erase(L.orc, bufs, n, at, count)
    assert st == 0
    d = H.to_device(bufs)
    P.erase(P.View(L.lib, n, d), n, at, count)
    assert P.sync() == 0, P.rl_last_error()
    footprint_equal(H.to_numpy(d), want, L, n - count, [], f"erase {at}+{count} {kind}")


@pytest.mark.parametrize("decl", [W.PLAIN8, W.CELL, W.SENSOR], ids=lambda d: d.name)
@pytest.mark.parametrize("kind", KINDS, ids=str)
@pytest.mark.parametrize("n,at,count", [(4000, 0, 37), (4000, 1234, 37), (4000, 4000, 37), (0, 0, 5),
                                        (999, 500, 2000)])
def test_insert_dense(decl, kind, n, at, count):
    sp = H.SchemaPair(decl)
    storage = H.narrowed_storage(decl) if decl is W.CELL else None
    L = sp.layout(*kind, storage=storage)
    NL = sp.layout("soa")
    v, new = values(decl, n, seed=n + at), values(decl, count, seed=count + 1)
    bufs = oracle.pack(sp.orc, v, L.orc)
    nb = oracle.pack(sp.orc, new, NL.orc)
    st, want, _ = oracle.insert(L.orc, bufs, n, at, NL.orc, nb, count)
    assert st == 0
    cap = n + count
    d = H.alloc_device(L.lib.buffer_bytes(cap))
    for t, b in zip(d, bufs):   # the current n objects at the front of buffers for n + count
        if t is not None and len(b):
            t[:len(b)] = torch.from_numpy(b).cuda()
    P.insert(P.View(L.lib, cap, d), n, at, P.View(NL.lib, count, H.to_device(nb)), count)
    assert P.sync() == 0, P.rl_last_error()
    footprint_equal(H.to_numpy(d), want, L, n + count, [], f"insert {count} at {at} of {n} {kind}")


def test_aosoa_shifts_over_several_scratch_bands():
    """3.2 M cell objects in AoSoA(64) (27 bytes each: 86 MB, two 64 MiB
    bands): erase near the front, then insert there again."""
    decl = W.CELL
    sp = H.SchemaPair(decl)
    L = sp.layout("aosoa", 64)
    NL = sp.layout("soa")
    n, at, count = 3_200_000, 1_000, 5_000
    v = values(decl, n, 21)
    bufs = oracle.pack(sp.orc, v, L.orc)
    st, want, _ = oracle.erase(L.orc, bufs, n, at, count)
    assert st == 0
    d = H.to_device(bufs)
    P.erase(P.View(L.lib, n, d), n, at, count)
    assert P.sync() == 0, P.rl_last_error()
    footprint_equal(H.to_numpy(d), want, L, n - count, [], "band erase")
    new = values(decl, count, 22)
    nb = oracle.pack(sp.orc, new, NL.orc)
    st, want2, _ = oracle.insert(L.orc, want, n - count, at, NL.orc, nb, count)
    assert st == 0
    P.insert(P.View(L.lib, n, d), n - count, at, P.View(NL.lib, count, H.to_device(nb)), count)
    assert P.sync() == 0, P.rl_last_error()
    footprint_equal(H.to_numpy(d), want2, L, n, [], "band insert")


@pytest.mark.parametrize("decl", [W.CLUSTER, W.PARTICLE], ids=lambda d: d.name)
@pytest.mark.parametrize("vk,sk", [(("soa", 0), ("soa", 0)), (("aosoa", 32), ("soa", 0)), (("soa", 0), ("aosoa", 8))],
                         ids=str)
@pytest.mark.parametrize("n,count", [(0, 100), (3000, 1), (3000, 2500)])
def test_jagged_append(decl, vk, sk, n, count):
    sp = H.SchemaPair(decl)
    L, SL = sp.layout(*vk), sp.layout(*sk)
    v, new = values(decl, n, seed=n + 31), values(decl, count, seed=count + 32)
    tot, ntot = v.total(0), new.total(0)
    bufs = oracle.pack(sp.orc, v, L.orc)
    nb = oracle.pack(sp.orc, new, SL.orc)
    st, want, tots = oracle.insert(L.orc, bufs, n, n, SL.orc, nb, count, [tot], [ntot])
    assert st == 0 and tots == [tot + ntot]
    cap, mcap = n + count, tot + ntot
    d = H.alloc_device(L.lib.buffer_bytes(cap, [mcap]))
    # the current collection placed in buffers sized for the result
    gb = oracle._group_buffers(L.orc, 0, bufs)
    for k, (t, b) in enumerate(zip(d, bufs)):
        if t is not None and len(b):
            t[:len(b)] = torch.from_numpy(b).cuda()
    P.insert(P.View(L.lib, cap, d, [mcap]), n, n, P.View(SL.lib, count, H.to_device(nb), [ntot]), count)
    assert P.sync() == 0, P.rl_last_error()
    footprint_equal(H.to_numpy(d), want, L, n + count, [mcap], f"append {count} to {n} {vk}<-{sk}")


def test_jagged_append_beyond_member_capacity_and_unsupported_cases():
    decl = W.CLUSTER
    sp = H.SchemaPair(decl)
    L = sp.layout("soa")
    n, count = 1000, 500
    v, new = values(decl, n, 41), values(decl, count, 42)
    tot, ntot = v.total(0), new.total(0)
    bufs = oracle.pack(sp.orc, v, L.orc)
    nb = oracle.pack(sp.orc, new, L.orc)
    cap, mcap = n + count, tot + ntot - 1
    d = H.alloc_device(L.lib.buffer_bytes(cap, [mcap]))
    for t, b in zip(d, bufs):
        if t is not None and len(b):
            t[:len(b)] = torch.from_numpy(b).cuda()
    before = [t.clone() for t in d[7:9]]
    P.insert(P.View(L.lib, cap, d, [mcap]), n, n, P.View(L.lib, count, H.to_device(nb), [ntot]), count)
    assert P.sync() == P.RL_ECAPACITY
    for a, b in zip(before, d[7:9]):   # no member appended
        assert torch.equal(a, b)
    import ctypes
    view = P.View(L.lib, cap, d, [mcap])
    st = P.lib().rl_insert(view.ref(), n, 3, P.View(L.lib, count, H.to_device(nb), [ntot]).ref(), count,
                           P.stream_ptr(None))
    assert st == P.RL_EUNSUPPORTED
    assert P.lib().rl_erase(view.ref(), n, 3, 4, P.stream_ptr(None)) == P.RL_EUNSUPPORTED
    # erasing the last objects of a jagged collection moves nothing
    P.erase(view, n, n - 10, 10)
    assert P.sync() == 0
