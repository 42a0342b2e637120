"""GPU parity of the single-pass jagged kernel (records with (pointer,
count) pairs -> offsets column + member columns in one launch, with a
look-back over earlier tiles for each tile's prefix, Sec. VI prefix sum).

Every case runs with the single-pass kernel required (RL_JAGGED_FUSED=2:
the conversion fails instead of falling back) and is compared byte for
byte with the oracle; the multi-kernel path (RL_JAGGED_FUSED=0) gives the
same bytes.  Covers: the full-size cluster collection (many look-back
rounds), every member word count 1..4 with each offset type, forced tile
sizes / block sizes / grids of a few persistent work-groups (tickets),
many launches back to back on one stream (look-back state reused across
launches of different sizes), two streams at once, and the error
statuses (capacity, a record outside its pool)."""
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


def _f(name, t, group=-1):
    return W.Field(name, t, 1, group, -1)


# member records of 1..4 packed 4-byte words, each offset type
DECLS = {
    1: W.SchemaDecl("jag_w1_u64", (_f("x", "f32"), _f("k", "u64"), _f("m0", "u32", 0)), offset_types=("u64",)),
    2: W.CLUSTER,
    3: W.SchemaDecl("jag_w3_i32", (_f("a", "i32"), _f("b", "u16"), _f("m0", "f32", 0), _f("m1", "i32", 0),
                                   _f("m2", "u32", 0), _f("c", "f64")), offset_types=("i32",)),
    4: W.SchemaDecl("jag_w4_u32", (_f("e", "f64"), _f("m0", "u32", 0), _f("m1", "f32", 0), _f("m2", "u32", 0),
                                   _f("m3", "i32", 0), _f("q", "u8")), offset_types=("u32",)),
}


def _values(decl, n, seed, mean_len=40.0):
    if decl is W.CLUSTER:
        return W.cluster_values(n, seed=seed, mean_len=mean_len)
    return W.generic_values(decl, n, seed=seed, mean_len=mean_len)


def _case(decl, v, dst_kind=("soa", 0), storage=None):
    sp = H.SchemaPair(decl)
    aos, dst = sp.layout("aos"), sp.layout(*dst_kind, storage=storage)
    tot = v.total(0)
    src = oracle.pack(sp.orc, v, aos.orc, pool_order=True)
    pool = len(src[1]) // aos.orc.member_stride[0]
    st, want, _ = H.oracle_convert(aos, src, dst, v.n, [pool], [tot])
    assert st == 0
    return aos, dst, src, pool, tot, want


def _run(aos, dst, src, pool, tot, n, fused, monkeypatch, stream=None):
    monkeypatch.setenv("RL_JAGGED_FUSED", str(fused))
    try:
        return H.run_lib_convert(aos, src, dst, n, [pool], [tot], stream=stream)
    finally:
        monkeypatch.delenv("RL_JAGGED_FUSED")


@pytest.mark.parametrize("dst_kind", [("soa", 0), ("aosoa", 64)], ids=str)
def test_full_size_cluster_collection(dst_kind, monkeypatch):
    """50,000 clusters, Poisson(40) members, shuffled pool: 782 tiles."""
    v = W.cluster_values(50_000, seed=1002)
    aos, dst, src, pool, tot, want = _case(W.CLUSTER, v, dst_kind)
    rc, rs, got = _run(aos, dst, src, pool, tot, v.n, 2, monkeypatch)
    assert rc == P.RL_OK and rs == P.RL_OK, P.rl_last_error()
    H.assert_same_bytes(got, want, f"single-pass {dst_kind}")
    rc, rs, old = _run(aos, dst, src, pool, tot, v.n, 0, monkeypatch)
    assert rc == P.RL_OK and rs == P.RL_OK, P.rl_last_error()
    H.assert_same_bytes(old, want, f"multi-kernel {dst_kind}")


@pytest.mark.parametrize("words", [1, 2, 3, 4])
@pytest.mark.parametrize("n", [1, 63, 1000, 20_011])
def test_member_word_counts_and_offset_types(words, n, monkeypatch):
    decl = DECLS[words]
    v = _values(decl, n, seed=100 + words * 7 + n, mean_len=9.0)
    storage = H.narrowed_storage(decl)
    for dst_kind in (("soa", 0), ("aosoa", 32)):
        aos, dst, src, pool, tot, want = _case(decl, v, dst_kind, storage)
        rc, rs, got = _run(aos, dst, src, pool, tot, v.n, 2, monkeypatch)
        assert rc == P.RL_OK and rs == P.RL_OK, P.rl_last_error()
        H.assert_same_bytes(got, want, f"{decl.name} n={n} {dst_kind}")


@pytest.mark.parametrize("tile,threads,grid", [(16, 64, 1), (64, 256, 3), (128, 128, 7), (512, 256, 0),
                                                (32, 64, 0)])
def test_forced_shapes(tile, threads, grid, monkeypatch):
    """Tiny tiles (thousands of look-back words), few persistent
    work-groups taking many tickets each, and member counts that need
    several staging passes in one tile."""
    lens = np.random.default_rng(5).poisson(30, size=9_001).astype(np.uint32)
    lens[17] = 9_000
    lens[4_000:4_600] = 0
    v = _values(W.CLUSTER, 9_001, seed=5)
    rng = np.random.default_rng(6)
    tot = int(lens.sum())
    v.lengths[0] = lens
    v.members["cell_index"] = rng.integers(0, 2**32 - 1, size=tot, dtype=np.uint32)
    v.members["cell_weight"] = rng.random(size=tot).astype(np.float32)
    aos, dst, src, pool, tot, want = _case(W.CLUSTER, v)
    monkeypatch.setenv("RL_TILE_OBJECTS", str(tile))
    monkeypatch.setenv("RL_BLOCK_THREADS", str(threads))
    if grid:
        monkeypatch.setenv("RL_GRID_BLOCKS", str(grid))
    rc, rs, got = _run(aos, dst, src, pool, tot, v.n, 2, monkeypatch)
    assert rc == P.RL_OK and rs == P.RL_OK, P.rl_last_error()
    H.assert_same_bytes(got, want, f"tile {tile} threads {threads} grid {grid}")


def test_back_to_back_launches_on_one_stream(monkeypatch):
    """Launches of different tile counts queued on one stream before any
    synchronisation: each reads only the look-back words of its own launch."""
    monkeypatch.setenv("RL_JAGGED_FUSED", "2")
    stream = torch.cuda.Stream()
    runs = []
    for k, n in enumerate([50_000, 777, 33_333, 5, 50_000, 12_345]):
        v = W.cluster_values(n, seed=300 + k)
        aos, dst, src, pool, tot, want = _case(W.CLUSTER, v)
        dsrc = H.to_device(src)
        ddst = H.alloc_device(dst.lib.buffer_bytes(n, [tot]))
        runs.append((n, aos, dst, dsrc, pool, tot, ddst, want))
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        for n, aos, dst, dsrc, pool, tot, ddst, want in runs:
            P.convert(P.View(aos.lib, n, dsrc, [pool]), P.View(dst.lib, n, ddst, [tot]), n, stream)
    assert P.sync(stream) == 0, P.rl_last_error()
    for n, aos, dst, dsrc, pool, tot, ddst, want in runs:
        H.assert_same_bytes(H.to_numpy(ddst), want, f"back to back n={n}")


def test_two_streams_at_once(monkeypatch):
    monkeypatch.setenv("RL_JAGGED_FUSED", "2")
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    runs = []
    for k, n in enumerate([40_000, 45_001]):
        v = W.cluster_values(n, seed=400 + k)
        aos, dst, src, pool, tot, want = _case(W.CLUSTER, v)
        runs.append((n, aos, dst, H.to_device(src), pool, tot, H.alloc_device(dst.lib.buffer_bytes(n, [tot])), want))
    torch.cuda.synchronize()
    for s, (n, aos, dst, dsrc, pool, tot, ddst, want) in zip(streams, runs):
        P.convert(P.View(aos.lib, n, dsrc, [pool]), P.View(dst.lib, n, ddst, [tot]), n, s)
    for s in streams:
        assert P.sync(s) == 0, P.rl_last_error()
    for n, aos, dst, dsrc, pool, tot, ddst, want in runs:
        H.assert_same_bytes(H.to_numpy(ddst), want, f"two streams n={n}")


def test_capacity_and_bounds_statuses(monkeypatch):
    """Too small a destination capacity -> RL_ECAPACITY (no write beyond
    it); a record pointing outside its pool -> RL_EBOUNDS.  The oracle
    reports the same statuses."""
    import ctypes
    monkeypatch.setenv("RL_JAGGED_FUSED", "2")
    v = W.cluster_values(3_000, seed=9)
    sp = H.SchemaPair(W.CLUSTER)
    aos, soa = sp.layout("aos"), sp.layout("soa")
    tot = v.total(0)
    src = oracle.pack(sp.orc, v, aos.orc, pool_order=True)
    pool = len(src[1]) // 8
    # capacity one short
    cap = tot - 1
    st, _, _ = H.oracle_convert(aos, src, soa, v.n, [pool], [cap])
    assert st == P.RL_ECAPACITY
    sizes = soa.lib.buffer_bytes(v.n, [cap])
    pad = [s + 64 for s in sizes]   # room past the capacity: must stay untouched
    ddst = H.alloc_device(pad)
    dsrc = H.to_device(src)
    P.convert(P.View(aos.lib, v.n, dsrc, [pool]), P.View(soa.lib, v.n, ddst, [cap]), v.n)
    assert P.sync() == P.RL_ECAPACITY
    got = H.to_numpy(ddst)
    for k in (7, 8):   # member columns: nothing written past the capacity
        assert np.all(got[k][sizes[k]:] == H.SENTINEL)
    # a record's pointer past its pool
    bad = [b.copy() for b in src]
    rec = bad[0].view(np.uint8).reshape(v.n, -1)
    ptr_off = aos.lib.slot_offsets[6]
    rec[1234, ptr_off:ptr_off + 8] = np.frombuffer(np.uint64(len(src[1]) + 8).tobytes(), np.uint8)
    st, _, _ = H.oracle_convert(aos, bad, soa, v.n, [pool], [tot])
    assert st == P.RL_EBOUNDS
    rc, rs, _ = H.run_lib_convert(aos, bad, soa, v.n, [pool], [tot])
    assert rc == P.RL_OK and rs == P.RL_EBOUNDS


def test_huge_count_outside_its_pool(monkeypatch):
    """A record whose count is 2^28 (past its pool): the single-pass
    kernel's scan then takes its 64-bit path (counts of 2^26 and more);
    the offsets column is the exact prefix sum of the counts as given,
    members are stored up to the capacity, and the status is the oracle's."""
    monkeypatch.setenv("RL_JAGGED_FUSED", "2")
    v = W.cluster_values(2_000, seed=23)
    sp = H.SchemaPair(W.CLUSTER)
    aos, soa = sp.layout("aos"), sp.layout("soa")
    tot = v.total(0)
    src = oracle.pack(sp.orc, v, aos.orc, pool_order=True)
    pool = len(src[1]) // 8
    bad = [b.copy() for b in src]
    rec = bad[0].view(np.uint8).reshape(v.n, -1)
    len_off = aos.lib.slot_offsets[7]
    lens = np.array(v.lengths[0], dtype=np.uint64)
    lens[777] = 1 << 28
    rec[777, len_off:len_off + 4] = np.frombuffer(np.uint32(1 << 28).tobytes(), np.uint8)
    st, _, _ = H.oracle_convert(aos, bad, soa, v.n, [pool], [tot])
    rc, rs, got = H.run_lib_convert(aos, bad, soa, v.n, [pool], [tot])
    assert rc == P.RL_OK and rs == st != P.RL_OK
    want = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint32)
    assert np.array_equal(got[6].view(np.uint32)[:v.n + 1], want)
