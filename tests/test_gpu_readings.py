"""GPU parity for the readings of the paper that the oracle pins: NaN
encodings through narrowing and widening, records restrided between C
natural alignment and a packed struct, offsets sources whose first entry is
not zero; and the isolation of device status between streams and between
batch items."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2511_04853_amd as P
import workloads as W
from tests import npref
from tests import rlhelp as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


def _convert_both(src, sbytes, dst, n, src_members=(), dst_members=()):
    st, want, _ = H.oracle_convert(src, sbytes, dst, n, list(src_members), list(dst_members))
    assert st == 0
    rc, rs, got = H.run_lib_convert(src, sbytes, dst, n, list(src_members), list(dst_members))
    assert rc == P.RL_OK, P.rl_last_error()
    assert rs == P.RL_OK, P.rl_last_error()
    return got, want


def _packed_pair(sp):
    """A packed record layout of a schema (numpy's unaligned structured
    dtype of the same fields: no padding) on both sides."""
    decl = sp.decl
    S = sp.orc
    pdt = npref.record_dtype(decl, align=False)
    offs = []
    for f, e in S.leaves:
        if f.subgroup >= 0:
            sub = pdt.fields[f"sub{f.subgroup}"]
            offs.append(sub[1] + sub[0].fields[f.name][1] + e * W.TYPE_SIZE[f.type])
        else:
            offs.append(pdt.fields[f.name][1] + e * W.TYPE_SIZE[f.type])
    return sp.layout("aos", slot_offsets=offs, stride=pdt.itemsize)


# ------------------------------------------------------------ NaN encodings (P9)

def _nan_cells(n, seed):
    """Cell values whose f64 energy holds every NaN class, the rounding edge
    cases and random doubles."""
    v = W.cell_values(n, seed=seed)
    d = np.array([0x7FF8000000000000, 0xFFF8000000000000, 0x7FF0000000000001, 0xFFF0000000000001,
                  0x7FFFFFFFFFFFFFFF, 0xFFFFFFFFFFFFFFFF, 0x7FF4000000000000, 0x7FF8DEADBEEF0001,
                  0xFFF0000020000000, 0x7FF000001FFFFFFF, 0x7FFA5A5A5A5A5A5A,
                  0x7FF0000000000000, 0xFFF0000000000000, 0x8000000000000000, 0x0000000000000001,
                  0x47EFFFFFF0000000, 0x47EFFFFFEFFFFFFF, 0x3FF0000010000000, 0x3FF0000030000000,
                  0x36A0000000000000, 0x3690000000000000, 0x3698000000000000], dtype=np.uint64)
    e = np.array(v.fields["energy_d"], dtype=np.float64)
    reps = np.resize(d, n // 3)
    e.view(np.uint64)[: reps.size * 3: 3] = reps
    v.fields["energy_d"] = e
    return v


@pytest.mark.parametrize("dst_kind", [("soa", 0), ("aosoa", 64), ("aosoa", 3), ("aos", 0)], ids=str)
def test_nan_narrowing_matches_oracle_bit_for_bit(dst_kind):
    sp = H.SchemaPair(W.CELL)
    v = _nan_cells(20_011, seed=5)
    src = sp.layout("aos")
    dst = sp.layout(*dst_kind, storage=H.narrowed_storage(W.CELL))
    got, want = _convert_both(src, oracle.pack(sp.orc, v, src.orc), dst, v.n)
    H.assert_same_bytes(got, want, f"narrow aos->{dst_kind}")


def test_nan_narrowing_through_packed_records_bit_for_bit():
    """A packed record puts the f64 at an offset that is not a multiple of 8
    (the byte-wise path of the kernels)."""
    sp = H.SchemaPair(W.CELL)
    v = _nan_cells(9_001, seed=6)
    src = _packed_pair(sp)
    dst = sp.layout("soa", storage=H.narrowed_storage(W.CELL))
    got, want = _convert_both(src, oracle.pack(sp.orc, v, src.orc), dst, v.n)
    H.assert_same_bytes(got, want, "narrow packed->soa")


@pytest.mark.parametrize("dst", ["aos", "packed"])
def test_nan_widening_matches_oracle_bit_for_bit(dst):
    sp = H.SchemaPair(W.CELL)
    v = _nan_cells(12_345, seed=7)
    narrow = H.narrowed_storage(W.CELL)
    mid = sp.layout("soa", storage=narrow)
    st, sbytes, _ = oracle.convert(oracle.values_layout(sp.orc), oracle.values_buffers(sp.orc, v), mid.orc, v.n)
    assert st == 0
    f = sbytes[6].view(np.uint32)
    f[::5] = np.resize(np.array([0x7FC00000, 0xFFC00000, 0x7F800001, 0xFF800001, 0x7FFFFFFF, 0xFFFFFFFF,
                                 0x7FA00000, 0x7FC0BEEF, 0xFF812345, 0x7F8FFFFF, 0x00000001, 0x80000000],
                                dtype=np.uint32), f[::5].size)
    if dst == "aos":
        out = sp.layout("aos")
    else:
        out = _packed_pair(sp)
    got, want = _convert_both(mid, sbytes, out, v.n)
    H.assert_same_bytes(got, want, f"widen soa(f32)->{dst}")


# ------------------------------------------------------------ records restrided (P2)

@pytest.mark.parametrize("decl", [W.PLAIN8, W.CELL, W.SENSOR], ids=lambda d: d.name)
@pytest.mark.parametrize("n", [1, 1037, 70_001])
def test_natural_records_restrided_to_packed_and_back(decl, n):
    """Filling back a pre-existing struct: C natural alignment <-> packed
    explicit slot offsets, padding zero-filled."""
    sp = H.SchemaPair(decl)
    v = W.generic_values(decl, n, seed=n + 3) if decl is not W.CELL else W.cell_values(n, seed=n)
    nat = sp.layout("aos")
    packed = _packed_pair(sp)
    src = oracle.pack(sp.orc, v, nat.orc)
    got, want = _convert_both(nat, src, packed, n)
    H.assert_same_bytes(got, want, f"{decl.name} natural->packed n={n}")
    back, want2 = _convert_both(packed, want, nat, n)
    H.assert_same_bytes(back, want2, f"{decl.name} packed->natural n={n}")
    H.assert_same_bytes(back, src, f"{decl.name} round trip n={n}")


@pytest.mark.parametrize("decl", [W.PLAIN8, W.CELL, W.SENSOR], ids=lambda d: d.name)
def test_natural_records_to_natural_records(decl):
    sp = H.SchemaPair(decl)
    n = 4099
    v = W.generic_values(decl, n, seed=41)
    nat = sp.layout("aos")
    src = oracle.pack(sp.orc, v, nat.orc)
    got, want = _convert_both(nat, src, nat, n)
    H.assert_same_bytes(got, want, f"{decl.name} aos->aos")
    H.assert_same_bytes(got, src, f"{decl.name} aos->aos copy")


# ------------------------------------------------------------ offsets sources not starting at 0 (P7, P8)

def _slice_soa(sp, v, k, n):
    """Objects k .. k+n-1 of a collection held as soa, viewed in place: the
    per-object columns start at object k, the offsets column is entries
    k .. k+n of the whole collection's (first entry = members before k), the
    member columns are the whole collection's."""
    S = sp.orc
    full = oracle.values_buffers(S, v)
    bufs = []
    for c, t in enumerate(S.leaf_types()):
        sz = W.TYPE_SIZE[t]
        bufs.append(full[c][k * sz:(k + n) * sz].copy())
    base = len(S.leaves)
    es = W.TYPE_SIZE[sp.decl.offset_types[0]]
    bufs.append(full[base][k * es:(k + n + 1) * es].copy())
    bufs += [full[base + 1 + m].copy() for m in range(len(S.members[0]))]
    member_cap = len(full[base + 1]) // W.TYPE_SIZE[S.member_types(0)[0]]
    return bufs, member_cap


@pytest.mark.parametrize("decl", [W.CLUSTER, W.PARTICLE], ids=lambda d: d.name)
@pytest.mark.parametrize("src_kind", [("soa", 0), ("aosoa", 32)], ids=str)
@pytest.mark.parametrize("dst_kind", [("aos", 0), ("soa", 0), ("aosoa", 16), ("aosoa", 128)], ids=str)
def test_offsets_source_with_a_nonzero_first_entry(decl, src_kind, dst_kind):
    if src_kind == dst_kind:
        pytest.skip("same layout")
    sp = H.SchemaPair(decl)
    v = W.generic_values(decl, 12_000, seed=17, mean_len=9.0)
    k, n = 3_001, 5_000
    soa = sp.layout("soa")
    bufs, cap = _slice_soa(sp, v, k, n)
    off = np.concatenate([[0], np.cumsum(v.lengths[0].astype(np.int64))])
    assert off[k] > 0
    total = int(off[k + n] - off[k])
    if src_kind[0] == "aosoa":
        src = sp.layout(*src_kind)
        st, blocks, _ = oracle.convert(soa.orc, bufs, src.orc, n, [cap], [total])
        assert st == 0
        # the object blocks of the slice, with the slice's own offsets and
        # the whole collection's member columns
        sbytes = [blocks[0]] + bufs[len(sp.orc.leaves):]
    else:
        src, sbytes = soa, bufs
    dst = sp.layout(*dst_kind)
    got, want = _convert_both(src, sbytes, dst, n, [cap], [total])
    H.assert_same_bytes(got, want, f"{decl.name} {src_kind}@{k}->{dst_kind}")
    # the same objects packed from index 0 give the same bytes
    sub = W.Values(decl, n)
    for f in decl.object_fields():
        sub.fields[f.name] = v.fields[f.name][k:k + n]
    sub.lengths = [v.lengths[0][k:k + n]]
    for f in decl.member_fields(0):
        sub.members[f.name] = v.members[f.name][off[k]:off[k + n]]
    sub.block_order = [np.arange(n)]
    H.assert_same_bytes(got, oracle.pack(sp.orc, sub, dst.orc), "slice vs packed from 0")


def test_offsets_source_past_its_member_columns_is_a_bounds_error():
    sp = H.SchemaPair(W.CLUSTER)
    v = W.generic_values(W.CLUSTER, 3_000, seed=19, mean_len=5.0)
    k, n = 1_000, 1_500
    soa = sp.layout("soa")
    bufs, cap = _slice_soa(sp, v, k, n)
    off = np.concatenate([[0], np.cumsum(v.lengths[0].astype(np.int64))])
    total = int(off[k + n] - off[k])
    short = int(off[k + n // 2])    # the columns are told to hold fewer members
    for dst_kind in (("aos", 0), ("soa", 0)):
        dst = sp.layout(*dst_kind)
        st, _, _ = oracle.convert(soa.orc, bufs, dst.orc, n, [short], [total])
        assert st == oracle.ST_BOUNDS
        rc, rs, _ = H.run_lib_convert(soa, bufs, dst, n, [short], [total])
        assert rc == P.RL_OK and rs == P.RL_EBOUNDS, (dst_kind, rc, rs)


# ------------------------------------------------------------ status words per stream

def _bad_cluster():
    sp = H.SchemaPair(W.CLUSTER)
    v = W.cluster_values(3_000, seed=23, mean_len=6.0)
    aos, soa = sp.layout("aos"), sp.layout("soa")
    src = oracle.pack(sp.orc, v, aos.orc, pool_order=True)
    bad = [b.copy() for b in src]
    rec = bad[0].view(npref.record_dtype(W.CLUSTER))
    i = int(np.nonzero(rec["len0"])[0][0])
    rec["ptr0"][i] = len(bad[1]) - 8      # its list runs past the end of the pool
    return sp, v, aos, soa, src, bad


def test_device_status_belongs_to_the_stream_that_ran_the_work():
    sp, v, aos, soa, good, bad = _bad_cluster()
    tot = v.total(0)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    keep = []

    def enqueue(src_bytes, stream):
        dsrc = H.to_device(src_bytes)
        ddst = H.alloc_device(soa.lib.buffer_bytes(v.n, [tot]))
        torch.cuda.synchronize()
        sv = P.View(aos.lib, v.n, dsrc, [len(src_bytes[1]) // 8])
        dv = P.View(soa.lib, v.n, ddst, [tot])
        keep.append((sv, dv))
        assert P.lib().rl_convert(sv.ref(), dv.ref(), v.n, P.stream_ptr(s1 if stream == 1 else s2)) == 0
        return ddst

    enqueue(bad, 1)
    out2 = enqueue(good, 2)
    # the good stream reports nothing, and does not clear the other's flag
    assert P.sync(s2) == P.RL_OK
    assert P.sync(s1) == P.RL_EBOUNDS
    assert P.sync(s1) == P.RL_OK        # cleared by the read
    st, want, _ = oracle.convert(aos.orc, good, soa.orc, v.n, [len(good[1]) // 8], [tot])
    H.assert_same_bytes(H.to_numpy(out2), want, "good stream")


# ------------------------------------------------------------ batch items

class _Batch:
    def __init__(self):
        h = ctypes.c_void_p()
        opts = P.rl_batch_opts(0, None)
        P.check(P.lib().rl_batch_create(ctypes.byref(opts), ctypes.byref(h)), "rl_batch_create")
        self.h, self.keep = h, []

    def add(self, sv, dv, n):
        self.keep += [sv, dv]
        P.check(P.lib().rl_batch_add(self.h, sv.ref(), dv.ref(), n), "rl_batch_add")

    def finalize(self):
        return P.lib().rl_batch_finalize(self.h, P.stream_ptr())

    def __del__(self):
        P.lib().rl_batch_destroy(self.h)


def test_batch_refuses_an_item_that_writes_another_items_buffers():
    sp = H.SchemaPair(W.PLAIN8)
    aos, soa = sp.layout("aos"), sp.layout("soa")
    n = 1000
    a = H.alloc_device(aos.lib.buffer_bytes(n))
    s = H.alloc_device(soa.lib.buffer_bytes(n))
    a2 = H.alloc_device(aos.lib.buffer_bytes(n))
    # chained: item 1 reads what item 0 writes
    b = _Batch()
    b.add(P.View(aos.lib, n, a), P.View(soa.lib, n, s), n)
    b.add(P.View(soa.lib, n, s), P.View(aos.lib, n, a2), n)
    assert b.finalize() == P.RL_EOVERLAP
    # two items writing the same destination
    b = _Batch()
    b.add(P.View(aos.lib, n, a), P.View(soa.lib, n, s), n)
    b.add(P.View(aos.lib, n, a2), P.View(soa.lib, n, s), n)
    assert b.finalize() == P.RL_EOVERLAP
    # a shared source is fine
    s2 = H.alloc_device(soa.lib.buffer_bytes(n))
    b = _Batch()
    b.add(P.View(aos.lib, n, a), P.View(soa.lib, n, s), n)
    b.add(P.View(aos.lib, n, a), P.View(soa.lib, n, s2), n)
    assert b.finalize() == P.RL_OK, P.rl_last_error()
