"""Pins for the oracle's gathers (insertion, deletion and compaction of a
collection, Sec. VII-B), each against something other than the gather
itself: numpy's own deletion, masking and insertion on structured record
arrays; the collection rebuilt from numpy-selected logical values and packed
through the (separately pinned) conversion; the identity gather against the
conversion; statuses."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import npref


def pick(v, idx):
    """Logical values of the objects idx of v, in that order (numpy)."""
    idx = np.asarray(idx, dtype=np.int64)
    out = W.Values(v.schema, len(idx))
    for f in v.schema.object_fields():
        out.fields[f.name] = np.asarray(v.fields[f.name])[idx]
    for g in range(len(v.schema.offset_types)):
        lens = np.asarray(v.lengths[g]).astype(np.int64)
        starts = np.concatenate([[0], np.cumsum(lens)])[:-1]
        out.lengths.append(lens[idx].astype(np.uint32))
        for f in v.schema.member_fields(g):
            a = np.asarray(v.members[f.name])
            parts = [a[starts[i]:starts[i] + lens[i]] for i in idx]
            out.members[f.name] = (np.concatenate(parts) if parts else a[:0]).copy()
        out.block_order.append(np.arange(len(idx)))
    return out


def concat(a, b):
    """Logical values of a's objects followed by b's."""
    out = W.Values(a.schema, a.n + b.n)
    for f in a.schema.object_fields():
        out.fields[f.name] = np.concatenate([np.asarray(a.fields[f.name]), np.asarray(b.fields[f.name])])
    for g in range(len(a.schema.offset_types)):
        out.lengths.append(np.concatenate([a.lengths[g], b.lengths[g]]).astype(np.uint32))
        for f in a.schema.member_fields(g):
            out.members[f.name] = np.concatenate([np.asarray(a.members[f.name]), np.asarray(b.members[f.name])])
        out.block_order.append(np.arange(out.n))
    return out


def values(decl, n, seed):
    if decl is W.CLUSTER:
        return W.cluster_values(n, seed=seed, mean_len=5.0)
    return W.generic_values(decl, n, seed=seed, mean_len=3.0)


def same(got, want, what):
    assert len(got) == len(want), what
    for k, (g, w) in enumerate(zip(got, want)):
        assert np.array_equal(np.asarray(g).view(np.uint8), np.asarray(w).view(np.uint8)), f"{what}: buffer {k}"


DECLS = [W.PLAIN8, W.CELL, W.SENSOR, W.CLUSTER, W.PARTICLE]
KINDS = [("aos", 0), ("soa", 0), ("aosoa", 4)]


def members_of(S, v):
    return [v.total(g) for g in range(S.n_groups)]


@pytest.mark.parametrize("decl", DECLS, ids=lambda d: d.name)
@pytest.mark.parametrize("kind", KINDS, ids=str)
def test_identity_gather_is_the_conversion(decl, kind):
    S = oracle.Schema(decl)
    v = values(decl, 23, 1)
    src = oracle.make_layout(S, "soa")
    dst = oracle.make_layout(S, *kind)
    sb = oracle.pack(S, v, src)
    mem = members_of(S, v)
    st, want, _ = oracle.convert(src, sb, dst, v.n, mem, mem)
    assert st == 0
    out = oracle.zeros_like_layout(dst, v.n, mem)
    st, ends = oracle.gather_into(src, sb, dst, out, np.arange(v.n), 0, [0] * S.n_groups, mem, mem)
    assert st == 0 and ends == mem
    same(out, want, "identity gather")


@pytest.mark.parametrize("decl", DECLS, ids=lambda d: d.name)
@pytest.mark.parametrize("kind", KINDS, ids=str)
@pytest.mark.parametrize("n,at,count", [(1, 0, 1), (17, 0, 5), (17, 12, 5), (40, 7, 9), (40, 39, 1), (9, 3, 0)])
def test_erase_matches_values_without_the_objects(decl, kind, n, at, count):
    S = oracle.Schema(decl)
    v = values(decl, n, 2 + n + at)
    L = oracle.make_layout(S, *kind)
    bufs = oracle.pack(S, v, L)
    st, got, tots = oracle.erase(L, bufs, n, at, count, members_of(S, v))
    assert st == 0
    keep = np.concatenate([np.arange(at), np.arange(at + count, n)])
    want_v = pick(v, keep)
    assert tots == members_of(S, want_v)
    same(got, oracle.pack(S, want_v, L), f"erase {at}+{count} of {n}")


@pytest.mark.parametrize("decl", DECLS, ids=lambda d: d.name)
@pytest.mark.parametrize("src_kind,dst_kind", [(("aos", 0), ("soa", 0)), (("soa", 0), ("aosoa", 8)),
                                               (("aosoa", 3), ("aos", 0)), (("soa", 0), ("soa", 0))], ids=str)
def test_select_matches_values_of_kept_objects(decl, src_kind, dst_kind):
    S = oracle.Schema(decl)
    n = 61
    v = values(decl, n, 3)
    src = oracle.make_layout(S, *src_kind)
    dst = oracle.make_layout(S, *dst_kind)
    sb = oracle.pack(S, v, src, pool_order=True)
    flags = (np.random.default_rng(4).random(n) < 0.4).astype(np.uint8)
    mem = [len(sb[1 + g]) // src.member_stride[g] for g in range(S.n_groups)] if src.kind == "aos" else members_of(S, v)
    st, got, count, tots = oracle.select(src, sb, dst, n, flags, mem)
    assert st == 0 and count == int(flags.sum())
    want_v = pick(v, np.nonzero(flags)[0])
    same(got, oracle.pack(S, want_v, dst), "select")


@pytest.mark.parametrize("decl", DECLS, ids=lambda d: d.name)
@pytest.mark.parametrize("kind", KINDS, ids=str)
@pytest.mark.parametrize("n,at,count", [(0, 0, 3), (10, 0, 4), (10, 10, 4), (10, 6, 1), (33, 17, 20)])
def test_insert_matches_concatenated_values(decl, kind, n, at, count):
    S = oracle.Schema(decl)
    v = values(decl, n, 5 + n)
    new = values(decl, count, 6 + count)
    L = oracle.make_layout(S, *kind)
    NL = oracle.make_layout(S, "soa")
    st, got, tots = oracle.insert(L, oracle.pack(S, v, L), n, at, NL, oracle.pack(S, new, NL), count,
                                  members_of(S, v), members_of(S, new))
    assert st == 0
    both = concat(v, new)
    order = np.concatenate([np.arange(at), n + np.arange(count), np.arange(at, n)])
    want_v = pick(both, order)
    same(got, oracle.pack(S, want_v, L), f"insert {count} at {at} of {n}")


def zero_padded(a):
    """The records of a structured array with their padding bytes zero
    (numpy copies structured items field by field, so the padding of its
    results is whatever the new memory held)."""
    out = np.zeros(a.shape, a.dtype)
    for name in a.dtype.names:
        out[name] = a[name]
    return out.view(np.uint8)


@pytest.mark.parametrize("decl", [W.PLAIN8, W.CELL, W.SENSOR], ids=lambda d: d.name)
def test_record_operations_against_numpy_structured_arrays(decl):
    """np.delete, boolean masks and np.insert on the records as a numpy
    structured array give the same bytes as the oracle's gathers (padding
    zero on both sides)."""
    S = oracle.Schema(decl)
    L = oracle.make_layout(S, "aos")
    dt = npref.record_dtype(decl)
    n = 50
    v = values(decl, n, 7)
    rec = oracle.pack(S, v, L)[0]
    arr = rec.view(dt)
    st, got, _ = oracle.erase(L, [rec], n, 11, 13)
    assert st == 0
    assert np.array_equal(got[0], zero_padded(np.delete(arr, np.arange(11, 24))))
    flags = (np.arange(n) % 3 == 1).astype(np.uint8)
    st, got, count, _ = oracle.select(L, [rec], L, n, flags)
    assert st == 0 and count == flags.sum()
    assert np.array_equal(got[0], zero_padded(arr[flags.astype(bool)]))
    new = values(decl, 6, 8)
    nrec = oracle.pack(S, new, L)[0]
    st, got, _ = oracle.insert(L, [rec], n, 20, L, [nrec], 6)
    assert st == 0
    assert np.array_equal(got[0], zero_padded(np.insert(arr, 20, nrec.view(dt))))


def test_jagged_offsets_and_members_by_hand():
    """Cluster objects 0..5 with counts 2,0,3,1,0,2; erase objects 1..2 and
    select objects {0, 3, 5}: offsets and member columns written out."""
    decl = W.CLUSTER
    S = oracle.Schema(decl)
    v = W.cluster_values(6, seed=9)
    v.lengths[0] = np.array([2, 0, 3, 1, 0, 2], dtype=np.uint32)
    v.members["cell_index"] = np.arange(100, 108, dtype=np.uint32)
    v.members["cell_weight"] = np.arange(8, dtype=np.float32) / 8
    L = oracle.make_layout(S, "soa")
    bufs = oracle.pack(S, v, L)
    st, got, tots = oracle.erase(L, bufs, 6, 1, 2, [8])
    assert st == 0 and tots == [5]
    assert list(got[6].view(np.uint32)) == [0, 2, 3, 3, 5]
    assert list(got[7].view(np.uint32)) == [100, 101, 105, 106, 107]
    st, got, count, tots = oracle.select(L, bufs, L, 6, np.array([1, 0, 0, 1, 0, 1], np.uint8), [8])
    assert st == 0 and count == 3 and tots == [5]
    assert list(got[6].view(np.uint32)) == [0, 2, 3, 5]
    assert list(got[7].view(np.uint32)) == [100, 101, 105, 106, 107]
    assert list(got[8].view(np.float32) * 8) == [0, 1, 5, 6, 7]


def test_statuses():
    decl = W.CLUSTER
    S = oracle.Schema(decl)
    v = W.cluster_values(30, seed=10, mean_len=4.0)
    L = oracle.make_layout(S, "aos")
    soa = oracle.make_layout(S, "soa")
    bufs = oracle.pack(S, v, L)
    pool = len(bufs[1]) // 8
    idx = np.arange(30)
    tot = v.total(0)
    # capacity one short
    out = oracle.zeros_like_layout(soa, 30, [tot])
    st, _ = oracle.gather_into(L, bufs, soa, out, idx, 0, [0], [pool], [tot - 1])
    assert st == oracle.ST_CAPACITY
    # a record outside its pool: only an error when that object is gathered
    bad = [b.copy() for b in bufs]
    ptr_off = L.slot_offsets[S.slots.index(("ptr", 0))]
    bad[0].reshape(30, L.stride)[7, ptr_off:ptr_off + 8] = np.frombuffer(np.uint64(len(bufs[1]) + 8).tobytes(),
                                                                         np.uint8)
    out = oracle.zeros_like_layout(soa, 30, [tot])
    st, _ = oracle.gather_into(L, bad, soa, out, idx, 0, [0], [pool], [tot])
    assert st == oracle.ST_BOUNDS
    keep = np.delete(idx, 7)
    tot2 = tot - int(v.lengths[0][7])
    out = oracle.zeros_like_layout(soa, 29, [tot2])
    st, _ = oracle.gather_into(L, bad, soa, out, keep, 0, [0], [pool], [tot2])
    assert st == 0
    # a member base that pushes the end past a u32 offset type
    out = oracle.zeros_like_layout(soa, 30, [tot])
    st, _ = oracle.gather_into(L, bufs, soa, out, idx, 0, [2**32 - 2], [pool], [2**40])
    assert st == oracle.ST_OVERFLOW
