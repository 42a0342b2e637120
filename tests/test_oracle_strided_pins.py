"""Pins for the oracle's strided layouts (Sec. VII-B: a layout's arrays need
not be contiguous, only map an object index to a value), each against numpy
doing the same placement by itself: fields of a foreign record type as numpy
structured arrays with their own offsets and padding, columns as numpy
strided slices, index tables as numpy fancy assignment and fancy indexing,
the narrowing as numpy's cast; statuses for indexes past the elements."""
import numpy as np
import pytest

import oracle
import workloads as W

DECLS = [W.PLAIN8, W.CELL, W.SENSOR]


def columns(decl, v):
    """Logical values per leaf in leaf order (numpy arrays)."""
    S = oracle.Schema(decl)
    out = []
    for f, e in S.leaves:
        a = np.asarray(v.fields[f.name])
        out.append(np.ascontiguousarray(a if f.extent == 1 else a[:, e]))
    return S, out


def foreign_dtype(S, order, pad, storage=None):
    """A numpy record type holding the leaves in the given order with `pad`
    bytes before each (its own offsets, computed here) and a trailing pad."""
    storage = storage or S.leaf_types()
    names, formats, offsets, at = [], [], [], 0
    for c in order:
        t = storage[c]
        at += pad
        at = -(-at // W.TYPE_SIZE[t]) * W.TYPE_SIZE[t]
        names.append(f"l{c}")
        formats.append(W.NP_DTYPE[t])
        offsets.append(at)
        at += W.TYPE_SIZE[t]
    size = -(-(at + pad) // 8) * 8
    return np.dtype({"names": names, "formats": formats, "offsets": offsets, "itemsize": size})


def leaf_views(raw, dt, nl):
    """Buffers of a strided layout over the records `raw` (uint8): buffer c
    starts at leaf c's field offset; every leaf has the record size as its
    stride."""
    return [raw[dt.fields[f"l{c}"][1]:] for c in range(nl)], [dt.itemsize] * nl


@pytest.mark.parametrize("decl", DECLS, ids=lambda d: d.name)
@pytest.mark.parametrize("n", [1, 7, 300])
def test_fields_of_a_foreign_record_type(decl, n):
    """Writing into the fields of an existing record array in place: every
    field gets its object's value, the padding keeps what it held."""
    v = W.generic_values(decl, n, seed=40 + n)
    S, cols = columns(decl, v)
    nl = len(S.leaves)
    order = list(reversed(range(nl)))
    dt = foreign_dtype(S, order, pad=3)
    rec = np.zeros(n, dtype=dt)
    raw = rec.view(np.uint8).reshape(-1)
    raw[:] = 0xA5
    want = raw.copy().view(dt)
    for c in range(nl):
        want[f"l{c}"] = cols[c]
    bufs, strides = leaf_views(raw, dt, nl)
    L = oracle.make_layout(S, "strided", leaf_strides=strides)
    st = oracle.convert_into(oracle.values_layout(S), oracle.values_buffers(S, v), L, bufs, n)
    assert st == oracle.ST_OK
    assert np.array_equal(raw, want.view(np.uint8).reshape(-1))
    # and back: reading the fields gives the values again
    back = oracle.zeros_like_layout(oracle.values_layout(S), n)
    assert oracle.convert_into(L, bufs, oracle.values_layout(S), back, n) == oracle.ST_OK
    for c in range(nl):
        assert np.array_equal(back[c], cols[c].view(np.uint8)), c


@pytest.mark.parametrize("decl", DECLS, ids=lambda d: d.name)
@pytest.mark.parametrize("step", [1, 2, 5])
def test_columns_with_gaps_are_numpy_strided_slices(decl, step):
    """Leaf c with stride step*size(c) (plus a per-leaf extra of c elements):
    the bytes are numpy's column[::step'] assignment into a zeroed array."""
    n = 129
    v = W.generic_values(decl, n, seed=77 + step)
    S, cols = columns(decl, v)
    steps = [step + c % 3 for c in range(len(S.leaves))]
    sizes = [W.TYPE_SIZE[t] for t in S.leaf_types()]
    L = oracle.make_layout(S, "strided", leaf_strides=[k * s for k, s in zip(steps, sizes)])
    bufs = oracle.zeros_like_layout(L, n)
    assert oracle.convert_into(oracle.values_layout(S), oracle.values_buffers(S, v), L, bufs, n) == oracle.ST_OK
    for c, (k, col) in enumerate(zip(steps, cols)):
        want = np.zeros((n - 1) * k + 1, dtype=col.dtype)
        want[::k] = col
        assert np.array_equal(bufs[c], want.view(np.uint8)), c


@pytest.mark.parametrize("decl", DECLS, ids=lambda d: d.name)
def test_index_table_scatter_and_gather(decl):
    """Indexed destination: element index[i] of every leaf takes object i's
    value (numpy fancy assignment), other elements keep theirs.  Indexed
    source: object i reads element index[i] (numpy fancy indexing)."""
    n, m = 250, 400
    rng = np.random.default_rng(5)
    v = W.generic_values(decl, n, seed=91)
    S, cols = columns(decl, v)
    idx = rng.permutation(m)[:n].astype(np.uint64)
    L = oracle.make_layout(S, "strided", indexed=True)
    bufs = oracle.zeros_like_layout(L, m)
    for b in bufs[:-1]:
        b[:] = 0x3C
    bufs[-1].view(np.uint64)[:n] = idx
    st = oracle.convert_into(oracle.values_layout(S), oracle.values_buffers(S, v), L, bufs, n)
    assert st == oracle.ST_OK
    for c, col in enumerate(cols):
        want = np.full(m * col.itemsize, 0x3C, dtype=np.uint8).view(col.dtype)
        want[idx.astype(np.int64)] = col
        assert np.array_equal(bufs[c], want.view(np.uint8)), c
    # gather through another index table
    g = rng.integers(0, m, size=n).astype(np.uint64)
    bufs[-1].view(np.uint64)[:n] = g
    out = oracle.zeros_like_layout(oracle.values_layout(S), n)
    assert oracle.convert_into(L, bufs, oracle.values_layout(S), out, n) == oracle.ST_OK
    for c in range(len(cols)):
        col = bufs[c].view(cols[c].dtype)
        assert np.array_equal(out[c], col[g.astype(np.int64)].view(np.uint8)), c


def test_indexed_to_indexed_with_narrowing():
    """Both sides indexed, f64 energy_d stored as f32 on the destination: the
    value of source element s[i] lands at destination element d[i], narrowed
    as numpy's cast to float32."""
    n, m = 300, 512
    rng = np.random.default_rng(8)
    v = W.cell_values(n, seed=12)
    S, cols = columns(W.CELL, v)
    storage = S.leaf_types()
    k = [f.name for f, _ in S.leaves].index("energy_d")
    narrow = list(storage)
    narrow[k] = "f32"
    src = oracle.make_layout(S, "strided", indexed=True)
    dst = oracle.make_layout(S, "strided", indexed=True, storage=narrow)
    sb = oracle.zeros_like_layout(src, m)
    db = oracle.zeros_like_layout(dst, m)
    s_idx = rng.permutation(m)[:n].astype(np.int64)
    d_idx = rng.permutation(m)[:n].astype(np.int64)
    for c, col in enumerate(cols):
        sb[c].view(col.dtype)[s_idx] = col
    sb[-1].view(np.uint64)[:n] = s_idx
    db[-1].view(np.uint64)[:n] = d_idx
    assert oracle.convert_into(src, sb, dst, db, n) == oracle.ST_OK
    for c, col in enumerate(cols):
        want = np.zeros(m, dtype=W.NP_DTYPE[narrow[c]])
        want[d_idx] = col.astype(want.dtype)
        assert np.array_equal(db[c], want.view(np.uint8)), c
    assert db[k].view(np.float32)[d_idx].tobytes() == cols[k].astype(np.float32).tobytes()


def test_gather_with_strided_sides():
    """The gather (insert/erase/compaction definition) with a strided
    source: destination object k0 + k takes element index[idx[k]]."""
    n, m = 60, 100
    rng = np.random.default_rng(21)
    v = W.generic_values(W.PLAIN8, n, seed=3)
    S, cols = columns(W.PLAIN8, v)
    L = oracle.make_layout(S, "strided", indexed=True)
    sb = oracle.zeros_like_layout(L, m)
    e = rng.permutation(m)[:n].astype(np.int64)
    for c, col in enumerate(cols):
        sb[c].view(col.dtype)[e] = col
    sb[-1].view(np.uint64)[:n] = e
    pick = rng.integers(0, n, size=25).astype(np.uint64)
    soa = oracle.make_layout(S, "soa")
    out = oracle.zeros_like_layout(soa, 30)
    st, _ = oracle.gather_into(L, sb, soa, out, pick, k0=5)
    assert st == oracle.ST_OK
    for c, col in enumerate(cols):
        got = out[c].view(col.dtype)
        assert np.array_equal(got[5:30], col[pick.astype(np.int64)]), c
        assert not got[:5].any()


def test_index_bound_is_strict():
    """An index equal to the element count is out of range; one below it is
    the last element."""
    S = oracle.Schema(W.PLAIN8)
    v = W.generic_values(W.PLAIN8, 4, seed=1)
    L = oracle.make_layout(S, "strided", indexed=True)
    src = oracle.values_buffers(S, v)
    for idx, want in [([0, 1, 2, 9], oracle.ST_OK), ([0, 1, 2, 10], oracle.ST_BOUNDS),
                      ([2**63, 0, 1, 2], oracle.ST_BOUNDS)]:
        bufs = oracle.zeros_like_layout(L, 10)
        bufs[-1].view(np.uint64)[:4] = idx
        assert oracle.convert_into(oracle.values_layout(S), src, L, bufs, 4) == want, idx
        st = oracle.convert_into(L, bufs, oracle.values_layout(S),
                                 oracle.zeros_like_layout(oracle.values_layout(S), 4), 4)
        assert st == want, idx
    # the elements come from the buffers: a shorter leaf buffer lowers the bound
    bufs = oracle.zeros_like_layout(L, 10)
    bufs[0] = bufs[0][:4 * 4]      # leaf 0 is f32: four elements
    bufs[-1].view(np.uint64)[:4] = [0, 1, 2, 4]
    assert oracle.convert_into(L, bufs, oracle.values_layout(S),
                               oracle.zeros_like_layout(oracle.values_layout(S), 4), 4) == oracle.ST_BOUNDS


def test_unindexed_natural_strides_hold_soa_bytes():
    """Natural strides and no index: the same buffers as numpy columns."""
    n = 33
    v = W.generic_values(W.SENSOR, n, seed=2)
    S, cols = columns(W.SENSOR, v)
    L = oracle.make_layout(S, "strided")
    bufs = oracle.zeros_like_layout(L, n)
    assert oracle.convert_into(oracle.values_layout(S), oracle.values_buffers(S, v), L, bufs, n) == oracle.ST_OK
    for c, col in enumerate(cols):
        assert np.array_equal(bufs[c], col.view(np.uint8)), c


def test_gather_index_bounds():
    """A gathered object whose element lies past the elements, on either
    side, is reported (ST_BOUNDS); in range it is not."""
    S = oracle.Schema(W.PLAIN8)
    v = W.generic_values(W.PLAIN8, 6, seed=4)
    L = oracle.make_layout(S, "strided", indexed=True)
    soa = oracle.make_layout(S, "soa")
    for e, want in [([0, 1, 2, 3, 4, 7], oracle.ST_OK), ([0, 1, 2, 3, 4, 8], oracle.ST_BOUNDS)]:
        sb = oracle.zeros_like_layout(L, 8)
        sb[-1].view(np.uint64)[:6] = e
        st, _ = oracle.gather_into(L, sb, soa, oracle.zeros_like_layout(soa, 6), [5, 0])
        assert st == want, e
        st, _ = oracle.gather_into(oracle.values_layout(S), oracle.values_buffers(S, v), L, sb, [1, 2], k0=4)
        assert st == want, e
