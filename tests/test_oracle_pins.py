"""Pins for the CPU oracle: each test checks it against something other than
itself (numpy's record layout rules, transposes, special block widths,
round-trip identities, cumsum, an independent bit-level rounding, brute
force through numpy views)."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
import workloads as W
from tests import npref

ALL = [W.PLAIN8, W.CELL, W.CLUSTER, W.SENSOR, W.PARTICLE]


# ------------------------------------------------------------ record layouts (P2)

@pytest.mark.parametrize("decl", ALL, ids=lambda d: d.name)
def test_natural_record_matches_numpy_aligned_dtype(decl):
    S = oracle.Schema(decl)
    offs, stride = oracle.natural_record(S)
    dt = npref.record_dtype(decl)
    assert stride == dt.itemsize
    # every leaf slot at numpy's offset
    for slot, off in zip(S.slots, offs):
        kind, idx = slot
        if kind == "leaf":
            f, e = S.leaves[idx]
            if f.subgroup >= 0:
                sub = dt.fields[f"sub{f.subgroup}"]
                base = sub[1] + sub[0].fields[f.name][1]
            else:
                base = dt.fields[f.name][1]
            assert off == base + e * W.TYPE_SIZE[f.type], (f.name, e)
        else:
            assert off == dt.fields[f"{kind}{idx}"][1]


def test_config_record_layouts_hand_derived():
    # C natural alignment worked out by hand for the three workload schemas
    assert oracle.natural_record(oracle.Schema(W.PLAIN8)) == ([0, 4, 8, 12, 16, 24, 26, 28], 32)
    assert oracle.natural_record(oracle.Schema(W.CELL)) == ([0, 4, 8, 10, 12, 16, 24], 32)
    assert oracle.natural_record(oracle.Schema(W.CLUSTER)) == ([0, 4, 8, 12, 16, 20, 24, 32], 40)


@pytest.mark.parametrize("decl", [W.PLAIN8, W.CELL, W.SENSOR, W.PARTICLE], ids=lambda d: d.name)
def test_packed_records_read_back_by_numpy(decl):
    S = oracle.Schema(decl)
    v = W.generic_values(decl, 37, seed=5)
    if decl is W.PARTICLE:
        v = W.generic_values(decl, 37, seed=5, mean_len=2.0)
    L = oracle.make_layout(S, "aos")
    bufs = oracle.pack(S, v, L)
    rec = bufs[0].view(npref.record_dtype(decl))
    for f in decl.object_fields():
        assert np.array_equal(npref.field_of(rec, decl, f.name), v.fields[f.name]), f.name
    # padding bytes are zero: zero every field through numpy and the rest must be zero
    r2 = bufs[0].copy().view(rec.dtype)   # byte copy (ndarray.copy may skip padding)
    for name in r2.dtype.names:
        r2[name] = 0
    assert not r2.view(np.uint8).any()


# ------------------------------------------------------------ transpose (P3)

def test_same_width_schema_aos_to_soa_is_a_transpose():
    decl = W.SchemaDecl("w4", tuple(W.Field(f"x{k}", t) for k, t in
                                    enumerate(["u32", "f32", "i32", "u32", "f32"])))
    S = oracle.Schema(decl)
    n = 101
    rng = np.random.default_rng(3)
    raw = rng.integers(0, 2**32, size=(n, 5), dtype=np.uint32)
    aos = oracle.make_layout(S, "aos")
    soa = oracle.make_layout(S, "soa")
    st, out, _ = oracle.convert(aos, [raw.view(np.uint8).reshape(-1)], soa, n)
    assert st == 0
    expect = raw.T.copy()
    for c in range(5):
        assert np.array_equal(out[c].view(np.uint32), expect[c])


# ------------------------------------------------------------ block width special cases (P6)

@pytest.mark.parametrize("decl", [W.PLAIN8, W.CELL, W.SENSOR], ids=lambda d: d.name)
def test_aosoa_width_one_is_a_packed_record(decl):
    S = oracle.Schema(decl)
    v = W.generic_values(decl, 29, seed=11)
    bufs = oracle.pack(S, v, oracle.make_layout(S, "aosoa", width=1))
    rec = bufs[0].view(npref.record_dtype(decl, align=False))
    for f in decl.object_fields():
        assert np.array_equal(npref.field_of(rec, decl, f.name), v.fields[f.name])


@pytest.mark.parametrize("decl", [W.PLAIN8, W.CELL], ids=lambda d: d.name)
def test_aosoa_width_n_is_back_to_back_columns(decl):
    S = oracle.Schema(decl)
    n = 23
    v = W.generic_values(decl, n, seed=12)
    blk = oracle.pack(S, v, oracle.make_layout(S, "aosoa", width=n))[0]
    cols = oracle.pack(S, v, oracle.make_layout(S, "soa"))
    assert np.array_equal(blk, np.concatenate(cols))


@pytest.mark.parametrize("width", [1, 2, 3, 7, 32, 64, 128])
def test_soa_aosoa_is_a_per_column_block_copy(width):
    decl = W.CELL
    S = oracle.Schema(decl)
    n = 301
    v = W.cell_values(n, seed=13)
    soa = oracle.pack(S, v, oracle.make_layout(S, "soa"))
    blk = oracle.pack(S, v, oracle.make_layout(S, "aosoa", width=width))[0]
    sizes = [W.TYPE_SIZE[t] for t in S.leaf_types()]
    for c, (f, _) in enumerate(S.leaves):
        col = npref.aosoa_column(blk, width, sizes, c, n, W.NP_DTYPE[f.type])
        assert np.array_equal(col.view(np.uint8), soa[c]), f.name
    # the unused slots of the last block are zero
    nblk = -(-n // width)
    assert len(blk) == nblk * width * sum(sizes)
    if n % width:
        blocks = blk.reshape(nblk, width * sum(sizes))
        last = blocks[-1]
        pos = 0
        for s in sizes:
            run = last[pos: pos + width * s]
            assert not run[(n % width) * s:].any()
            pos += width * s


# ------------------------------------------------------------ round trips and byte counts (P5)

@pytest.mark.parametrize("decl", ALL, ids=lambda d: d.name)
@pytest.mark.parametrize("mid", ["soa", "aosoa3", "aosoa64"])
def test_round_trips_are_identities(decl, mid):
    S = oracle.Schema(decl)
    v = W.generic_values(decl, 130, seed=21, mean_len=3.0, shuffle_pool=False)
    aos = oracle.make_layout(S, "aos")
    src = oracle.pack(S, v, aos)
    M = (oracle.make_layout(S, "soa") if mid == "soa"
         else oracle.make_layout(S, "aosoa", width=int(mid[5:])))
    tot = [v.total(g) for g in range(S.n_groups)]
    st, mb, t1 = oracle.convert(aos, src, M, v.n, tot)
    assert st == 0 and t1 == tot
    st, back, t2 = oracle.convert(M, mb, aos, v.n, tot)
    assert st == 0 and t2 == tot
    for a, b in zip(src, back):
        assert np.array_equal(a, b)
    # payload bytes agree across layouts (AoS record minus padding and ptr/len slots)
    payload = sum(W.TYPE_SIZE[t] for t in S.leaf_types()) * v.n
    if M.kind == "soa":
        assert sum(len(b) for b in mb[:len(S.leaves)]) == payload


def test_narrow_then_widen_round_trip_on_representable_values():
    S = oracle.Schema(W.CELL)
    v = W.cell_values(500, seed=31)
    v.fields["energy_d"] = v.fields["energy"].astype(np.float64)  # exactly representable
    soa32 = oracle.make_layout(S, "soa", storage=["f32", "f32", "i8", "u16", "u32", "u32", "f32"])
    aos64 = oracle.make_layout(S, "aos")
    src = oracle.pack(S, v, soa32)
    st, a, _ = oracle.convert(soa32, src, aos64, v.n)
    assert st == 0
    st, back, _ = oracle.convert(aos64, a, soa32, v.n)
    assert st == 0
    for x, y in zip(src, back):
        assert np.array_equal(x, y)


def test_cell_order_and_narrowing_invariants():
    # hash[i] == i survives (order preserved) and the narrowed energy_d equals
    # energy, which the generator rounded with numpy's own cast
    S = oracle.Schema(W.CELL)
    v = W.cell_values(5000)
    aos = oracle.make_layout(S, "aos")
    soa = oracle.make_layout(S, "soa", storage=["f32", "f32", "i8", "u16", "u32", "u32", "f32"])
    st, out, _ = oracle.convert(aos, oracle.pack(S, v, aos), soa, v.n)
    assert st == 0
    assert np.array_equal(out[4].view(np.uint32), np.arange(v.n, dtype=np.uint32))
    assert np.array_equal(out[6], out[0])
    assert len(out[6]) == 4 * v.n


def test_copies_keep_nan_payloads_and_signed_zero():
    decl = W.SchemaDecl("fp", (W.Field("x", "f64"), W.Field("y", "f32")))
    S = oracle.Schema(decl)
    xs = np.array([0x7FF0000000000001, 0xFFF8DEADBEEF0001, 0x8000000000000000], dtype=np.uint64)
    ys = np.array([0x7F800001, 0xFFC0BEEF, 0x80000000], dtype=np.uint32)
    aos = oracle.make_layout(S, "aos")
    soa = oracle.make_layout(S, "soa")
    st, out, _ = oracle.convert(soa, [xs.view(np.uint8), ys.view(np.uint8)], aos, 3)
    assert st == 0
    st, back, _ = oracle.convert(aos, out, soa, 3)
    assert np.array_equal(back[0].view(np.uint64), xs)
    assert np.array_equal(back[1].view(np.uint32), ys)


# ------------------------------------------------------------ offsets (P7)

@pytest.mark.parametrize("off_type", ["u32", "i32", "u64"])
def test_exclusive_scan_is_cumsum(off_type):
    rng = np.random.default_rng(7)
    lens = rng.poisson(40, size=10_001).astype(np.uint32)
    st, offs, tot = oracle.exclusive_scan(lens, off_type)
    assert st == 0 and tot == int(lens.sum())
    expect = np.concatenate([[0], np.cumsum(lens.astype(np.int64))])
    assert np.array_equal(offs.astype(np.int64), expect)
    assert offs[0] == 0 and np.all(np.diff(offs.astype(np.int64)) == lens)


def test_exclusive_scan_overflow_detection():
    # the total must fit the offset type: 2**32 - 1 fits u32, 2**32 does not
    assert oracle.exclusive_scan(np.array([2**31, 2**31 - 1], dtype=np.uint32), "u32")[0] == oracle.ST_OK
    assert oracle.exclusive_scan(np.array([2**31, 2**31], dtype=np.uint32), "u32")[0] == oracle.ST_OVERFLOW
    assert oracle.exclusive_scan(np.array([2**31, 2**31], dtype=np.uint32), "u64")[0] == oracle.ST_OK
    assert oracle.exclusive_scan(np.array([2**30, 2**30 - 1], dtype=np.uint32), "i32")[0] == oracle.ST_OK
    assert oracle.exclusive_scan(np.array([2**30, 2**30], dtype=np.uint32), "i32")[0] == oracle.ST_OVERFLOW


# ------------------------------------------------------------ jagged members (P8)

def _cluster_layouts():
    S = oracle.Schema(W.CLUSTER)
    return S, oracle.make_layout(S, "aos"), oracle.make_layout(S, "soa")


def test_jagged_gather_matches_numpy_member_views():
    S, aos, soa = _cluster_layouts()
    v = W.cluster_values(2000, seed=41)
    src = oracle.pack(S, v, aos, pool_order=True)
    tot = v.total(0)
    st, out, totals = oracle.convert(aos, src, soa, v.n, [tot])
    assert st == 0 and totals == [tot]
    rec = src[0].view(npref.record_dtype(W.CLUSTER))
    pool = src[1].view(npref.member_dtype(W.CLUSTER, 0))
    offs = out[6].view(np.uint32)
    idx, wgt = out[7].view(np.uint32), out[8].view(np.float32)
    assert np.array_equal(np.diff(offs.astype(np.int64)), rec["len0"].astype(np.int64))
    rng = np.random.default_rng(0)
    for i in rng.choice(v.n, size=200, replace=False):
        first = int(rec["ptr0"][i]) // pool.dtype.itemsize
        ln = int(rec["len0"][i])
        assert np.array_equal(idx[offs[i]:offs[i] + ln], pool["cell_index"][first:first + ln])
        assert np.array_equal(wgt[offs[i]:offs[i] + ln], pool["cell_weight"][first:first + ln])
    # and against the generator's values in object order
    assert np.array_equal(idx, v.members["cell_index"])
    assert np.array_equal(wgt, v.members["cell_weight"])


def test_jagged_pool_order_does_not_change_the_result():
    S, aos, soa = _cluster_layouts()
    v = W.cluster_values(777, seed=42)
    a = oracle.pack(S, v, aos, pool_order=True)
    b = oracle.pack(S, v, aos, pool_order=False)
    assert not np.array_equal(a[1], b[1])        # the pools differ
    tot = [v.total(0)]
    ra = oracle.convert(aos, a, soa, v.n, tot)[1]
    rb = oracle.convert(aos, b, soa, v.n, tot)[1]
    for x, y in zip(ra, rb):
        assert np.array_equal(x, y)


def test_jagged_reverse_is_canonical_packing():
    S, aos, soa = _cluster_layouts()
    v = W.cluster_values(500, seed=43)
    shuffled = oracle.pack(S, v, aos, pool_order=True)
    tot = [v.total(0)]
    st, mid, _ = oracle.convert(aos, shuffled, soa, v.n, tot)
    st, back, _ = oracle.convert(soa, mid, aos, v.n, tot)
    assert st == 0
    rec = back[0].view(npref.record_dtype(W.CLUSTER))
    lens = v.lengths[0].astype(np.uint64)
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint64)
    assert np.array_equal(rec["ptr0"], starts * 8)
    assert np.array_equal(rec["len0"], v.lengths[0])
    pool = back[1].view(npref.member_dtype(W.CLUSTER, 0))
    assert np.array_equal(pool["cell_index"], v.members["cell_index"])
    assert np.array_equal(pool["cell_weight"], v.members["cell_weight"])


def test_jagged_error_statuses():
    S, aos, soa = _cluster_layouts()
    v = W.cluster_values(50, seed=44)
    src = oracle.pack(S, v, aos, pool_order=False)
    tot = v.total(0)
    # destination too small
    st, _, _ = oracle.convert(aos, src, soa, v.n, [tot], [tot - 1])
    assert st == oracle.ST_CAPACITY
    # a member block beyond the end of the pool
    bad = [b.copy() for b in src]
    rec = bad[0].view(npref.record_dtype(W.CLUSTER))
    rec["ptr0"][3] = len(bad[1])
    st, _, _ = oracle.convert(aos, bad, soa, v.n, [tot], [tot])
    assert st == oracle.ST_BOUNDS if rec["len0"][3] else st == 0
    # a misaligned member block
    bad = [b.copy() for b in src]
    rec = bad[0].view(npref.record_dtype(W.CLUSTER))
    rec["ptr0"][0] += 2
    assert oracle.convert(aos, bad, soa, v.n, [tot], [tot])[0] == oracle.ST_BOUNDS
    # a total beyond the offset type
    bad = [b.copy() for b in src]
    rec = bad[0].view(npref.record_dtype(W.CLUSTER))
    rec["len0"][:3] = 2**31
    assert oracle.convert(aos, bad, soa, v.n, [tot], [tot], dst_capacity=[2**40])[0] == oracle.ST_OVERFLOW


def test_paper_particle_schema_flattening():
    # Particle (Sec. III listing, declared in Sec. VI): 6 scalar leaves, three
    # arrays of extent 4 (12 leaves), one jagged u64 list with an int prefix sum
    S = oracle.Schema(W.PARTICLE)
    assert len(S.leaves) == 6 + 3 * W.N_SENSOR_TYPES
    assert S.n_groups == 1 and S.member_types(0) == ["u64"]
    assert W.PARTICLE.offset_types == ("i32",)
    names = [f.name for f, _ in S.leaves]
    assert names[:6] == ["energy", "x", "y", "origin", "x_variance", "y_variance"]
    # Sensor: the calibration sub-group flattens into five separate leaves
    S2 = oracle.Schema(W.SENSOR)
    assert [f.name for f, _ in S2.leaves] == [
        "type", "counts", "energy", "noisy", "parameter_A", "parameter_B", "noise_A", "noise_B"]


# ------------------------------------------------------------ narrowing (P9)

def _rne_bits(d):
    """Independent double -> float rounding to nearest even, on the IEEE-754
    bit fields only (no floating-point arithmetic).  NaNs excluded."""
    b = np.asarray(d, dtype=np.float64).view(np.uint64)
    sign = (b >> np.uint64(63)).astype(np.uint64)
    exp = ((b >> np.uint64(52)) & np.uint64(0x7FF)).astype(np.int64)
    man = b & np.uint64((1 << 52) - 1)
    out = np.zeros(b.shape, dtype=np.uint64)
    for k in range(b.size):
        e, m, s = int(exp.flat[k]), int(man.flat[k]), int(sign.flat[k])
        if e == 0x7FF:                       # infinity
            r = 0xFF << 23
        elif e == 0:                         # double subnormals underflow to zero
            r = 0
        else:
            full = (1 << 52) | m
            ue = e - 1023
            if ue >= -126:
                shift = 29
                q, rem = full >> shift, full & ((1 << shift) - 1)
                half = 1 << (shift - 1)
                if rem > half or (rem == half and (q & 1)):
                    q += 1
                if q == 1 << 24:
                    q >>= 1
                    ue += 1
                r = (0xFF << 23) if ue > 127 else ((ue + 127) << 23) | (q & ((1 << 23) - 1))
            else:                            # result in the subnormal range (units of 2**-149)
                shift = -(ue + 97)
                if shift > 60:
                    q, rem, half = 0, 1, 2
                else:
                    q, rem = full >> shift, full & ((1 << shift) - 1)
                    half = 1 << (shift - 1)
                if rem > half or (rem == half and (q & 1)):
                    q += 1
                r = q                        # q == 2**23 encodes the smallest normal
        out.flat[k] = (s << 31) | r
    return out.astype(np.uint32)


def _oracle_narrow(d):
    decl = W.SchemaDecl("n1", (W.Field("x", "f64"),))
    S = oracle.Schema(decl)
    src = oracle.make_layout(S, "soa")
    dst = oracle.make_layout(S, "soa", storage=["f32"])
    d = np.ascontiguousarray(d, dtype=np.float64)
    st, out, _ = oracle.convert(src, [d.view(np.uint8)], dst, d.size)
    assert st == 0
    return out[0].view(np.uint32)


def narrowing_edge_vector():
    fmax = float(np.finfo(np.float32).max)
    cases = [
        (1.0, 1.0), (-2.5, -2.5),
        (1.0 + 2.0**-24, 1.0),                          # tie -> even (down)
        (1.0 + 3 * 2.0**-24, 1.0 + 2.0**-22),           # tie -> even (up)
        (1.0 + 2.0**-24 + 2.0**-40, 1.0 + 2.0**-23),    # above the tie
        (fmax, fmax),
        (fmax + 2.0**103, np.inf),                      # tie above FLT_MAX -> inf
        (fmax + 2.0**103 - 2.0**80, fmax),              # just below it
        (2.0**-126, 2.0**-126), (2.0**-149, 2.0**-149),
        (2.0**-150, 0.0),                               # tie -> even (zero)
        (3 * 2.0**-151, 2.0**-149),
        (2.0**-150 + 2.0**-170, 2.0**-149),
        (-0.0, -0.0), (np.inf, np.inf), (-np.inf, -np.inf),
        (1e300, np.inf), (-1e300, -np.inf), (1e-300, 0.0), (-1e-300, -0.0),
        (5e-324, 0.0),
    ]
    return cases


def test_narrowing_edge_vector_closed_forms():
    cases = narrowing_edge_vector()
    d = np.array([c[0] for c in cases])
    want = np.array([c[1] for c in cases], dtype=np.float32).view(np.uint32)
    assert np.array_equal(_oracle_narrow(d), want)
    assert np.array_equal(_rne_bits(d), want)


def test_narrowing_agrees_with_bitwise_rounding_on_random_doubles():
    rng = np.random.default_rng(99)
    bits = rng.integers(0, 2**64, size=40_000, dtype=np.uint64)
    d = bits.view(np.float64)
    d = d[np.isfinite(d)]
    # bias towards the float range, the subnormal range and exact ties
    span = np.ldexp(rng.uniform(1, 2, 20_000), rng.integers(-160, 130, 20_000))
    ties = (np.ldexp(rng.integers(1 << 23, 1 << 24, 5000).astype(np.float64) + 0.5,
                     rng.integers(-150, 100, 5000)))
    d = np.concatenate([d, span, -span, ties])
    got = _oracle_narrow(d)
    assert np.array_equal(got, _rne_bits(d))
    assert np.array_equal(got, d.astype(np.float32).view(np.uint32))


# ------------------------------------------------------------ brute force (P1)

TYPES = list(W.NP_DTYPE)


@st.composite
def schemas(draw):
    n_fields = draw(st.integers(1, 9))
    n_groups = draw(st.integers(0, 2))
    fields, sub = [], -1
    for k in range(n_fields):
        t = draw(st.sampled_from(TYPES))
        ext = draw(st.integers(1, 3))
        sg = -1
        if draw(st.booleans()) and draw(st.booleans()):
            sg = draw(st.integers(0, 1))
        fields.append(W.Field(f"f{k}", t, ext, -1, sg))
    for g in range(n_groups):
        pos = draw(st.integers(0, len(fields)))
        for m in range(draw(st.integers(1, 3))):
            fields.insert(pos + m, W.Field(f"g{g}m{m}", draw(st.sampled_from(TYPES)), 1, g, -1))
    # sub-group ids must label contiguous runs: renumber runs
    out, run_id, prev = [], -1, None
    for f in fields:
        if f.subgroup >= 0:
            if prev is None or prev.subgroup != f.subgroup or prev.group >= 0:
                run_id += 1
            out.append(W.Field(f.name, f.type, f.extent, f.group, run_id))
        else:
            out.append(f)
        prev = f
    offs = tuple(draw(st.sampled_from(["u32", "i32", "u64"])) for _ in range(n_groups))
    return W.SchemaDecl("h", tuple(out), offs)


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(decl=schemas(), width=st.sampled_from([1, 2, 3, 4, 8]), nsel=st.integers(0, 7))
def test_brute_force_random_schemas(decl, width, nsel):
    n = [0, 1, 2, 3, width - 1, width, width + 1, 2 * width + 1][nsel]
    n = max(n, 0)
    S = oracle.Schema(decl)
    v = W.generic_values(decl, n, seed=nsel + 100 * width, mean_len=1.5)
    aos = oracle.make_layout(S, "aos")
    soa = oracle.make_layout(S, "soa")
    blk = oracle.make_layout(S, "aosoa", width=width)
    src = oracle.pack(S, v, aos, pool_order=True)
    tot = [v.total(g) for g in range(S.n_groups)]
    # AoS read back through numpy's own record layout
    if n:
        rec = src[0].view(npref.record_dtype(decl))
        for f in decl.object_fields():
            assert np.array_equal(npref.field_of(rec, decl, f.name), v.fields[f.name])
    for dstL in (soa, blk):
        st_, out, totals = oracle.convert(aos, src, dstL, n, tot)
        assert st_ == 0 and totals == tot
        sizes = [W.TYPE_SIZE[t] for t in S.leaf_types()]
        for c, (f, e) in enumerate(S.leaves):
            want = v.fields[f.name] if f.extent == 1 else v.fields[f.name][:, e]
            if dstL.kind == "soa":
                got = out[c].view(W.NP_DTYPE[f.type])
            else:
                got = npref.aosoa_column(out[0], width, sizes, c, n, W.NP_DTYPE[f.type])
            assert np.array_equal(got, want), (f.name, e)
        # groups: offsets and member columns
        base = len(S.leaves) if dstL.kind == "soa" else 1
        for g in range(S.n_groups):
            offs = out[base].view(W.NP_DTYPE[decl.offset_types[g]]).astype(np.int64)
            assert np.array_equal(offs, np.concatenate([[0], np.cumsum(v.lengths[g].astype(np.int64))]))
            for k, (f, e) in enumerate(S.members[g]):
                assert np.array_equal(out[base + 1 + k].view(W.NP_DTYPE[f.type]), v.members[f.name])
            base += 1 + len(S.members[g])
        st_, back, _ = oracle.convert(dstL, out, aos, n, tot)
        assert st_ == 0
        # reverse gives canonical pools: compare with an in-order pack
        canon = oracle.pack(S, v, aos, pool_order=False)
        for x, y in zip(back, canon):
            assert np.array_equal(x, y)


# ------------------------------------------------------------ widening and NaNs (P9)

def _oracle_widen(f):
    decl = W.SchemaDecl("w1", (W.Field("x", "f32"),))
    S = oracle.Schema(decl)
    src = oracle.make_layout(S, "soa")
    dst = oracle.make_layout(S, "soa", storage=["f64"])
    f = np.ascontiguousarray(f, dtype=np.float32)
    st, out, _ = oracle.convert(src, [f.view(np.uint8)], dst, f.size)
    assert st == 0
    return out[0].view(np.uint64)


def widening_vector():
    """Every class of single-precision value: zeros, subnormals, normals,
    the extremes, infinities (NaNs are covered separately)."""
    rng = np.random.default_rng(123)
    fi = np.finfo(np.float32)
    special = np.array([0.0, -0.0, 2.0**-149, -2.0**-149, 2.0**-127, 2.0**-126, fi.max, -fi.max,
                        np.inf, -np.inf, 1.0, -1.0, 0.1, 1e-30], dtype=np.float32)
    bits = rng.integers(0, 2**32, size=50_000, dtype=np.uint64).astype(np.uint32)
    rand = bits.view(np.float32)
    return np.concatenate([special, rand[np.isfinite(rand)]])


def test_widening_is_exact_and_matches_numpy():
    f = widening_vector()
    got = _oracle_widen(f)
    assert np.array_equal(got, f.astype(np.float64).view(np.uint64))
    # exactness: narrowing the widened value gives back the same bits
    assert np.array_equal(got.view(np.float64).astype(np.float32).view(np.uint32), f.view(np.uint32))


def nan_vectors():
    """NaN encodings: quiet and signalling, both signs, empty and full
    payloads, payload bits at both ends."""
    d = np.array([0x7FF8000000000000, 0xFFF8000000000000, 0x7FF0000000000001, 0xFFF0000000000001,
                  0x7FFFFFFFFFFFFFFF, 0xFFFFFFFFFFFFFFFF, 0x7FF4000000000000, 0x7FF8DEADBEEF0001,
                  0xFFF0000020000000, 0x7FF000001FFFFFFF, 0x7FFA5A5A5A5A5A5A], dtype=np.uint64)
    f = np.array([0x7FC00000, 0xFFC00000, 0x7F800001, 0xFF800001, 0x7FFFFFFF, 0xFFFFFFFF,
                  0x7FA00000, 0x7FC0BEEF, 0xFF812345, 0x7F8FFFFF], dtype=np.uint32)
    return d, f


def _nan_narrow_bits(b):
    """Reading of a NaN through narrowing: quiet, sign kept, leading 22
    payload bits kept (IEEE 754-2008 6.2.3 recommends keeping the payload
    as far as the destination format allows)."""
    b = np.asarray(b, dtype=np.uint64)
    return (((b >> np.uint64(63)) << np.uint64(31)) | np.uint64(0x7FC00000)
            | ((b & np.uint64((1 << 52) - 1)) >> np.uint64(29))).astype(np.uint32)


def _nan_widen_bits(b):
    b = np.asarray(b, dtype=np.uint32).astype(np.uint64)
    return (((b >> np.uint64(31)) << np.uint64(63)) | np.uint64(0x7FF8000000000000)
            | ((b & np.uint64(0x7FFFFF)) << np.uint64(29)))


def test_nan_through_narrowing_and_widening():
    d, f = nan_vectors()
    # the bit-field reading, and numpy's own casts (IEEE hardware conversion)
    assert np.array_equal(_oracle_narrow(d.view(np.float64)), _nan_narrow_bits(d))
    with np.errstate(invalid="ignore"):
        assert np.array_equal(_oracle_narrow(d.view(np.float64)), d.view(np.float64).astype(np.float32).view(np.uint32))
        assert np.array_equal(_oracle_widen(f.view(np.float32)), f.view(np.float32).astype(np.float64).view(np.uint64))
    assert np.array_equal(_oracle_widen(f.view(np.float32)), _nan_widen_bits(f))
    # every result is a quiet NaN with the input's sign
    nb = _oracle_narrow(d.view(np.float64))
    assert np.all((nb & 0x7FC00000) == 0x7FC00000)
    assert np.array_equal(nb >> 31, (d >> np.uint64(63)).astype(np.uint32))


# ------------------------------------------------------------ offsets sources not starting at 0 (P7, P8)

def _slice_view(v, k, n):
    """Objects k .. k+n-1 of a collection held in soa form, viewed in place:
    each per-object column starts at object k, the offsets column is entries
    k .. k+n of the whole collection's (so its first entry is the number of
    members before object k), and the member columns are the whole
    collection's."""
    S = oracle.Schema(v.schema)
    soa = oracle.make_layout(S, "soa")
    full = oracle.values_buffers(S, v)
    bufs = []
    for c, t in enumerate(S.leaf_types()):
        sz = W.TYPE_SIZE[t]
        bufs.append(full[c][k * sz:(k + n) * sz].copy())
    base = len(S.leaves)
    for g in range(S.n_groups):
        es = W.TYPE_SIZE[v.schema.offset_types[g]]
        bufs.append(full[base][k * es:(k + n + 1) * es].copy())
        bufs += [full[base + 1 + m].copy() for m in range(len(S.members[g]))]
        base += 1 + len(S.members[g])
    return S, soa, bufs


@pytest.mark.parametrize("decl", [W.CLUSTER, W.PARTICLE], ids=lambda d: d.name)
@pytest.mark.parametrize("dst_kind", ["aos", "soa", "aosoa"])
def test_offsets_source_with_a_nonzero_first_entry(decl, dst_kind):
    v = W.generic_values(decl, 300, seed=8, mean_len=3.0)
    k, n = 117, 150
    S, soa, bufs = _slice_view(v, k, n)
    off = np.concatenate([[0], np.cumsum(v.lengths[0].astype(np.int64))])
    assert off[k] > 0
    total = int(off[k + n] - off[k])
    cap = [len(bufs[len(S.leaves) + 1]) // W.TYPE_SIZE[S.member_types(0)[0]]]
    dst = oracle.make_layout(S, dst_kind, width=16 if dst_kind == "aosoa" else 0)
    st, out, tots = oracle.convert(soa, bufs, dst, n, cap, [total])
    assert st == 0 and tots == [total]
    # the same objects packed from index 0 give the same bytes
    sub = W.Values(decl, n)
    for f in decl.object_fields():
        sub.fields[f.name] = v.fields[f.name][k:k + n]
    sub.lengths = [v.lengths[0][k:k + n]]
    for f in decl.member_fields(0):
        sub.members[f.name] = v.members[f.name][off[k]:off[k + n]]
    sub.block_order = [np.arange(n)]
    want = oracle.pack(S, sub, dst)
    for x, y in zip(out, want):
        assert np.array_equal(x, y)
    # and directly: member j of object i is entry off[k + i] + j of the columns
    if dst_kind == "soa":
        got_off = out[len(S.leaves)].view(W.NP_DTYPE[decl.offset_types[0]]).astype(np.int64)
        assert np.array_equal(got_off, off[k:k + n + 1] - off[k])
        f0 = decl.member_fields(0)[0]
        col = out[len(S.leaves) + 1].view(W.NP_DTYPE[f0.type])
        for i in (0, 1, n // 2, n - 1):
            ln = int(v.lengths[0][k + i])
            assert np.array_equal(col[got_off[i]:got_off[i] + ln],
                                  v.members[f0.name][off[k + i]:off[k + i] + ln])


def test_offsets_source_past_its_member_columns_is_a_bounds_error():
    v = W.generic_values(W.CLUSTER, 100, seed=9, mean_len=3.0)
    S, soa, bufs = _slice_view(v, 40, 50)
    off = np.concatenate([[0], np.cumsum(v.lengths[0].astype(np.int64))])
    total = int(off[90] - off[40])
    aos = oracle.make_layout(S, "aos")
    # the member columns hold only the first off[60] members
    st, _, _ = oracle.convert(soa, bufs, aos, 50, [int(off[60])], [total])
    assert st == oracle.ST_BOUNDS
    st, _, _ = oracle.convert(soa, bufs, aos, 50, [int(off[90])], [total])
    assert st == oracle.ST_OK


# ------------------------------------------------------------ records restrided (P2)

@pytest.mark.parametrize("decl", [W.PLAIN8, W.CELL, W.SENSOR], ids=lambda d: d.name)
def test_natural_records_to_packed_records_match_numpy(decl):
    """AoS -> AoS between C natural alignment and a packed struct (explicit
    slot offsets, no padding): numpy's unaligned structured dtype of the
    same fields is the packed record."""
    S = oracle.Schema(decl)
    v = W.generic_values(decl, 301, seed=12)
    nat = oracle.make_layout(S, "aos")
    pdt = npref.record_dtype(decl, align=False)
    offs = []
    for f, e in S.leaves:
        if f.subgroup >= 0:
            sub = pdt.fields[f"sub{f.subgroup}"]
            offs.append(sub[1] + sub[0].fields[f.name][1] + e * W.TYPE_SIZE[f.type])
        else:
            offs.append(pdt.fields[f.name][1] + e * W.TYPE_SIZE[f.type])
    packed = oracle.make_layout(S, "aos", slot_offsets=offs, stride=pdt.itemsize)
    src = oracle.pack(S, v, nat)
    st, out, _ = oracle.convert(nat, src, packed, v.n)
    assert st == 0 and len(out[0]) == v.n * pdt.itemsize
    want = np.zeros(v.n, dtype=pdt)
    natural = src[0].view(npref.record_dtype(decl))
    for name in pdt.names:
        want[name] = natural[name]
    assert np.array_equal(out[0], want.view(np.uint8))
    # and back: padding of the natural records comes out zero
    st, back, _ = oracle.convert(packed, out, nat, v.n)
    assert st == 0 and np.array_equal(back[0], src[0])
