"""Pins for the oracle's property trees (Sec. VI: array properties holding
several properties, sub-groups and jagged vectors inside arrays, arrays and
sub-groups inside jagged vectors), each against numpy doing the same by
itself: record and member-record offsets against numpy's nested structured
dtypes with C alignment (align=True), the flattening order against the
order of the dtype's scalars, packed records, pools and columns against
structured arrays and columns filled path by path from the logical values."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import npref

TREES = [W.TRACKER, W.DETECTOR]


def record_scalars(decl, leaf_type=None):
    dt = npref.tree_dtype(decl.props, leaf_type)
    return dt, npref.flatten_dtype(dt)


def jagged_node(decl, path):
    """The Jagged property a group path names (array indexes dropped)."""
    props = decl.props
    node = None
    for part in path.split("."):
        name = part.split("[")[0]
        node = next(p for p in props if p.name == name)
        props = getattr(node, "props", ())
    assert type(node).__name__ == "Jagged"
    return node


def groups_of(decl):
    """Group paths in the order the record's pointer fields come."""
    _, flat = record_scalars(decl)
    return [p[:-4] for p, _, _ in flat if p.endswith("#ptr")]


@pytest.mark.parametrize("decl", TREES, ids=lambda d: d.name)
def test_natural_record_and_order_match_numpy(decl):
    S = oracle.Schema(decl)
    dt, flat = record_scalars(decl)
    offs, stride = oracle.natural_record(S)
    assert stride == dt.itemsize
    assert offs == [o for _, o, _ in flat]
    # slot k of the oracle is scalar k of the dtype: leaves by path, pairs
    names = []
    for kind, idx in S.slots:
        names.append(S.leaves[idx][0].name if kind == "leaf" else kind)
    want = [p if "#" not in p else p.split("#")[1] for p, _, _ in flat]
    assert names == want
    assert S.offset_types == list(decl.offset_types)


def test_narrowed_elements_are_their_own_structs():
    """Narrowing every f64 of an array, or only one element's, gives the
    record numpy builds with those types (element structs of different
    sizes where only some are narrowed)."""
    decl = W.DETECTOR
    S = oracle.Schema(decl)
    paths = [f.name for f, _ in S.leaves]
    for rule in (lambda p: p.endswith("gain"), lambda p: p == "modules[1].cal.gain", lambda p: p == "t0"):
        types = ["f32" if rule(p) and t == "f64" else t for p, t in zip(paths, S.leaf_types())]
        dt, flat = record_scalars(decl, lambda p, t: "f32" if rule(p) and t == "f64" else t)
        offs, stride = oracle.natural_record(S, types)
        assert stride == dt.itemsize
        assert offs == [o for _, o, _ in flat]


@pytest.mark.parametrize("decl", TREES, ids=lambda d: d.name)
def test_member_records_match_numpy(decl):
    S = oracle.Schema(decl)
    gpaths = groups_of(decl)
    assert len(gpaths) == S.n_groups
    for g, gp in enumerate(gpaths):
        node = jagged_node(decl, gp)
        dt = npref.tree_dtype(node.props)
        flat = npref.flatten_dtype(dt)
        offs, stride, align = oracle.natural_member_record(S, g)
        assert offs == [o for _, o, _ in flat], gp
        assert stride == dt.itemsize and align == dt.alignment, gp
        assert [f.name for f, _ in S.members[g]] == [f"{gp}.{p}" for p, _, _ in flat]


@pytest.mark.parametrize("decl", TREES, ids=lambda d: d.name)
@pytest.mark.parametrize("n", [1, 37])
def test_packed_records_and_pools_match_structured_arrays(decl, n):
    S = oracle.Schema(decl)
    v = W.tree_values(decl, n, seed=n + 5)
    L = oracle.make_layout(S, "aos")
    got = oracle.pack(S, v, L)
    dt, flat = record_scalars(decl)
    rec = np.zeros(n, dtype=dt)
    raw = rec.view(np.uint8).reshape(n, dt.itemsize)
    gpaths = groups_of(decl)
    for path, off, sdt in flat:
        if path.endswith("#ptr") or path.endswith("#len"):
            g = gpaths.index(path[:-4])
            lens = v.lengths[g].astype(np.uint64)
            if path.endswith("#len"):
                col = lens.astype(np.uint32)
            else:
                mstride = npref.tree_dtype(jagged_node(decl, gpaths[g]).props).itemsize
                col = (np.concatenate([[0], np.cumsum(lens)])[:-1] * mstride).astype(np.uint64)
        else:
            col = np.asarray(v.fields[path]).astype(sdt)
        raw[:, off:off + sdt.itemsize] = col.view(np.uint8).reshape(n, sdt.itemsize)
    assert np.array_equal(got[0], rec.view(np.uint8).reshape(-1))
    for g, gp in enumerate(gpaths):
        mdt = npref.tree_dtype(jagged_node(decl, gp).props)
        tot = v.total(g)
        pool = np.zeros(tot, dtype=mdt)
        praw = pool.view(np.uint8).reshape(tot, mdt.itemsize)
        for p, off, sdt in npref.flatten_dtype(mdt):
            col = np.asarray(v.members[f"{gp}.{p}"]).astype(sdt)
            praw[:, off:off + sdt.itemsize] = col.view(np.uint8).reshape(tot, sdt.itemsize)
        assert np.array_equal(got[1 + g], pool.view(np.uint8).reshape(-1)), gp


@pytest.mark.parametrize("decl", TREES, ids=lambda d: d.name)
def test_columns_follow_the_walk(decl):
    """SoA: one column per scalar of the record in the dtype's order, then
    per group (in pointer order) the offsets and the member columns."""
    n = 50
    S = oracle.Schema(decl)
    v = W.tree_values(decl, n, seed=2)
    got = oracle.pack(S, v, oracle.make_layout(S, "soa"))
    _, flat = record_scalars(decl)
    want = [np.asarray(v.fields[p]).astype(sdt).view(np.uint8)
            for p, _, sdt in flat if "#" not in p]
    for g, gp in enumerate(groups_of(decl)):
        t = decl.offset_types[g]
        offs = np.concatenate([[0], np.cumsum(v.lengths[g].astype(np.int64))]).astype(W.NP_DTYPE[t])
        want.append(offs.view(np.uint8))
        mdt = npref.tree_dtype(jagged_node(decl, gp).props)
        for p, _, sdt in npref.flatten_dtype(mdt):
            want.append(np.asarray(v.members[f"{gp}.{p}"]).astype(sdt).view(np.uint8))
    assert len(got) == len(want)
    for k, (a, b) in enumerate(zip(got, want)):
        assert np.array_equal(a, b), k


def test_flat_declaration_as_a_tree_has_the_same_layout():
    """The paper's particle (extent-4 arrays, a jagged vector of u64 with
    i32 prefix sums) declared as a tree gives the record, member record and
    leaf order of its flat declaration."""
    tree = W.TreeDecl("particle_tree", (
        W.Item("energy", "f32"), W.Item("x", "f32"), W.Item("y", "f32"), W.Item("origin", "u64"),
        W.Jagged("sensors", "i32", (W.Item("sensors", "u64"),)),
        W.Item("x_variance", "f32"), W.Item("y_variance", "f32"),
        W.Array("significance", 4, (W.Item("v", "f32"),)),
        W.Array("E_contribution", 4, (W.Item("v", "f32"),)),
        W.Array("noisy_count", 4, (W.Item("v", "u8"),)),
    ))
    a, b = oracle.Schema(W.PARTICLE), oracle.Schema(tree)
    assert oracle.natural_record(a) == oracle.natural_record(b)
    assert oracle.natural_member_record(a, 0) == oracle.natural_member_record(b, 0)
    assert a.leaf_types() == b.leaf_types() and a.slots == b.slots
