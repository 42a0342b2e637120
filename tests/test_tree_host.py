"""Property-tree schemas in the library (Sec. VI, nested properties) on the
host: validation of the pre-order node list, and the record layouts and
buffer sizes against the oracle's (which are pinned against numpy)."""
import ctypes

import pytest

import oracle
import paper_2511_04853_amd as P
import workloads as W

TREES = [W.TRACKER, W.DETECTOR]


def create(entries):
    arr = (P.rl_prop * max(1, len(entries)))(*entries)
    h = ctypes.c_void_p()
    st = P.lib().rl_schema_create_tree(arr, len(entries), ctypes.byref(h))
    if st == P.RL_OK:
        P.lib().rl_schema_destroy(h)
    return st


def item(t="f32"):
    return P.rl_prop(P.PROP_ITEM, b"x", P.TYPES.index(t), 1, 0)


def test_tree_validation():
    A, S, J = P.PROP_ARRAY, P.PROP_SUBGROUP, P.PROP_JAGGED
    u32 = P.TYPES.index("u32")
    assert create([item()]) == P.RL_OK
    assert create([P.rl_prop(A, b"a", 0, 3, 2), item(), item("u8")]) == P.RL_OK
    assert create([P.rl_prop(A, b"a", 0, 0, 1), item()]) == P.RL_EINVAL       # extent 0
    assert create([P.rl_prop(A, b"a", 0, 65, 1), item()]) == P.RL_EINVAL      # extent over 64
    assert create([P.rl_prop(S, b"s", 0, 1, 0)]) == P.RL_EINVAL               # empty sub-group
    assert create([P.rl_prop(S, b"s", 0, 1, 3), item(), item()]) == P.RL_EINVAL  # children past the end
    assert create([P.rl_prop(7, b"?", 0, 1, 0)]) == P.RL_EINVAL               # bad kind
    assert create([P.rl_prop(P.PROP_ITEM, b"x", 11, 1, 0)]) == P.RL_EINVAL    # bad type
    assert create([P.rl_prop(P.PROP_ITEM, b"x", 8, 1, 1), item()]) == P.RL_EINVAL  # item with children
    assert create([P.rl_prop(J, b"j", P.TYPES.index("f32"), 1, 1), item()]) == P.RL_EINVAL  # offset type
    nested = [P.rl_prop(J, b"j", u32, 1, 1), P.rl_prop(J, b"k", u32, 1, 1), item()]
    assert create(nested) == P.RL_EUNSUPPORTED                                 # jagged in jagged
    five = [P.rl_prop(A, b"a", 0, 5, 1), P.rl_prop(J, b"j", u32, 1, 1), item()]
    assert create(five) == P.RL_EINVAL                                         # 5 groups
    four = [P.rl_prop(A, b"a", 0, 4, 1), P.rl_prop(J, b"j", u32, 1, 1), item()]
    assert create(four) == P.RL_OK
    wide = [P.rl_prop(A, b"a", 0, 64, 1), item("u8"), item()]
    assert create(wide) == P.RL_EINVAL                                         # 128 leaves
    members = [P.rl_prop(J, b"j", u32, 1, 1), P.rl_prop(A, b"a", 0, 9, 1), item()]
    assert create(members) == P.RL_EINVAL                                      # 9 member leaves


@pytest.mark.parametrize("decl", TREES, ids=lambda d: d.name)
@pytest.mark.parametrize("narrow", [False, True])
def test_records_match_oracle(decl, narrow):
    S = oracle.Schema(decl)
    storage = [("f32" if narrow and t == "f64" else t) for t in S.leaf_types()]
    lay = P.Layout(P.Schema(decl), "aos", storage=storage)
    offs, stride = oracle.natural_record(S, storage)
    assert lay.stride == stride and lay.slot_offsets == offs


@pytest.mark.parametrize("decl", TREES, ids=lambda d: d.name)
@pytest.mark.parametrize("kind,width", [("aos", 0), ("soa", 0), ("aosoa", 8)])
def test_buffer_sizes_match_oracle(decl, kind, width):
    S = oracle.Schema(decl)
    lib = P.Layout(P.Schema(decl), kind, width=width)
    orc = oracle.make_layout(S, kind, width=width)
    members = [5 + 3 * g for g in range(S.n_groups)]
    for n in (0, 1, 77):
        assert lib.buffer_bytes(n, members) == oracle.buffer_sizes(orc, n, members)
