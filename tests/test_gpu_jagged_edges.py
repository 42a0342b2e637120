"""GPU parity for jagged groups at the edges of the member gather: objects
with more members than one staging pass, long runs of empty objects, a
single huge object, all-empty collections, and the reverse direction on the
same data.  Byte for byte against the oracle."""
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


def _with_lengths(decl, lens, seed):
    """Values of `decl` (one jagged group) with the given member counts."""
    n = len(lens)
    v = W.generic_values(decl, n, seed=seed) if decl is not W.CLUSTER else W.cluster_values(n, seed=seed)
    rng = np.random.default_rng(seed + 1)
    lens = np.asarray(lens, dtype=np.uint32)
    tot = int(lens.sum())
    v.lengths[0] = lens
    for f in decl.member_fields(0):
        shape = (tot,) if f.extent == 1 else (tot, f.extent)
        if f.type == "f32":
            v.members[f.name] = (1.0 - rng.random(size=shape)).astype(np.float32)
        else:
            info = np.iinfo(W.NP_DTYPE[f.type])
            v.members[f.name] = rng.integers(0, info.max, size=shape, dtype=W.NP_DTYPE[f.type], endpoint=True)
    v.block_order[0] = rng.permutation(n)
    return v


def _roundtrip(decl, v, fwd_dst=("soa", 0)):
    sp = H.SchemaPair(decl)
    aos, dst = sp.layout("aos"), sp.layout(*fwd_dst)
    tot = v.total(0)
    src = oracle.pack(sp.orc, v, aos.orc, pool_order=True)
    pool_members = len(src[1]) // aos.orc.member_stride[0]
    st, want, _ = H.oracle_convert(aos, src, dst, v.n, [pool_members], [tot])
    assert st == 0
    rc, rs, got = H.run_lib_convert(aos, src, dst, v.n, [pool_members], [tot])
    assert rc == P.RL_OK and rs == P.RL_OK, P.rl_last_error()
    H.assert_same_bytes(got, want, f"{decl.name} aos->{fwd_dst} n={v.n} tot={tot}")
    # and back into records with a canonical pool
    st, want2, _ = H.oracle_convert(dst, want, aos, v.n, [tot], [tot])
    assert st == 0
    rc, rs, back = H.run_lib_convert(dst, want, aos, v.n, [tot], [tot])
    assert rc == P.RL_OK and rs == P.RL_OK, P.rl_last_error()
    H.assert_same_bytes(back, want2, f"{decl.name} {fwd_dst}->aos n={v.n}")


def _skewed(n, seed):
    rng = np.random.default_rng(seed)
    lens = rng.choice([0, 0, 0, 1, 2, 7, 40], size=n).astype(np.uint32)
    lens[100:700] = 0                   # a long run of empty objects
    lens[5] = 5000                      # several staging passes in one work-group
    lens[1234 % n] = 1500
    lens[n - 1] = 1025                  # one member past a pass
    return lens


@pytest.mark.parametrize("dst", [("soa", 0), ("aosoa", 32), ("aosoa", 3)], ids=str)
def test_skewed_member_counts(dst):
    _roundtrip(W.CLUSTER, _with_lengths(W.CLUSTER, _skewed(3001, 11), 11), dst)


def test_one_huge_object():
    _roundtrip(W.CLUSTER, _with_lengths(W.CLUSTER, [100_000], 12))


def test_huge_object_among_empty_ones():
    lens = np.zeros(4096, dtype=np.uint32)
    lens[2047] = 70_001
    _roundtrip(W.CLUSTER, _with_lengths(W.CLUSTER, lens, 13))


def test_all_objects_empty():
    _roundtrip(W.CLUSTER, _with_lengths(W.CLUSTER, np.zeros(5000, dtype=np.uint32), 14))


@pytest.mark.parametrize("n", [1, 16, 17, 513])
def test_member_counts_of_one(n):
    _roundtrip(W.CLUSTER, _with_lengths(W.CLUSTER, np.ones(n, dtype=np.uint32), 15 + n))


def test_skewed_generic_members_i32_offsets():
    """The particle schema: u64 members (generic member path), int offsets."""
    _roundtrip(W.PARTICLE, _with_lengths(W.PARTICLE, _skewed(2500, 21), 21))
