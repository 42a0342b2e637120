"""GPU parity of property-tree schemas (Sec. VI: array properties holding
several properties, sub-groups and jagged vectors inside arrays, arrays and
sub-groups inside jagged vectors) against the oracle byte for byte: every
layout pair, narrowing, member pools in heap order, several jagged groups
with different offset types, transfers, compaction and a batch."""
import numpy as np
import pytest

import oracle
import paper_2511_04853_amd as P
import workloads as W
from tests import rlhelp as H
from tests.test_gpu_batch import Batch

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TREES = [W.TRACKER, W.DETECTOR]
KINDS = [("aos", 0), ("soa", 0), ("aosoa", 1), ("aosoa", 32)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


def source(sp, decl, kind, n, seed):
    v = W.tree_values(decl, n, seed=seed, mean_len=3.0)
    src = sp.layout(*kind)
    sb = oracle.pack(sp.orc, v, src.orc, pool_order=True)
    tot = H.totals(v)
    mem = ([len(sb[1 + g]) // src.orc.member_stride[g] for g in range(sp.orc.n_groups)]
           if kind[0] == "aos" else tot)
    return v, src, sb, tot, mem


@pytest.mark.parametrize("decl", TREES, ids=lambda d: d.name)
@pytest.mark.parametrize("sk", KINDS, ids=str)
@pytest.mark.parametrize("dk", KINDS, ids=str)
@pytest.mark.parametrize("n", [1, 1037, 20_000])
def test_every_pair(decl, sk, dk, n):
    if sk[0] == "aos" and dk[0] == "aos":
        pytest.skip("records to records with jagged groups is not supported")
    sp = H.SchemaPair(decl)
    v, src, sb, tot, mem = source(sp, decl, sk, n, seed=n + 3)
    storage = H.narrowed_storage(decl) if decl is W.DETECTOR and dk[0] != "aos" else None
    dst = sp.layout(*dk, storage=storage)
    st, want, wt = H.oracle_convert(src, sb, dst, n, mem, tot)
    assert st == 0 and wt == tot
    rc, rs, got = H.run_lib_convert(src, sb, dst, n, mem, tot)
    assert rc == P.RL_OK and rs == P.RL_OK, P.rl_last_error()
    H.assert_same_bytes(got, want, f"{decl.name} {sk}->{dk} n={n}")


@pytest.mark.parametrize("mode", ["staged", "zero_copy"])
def test_transfers_both_ways(mode):
    """Pinned host records with member pools -> device SoA -> pinned host
    records again (every group's pool refilled in object order)."""
    decl, n = W.TRACKER, 5000
    sp = H.SchemaPair(decl)
    v, src, sb, tot, mem = source(sp, decl, ("aos", 0), n, seed=11)
    hsrc = sp.layout("aos", space="pinned")
    dev = sp.layout("soa")
    st, want, _ = H.oracle_convert(src, sb, dev, n, mem, tot)
    assert st == 0
    hb = H.alloc_pinned([len(b) for b in sb])
    for t, b in zip(hb, sb):
        if t is not None:
            t.copy_(torch.from_numpy(b))
    dbufs = H.alloc_device(dev.lib.buffer_bytes(n, tot))
    P.transfer(P.View(hsrc.lib, n, hb, mem), P.View(dev.lib, n, dbufs, tot), n, mode=mode)
    assert P.sync() == 0, P.rl_last_error()
    torch.cuda.synchronize()
    H.assert_same_bytes(H.to_numpy(dbufs), want, f"h2d {mode}")
    st, back, _ = H.oracle_convert(dev, want, src, n, tot, tot)
    assert st == 0
    hout = H.alloc_pinned(src.lib.buffer_bytes(n, tot))
    P.transfer(P.View(dev.lib, n, dbufs, tot), P.View(hsrc.lib, n, hout, tot), n, mode=mode)
    assert P.sync() == 0, P.rl_last_error()
    torch.cuda.synchronize()
    H.assert_same_bytes(H.to_numpy(hout), back, f"d2h {mode}")


@pytest.mark.parametrize("dk", [("soa", 0), ("aosoa", 16)], ids=str)
def test_compaction_moves_every_groups_members(dk):
    decl, n = W.TRACKER, 3001
    sp = H.SchemaPair(decl)
    v, src, sb, tot, mem = source(sp, decl, ("aos", 0), n, seed=21)
    dst = sp.layout(*dk)
    keep = (np.random.default_rng(4).random(n) < 0.45).astype(np.uint8)
    st, want, count, tots = oracle.select(src.orc, sb, dst.orc, n, keep, mem)
    assert st == 0
    out = H.alloc_device(dst.lib.buffer_bytes(n, tot))
    kept = torch.zeros(1, dtype=torch.int64, device="cuda")
    P.select(P.View(src.lib, n, H.to_device(sb), mem), P.View(dst.lib, n, out, tot), n,
             torch.from_numpy(keep).cuda(), kept)
    assert P.sync() == 0, P.rl_last_error()
    assert int(kept.item()) == count
    sizes = oracle.buffer_sizes(dst.orc, count, tots)
    got = H.to_numpy(out)
    H.assert_same_bytes([g[:s] for g, s in zip(got, sizes)], [w[:s] for w, s in zip(want, sizes)],
                        f"select into {dk}")


def test_batch_of_trees():
    """Both trees in one batch launch, against the oracle."""
    items = []
    b = Batch()
    for decl, sk, dk, n in [(W.TRACKER, ("aos", 0), ("soa", 0), 4000),
                            (W.DETECTOR, ("aos", 0), ("aosoa", 64), 9000),
                            (W.TRACKER, ("soa", 0), ("aosoa", 8), 777)]:
        sp = H.SchemaPair(decl)
        v, src, sb, tot, mem = source(sp, decl, sk, n, seed=n)
        dst = sp.layout(*dk)
        st, want, _ = H.oracle_convert(src, sb, dst, n, mem, tot)
        assert st == 0
        dsrc = H.to_device(sb)
        ddst = H.alloc_device(dst.lib.buffer_bytes(n, tot))
        b.add(P.View(src.lib, n, dsrc, mem), P.View(dst.lib, n, ddst, tot), n)
        items.append((sp, src, dst, dsrc, ddst, want))
    b.finalize()
    b.launch()
    assert P.sync() == 0, P.rl_last_error()
    torch.cuda.synchronize()
    for k, (_, _, _, _, ddst, want) in enumerate(items):
        H.assert_same_bytes(H.to_numpy(ddst), want, f"batch item {k}")
