"""Batched conversion on the GPU: one graph launch over many collections
gives, item by item, the oracle's bytes; replays and the per-collection
launch loop give the same bytes."""
import ctypes
import json
import os

import numpy as np
import pytest

import oracle
import paper_2511_04853_amd as P
import workloads as W
from tests import rlhelp as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DECLS = {"plain8": W.PLAIN8, "cell": W.CELL, "cluster": W.CLUSTER}
KIND = {"aos": ("aos", 0), "soa": ("soa", 0), "aosoa": ("aosoa", 64)}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


class Batch:
    def __init__(self, autotune=0, cache=None):
        self.keep = []
        h = ctypes.c_void_p()
        opts = P.rl_batch_opts(autotune, cache.encode() if cache else None)
        P.check(P.lib().rl_batch_create(ctypes.byref(opts), ctypes.byref(h)), "rl_batch_create")
        self.h = h

    def add(self, sv, dv, n):
        self.keep += [sv, dv]
        P.check(P.lib().rl_batch_add(self.h, sv.ref(), dv.ref(), n), "rl_batch_add")

    def finalize(self):
        P.check(P.lib().rl_batch_finalize(self.h, P.stream_ptr()), "rl_batch_finalize")

    def launch(self):
        P.check(P.lib().rl_batch_launch(self.h, P.stream_ptr()), "rl_batch_launch")

    def loop(self):
        P.check(P.lib().rl_batch_launch_loop(self.h, P.stream_ptr()), "rl_batch_launch_loop")

    def width(self, k):
        w = ctypes.c_uint32()
        P.check(P.lib().rl_batch_item_width(self.h, k, ctypes.byref(w)), "rl_batch_item_width")
        return w.value

    def shape(self):
        a, b, c = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        P.check(P.lib().rl_batch_shape(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), None), "shape")
        return a.value, b.value, c.value

    def info(self):
        i = P.rl_batch_info()
        P.check(P.lib().rl_batch_get_info(self.h, ctypes.byref(i)), "rl_batch_get_info")
        return i

    def __del__(self):
        if getattr(self, "h", None):
            P.lib().rl_batch_destroy(self.h)


_VALUES = {}


def values_for(sname, n, seed):
    """Values of the first n objects of a per-schema pool of 200,000."""
    key = (sname, seed)
    if key not in _VALUES:
        if sname == "plain8":
            _VALUES[key] = W.plain_values(200_000, seed)
        elif sname == "cell":
            _VALUES[key] = W.cell_values(200_000, seed)
        else:
            _VALUES[key] = W.cluster_values(200_000, seed)
    v = _VALUES[key]
    out = W.Values(v.schema, n)
    out.fields = {k: a[:n] for k, a in v.fields.items()}
    if v.lengths:
        lens = v.lengths[0][:n]
        tot = int(lens.astype(np.int64).sum())
        out.lengths = [lens]
        out.members = {k: a[:tot] for k, a in v.members.items()}
        out.block_order = [np.random.default_rng(n).permutation(n)]
    return out


class Item:
    """One batch item: oracle-packed source on the device, sentinel-filled
    destination, and what the oracle says the destination must hold."""

    def __init__(self, schemas, spec, auto_width=False):
        sname = spec["schema"]
        decl = DECLS[sname]
        sp = schemas[sname]
        self.n = n = spec["n"]
        v = values_for(sname, n, 1003)
        self.src = sp.layout(*KIND[spec["src"]])
        narrow = H.narrowed_storage(decl) if sname == "cell" and spec["dst"] != "aos" else None
        dk = KIND[spec["dst"]]
        self.auto = auto_width and dk[0] == "aosoa"
        self.dst_kind = dk
        self.sp, self.decl, self.narrow = sp, decl, narrow
        self.dst = sp.layout(dk[0], 0 if self.auto else dk[1], storage=narrow)
        self.tot = H.totals(v)
        self.sbytes = oracle.pack(sp.orc, v, self.src.orc, pool_order=True)
        self.src_mem = ([len(self.sbytes[1]) // self.src.orc.member_stride[0]] if self.src.kind == "aos" and
                        self.tot else self.tot)
        self.dsrc = H.to_device(self.sbytes)
        self.ddst = H.alloc_device(self.dst.lib.buffer_bytes(n, self.tot))
        self.sv = P.View(self.src.lib, n, self.dsrc, self.src_mem)
        self.dv = P.View(self.dst.lib, n, self.ddst, self.tot)

    def expected(self, width):
        dst = oracle.make_layout(self.sp.orc, self.dst_kind[0], width or self.dst_kind[1],
                                 storage=self.narrow)
        st, want, _ = oracle.convert(self.src.orc, self.sbytes, dst, self.n, self.src_mem, self.tot)
        assert st == 0
        return want

    def got(self):
        """Destination bytes, trimmed to the footprint of the chosen width."""
        return H.to_numpy(self.ddst)


def _check_against_oracle(items, b):
    for k, it in enumerate(items):
        w = b.width(k)
        want = it.expected(w)
        got = it.got()
        if it.auto:
            assert w in (32, 64, 128)
            got = [got[0][:len(want[0])]] + got[1:]
        H.assert_same_bytes(got, want, f"item {k} {it.decl.name} {it.src.kind}->{it.dst_kind} w={w}")


def _small_specs(k=24, seed=77):
    rng = np.random.default_rng(seed)
    specs = []
    kinds = ["aos", "soa", "aosoa"]
    for j in range(k):
        s = ["plain8", "cell", "cluster"][j % 3]
        src = kinds[(j // 3) % 3]
        dst = [x for x in kinds if x != src][(j // 9) % 2]
        specs.append(dict(schema=s, n=int(rng.integers(1, 20_000)), src=src, dst=dst))
    specs[0]["n"] = 1
    specs[1]["n"] = 0
    return specs


def test_small_batch_matches_oracle():
    schemas = {k: H.SchemaPair(d) for k, d in DECLS.items()}
    items = [Item(schemas, s, auto_width=True) for s in _small_specs()]
    b = Batch()
    for it in items:
        b.add(it.sv, it.dv, it.n)
    b.finalize()
    b.launch()
    assert P.sync() == 0, P.rl_last_error()
    _check_against_oracle(items, b)
    # replays give the same bytes (sentinel-refilled destinations)
    for rep in range(3):
        for it in items:
            for t in it.ddst:
                if t is not None:
                    t.fill_(H.SENTINEL)
        b.launch()
        assert P.sync() == 0
        _check_against_oracle(items, b)
    # and so does the launch loop
    for it in items:
        for t in it.ddst:
            if t is not None:
                t.fill_(H.SENTINEL)
    b.loop()
    assert P.sync() == 0
    _check_against_oracle(items, b)


@pytest.mark.timeout(400)
def test_full_batch_graph_equals_loop_and_oracle():
    """512 collections, sizes log-uniform over 1k..200k, three schemas,
    mixed source and destination kinds, auto block widths."""
    schemas = {k: H.SchemaPair(d) for k, d in DECLS.items()}
    specs = W.batch_items()
    items = [Item(schemas, s, auto_width=True) for s in specs]
    b = Batch()
    for it in items:
        b.add(it.sv, it.dv, it.n)
    b.finalize()
    b.launch()
    assert P.sync() == 0, P.rl_last_error()
    first = [[None if t is None else t.clone() for t in it.ddst] for it in items]
    for it in items:
        for t in it.ddst:
            if t is not None:
                t.fill_(H.SENTINEL)
    b.loop()
    assert P.sync() == 0
    for k, it in enumerate(items):
        for a, c in zip(first[k], it.ddst):
            assert (a is None) == (c is None)
            if a is not None:
                assert torch.equal(a, c), f"item {k}: graph and loop differ"
    # every item against the oracle, one at a time (host memory)
    for k, it in enumerate(items):
        _check_against_oracle([it], _SubBatch(b, [k]))


class _SubBatch:
    def __init__(self, b, idx):
        self.b, self.idx = b, idx

    def width(self, k):
        return self.b.width(self.idx[k])


def test_autotune_writes_and_reuses_cache(tmp_path):
    cache = str(tmp_path / "tune.json")
    schemas = {k: H.SchemaPair(d) for k, d in DECLS.items()}
    specs = _small_specs(12, seed=5)
    items = [Item(schemas, s, auto_width=True) for s in specs]
    b = Batch(autotune=1, cache=cache)
    for it in items:
        b.add(it.sv, it.dv, it.n)
    b.finalize()
    shape = b.shape()
    widths = [b.width(k) for k in range(len(items))]
    b.launch()
    assert P.sync() == 0
    _check_against_oracle(items, b)
    data = json.load(open(cache))
    assert len(data) == 1
    entry = next(iter(data.values()))
    assert (entry["tile"], entry["threads"]) == shape[:2]
    # grid 0 in the cache means "as many work-groups as fit at once"; the
    # shape reports the work-groups launched (at most one per tile)
    assert shape[2] > 0 and (entry["grid"] == 0 or entry["grid"] >= shape[2])
    assert entry["gather_threads"] in (64, 128, 256)
    # a second batch of the same shape takes the cached choice
    items2 = [Item(schemas, s, auto_width=True) for s in specs]
    b2 = Batch(autotune=0, cache=cache)
    for it in items2:
        b2.add(it.sv, it.dv, it.n)
    b2.finalize()
    assert b2.shape() == shape
    assert [b2.width(k) for k in range(len(items2))] == widths
    b2.launch()
    assert P.sync() == 0
    _check_against_oracle(items2, b2)


@pytest.mark.parametrize("gather_threads", [64, 256])
def test_member_gather_work_group_sizes(gather_threads, monkeypatch):
    """The member gather of a batch at each work-group size the tuner may
    pick, against the oracle."""
    monkeypatch.setenv("RL_BATCH_GATHER_THREADS", str(gather_threads))
    schemas = {k: H.SchemaPair(d) for k, d in DECLS.items()}
    specs = _small_specs(12, seed=7)
    assert any(s["schema"] == "cluster" and s["src"] == "aos" for s in specs)   # member gathers
    items = [Item(schemas, s) for s in specs]
    b = Batch()
    for it in items:
        b.add(it.sv, it.dv, it.n)
    b.finalize()
    b.launch()
    assert P.sync() == 0
    _check_against_oracle(items, b)


class SharedSourceItem(Item):
    """Another destination for the source of an existing item (the batch
    converts one source into several layouts)."""

    def __init__(self, base, dst_kind, narrow=None, width=None):
        self.n, self.sp, self.decl = base.n, base.sp, base.decl
        self.src, self.sbytes, self.src_mem, self.tot = base.src, base.sbytes, base.src_mem, base.tot
        self.dsrc, self.sv = base.dsrc, base.sv
        self.auto = dst_kind == "aosoa" and width is None
        self.dst_kind = ("aosoa", width or 64) if dst_kind == "aosoa" else (dst_kind, 0)
        self.narrow = narrow
        self.dst = self.sp.layout(self.dst_kind[0], 0 if self.auto else self.dst_kind[1], storage=narrow)
        self.ddst = H.alloc_device(self.dst.lib.buffer_bytes(self.n, self.tot))
        self.dv = P.View(self.dst.lib, self.n, self.ddst, self.tot)


@pytest.mark.parametrize("src", ["aos", "soa", "aosoa"])
def test_one_source_into_several_layouts(src):
    """Steps reading the same source tiles are converted from one load of
    each tile: every destination must still be the oracle's."""
    schemas = {k: H.SchemaPair(d) for k, d in DECLS.items()}
    items = []
    for sname in ("plain8", "cell", "cluster"):
        base = Item(schemas, dict(schema=sname, n=30_001, src=src, dst="soa" if src != "soa" else "aos"))
        items.append(base)
        narrow = H.narrowed_storage(DECLS[sname]) if sname == "cell" else None
        for dk, w in (("soa", None), ("aosoa", None), ("aosoa", 3), ("aosoa", 128), ("aos", None)):
            if dk == src:
                continue
            items.append(SharedSourceItem(base, dk, narrow=None if dk == "aos" else narrow, width=w))
    # unrelated collections in the same batch
    items += [Item(schemas, s, auto_width=True) for s in _small_specs(6, seed=91)]
    b = Batch()
    for it in items:
        b.add(it.sv, it.dv, it.n)
    b.finalize()
    for mode in ("graph", "loop"):
        for it in items:
            for t in it.ddst:
                if t is not None:
                    t.fill_(H.SENTINEL)
        (b.launch if mode == "graph" else b.loop)()
        assert P.sync() == 0, P.rl_last_error()
        _check_against_oracle(items, b)
