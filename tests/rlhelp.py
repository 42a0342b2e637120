"""Helpers shared by the tests: build the same layout on the library side and
on the oracle side, feed both the same bytes, compare bytes."""
import numpy as np

import oracle
import paper_2511_04853_amd as P
import workloads as W

SENTINEL = 0xAB


class Pair:
    """A layout built twice: in the library and in the oracle."""

    def __init__(self, schema_pair, kind, width=0, storage=None, space="device", slot_offsets=None,
                 stride=None):
        self.sp = schema_pair
        self.kind, self.width, self.storage = kind, width, storage
        self.lib = P.Layout(schema_pair.lib, kind, space=space, width=width, storage=storage,
                            slot_offsets=slot_offsets, stride=stride or 0)
        # an AoSoA width of 0 ("auto", chosen by a batch) has no oracle layout until resolved
        self.orc = (None if kind == "aosoa" and width == 0
                    else oracle.make_layout(schema_pair.orc, kind, width=width, storage=storage,
                                            slot_offsets=slot_offsets, stride=stride))


class SchemaPair:
    def __init__(self, decl):
        self.decl = decl
        self.lib = P.Schema(decl)
        self.orc = oracle.Schema(decl)

    def layout(self, kind, width=0, storage=None, space="device", slot_offsets=None, stride=None):
        return Pair(self, kind, width, storage, space, slot_offsets, stride)


def narrowed_storage(decl):
    """Storage types with every f64 leaf kept as f32."""
    S = oracle.Schema(decl)
    return ["f32" if t == "f64" else t for t in S.leaf_types()]


def totals(v):
    return [v.total(g) for g in range(len(v.schema.offset_types))]


def to_device(bufs, device="cuda"):
    import torch
    out = []
    for b in bufs:
        if len(b) == 0:
            out.append(None)
        else:
            out.append(torch.from_numpy(np.ascontiguousarray(b)).to(device))
    return out


def alloc_device(sizes, fill=SENTINEL, device="cuda"):
    import torch
    return [None if s == 0 else torch.full((s,), fill, dtype=torch.uint8, device=device) for s in sizes]


def alloc_pinned(sizes, fill=SENTINEL):
    import torch
    out = []
    for s in sizes:
        if s == 0:
            out.append(None)
        else:
            t = torch.empty((s,), dtype=torch.uint8, pin_memory=True)
            t.fill_(fill)
            out.append(t)
    return out


def to_numpy(ts):
    return [np.zeros(0, np.uint8) if t is None else t.cpu().numpy() for t in ts]


def run_lib_convert(src_pair, src_bufs_np, dst_pair, n, src_members, dst_members, stream=None):
    """Upload src bytes, convert on the device with rl_convert, return
    (status of rl_convert, status of rl_sync, dst bytes)."""
    import torch
    dsrc = to_device(src_bufs_np)
    sizes = dst_pair.lib.buffer_bytes(n, dst_members)
    ddst = alloc_device(sizes)
    sv = P.View(src_pair.lib, n, dsrc, src_members)
    dv = P.View(dst_pair.lib, n, ddst, dst_members)
    st = P.lib().rl_convert(sv.ref(), dv.ref(), n, P.stream_ptr(stream))
    st2 = P.sync(stream)
    torch.cuda.synchronize()
    return st, st2, to_numpy(ddst)


def oracle_convert(src_pair, src_bufs_np, dst_pair, n, src_members, dst_members):
    return oracle.convert(src_pair.orc, src_bufs_np, dst_pair.orc, n, src_members, dst_members)


def assert_same_bytes(got, want, what=""):
    assert len(got) == len(want), (what, len(got), len(want))
    for k, (g, w) in enumerate(zip(got, want)):
        g = np.asarray(g).reshape(-1)
        w = np.asarray(w).reshape(-1)
        assert g.size == w.size, (what, k, g.size, w.size)
        if not np.array_equal(g, w):
            bad = np.nonzero(g != w)[0]
            raise AssertionError(f"{what}: buffer {k} differs at {bad.size} bytes, first at {bad[:8]}: "
                                 f"got {g[bad[:8]]} want {w[bad[:8]]}")
