"""The C ABI on the host: the library loads, exports every declared symbol,
and its host logic (schema flattening, record layouts, buffer sizes,
argument validation) agrees with the oracle and the header.  No kernel is
launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2511_04853_amd as P
import workloads as W
from tests.rlhelp import SchemaPair

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "relayout.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"typedef[^;]*;", "", text, flags=re.S)   # types, including function pointer types
    return sorted(set(re.findall(r"\b(rl_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    syms = declared_symbols()
    assert len(syms) >= 20
    L = ctypes.CDLL(P.LIB_PATH)
    missing = [s for s in syms if not hasattr(L, s)]
    assert not missing, missing
    # and the binding knows every one of them
    assert sorted(P.SIGNATURES) == syms


@pytest.mark.parametrize("decl", [W.PLAIN8, W.CELL, W.CLUSTER, W.SENSOR, W.PARTICLE],
                         ids=lambda d: d.name)
def test_record_layout_matches_oracle(decl):
    sp = SchemaPair(decl)
    assert sp.lib.n_leaves == len(sp.orc.leaves)
    assert sp.lib.n_slots == len(sp.orc.slots)
    lay = P.Layout(sp.lib, "aos")
    offs, stride = oracle.natural_record(sp.orc)
    assert lay.slot_offsets == offs and lay.stride == stride


@pytest.mark.parametrize("decl", [W.PLAIN8, W.CELL, W.CLUSTER, W.PARTICLE], ids=lambda d: d.name)
@pytest.mark.parametrize("kind,width", [("aos", 0), ("soa", 0), ("aosoa", 1), ("aosoa", 3), ("aosoa", 64)])
@pytest.mark.parametrize("n", [0, 1, 17, 1000])
def test_buffer_sizes_match_oracle(decl, kind, width, n):
    sp = SchemaPair(decl)
    mem = [5 * n + 3 for _ in decl.offset_types]
    lay = sp.layout(kind, width)
    assert lay.lib.buffer_bytes(n, mem) == oracle.buffer_sizes(lay.orc, n, mem)


def test_narrowed_storage_sizes():
    sp = SchemaPair(W.CELL)
    st = ["f32", "f32", "i8", "u16", "u32", "u32", "f32"]
    soa = sp.layout("soa", storage=st)
    assert soa.lib.buffer_bytes(190_000) == [4 * 190_000] * 2 + [190_000, 2 * 190_000] + [4 * 190_000] * 3
    blk = sp.layout("aosoa", width=32, storage=st)
    assert blk.lib.buffer_bytes(190_000) == [5938 * 32 * 23]


def _schema(fields, groups=()):
    arr = (P.rl_field * max(1, len(fields)))(*[P.rl_field(None, *f) for f in fields])
    g = (P.rl_jagged * max(1, len(groups)))(*[P.rl_jagged(t) for t in groups])
    h = ctypes.c_void_p()
    st = P.lib().rl_schema_create(arr, len(fields), g, len(groups), ctypes.byref(h))
    if st == 0:
        P.lib().rl_schema_destroy(h)
    return st


def test_schema_validation():
    U32, F64 = 4, 9
    assert _schema([(U32, 1, -1, -1)]) == P.RL_OK
    assert _schema([(42, 1, -1, -1)]) == P.RL_EINVAL              # bad type
    assert _schema([(U32, 0, -1, -1)]) == P.RL_EINVAL              # extent 0
    assert _schema([(U32, 1, 0, -1)]) == P.RL_EINVAL               # group without declaration
    assert _schema([(U32, 1, 0, -1)], [U32]) == P.RL_OK
    assert _schema([(U32, 1, -1, -1)], [U32]) == P.RL_EINVAL       # group with no member
    assert _schema([(U32, 1, 0, -1)], [F64]) == P.RL_EINVAL        # bad offset type
    assert _schema([(U32, 1, 0, 0)], [U32]) == P.RL_EINVAL         # member inside a sub-group
    # sub-group ids must label consecutive runs
    assert _schema([(U32, 1, -1, 0), (U32, 1, -1, -1), (U32, 1, -1, 0)]) == P.RL_EINVAL
    assert _schema([(U32, 1, -1, 0), (U32, 1, -1, 0), (U32, 1, -1, 1)]) == P.RL_OK
    assert _schema([(U32, 65, -1, -1)]) == P.RL_EINVAL             # extent limit
    assert _schema([(U32, 33, -1, -1), (U32, 32, -1, -1)]) == P.RL_EINVAL  # leaf limit


def test_layout_validation():
    sp = SchemaPair(W.CELL)
    with pytest.raises(P.RelayoutError) as e:
        P.Layout(sp.lib, "aosoa", width=70_000)
    assert e.value.status == P.RL_EINVAL
    with pytest.raises(P.RelayoutError):
        P.Layout(sp.lib, "soa", storage=["f32", "f32", "i8", "u16", "u32", "u32", "u64"])
    # explicit record: overlapping slots
    with pytest.raises(P.RelayoutError):
        P.Layout(sp.lib, "aos", slot_offsets=[0, 2, 8, 10, 12, 16, 24], stride=32)
    # explicit record: slot beyond stride
    with pytest.raises(P.RelayoutError):
        P.Layout(sp.lib, "aos", slot_offsets=[0, 4, 8, 10, 12, 16, 24], stride=30)
    # a packed record is fine
    lay = P.Layout(sp.lib, "aos", slot_offsets=[0, 4, 8, 9, 11, 15, 19], stride=27)
    assert lay.stride == 27 and lay.slot_offsets == [0, 4, 8, 9, 11, 15, 19]


def _fake_view(pair, n, base, members=(), step=1 << 24):
    """A view over fake (never dereferenced) addresses."""
    sizes = pair.lib.buffer_bytes(n, members)
    ptrs = [base + k * step for k in range(len(sizes))]
    return P.View(pair.lib, n, ptrs, members)


def test_convert_validation_on_the_host():
    # every check below fails before any device work, so it runs without a GPU
    sp = SchemaPair(W.PLAIN8)
    aos, soa = sp.layout("aos"), sp.layout("soa")
    src = _fake_view(aos, 100, 1 << 40)
    dst = _fake_view(soa, 100, 1 << 41)
    rc = P.lib().rl_convert
    s0 = ctypes.c_void_p(0)
    assert rc(src.ref(), dst.ref(), 101, s0) == P.RL_EINVAL            # n over capacity
    assert rc(src.ref(), dst.ref(), 0, s0) == P.RL_OK                  # nothing to do
    over = _fake_view(soa, 100, (1 << 40) + 64)                         # inside the source records
    assert rc(src.ref(), over.ref(), 10, s0) == P.RL_EOVERLAP
    mis = _fake_view(soa, 100, (1 << 41) + 2)                           # f32 column at +2
    assert rc(src.ref(), mis.ref(), 10, s0) == P.RL_EALIGN
    other = SchemaPair(W.PLAIN8)
    odst = _fake_view(other.layout("soa"), 100, 1 << 41)
    assert rc(src.ref(), odst.ref(), 10, s0) == P.RL_EINVAL            # different schema objects
    hsrc = _fake_view(sp.layout("aos", space="pinned"), 100, 1 << 40)
    assert rc(hsrc.ref(), dst.ref(), 10, s0) == P.RL_EUNSUPPORTED      # host view in rl_convert
    null = P.View(soa.lib, 100, [None] * 8)
    assert rc(src.ref(), null.ref(), 10, s0) == P.RL_EINVAL
    assert "NULL" in P.rl_last_error()


def test_transfer_validation_on_the_host():
    sp = SchemaPair(W.CELL)
    dev = _fake_view(sp.layout("soa"), 100, 1 << 41)
    dev2 = _fake_view(sp.layout("aos"), 100, 1 << 40)
    s0 = ctypes.c_void_p(0)
    # two device views: use rl_convert
    assert P.lib().rl_transfer(dev2.ref(), dev.ref(), 10, s0, None) == P.RL_EUNSUPPORTED
    host = _fake_view(sp.layout("aos", space="host"), 100, 1 << 40)
    o = P.rl_xfer_opts(2)          # zero-copy from pageable memory
    assert P.lib().rl_transfer(host.ref(), dev.ref(), 10, s0, ctypes.byref(o)) == P.RL_EUNSUPPORTED
    o = P.rl_xfer_opts(7)          # no such mode
    assert P.lib().rl_transfer(host.ref(), dev.ref(), 10, s0, ctypes.byref(o)) == P.RL_EINVAL


def test_jagged_aos_to_aos_is_unsupported():
    sp = SchemaPair(W.CLUSTER)
    a = _fake_view(sp.layout("aos"), 10, 1 << 40, [100])
    b = _fake_view(sp.layout("aos"), 10, 1 << 42, [100])
    assert P.lib().rl_convert(a.ref(), b.ref(), 0, ctypes.c_void_p(0)) == P.RL_EUNSUPPORTED


def test_batch_validation_on_the_host():
    sp = SchemaPair(W.CELL)
    h = ctypes.c_void_p()
    assert P.lib().rl_batch_create(None, ctypes.byref(h)) == P.RL_OK
    a = _fake_view(sp.layout("aos"), 100, 1 << 40)
    s = _fake_view(sp.layout("soa"), 100, 1 << 42)
    auto = _fake_view(sp.layout("aosoa", width=0), 100, 1 << 43)
    assert P.lib().rl_batch_add(h, a.ref(), s.ref(), 101) == P.RL_EINVAL        # over capacity
    assert P.lib().rl_batch_add(h, auto.ref(), s.ref(), 10) == P.RL_EINVAL      # auto width as source
    over = _fake_view(sp.layout("soa"), 100, (1 << 40) + 256)
    assert P.lib().rl_batch_add(h, a.ref(), over.ref(), 10) == P.RL_EOVERLAP
    assert P.lib().rl_batch_add(h, a.ref(), auto.ref(), 10) == P.RL_OK          # auto width as destination
    w = ctypes.c_uint32()
    assert P.lib().rl_batch_item_width(h, 0, ctypes.byref(w)) == P.RL_EINVAL    # not finalized
    assert P.lib().rl_batch_launch(h, ctypes.c_void_p(0)) == P.RL_EINVAL
    info = P.rl_batch_info()
    assert P.lib().rl_batch_get_info(h, ctypes.byref(info)) == P.RL_EINVAL     # not finalized
    assert P.lib().rl_batch_get_info(h, None) == P.RL_EINVAL
    assert P.lib().rl_batch_get_info(None, ctypes.byref(info)) == P.RL_EINVAL
    P.lib().rl_batch_destroy(h)


def test_batch_info_struct_matches_header():
    """rl_batch_info is eight 32-bit words in the header's order."""
    assert ctypes.sizeof(P.rl_batch_info) == 32
    names = [f[0] for f in P.rl_batch_info._fields_]
    assert names == ["double_buffered", "fanout_threads", "fanout_groups", "fanout_steps", "dense_steps",
                     "stream_stores", "reserved"]
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "relayout.h")).read()
    body = hdr[hdr.index("typedef struct rl_batch_info {"):hdr.index("} rl_batch_info;")]
    assert [n for n in names[:-1] if n in body] == names[:-1]
    assert body.index("double_buffered") < body.index("fanout_threads") < body.index("stream_stores") < body.index("reserved[2]")


def test_auto_width_layout_is_batch_only():
    sp = SchemaPair(W.CELL)
    auto = sp.layout("aosoa", width=0)
    # buffers are sized for the widest candidate (128)
    assert auto.lib.buffer_bytes(1000) == [8 * 128 * 27]
    a = _fake_view(sp.layout("aos"), 100, 1 << 40)
    d = _fake_view(auto, 100, 1 << 42)
    assert P.lib().rl_convert(a.ref(), d.ref(), 10, ctypes.c_void_p(0)) == P.RL_EINVAL


def test_noalloc_limit_matches_header():
    text = open(HEADER).read()
    m = re.search(r"#define\s+RL_TRANSFER_NOALLOC_LIMIT\s+\((\d+)ull\s*<<\s*(\d+)\)", text)
    assert m, "RL_TRANSFER_NOALLOC_LIMIT not found"
    assert int(m.group(1)) << int(m.group(2)) == P.TRANSFER_NOALLOC_LIMIT
    src = open(os.path.join(ROOT, "paper_2511_04853_amd", "csrc", "transfer.cpp")).read()
    # the staging array is a fixed device array, reached only through hipGetSymbolAddress
    assert re.search(r"__device__\s+__align__\(256\)\s+uint8_t\s+scratch\[", src)
    assert "hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))" in src
