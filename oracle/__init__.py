"""CPU oracle for schema-driven layout conversion.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline of the benchmark may import this package; the library never does and
shares no code with it.

What it computes (the plain definition, Sec. VI and VII-B of the paper):

* A schema is a list of properties.  Per-item properties give one value per
  object; an array property of extent E gives E values, kept as E separate
  leaf columns; a sub-group's members are flattened into leaves in
  declaration order; a jagged vector property gives each object a list of
  members, whose sizes are kept as a prefix sum of a stated offset type.
* A layout says where every leaf value of every object lives:
    - ``aos``:   record i at ``i * stride``, leaf c at a fixed byte offset in
                 the record; each jagged group has a (u64 byte pointer into a
                 member pool, u32 count) pair in the record;
    - ``soa``:   one column per leaf; jagged groups as an offsets column of
                 n + 1 entries plus one column per member leaf;
    - ``aosoa``: blocks of W objects; inside a block each leaf is a run of W
                 values, runs in leaf order; jagged groups as in ``soa``.
* A conversion moves every value of objects 0..n-1 from the source address to
  the destination address (copy; or double -> float rounding to nearest
  even; or float -> double), into a zero-filled destination.

The default record layout is C's natural alignment: a scalar sits at a
multiple of its size, an array at a multiple of its element size, a
sub-group is a nested struct aligned to its largest member, and the record
stride is rounded up to the largest alignment.

Pins (see tests/test_oracle_*.py): numpy structured dtypes for record
layouts, transposes for same-width schemas, special block widths (W = 1 is a
packed record, W = n is back-to-back columns), round trips, cumsum for
offsets, an independent bit-level rounding for narrowing, brute force on tiny
inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from workloads import NP_DTYPE, TYPE_CODES, TYPE_SIZE, SchemaDecl, Values

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ST_OK, ST_ALIGN, ST_CAPACITY, ST_OVERFLOW, ST_UNSUPPORTED, ST_BOUNDS = 0, 2, 4, 5, 8, 11
KIND = {"aos": 0, "soa": 1, "aosoa": 2}


def build() -> str:
    """Compile the C part of the oracle (plain -O2, IEEE semantics)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-shared", "-fPIC",
           "-o", _LIB + ".tmp", _SRC]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if (not os.path.exists(_LIB)
                or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        _lib = ctypes.CDLL(_LIB)
        _lib.or_convert_objects.restype = ctypes.c_int
        _lib.or_convert_objects_range.restype = ctypes.c_int
        _lib.or_gather_objects.restype = ctypes.c_int
        _lib.or_gather_group.restype = ctypes.c_int
        _lib.or_convert_group.restype = ctypes.c_int
        _lib.or_exclusive_scan.restype = ctypes.c_int
        _lib.or_rounding_is_nearest.restype = ctypes.c_int
    return _lib


# ---------------------------------------------------------------- ctypes structs

class _Objects(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("stride", ctypes.c_uint64),
                ("width", ctypes.c_uint64), ("obj_bytes", ctypes.c_uint64),
                ("offset", ctypes.POINTER(ctypes.c_uint64)),
                ("type", ctypes.POINTER(ctypes.c_int32)),
                ("base", ctypes.POINTER(ctypes.c_void_p)),
                ("index", ctypes.POINTER(ctypes.c_uint64)),
                ("elements", ctypes.c_uint64)]


class _Group(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("n_members", ctypes.c_uint32),
                ("type", ctypes.POINTER(ctypes.c_int32)),
                ("capacity", ctypes.c_uint64),
                ("records", ctypes.c_void_p), ("rec_stride", ctypes.c_uint64),
                ("ptr_off", ctypes.c_uint64), ("len_off", ctypes.c_uint64),
                ("pool", ctypes.c_void_p), ("mstride", ctypes.c_uint64),
                ("malign", ctypes.c_uint64),
                ("moff", ctypes.POINTER(ctypes.c_uint64)),
                ("offsets", ctypes.c_void_p), ("off_type", ctypes.c_int32),
                ("mcol", ctypes.POINTER(ctypes.c_void_p))]


def _u64s(xs):
    return (ctypes.c_uint64 * max(1, len(xs)))(*xs)


def _i32s(xs):
    return (ctypes.c_int32 * max(1, len(xs)))(*xs)


def _ptrs(arrs):
    return (ctypes.c_void_p * max(1, len(arrs)))(*[a.ctypes.data for a in arrs])


# ---------------------------------------------------------------- schema

class Schema:
    """Flattened view of a schema declaration.

    ``leaves``: per-object leaf values in order, as (field, element) pairs.
    ``members[g]``: member leaves of jagged group g, as (field, element).
    ``slots``: the entries of an object record, in order: ('leaf', k) for
    leaf k, ('ptr', g) and ('len', g) for jagged group g, placed where the
    group's first field is declared.
    """

    def __init__(self, decl):
        self.decl = decl
        self.tree = None
        if hasattr(decl, "props"):
            self._from_tree(decl)
            return
        self.offset_types = list(decl.offset_types)
        self.leaves, self.slots = [], []
        self.members = [[] for _ in decl.offset_types]
        seen_groups = set()
        for f in decl.fields:
            if f.group < 0:
                for e in range(f.extent):
                    self.slots.append(("leaf", len(self.leaves)))
                    self.leaves.append((f, e))
            else:
                if f.group not in seen_groups:
                    seen_groups.add(f.group)
                    self.slots.append(("ptr", f.group))
                    self.slots.append(("len", f.group))
                for e in range(f.extent):
                    self.members[f.group].append((f, e))
        self.n_groups = len(decl.offset_types)

    def _from_tree(self, decl):
        """A property tree (Sec. VI: array properties holding a list of
        properties, sub-groups and jagged vectors nested in them): walked in
        pre-order, each array element in turn.  An item outside a jagged
        vector is a per-object leaf and a record slot; each jagged vector
        reached (one per element of an array holding it) is the next group,
        its (ptr, len) slots where it is reached, its items the group's
        member leaves.  Leaves are named by path (names joined by '.', an
        element as '[e]')."""
        self.tree = decl.props
        self.leaves, self.slots, self.members, self.offset_types = [], [], [], []

        def visit(p, path, group):
            name = f"{path}.{p.name}" if path else p.name
            kind = type(p).__name__
            if kind == "Item":
                ref = _PathLeaf(name, p.type)
                if group is None:
                    self.slots.append(("leaf", len(self.leaves)))
                    self.leaves.append((ref, 0))
                else:
                    self.members[group].append((ref, 0))
            elif kind == "Array":
                for e in range(p.extent):
                    for c in p.props:
                        visit(c, f"{name}[{e}]", group)
            elif kind == "SubGroup":
                for c in p.props:
                    visit(c, name, group)
            else:
                assert group is None, "a jagged vector inside another"
                g = len(self.members)
                self.members.append([])
                self.offset_types.append(p.offset_type)
                self.slots += [("ptr", g), ("len", g)]
                for c in p.props:
                    visit(c, name, g)

        for p in decl.props:
            visit(p, "", None)
        self.n_groups = len(self.members)

    def leaf_types(self):
        return [f.type for f, _ in self.leaves]

    def member_types(self, g):
        return [f.type for f, _ in self.members[g]]

    def slot_type(self, slot):
        k, idx = slot
        if k == "leaf":
            return self.leaves[idx][0].type
        return "u64" if k == "ptr" else "u32"


@dataclass(frozen=True)
class _PathLeaf:
    """A leaf of a property tree: its path, its type, one value per object."""
    name: str
    type: str
    extent: int = 1


def _round_up(x, a):
    return (x + a - 1) // a * a


def _tree_struct(props, sizes):
    """C layout of a struct whose members are `props` (Sec. VI property
    kinds): an item is a scalar member; a sub-group a nested struct; an
    array `extent` nested structs, one per element, each made of the
    element's properties; a jagged vector two members, u64 ptr and u32 len.
    `sizes` yields the byte size of each item (and 8, 4 for each ptr, len)
    in walk order.  Returns (offsets in walk order, size, alignment):
    members aligned to their own alignment, the size rounded up to the
    largest."""
    offs, pos, align = [], 0, 1

    def place(o_rel, size, al):
        nonlocal pos, align
        pos = _round_up(pos, al)
        offs.extend(pos + o for o in o_rel)
        pos += size
        align = max(align, al)

    for p in props:
        kind = type(p).__name__
        if kind == "Item":
            sz = next(sizes)
            place([0], sz, sz)
        elif kind == "Jagged":
            place([0], next(sizes), 8)
            place([0], next(sizes), 4)
        elif kind == "SubGroup":
            place(*_tree_struct(p.props, sizes))
        else:
            for _ in range(p.extent):
                place(*_tree_struct(p.props, sizes))
    return offs, (_round_up(pos, align) if pos else 0), align


def _group_props(schema, g):
    """The property of jagged group g (the g-th reached by the walk)."""
    found = []

    def visit(p):
        kind = type(p).__name__
        if kind == "Jagged":
            found.append(p)
        elif kind != "Item":
            for _ in range(getattr(p, "extent", 1)):
                for c in p.props:
                    visit(c)

    for p in schema.tree:
        visit(p)
    return found[g]


def natural_record(schema: Schema, leaf_types=None):
    """C natural-alignment offsets of every record slot and the stride.

    Sub-groups (runs of fields sharing a subgroup id) are nested structs:
    members are placed from offset 0 of the nested struct, whose size is
    rounded up to, and whose start aligned to, its largest member alignment.
    """
    types = leaf_types or schema.leaf_types()

    def slot_size(slot):
        k, idx = slot
        if k == "leaf":
            return TYPE_SIZE[types[idx]]
        return 8 if k == "ptr" else 4

    if schema.tree is not None:
        offs, stride, _ = _tree_struct(schema.tree, iter([slot_size(sl) for sl in schema.slots]))
        return offs, stride

    # the sub-group id of each record slot (ptr/len pairs are top level)
    sub_of_slot = []
    seen = set()
    for f in schema.decl.fields:
        if f.group < 0:
            sub_of_slot += [f.subgroup] * f.extent
        elif f.group not in seen:
            seen.add(f.group)
            sub_of_slot += [-1, -1]
    # consecutive slots of one sub-group form a nested struct item
    items = []   # (is_nested, [slots])
    prev = -1
    for slot, sub in zip(schema.slots, sub_of_slot):
        if sub >= 0 and sub == prev:
            items[-1][1].append(slot)
        else:
            items.append((sub >= 0, [slot]))
        prev = sub
    offsets = {}
    pos, max_align = 0, 1
    for nested, it in items:
        if not nested:
            s = slot_size(it[0])
            pos = _round_up(pos, s)
            offsets[it[0]] = pos
            pos += s
            max_align = max(max_align, s)
        else:
            inner, ia = 0, 1
            local = {}
            for sl in it:
                s = slot_size(sl)
                inner = _round_up(inner, s)
                local[sl] = inner
                inner += s
                ia = max(ia, s)
            inner = _round_up(inner, ia)
            pos = _round_up(pos, ia)
            for sl, o in local.items():
                offsets[sl] = pos + o
            pos += inner
            max_align = max(max_align, ia)
    stride = _round_up(pos, max_align) if pos else 0
    return [offsets[s] for s in schema.slots], stride


def natural_member_record(schema: Schema, g: int, member_types=None):
    types = member_types or schema.member_types(g)
    if schema.tree is not None:
        return _tree_struct(_group_props(schema, g).props, iter([TYPE_SIZE[t] for t in types]))
    pos, ma, offs = 0, 1, []
    for t in types:
        s = TYPE_SIZE[t]
        pos = _round_up(pos, s)
        offs.append(pos)
        pos += s
        ma = max(ma, s)
    return offs, _round_up(pos, ma), ma


# ---------------------------------------------------------------- layout

@dataclass
class Layout:
    schema: Schema
    kind: str
    width: int = 0                 # aosoa block width
    storage: list = None           # per-object leaf storage types
    member_storage: list = None    # per group: member leaf storage types
    slot_offsets: list = None      # aos: per record slot
    stride: int = 0                # aos: record stride
    member_offsets: list = None    # aos: per group, offsets in member record
    member_stride: list = None     # aos: per group
    member_align: list = None      # aos: per group
    leaf_strides: list = None      # strided: bytes between elements, per leaf
    indexed: bool = False          # strided: objects reach elements through an index table


def make_layout(schema: Schema, kind: str, width: int = 0, storage=None,
                slot_offsets=None, stride=None, member_storage=None,
                leaf_strides=None, indexed=False) -> Layout:
    """kind: "aos", "soa", "aosoa" or "strided" (Sec. VII-B: a layout whose
    arrays map an object index to a value anywhere: leaf c of object i at
    byte e * leaf_strides[c] of buffer c, e = i, or e = index[i] from an
    index table, the buffer after the leaves, when indexed).  Strided
    layouts hold per-object leaves only."""
    storage = list(storage) if storage is not None else schema.leaf_types()
    mstor = (list(member_storage) if member_storage is not None
             else [schema.member_types(g) for g in range(schema.n_groups)])
    L = Layout(schema, kind, width, storage, mstor)
    if kind == "aos":
        nat_off, nat_stride = natural_record(schema, storage)
        L.slot_offsets = list(slot_offsets) if slot_offsets is not None else nat_off
        L.stride = stride if stride is not None else nat_stride
        L.member_offsets, L.member_stride, L.member_align = [], [], []
        for g in range(schema.n_groups):
            mo, ms, ma = natural_member_record(schema, g, mstor[g])
            L.member_offsets.append(mo)
            L.member_stride.append(ms)
            L.member_align.append(ma)
    elif kind == "aosoa":
        assert width >= 1
    elif kind == "strided":
        assert schema.n_groups == 0, "strided layouts hold per-object leaves only"
        L.leaf_strides = (list(leaf_strides) if leaf_strides is not None
                          else [TYPE_SIZE[t] for t in storage])
        L.indexed = bool(indexed)
    return L


def obj_bytes(L: Layout) -> int:
    return sum(TYPE_SIZE[t] for t in L.storage)


def leaf_prefix(L: Layout):
    pre, acc = [], 0
    for t in L.storage:
        pre.append(acc)
        acc += TYPE_SIZE[t]
    return pre


def buffer_sizes(L: Layout, n: int, members=()):
    """Byte sizes of the layout's buffers holding n objects and members[g]
    members per group, in the buffer order of the layout:
    aos: records, then a pool per group; soa: one column per leaf, then per
    group the offsets column and one column per member leaf; aosoa: the
    blocks, then per group as soa; strided: one buffer per leaf reaching n
    elements (the last element's end), then the index table (n entries)
    when indexed."""
    S = L.schema
    out = []
    if L.kind == "strided":
        out += [(n - 1) * st + TYPE_SIZE[t] if n else 0
                for st, t in zip(L.leaf_strides, L.storage)]
        if L.indexed:
            out.append(8 * n)
        return out
    if L.kind == "aos":
        out.append(n * L.stride)
        for g in range(S.n_groups):
            out.append(members[g] * L.member_stride[g])
        return out
    if L.kind == "soa":
        out += [n * TYPE_SIZE[t] for t in L.storage]
    else:
        nblk = -(-n // L.width)
        out.append(nblk * L.width * obj_bytes(L))
    for g in range(S.n_groups):
        out.append((n + 1) * TYPE_SIZE[S.offset_types[g]])
        out += [members[g] * TYPE_SIZE[t] for t in L.member_storage[g]]
    return out


def zeros_like_layout(L: Layout, n: int, members=()):
    return [np.zeros(s, dtype=np.uint8) for s in buffer_sizes(L, n, members)]


def _objects_struct(L: Layout, bufs, keep, elements=0):
    """The C description of a layout's per-object leaves.  ``elements``:
    for an indexed strided layout, the elements each leaf holds."""
    S = L.schema
    types = [TYPE_CODES.index(t) for t in L.storage]
    if L.kind == "strided":
        nl = len(S.leaves)
        o = _Objects(3, 0, 0, 0, _u64s(L.leaf_strides), _i32s(types), _ptrs(bufs[:nl]))
        if L.indexed:
            idx = bufs[nl].view(np.uint64)
            keep.append(idx)
            o.index = idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
            if not elements:   # the whole elements every leaf buffer holds
                elements = min(((len(b) - TYPE_SIZE[t]) // st + 1 if len(b) >= TYPE_SIZE[t] else 0)
                               for b, st, t in zip(bufs[:nl], L.leaf_strides, L.storage))
            o.elements = elements
    elif L.kind == "aos":
        offs = [L.slot_offsets[S.slots.index(("leaf", k))] for k in range(len(S.leaves))]
        base = [bufs[0]]
        o = _Objects(0, L.stride, 0, 0, _u64s(offs), _i32s(types), _ptrs(base))
    elif L.kind == "soa":
        base = bufs[:len(S.leaves)]
        o = _Objects(1, 0, 0, 0, _u64s([0] * len(types)), _i32s(types), _ptrs(base))
    else:
        o = _Objects(2, 0, L.width, obj_bytes(L), _u64s(leaf_prefix(L)),
                     _i32s(types), _ptrs([bufs[0]]))
    keep.append(o)
    return o


def _group_buffers(L: Layout, g: int, bufs):
    """(first buffer index of group g's storage) in the layout's buffer list."""
    S = L.schema
    if L.kind == "aos":
        return 1 + g
    idx = len(S.leaves) if L.kind == "soa" else 1
    for h in range(g):
        idx += 1 + len(S.members[h])
    return idx


def _group_struct(L: Layout, g: int, bufs, capacity: int, keep):
    S = L.schema
    types = [TYPE_CODES.index(t) for t in L.member_storage[g]]
    gs = _Group()
    gs.n_members = len(types)
    gs.type = _i32s(types)
    gs.capacity = capacity
    keep.append(gs.type)
    i0 = _group_buffers(L, g, bufs)
    if L.kind == "aos":
        gs.form = 0
        gs.records = bufs[0].ctypes.data
        gs.rec_stride = L.stride
        gs.ptr_off = L.slot_offsets[S.slots.index(("ptr", g))]
        gs.len_off = L.slot_offsets[S.slots.index(("len", g))]
        gs.pool = bufs[i0].ctypes.data
        gs.mstride = L.member_stride[g]
        gs.malign = L.member_align[g]
        gs.moff = _u64s(L.member_offsets[g])
        keep.append(gs.moff)
    else:
        gs.form = 1
        gs.offsets = bufs[i0].ctypes.data
        gs.off_type = TYPE_CODES.index(S.offset_types[g])
        gs.mcol = _ptrs(bufs[i0 + 1: i0 + 1 + len(types)])
        keep.append(gs.mcol)
    keep.append(gs)
    return gs


def convert(src: Layout, src_bufs, dst: Layout, n: int, src_members=(),
            dst_members=None, dst_capacity=None):
    """Convert objects 0..n-1 from src_bufs (layout src) into freshly
    zero-filled buffers of layout dst.  ``src_members[g]`` is the member
    capacity of the source group g (pool records or member column length);
    ``dst_members[g]`` the destination's (default: the group total), which
    sizes the destination buffers; ``dst_capacity`` (default dst_members) is
    the capacity the conversion is told about.
    Returns (status, dst_bufs, totals)."""
    lib = _load()
    S = src.schema
    assert dst.schema is S or dst.schema.decl == S.decl
    src_bufs = [np.ascontiguousarray(b).view(np.uint8).reshape(-1) for b in src_bufs]
    totals = []
    if dst_members is None:
        dst_members = [_count_members(src, src_bufs, g, n) for g in range(S.n_groups)]
    dst_bufs = zeros_like_layout(dst, n, dst_members)
    keep = []
    so = _objects_struct(src, src_bufs, keep)
    do = _objects_struct(dst, dst_bufs, keep)
    st = lib.or_convert_objects(ctypes.byref(so), ctypes.byref(do),
                                ctypes.c_uint32(len(S.leaves)), ctypes.c_uint64(n))
    if st != ST_OK:
        return st, dst_bufs, totals
    for g in range(S.n_groups):
        sg = _group_struct(src, g, src_bufs, src_members[g], keep)
        cap = dst_members[g] if dst_capacity is None else dst_capacity[g]
        dg = _group_struct(dst, g, dst_bufs, cap, keep)
        tot = ctypes.c_uint64(0)
        st = lib.or_convert_group(ctypes.byref(sg), ctypes.byref(dg), ctypes.c_uint64(n),
                                  ctypes.byref(tot))
        totals.append(tot.value)
        if st != ST_OK:
            return st, dst_bufs, totals
    return ST_OK, dst_bufs, totals


def convert_into(src: Layout, src_bufs, dst: Layout, dst_bufs, n: int, src_elements=0,
                 dst_elements=0):
    """Per-object leaves of objects 0..n-1 from src_bufs into dst_bufs
    (numpy uint8 arrays, modified in place; what the conversion does not
    address is left as it is).  ``*_elements``: the elements each leaf of an
    indexed strided side holds.  For schemas without jagged groups.
    Returns the status."""
    lib = _load()
    S = src.schema
    assert S.n_groups == 0
    src_bufs = [np.ascontiguousarray(b).view(np.uint8).reshape(-1) for b in src_bufs]
    keep = []
    so = _objects_struct(src, src_bufs, keep, src_elements)
    do = _objects_struct(dst, dst_bufs, keep, dst_elements)
    return lib.or_convert_objects(ctypes.byref(so), ctypes.byref(do),
                                  ctypes.c_uint32(len(S.leaves)), ctypes.c_uint64(n))


def gather_into(src: Layout, src_bufs, dst: Layout, dst_bufs, idx, k0=0, base=(), src_members=(),
                dst_capacity=(), src_elements=0, dst_elements=0):
    """Gather (the plain definition behind insertion, deletion and
    compaction, Sec. VII-B): destination object k0 + k takes every value of
    source object idx[k]; per jagged group g the members of the gathered
    objects are placed one object after the other from destination member
    base[g] on.  dst_bufs (numpy uint8 arrays of the destination layout) are
    modified in place.  Returns (status, ends) with ends[g] the member index
    after the last one placed."""
    lib = _load()
    S = src.schema
    src_bufs = [np.ascontiguousarray(b).view(np.uint8).reshape(-1) for b in src_bufs]
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
    m = len(idx)
    keep = [idx]
    so = _objects_struct(src, src_bufs, keep, src_elements)
    do = _objects_struct(dst, dst_bufs, keep, dst_elements)
    ip = idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    st = lib.or_gather_objects(ctypes.byref(so), ctypes.byref(do), ctypes.c_uint32(len(S.leaves)), ip,
                               ctypes.c_uint64(m), ctypes.c_uint64(k0))
    ends = []
    if st != ST_OK:
        return st, ends
    for g in range(S.n_groups):
        sg = _group_struct(src, g, src_bufs, src_members[g], keep)
        dg = _group_struct(dst, g, dst_bufs, dst_capacity[g], keep)
        end = ctypes.c_uint64(0)
        st = lib.or_gather_group(ctypes.byref(sg), ctypes.byref(dg), ip, ctypes.c_uint64(m), ctypes.c_uint64(k0),
                                 ctypes.c_uint64(base[g] if base else 0), ctypes.byref(end))
        ends.append(end.value)
        if st != ST_OK:
            return st, ends
    return ST_OK, ends


def _lengths(L: Layout, bufs, g, n):
    """Member counts of objects 0..n-1 of group g (records' counts, or
    differences of the offsets)."""
    S = L.schema
    if L.kind == "aos":
        off = L.slot_offsets[S.slots.index(("len", g))]
        rec = np.ascontiguousarray(bufs[0]).view(np.uint8)[:n * L.stride].reshape(n, L.stride)
        return rec[:, off:off + 4].copy().view(np.uint32).reshape(-1).astype(np.uint64)
    o = np.ascontiguousarray(bufs[_group_buffers(L, g, bufs)]).view(NP_DTYPE[S.offset_types[g]])
    return (o[1:n + 1].astype(np.int64) - o[:n].astype(np.int64)).astype(np.uint64)


def select(src: Layout, src_bufs, dst: Layout, n: int, keep_flags, src_members=()):
    """Compaction after a filter: the objects i < n with keep_flags[i] != 0,
    in order, into fresh zero-filled buffers of layout dst (members of each
    group packed from 0).  Returns (status, dst_bufs, count, totals)."""
    idx = np.nonzero(np.asarray(keep_flags)[:n])[0].astype(np.uint64)
    S = src.schema
    tots = [int(_lengths(src, src_bufs, g, n)[idx].sum()) for g in range(S.n_groups)]
    out = zeros_like_layout(dst, len(idx), tots)
    st, _ = gather_into(src, src_bufs, dst, out, idx, 0, [0] * S.n_groups, src_members, tots)
    return st, out, len(idx), tots


def erase(L: Layout, bufs, n: int, at: int, count: int, members=()):
    """Objects [at, at + count) removed from a collection of n objects: the
    objects before and after them, in order, in fresh buffers of the same
    layout.  Returns (status, bufs, totals)."""
    idx = np.concatenate([np.arange(at, dtype=np.uint64), np.arange(at + count, n, dtype=np.uint64)])
    S = L.schema
    tots = [int(_lengths(L, bufs, g, n)[idx].sum()) for g in range(S.n_groups)]
    out = zeros_like_layout(L, len(idx), tots)
    st, _ = gather_into(L, bufs, L, out, idx, 0, [0] * S.n_groups, members, tots)
    return st, out, tots


def insert(L: Layout, bufs, n: int, at: int, new_L: Layout, new_bufs, count: int, members=(), new_members=()):
    """`count` objects of a second collection (layout new_L) inserted before
    object `at` of a collection of n objects (at == n appends): objects
    0..at-1, then the new ones, then objects at..n-1, in fresh buffers of
    layout L; members follow their objects.  Returns (status, bufs, totals)."""
    S = L.schema
    old_len = [_lengths(L, bufs, g, n) for g in range(S.n_groups)]
    new_len = [_lengths(new_L, new_bufs, g, count) for g in range(S.n_groups)]
    tots = [int(old_len[g].sum() + new_len[g].sum()) for g in range(S.n_groups)]
    out = zeros_like_layout(L, n + count, tots)
    base = [0] * S.n_groups
    parts = [(L, bufs, np.arange(at, dtype=np.uint64), 0, members),
             (new_L, new_bufs, np.arange(count, dtype=np.uint64), at, new_members),
             (L, bufs, np.arange(at, n, dtype=np.uint64), at + count, members)]
    for sl, sb, idx, k0, mem in parts:
        st, ends = gather_into(sl, sb, L, out, idx, k0, base, mem, tots)
        if st != ST_OK:
            return st, out, tots
        base = ends if ends else base
    return ST_OK, out, tots


class Prepared:
    """One dense conversion with its buffers set up once, for timing the
    oracle's loop alone (no allocation or packing per run): ``run(threads)``
    converts objects 0..n-1 split into ``threads`` contiguous ranges, one
    host thread each (ctypes releases the GIL during the C call)."""

    def __init__(self, src: Layout, src_bufs, dst: Layout, n: int):
        self.n = n
        self.src_bufs = [np.ascontiguousarray(b).view(np.uint8).reshape(-1) for b in src_bufs]
        self.dst_bufs = zeros_like_layout(dst, n, [0] * dst.schema.n_groups)
        self.keep = []
        self.so = _objects_struct(src, self.src_bufs, self.keep)
        self.do = _objects_struct(dst, self.dst_bufs, self.keep)
        self.n_leaves = len(src.schema.leaves)

    def _range(self, i0, i1):
        return _load().or_convert_objects_range(ctypes.byref(self.so), ctypes.byref(self.do),
                                                ctypes.c_uint32(self.n_leaves), ctypes.c_uint64(i0),
                                                ctypes.c_uint64(i1))

    def run(self, threads=1, pool=None):
        if threads <= 1:
            return self._range(0, self.n)
        step = (self.n + threads - 1) // threads
        futs = [pool.submit(self._range, k * step, min(self.n, (k + 1) * step)) for k in range(threads)]
        sts = [f.result() for f in futs]
        return max(sts)


def _count_members(L: Layout, bufs, g, n):
    """Total member count of group g over objects 0..n-1 of a source."""
    S = L.schema
    if L.kind == "aos":
        if n == 0:
            return 0
        lo = L.slot_offsets[S.slots.index(("len", g))]
        lens = np.ndarray((n,), dtype=np.uint32, buffer=bufs[0], offset=lo,
                          strides=(L.stride,))
        return int(lens.astype(np.uint64).sum())
    i0 = _group_buffers(L, g, bufs)
    t = S.offset_types[g]
    offs = np.frombuffer(bufs[i0].tobytes(), dtype=NP_DTYPE[t])
    return int(offs[n]) - int(offs[0]) if n >= 0 else 0


def exclusive_scan(lengths: np.ndarray, off_type: str = "u32"):
    lib = _load()
    lengths = np.ascontiguousarray(lengths, dtype=np.uint32)
    n = lengths.size
    out = np.zeros((n + 1) * TYPE_SIZE[off_type], dtype=np.uint8)
    tot = ctypes.c_uint64(0)
    st = lib.or_exclusive_scan(ctypes.c_void_p(lengths.ctypes.data), ctypes.c_uint64(n),
                               ctypes.c_void_p(out.ctypes.data),
                               ctypes.c_int32(TYPE_CODES.index(off_type)), ctypes.byref(tot))
    return st, out.view(NP_DTYPE[off_type]), tot.value


# ---------------------------------------------------------------- sources from values

def values_layout(schema: Schema) -> Layout:
    """The layout in which Values hold their content: one column per leaf in
    schema types, jagged members in object order with u64 offsets."""
    return make_layout(schema, "soa")


def values_buffers(schema: Schema, v: Values):
    """Buffers of the ``soa`` layout holding v's content (the value layout),
    with group offsets in the schema's offset type."""
    bufs = []
    for f, e in schema.leaves:
        a = np.asarray(v.fields[f.name])
        col = a if f.extent == 1 else a[:, e]
        bufs.append(np.ascontiguousarray(col, dtype=NP_DTYPE[f.type]).view(np.uint8).copy())
    for g in range(schema.n_groups):
        t = schema.offset_types[g]
        offs = np.zeros(v.n + 1, dtype=np.uint64)
        np.cumsum(v.lengths[g].astype(np.uint64), out=offs[1:])
        bufs.append(offs.astype(NP_DTYPE[t]).view(np.uint8).copy())
        for f, e in schema.members[g]:
            a = np.asarray(v.members[f.name])
            col = a if f.extent == 1 else a[:, e]
            bufs.append(np.ascontiguousarray(col, dtype=NP_DTYPE[f.type]).view(np.uint8).copy())
    return bufs


def pack(schema: Schema, v: Values, dst: Layout, pool_order: bool = False):
    """Bytes of layout dst holding v's content.  For an aos destination with
    pool_order=True, each group's member blocks are placed in the pool in
    v.block_order (a heap-like source) instead of object order."""
    src = values_layout(schema)
    bufs = values_buffers(schema, v)
    tot = [v.total(g) for g in range(schema.n_groups)]
    st, out, _ = convert(src, bufs, dst, v.n, tot, tot)
    assert st == ST_OK, st
    if pool_order and dst.kind == "aos":
        for g in range(schema.n_groups):
            _reorder_pool(dst, out, g, v.block_order[g], v.n)
    return out


def _reorder_pool(L: Layout, bufs, g, order, n):
    """Move group g's member blocks into the pool in the given object order,
    rewriting each record's pointer."""
    S = L.schema
    po = L.slot_offsets[S.slots.index(("ptr", g))]
    lo = L.slot_offsets[S.slots.index(("len", g))]
    ms = L.member_stride[g]
    rec = bufs[0]
    pool = bufs[1 + g]
    new_pool = np.zeros_like(pool)
    pos = 0
    ptr_col = np.ndarray((n,), dtype=np.uint64, buffer=rec, offset=po, strides=(L.stride,)) if n else None
    len_col = np.ndarray((n,), dtype=np.uint32, buffer=rec, offset=lo, strides=(L.stride,)) if n else None
    for i in order:
        p, ln = int(ptr_col[i]), int(len_col[i])
        new_pool[pos: pos + ln * ms] = pool[p: p + ln * ms]
        ptr_col[i] = pos
        pos += ln * ms
    pool[:] = new_pool


def unpack_fields(schema: Schema, L: Layout, bufs, n: int, totals=None):
    """Inverse of pack: logical values (per field arrays) read back from a
    layout by converting into the value layout."""
    src_members = totals if totals is not None else [
        _count_members(L, bufs, g, n) for g in range(schema.n_groups)]
    if L.kind == "aos":
        src_members = [len(bufs[1 + g]) // L.member_stride[g] if L.member_stride[g] else 0
                       for g in range(schema.n_groups)]
    vl = values_layout(schema)
    st, out, tots = convert(L, bufs, vl, n, src_members)
    assert st == ST_OK, st
    return out, tots
