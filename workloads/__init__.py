"""Seeded synthetic workloads: schema declarations and field values.

This module is shared by the product's tests and benchmark and by the CPU
oracle's tests.  It holds no layout arithmetic at all: it declares schemas as
plain field lists and draws *logical* field values (one numpy array per field,
members of jagged groups in object order).  Turning those values into bytes of
a particular memory layout is the job of the code under test (and, separately,
of the oracle).

A schema follows the property kinds of the paper (Sec. VI): a per-item property
is a field with extent 1, an array property a field with extent E > 1, a
sub-group property a run of fields sharing a ``subgroup`` id, and a jagged
vector property a set of fields sharing a ``group`` id, whose sizes are kept as
a prefix sum of the declared offset type.

Value recipes follow the workloads of the case study (Sec. VIII): sensor-like
"cell" collections and particle-like "cluster" collections whose member list
is a variable-length list of (index, weight) pairs.
"""
from __future__ import annotations

from dataclasses import dataclass, field as dc_field

import numpy as np

# name -> (numpy dtype, size in bytes, code shared with the C ABI enum order)
TYPE_CODES = ["u8", "i8", "u16", "i16", "u32", "i32", "u64", "i64", "f32", "f64"]
NP_DTYPE = {
    "u8": np.uint8, "i8": np.int8, "u16": np.uint16, "i16": np.int16,
    "u32": np.uint32, "i32": np.int32, "u64": np.uint64, "i64": np.int64,
    "f32": np.float32, "f64": np.float64,
}
TYPE_SIZE = {t: np.dtype(d).itemsize for t, d in NP_DTYPE.items()}


@dataclass(frozen=True)
class Field:
    name: str
    type: str
    extent: int = 1
    group: int = -1      # -1: one value per object; g >= 0: member of jagged group g
    subgroup: int = -1   # -1: top level; s >= 0: part of nested sub-group s


@dataclass(frozen=True)
class SchemaDecl:
    name: str
    fields: tuple
    offset_types: tuple = ()   # one per jagged group: "u32", "i32" or "u64"

    def object_fields(self):
        return [f for f in self.fields if f.group < 0]

    def member_fields(self, g):
        return [f for f in self.fields if f.group == g]


def _f(name, t, extent=1, group=-1, subgroup=-1):
    return Field(name, t, extent, group, subgroup)


# Plain method, small case: eight scalar fields of mixed width.
PLAIN8 = SchemaDecl("plain8", (
    _f("a", "f32"), _f("b", "f32"), _f("c", "i32"), _f("d", "i32"),
    _f("e", "f64"), _f("f", "u16"), _f("g", "u8"), _f("h", "u32"),
))

# Sensor-like cell collection; energy_d is kept in double precision at the
# source and narrowed to single precision in device layouts.
CELL = SchemaDecl("cell", (
    _f("energy", "f32"), _f("time", "f32"), _f("gain", "i8"),
    _f("quality", "u16"), _f("hash", "u32"), _f("flags", "u32"),
    _f("energy_d", "f64"),
))

# Particle-like cluster collection with a jagged list of (index, weight).
CLUSTER = SchemaDecl("cluster", (
    _f("energy", "f32"), _f("eta", "f32"), _f("phi", "f32"), _f("time", "f32"),
    _f("n_cells", "i32"), _f("seed", "i32"),
    _f("cell_index", "u32", group=0), _f("cell_weight", "f32", group=0),
), offset_types=("u32",))

# The two example classes of the paper (Sec. III listings and their Sec. VI
# property declarations).  The enumeration's underlying type and its number
# of sensor types are not stated; u8 and 4 are used.
N_SENSOR_TYPES = 4
SENSOR = SchemaDecl("sensor", (
    _f("type", "u8"), _f("counts", "u64"), _f("energy", "f32"),
    _f("noisy", "u8", subgroup=0), _f("parameter_A", "f32", subgroup=0),
    _f("parameter_B", "f32", subgroup=0), _f("noise_A", "f32", subgroup=0),
    _f("noise_B", "f32", subgroup=0),
))
PARTICLE = SchemaDecl("particle", (
    _f("energy", "f32"), _f("x", "f32"), _f("y", "f32"), _f("origin", "u64"),
    _f("sensors", "u64", group=0),
    _f("x_variance", "f32"), _f("y_variance", "f32"),
    _f("significance", "f32", extent=N_SENSOR_TYPES),
    _f("E_contribution", "f32", extent=N_SENSOR_TYPES),
    _f("noisy_count", "u8", extent=N_SENSOR_TYPES),
), offset_types=("i32",))

SCHEMAS = {s.name: s for s in (PLAIN8, CELL, CLUSTER, SENSOR, PARTICLE)}


# ---------------------------------------------------------------- property trees
#
# Schemas whose properties nest (Sec. VI): an array property holds a list of
# properties, and sub-groups and jagged vectors may sit inside arrays.  A
# tree's logical values are named by paths: names joined by ".", an array
# element as "[e]" after the array's name (e.g. "layers[1].pos.x").  Each
# jagged vector reached -- each element of an array holding one is its own
# -- is a jagged group; groups are numbered in the order a pre-order walk
# reaches them, array elements in turn.

@dataclass(frozen=True)
class Item:
    name: str
    type: str


@dataclass(frozen=True)
class Array:
    name: str
    extent: int
    props: tuple


@dataclass(frozen=True)
class SubGroup:
    name: str
    props: tuple


@dataclass(frozen=True)
class Jagged:
    name: str
    offset_type: str
    props: tuple


@dataclass(frozen=True)
class TreeDecl:
    name: str
    props: tuple

    def _walk(self):
        """(object paths and types, [(offset type, member paths and types)])
        in walk order."""
        objs, groups = [], []

        def go(p, prefix, members):
            path = f"{prefix}.{p.name}" if prefix else p.name
            if isinstance(p, Item):
                (members if members is not None else objs).append((path, p.type))
            elif isinstance(p, Array):
                for e in range(p.extent):
                    for c in p.props:
                        go(c, f"{path}[{e}]", members)
            elif isinstance(p, SubGroup):
                for c in p.props:
                    go(c, path, members)
            else:
                assert members is None, "jagged vectors do not nest"
                mem = []
                groups.append((path, p.offset_type, mem))
                for c in p.props:
                    go(c, path, mem)

        for p in self.props:
            go(p, "", None)
        return objs, groups

    @property
    def offset_types(self):
        return tuple(t for _, t, _ in self._walk()[1])

    def object_paths(self):
        return self._walk()[0]

    def group_paths(self):
        """Per group: (path of the jagged vector, offset type, member paths and types)."""
        return self._walk()[1]


def tree_values(decl: TreeDecl, n: int, seed: int, mean_len: float = 4.0,
                shuffle_pool: bool = True) -> Values:
    """Uniform values for a property tree, keyed by path: floats in
    [-1e3, 1e3], integers over their full range, member counts of every
    group Poisson(mean_len)."""
    rng = np.random.default_rng(seed)
    v = Values(decl, n)
    for path, t in decl.object_paths():
        v.fields[path] = _uniform_values(rng, Field(path, t), (n,))
    for _, _, mem in decl.group_paths():
        lens = rng.poisson(mean_len, size=n).astype(np.uint32)
        v.lengths.append(lens)
        tot = int(lens.sum())
        for path, t in mem:
            v.members[path] = _uniform_values(rng, Field(path, t), (tot,))
        v.block_order.append(rng.permutation(n) if shuffle_pool else np.arange(n))
    return v


# Event-like record with nesting at every level: per-layer arrays of a
# sub-group and items, per-calorimeter-side jagged cell lists (an array of
# jagged vectors, u32 prefix sums) whose members hold an array, and a
# track list with a sub-group inside each member (u64 prefix sums).
TRACKER = TreeDecl("tracker", (
    Item("energy", "f32"),
    Array("layers", 3, (Item("hits", "u16"),
                        SubGroup("pos", (Item("x", "f32"), Item("y", "f32"))),
                        Item("flag", "u8"))),
    Array("calo", 2, (Jagged("cells", "u32", (Item("id", "u32"),
                                              Array("w", 2, (Item("v", "f32"),)))),)),
    Item("id", "u64"),
    Jagged("tracks", "u64", (Item("pt", "f32"),
                             SubGroup("dir", (Item("eta", "f32"), Item("phi", "f32"))))),
))

# Arrays of sub-groups holding arrays (properties nested inside arrays,
# extents multiplying), an f64 item to narrow, and an i32-offset jagged
# vector of 8-byte members.
DETECTOR = TreeDecl("detector", (
    Item("flags", "u8"),
    Array("modules", 4, (SubGroup("cal", (Item("gain", "f64"), Array("ped", 2, (Item("v", "i16"),)))),
                         Item("ok", "u8"))),
    Item("t0", "f64"),
    Jagged("hits", "i32", (Item("adc", "u64"),)),
))

TREES = {t.name: t for t in (TRACKER, DETECTOR)}


@dataclass
class Values:
    """Logical content of a collection of ``n`` objects.

    ``fields[name]`` has shape (n,) or (n, extent) for per-object fields.
    For jagged group g: ``lengths[g]`` (n,) uint32, ``members[name]`` of
    shape (total,) or (total, extent) in object order, and
    ``block_order[g]``, a permutation of range(n) giving the order in which
    the objects' member blocks sit in a heap-like source pool.
    """
    schema: SchemaDecl
    n: int
    fields: dict = dc_field(default_factory=dict)
    lengths: list = dc_field(default_factory=list)
    members: dict = dc_field(default_factory=dict)
    block_order: list = dc_field(default_factory=list)

    def total(self, g):
        return int(self.lengths[g].astype(np.uint64).sum())


def _full_range(rng, t, shape):
    info = np.iinfo(NP_DTYPE[t])
    return rng.integers(info.min, info.max, size=shape, dtype=NP_DTYPE[t],
                        endpoint=True)


def _uniform_values(rng, f, shape):
    if f.type in ("f32", "f64"):
        # single precision values are drawn in double and rounded by numpy
        return rng.uniform(-1e3, 1e3, size=shape).astype(NP_DTYPE[f.type])
    return _full_range(rng, f.type, shape)


def _shape(n, f):
    return (n,) if f.extent == 1 else (n, f.extent)


def generic_values(schema: SchemaDecl, n: int, seed: int, mean_len: float = 4.0,
                   shuffle_pool: bool = True) -> Values:
    """Uniform values for any schema: floats in [-1e3, 1e3], integers over
    their full range, jagged lengths Poisson(mean_len)."""
    rng = np.random.default_rng(seed)
    v = Values(schema, n)
    for f in schema.object_fields():
        v.fields[f.name] = _uniform_values(rng, f, _shape(n, f))
    for g in range(len(schema.offset_types)):
        lens = rng.poisson(mean_len, size=n).astype(np.uint32)
        v.lengths.append(lens)
        tot = int(lens.sum())
        for f in schema.member_fields(g):
            v.members[f.name] = _uniform_values(rng, f, _shape(tot, f))
        v.block_order.append(rng.permutation(n) if shuffle_pool
                             else np.arange(n))
    return v


def plain_values(n: int = 10_000, seed: int = 1000) -> Values:
    """Plain method, small case: 8 scalar fields, uniform values."""
    return generic_values(PLAIN8, n, seed)


def cell_values(n: int = 190_000, seed: int = 1001) -> Values:
    """Cell-like collection: energy_d log-normal (mu 3, sigma 1.5) in double,
    energy its single-precision rounding (numpy's cast), time normal(0, 5),
    gain in {0,1,2}, quality full range, hash = object index, flags random
    bits."""
    rng = np.random.default_rng(seed)
    v = Values(CELL, n)
    energy_d = rng.lognormal(3.0, 1.5, size=n)
    v.fields["energy_d"] = energy_d
    v.fields["energy"] = energy_d.astype(np.float32)
    v.fields["time"] = rng.normal(0.0, 5.0, size=n).astype(np.float32)
    v.fields["gain"] = rng.integers(0, 3, size=n, dtype=np.int8)
    v.fields["quality"] = _full_range(rng, "u16", (n,))
    v.fields["hash"] = np.arange(n, dtype=np.uint32)
    v.fields["flags"] = _full_range(rng, "u32", (n,))
    return v


def cluster_values(n: int = 50_000, seed: int = 1002, mean_len: float = 40.0,
                   shuffle_pool: bool = True, n_cells: int = 190_000) -> Values:
    """Cluster-like jagged collection: 4 float fields uniform in [-1e3, 1e3],
    2 int fields over their full range, Poisson(mean_len) member counts,
    member cell_index uniform in [0, n_cells), cell_weight uniform in (0, 1]."""
    rng = np.random.default_rng(seed)
    v = Values(CLUSTER, n)
    for name in ("energy", "eta", "phi", "time"):
        v.fields[name] = rng.uniform(-1e3, 1e3, size=n).astype(np.float32)
    for name in ("n_cells", "seed"):
        v.fields[name] = _full_range(rng, "i32", (n,))
    lens = rng.poisson(mean_len, size=n).astype(np.uint32)
    tot = int(lens.sum())
    v.lengths.append(lens)
    v.members["cell_index"] = rng.integers(0, n_cells, size=tot, dtype=np.uint32)
    v.members["cell_weight"] = (1.0 - rng.random(size=tot)).astype(np.float32)
    v.block_order.append(rng.permutation(n) if shuffle_pool else np.arange(n))
    return v


def batch_items(n_items: int = 512, seed: int = 1003, lo: int = 1_000,
                hi: int = 200_000):
    """Heterogeneous batch: per item a schema (plain8 / cell / cluster,
    uniform), an object count log-uniform over [lo, hi], a source kind
    uniform over {aos, soa, aosoa64} and a destination kind drawn from the
    two others.  Returns a list of dicts; values are drawn lazily per item
    with seed + 1 + item index."""
    rng = np.random.default_rng(seed)
    names = ["plain8", "cell", "cluster"]
    kinds = ["aos", "soa", "aosoa"]
    out = []
    for k in range(n_items):
        sname = names[int(rng.integers(0, 3))]
        n = int(np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        src = kinds[int(rng.integers(0, 3))]
        others = [x for x in kinds if x != src]
        dst = others[int(rng.integers(0, 2))]
        out.append(dict(schema=sname, n=n, src=src, dst=dst, seed=seed + 1 + k))
    return out


def item_values(item) -> Values:
    s = item["schema"]
    if s == "plain8":
        return plain_values(item["n"], item["seed"])
    if s == "cell":
        return cell_values(item["n"], item["seed"])
    return cluster_values(item["n"], item["seed"])


def serving_events(n_events: int, seed: int = 1004, medians=(10_000, 100_000, 20_000),
                   sigma: float = 0.5, cap: int = 1_000_000):
    """Per event object counts for (plain8, cell, cluster), log-normal with the
    given medians and sigma, clipped to [1, cap]."""
    rng = np.random.default_rng(seed)
    sizes = np.empty((n_events, 3), dtype=np.int64)
    for j, med in enumerate(medians):
        sizes[:, j] = np.clip(np.floor(rng.lognormal(np.log(med), sigma, size=n_events)),
                              1, cap).astype(np.int64)
    return sizes


def poisson_arrivals(n_events: int, rate_hz: float, seed: int = 1004):
    """Open-loop Poisson arrival times in seconds (exponential gaps)."""
    rng = np.random.default_rng(seed + 7)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n_events))
