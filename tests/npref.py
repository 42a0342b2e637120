"""numpy-side helpers for pinning the oracle: record layouts built by
numpy's own structured-dtype rules, and block views built by reshaping.
None of this is used by the oracle or by the library."""
import numpy as np

from workloads import NP_DTYPE


def record_dtype(decl, align=True):
    """numpy structured dtype of one object record: per-object fields (arrays
    as sub-arrays, sub-groups as nested structs) and, where a jagged group is
    first declared, a (u64 ptr, u32 len) pair."""
    names, formats = [], []
    seen = set()
    sub_names, sub_formats, cur = [], [], None

    def flush():
        nonlocal sub_names, sub_formats, cur
        if cur is not None:
            names.append(f"sub{cur}")
            formats.append(np.dtype({"names": sub_names, "formats": sub_formats}, align=align))
        sub_names, sub_formats, cur = [], [], None

    for f in decl.fields:
        if f.group >= 0:
            if f.group not in seen:
                flush()
                seen.add(f.group)
                names += [f"ptr{f.group}", f"len{f.group}"]
                formats += [np.uint64, np.uint32]
            continue
        fmt = NP_DTYPE[f.type] if f.extent == 1 else (NP_DTYPE[f.type], (f.extent,))
        if f.subgroup >= 0:
            if cur != f.subgroup:
                flush()
                cur = f.subgroup
            sub_names.append(f.name)
            sub_formats.append(fmt)
        else:
            flush()
            names.append(f.name)
            formats.append(fmt)
    flush()
    return np.dtype({"names": names, "formats": formats}, align=align)


def field_of(rec, decl, name):
    """Values of a per-object field from a record array, looking through
    nested sub-group structs."""
    for f in decl.fields:
        if f.name == name and f.subgroup >= 0:
            return rec[f"sub{f.subgroup}"][name]
    return rec[name]


def member_dtype(decl, g, align=True):
    fs = decl.member_fields(g)
    return np.dtype({"names": [f.name for f in fs],
                     "formats": [NP_DTYPE[f.type] if f.extent == 1 else (NP_DTYPE[f.type], (f.extent,))
                                 for f in fs]}, align=align)


def aosoa_column(buf, width, sizes, c, n, dtype):
    """Leaf c of an AoSoA buffer (blocks of `width` objects, each block the
    leaves' runs back to back) by reshaping into blocks and slicing."""
    B = sum(sizes)
    nblk = len(buf) // (width * B) if B else 0
    blocks = np.asarray(buf).reshape(nblk, width * B)
    start = width * sum(sizes[:c])
    run = blocks[:, start:start + width * sizes[c]]
    return np.ascontiguousarray(run).reshape(-1).view(dtype)[:n]


# ---- property trees (nested structured dtypes)

def tree_dtype(props, leaf_type=None):
    """numpy structured dtype (C alignment, align=True) of a struct made of
    tree properties: an item a scalar field, a sub-group a nested struct, an
    array a sub-array of element structs, a jagged vector two fields
    '<name>#ptr' (u64) and '<name>#len' (u32).  leaf_type(path, type) may
    change an item's type (paths as the workloads name them)."""
    return _tree_dtype(props, "", leaf_type)


def _tree_dtype(props, prefix, leaf_type):
    names, formats = [], []
    for p in props:
        path = f"{prefix}.{p.name}" if prefix else p.name
        kind = type(p).__name__
        if kind == "Item":
            t = leaf_type(path, p.type) if leaf_type else p.type
            names.append(p.name)
            formats.append(NP_DTYPE[t])
        elif kind == "Jagged":
            names += [p.name + "#ptr", p.name + "#len"]
            formats += [np.uint64, np.uint32]
        elif kind == "SubGroup":
            names.append(p.name)
            formats.append(_tree_dtype(p.props, path, leaf_type))
        else:
            # element structs may differ when leaf_type narrows some elements
            elems = [_tree_dtype(p.props, f"{path}[{e}]", leaf_type) for e in range(p.extent)]
            if all(el == elems[0] for el in elems):
                names.append(p.name)
                formats.append((elems[0], (p.extent,)))
            else:
                for e, el in enumerate(elems):
                    names.append(f"{p.name}@{e}")
                    formats.append(el)
    return np.dtype({"names": names, "formats": formats}, align=True)


def flatten_dtype(dt, prefix="", base=0):
    """(path, byte offset, dtype) of every scalar of a structured dtype in
    declaration order, sub-arrays element by element; sub-array elements
    named '<name>[e]', split arrays' '<name>@e' named the same way."""
    out = []
    for name in dt.names:
        sub, off = dt.fields[name][0], dt.fields[name][1]
        nm = name
        if "@" in nm:
            a, e = nm.split("@")
            nm = f"{a}[{e}]"
        path = f"{prefix}.{nm}" if prefix else nm
        if sub.subdtype is not None:
            el, shape = sub.subdtype
            for e in range(shape[0]):
                ep = f"{path}[{e}]"
                if el.names:
                    out += flatten_dtype(el, ep, base + off + e * el.itemsize)
                else:
                    out.append((ep, base + off + e * el.itemsize, el))
        elif sub.names:
            out += flatten_dtype(sub, path, base + off)
        else:
            out.append((path, base + off, sub))
    return out
