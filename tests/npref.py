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
