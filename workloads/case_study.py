"""The case study's two pipelines as synthetic stand-ins (Sec. VIII, the
sensor-grid example of Sec. III): what the paper times is fill -> transfer
to the device -> energy per sensor, and particle reconstruction ->
transfer back -> fill of the original records.  The energy calibration and
the particle reconstruction are not given in the paper; the arithmetic here
is a stand-in of the same shape (an elementwise formula over every sensor
property; per particle, sums over the 5 x 5 neighbourhood of a seed sensor,
with the neighbourhood's sensor indices as its jagged member list) and only
the layout steps around it carry parity claims.

Device code here is plain torch (the stand-in compute is not part of the
conversion path)."""
import numpy as np

from workloads import N_SENSOR_TYPES, PARTICLE, SENSOR, Values


def sensor_grid(side: int, seed: int) -> Values:
    """Raw sensor information for a side x side grid: type uniform over the
    sensor types, counts Poisson(200), calibration parameters A in [0.5,
    1.5], B in [-5, 5], noise flag on one sensor in eight, noise A in
    [0, 0.1], noise B in [0, 2]; energy left 0 (computed on the device)."""
    rng = np.random.default_rng(seed)
    n = side * side
    v = Values(SENSOR, n)
    v.fields["type"] = rng.integers(0, N_SENSOR_TYPES, size=n, dtype=np.uint8)
    v.fields["counts"] = rng.poisson(200.0, size=n).astype(np.uint64)
    v.fields["energy"] = np.zeros(n, dtype=np.float32)
    v.fields["noisy"] = (rng.random(n) < 0.125).astype(np.uint8)
    v.fields["parameter_A"] = rng.uniform(0.5, 1.5, size=n).astype(np.float32)
    v.fields["parameter_B"] = rng.uniform(-5, 5, size=n).astype(np.float32)
    v.fields["noise_A"] = rng.uniform(0, 0.1, size=n).astype(np.float32)
    v.fields["noise_B"] = rng.uniform(0, 2, size=n).astype(np.float32)
    return v


def sensor_energy(cols):
    """Stand-in calibration on device SoA columns (torch float32 views, in
    the schema's leaf order): energy = A * counts + B, less the noise
    A' * counts + B' on noisy sensors; written into the energy column."""
    import torch
    typ, counts, energy, noisy, pa, pb, na, nb = cols
    c = counts.to(torch.float32)
    e = pa * c + pb - noisy.to(torch.float32) * (na * c + nb)
    energy.copy_(e)
    return energy


def sensor_energy_numpy(v: Values):
    c = v.fields["counts"].astype(np.float32)
    f = {k: v.fields[k] for k in ("parameter_A", "parameter_B", "noise_A", "noise_B")}
    return (f["parameter_A"] * c + f["parameter_B"]
            - v.fields["noisy"].astype(np.float32) * (f["noise_A"] * c + f["noise_B"])).astype(np.float32)


def seed_sensors(side: int, n_particles: int, seed: int):
    """Seed sensor of each particle: distinct grid positions, uniform."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(side * side, size=n_particles, replace=False)).astype(np.int64)


def reconstruct(side: int, seeds, typ, energy, noisy):
    """Stand-in reconstruction on the device (torch): per seed, the sensors
    of its 5 x 5 neighbourhood inside the grid (the particle's jagged member
    list, their indices), energy = their energy sum, (x, y) the
    energy-weighted centroid, variances about it, and per sensor type the
    energy share (significance), energy sum (E_contribution) and noisy
    count.  Returns (per-leaf columns in the schema's leaf order, member
    counts, member indices), all torch tensors on the device."""
    import torch
    dev = energy.device
    s = torch.as_tensor(seeds, device=dev)
    sx, sy = s % side, s // side
    d = torch.arange(-2, 3, device=dev)
    nx = sx[:, None, None] + d[None, None, :]
    ny = sy[:, None, None] + d[None, :, None]
    nx, ny = nx.expand(-1, 5, 5).reshape(-1, 25), ny.expand(-1, 5, 5).reshape(-1, 25)
    inside = (nx >= 0) & (nx < side) & (ny >= 0) & (ny < side)
    idx = torch.where(inside, ny * side + nx, torch.zeros_like(nx))
    e = torch.where(inside, energy[idx], torch.zeros((), device=dev))
    etot = e.sum(1)
    w = e / torch.where(etot == 0, torch.ones_like(etot), etot)[:, None]
    x = (w * nx.to(torch.float32)).sum(1)
    y = (w * ny.to(torch.float32)).sum(1)
    xv = (w * (nx.to(torch.float32) - x[:, None]) ** 2).sum(1)
    yv = (w * (ny.to(torch.float32) - y[:, None]) ** 2).sum(1)
    t = typ[idx].to(torch.int64)
    nz = noisy[idx].to(torch.int64)
    sig, econ, ncount = [], [], []
    for k in range(N_SENSOR_TYPES):
        m = inside & (t == k)
        ek = torch.where(m, e, torch.zeros((), device=dev)).sum(1)
        econ.append(ek)
        sig.append(ek / torch.where(etot == 0, torch.ones_like(etot), etot))
        ncount.append((m & (nz != 0)).sum(1).to(torch.uint8))
    cols = [etot, x, y, s.to(torch.int64), xv, yv] + sig + econ + ncount
    counts = inside.sum(1)
    members = idx[inside].to(torch.int64)   # row-major: each particle's members in order
    return cols, counts, members


def particle_leaf_order():
    """Leaf names of the particle schema in leaf order (arrays expanded)."""
    out = []
    for f in PARTICLE.object_fields():
        out += [f.name] if f.extent == 1 else [f"{f.name}[{e}]" for e in range(f.extent)]
    return out


def _field_slots(decl):
    """Record slot index of the first leaf of every per-object field: slots
    are the per-object leaves in declaration order, with a jagged group's
    (pointer, count) pair where the group's first field is declared."""
    out, slot, seen = {}, 0, set()
    for f in decl.fields:
        if f.group >= 0:
            if f.group not in seen:
                seen.add(f.group)
                slot += 2
            continue
        out[f.name] = slot
        slot += f.extent
    return out


def record_dtype(layout, decl):
    """numpy structured dtype of a record layout of the library (its slot
    offsets and stride), for filling records on the host."""
    from workloads import NP_DTYPE
    slots = _field_slots(decl)
    names, formats, offsets = [], [], []
    for f in decl.fields:
        if f.group >= 0:
            continue
        names.append(f.name)
        formats.append(NP_DTYPE[f.type] if f.extent == 1 else (NP_DTYPE[f.type], f.extent))
        offsets.append(layout.slot_offsets[slots[f.name]])
    return np.dtype({"names": names, "formats": formats, "offsets": offsets, "itemsize": layout.stride})


def sensor_pipeline(P, torch, side, v, stream, reps=5):
    """Fill pinned host records with v's raw sensor information, transfer
    them to device SoA columns (conversion included), compute the energy.
    Returns per-run timings in ms (after one warm-up run), the pinned
    records and the device columns of the last run."""
    import time
    S = P.Schema(SENSOR)
    aos_h = P.Layout(S, "aos", space="pinned")
    soa = P.Layout(S, "soa")
    n = v.n
    host = torch.zeros(aos_h.buffer_bytes(n)[0], dtype=torch.uint8).pin_memory()   # padding zero
    rec = host.numpy().view(record_dtype(aos_h, SENSOR))
    cols = [torch.empty(b, dtype=torch.uint8, device="cuda") for b in soa.buffer_bytes(n)]
    tv = {"u8": torch.uint8, "u64": torch.int64, "f32": torch.float32}
    typed = [c.view(tv[f.type]) for c, f in zip(cols, SENSOR.fields)]
    sv, dv = P.View(aos_h, n, [host]), P.View(soa, n, cols)
    runs = []
    for _ in range(reps + 1):   # the first run is a warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in SENSOR.fields:   # fill the records from the raw information
            rec[f.name] = v.fields[f.name]
        t1 = time.perf_counter()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        P.transfer(sv, dv, n, stream)
        e1.record(stream)
        sensor_energy(typed)
        e2.record(stream)
        torch.cuda.synchronize()
        runs.append({"fill": (t1 - t0) * 1e3, "h2d_convert": e0.elapsed_time(e1), "energy": e1.elapsed_time(e2)})
    return runs[1:], host, cols, typed


def particle_pipeline(P, torch, side, seeds, typed, stream, reps=5):
    """Reconstruct particles from the device sensor columns (stand-in),
    write them as device SoA (offsets from the member counts), transfer
    them back into pinned host records + member pool (conversion
    included).  Returns per-run timings in ms (after one warm-up run), the
    device particle buffers and the pinned host buffers of the last run."""
    S = P.Schema(PARTICLE)
    soa = P.Layout(S, "soa")
    aos_h = P.Layout(S, "aos", space="pinned")
    npart = len(seeds)
    mcap = 25 * npart
    dbufs = [torch.empty(b, dtype=torch.uint8, device="cuda") for b in soa.buffer_bytes(npart, [mcap])]
    hbufs = [torch.empty(b, dtype=torch.uint8).pin_memory() for b in aos_h.buffer_bytes(npart, [mcap])]
    leaf_types = [f.type for f in PARTICLE.object_fields() for _ in range(f.extent)]
    tv = {"u8": torch.uint8, "u64": torch.int64, "f32": torch.float32}
    runs = []
    seeds_d = torch.as_tensor(seeds, device="cuda")
    typ, energy, noisy = typed[0], typed[2], typed[3]
    for _ in range(reps + 1):   # the first run is a warm-up
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        torch.cuda.synchronize()
        e0.record(stream)
        cols, counts, members = reconstruct(side, seeds_d, typ, energy, noisy)
        for c, (buf, t) in enumerate(zip(dbufs, leaf_types)):
            buf.view(tv[t]).copy_(cols[c].to(tv[t]))
        offs = dbufs[len(leaf_types)].view(torch.int32)
        offs[0] = 0
        offs[1:] = torch.cumsum(counts, 0).to(torch.int32)
        tot = int(members.numel())
        dbufs[len(leaf_types) + 1][:8 * tot].view(torch.int64).copy_(members)
        e1.record(stream)
        P.transfer(P.View(soa, npart, dbufs, [tot]), P.View(aos_h, npart, hbufs, [mcap]), npart, stream)
        e2.record(stream)
        torch.cuda.synchronize()
        runs.append({"reconstruct": e0.elapsed_time(e1), "d2h_convert": e1.elapsed_time(e2), "members": tot})
    return runs[1:], dbufs, hbufs
