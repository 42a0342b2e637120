"""Benchmark of the layout-conversion hot path on one MI355X.

Step: the cell-like collection of the case study (190,000 objects: energy
f32, time f32, gain i8, quality u16, hash u32, flags u32, energy_d f64),
resident in HBM as AoS records, converted into the four device layouts the
workload asks for: SoA (energy_d narrowed to f32) and AoSoA with block
widths 32, 64 and 128 (same narrowing).  Each step uses its own copy of the
source and destinations, rotating over enough copies that the working set
is several times the 256 MB Infinity Cache; the timed steps use copies the
warm-up did not touch.

Value: algorithmic bytes (source footprint read + destination footprint
written, per conversion) per second of the timed region.  The four
conversions share their source, so the HBM traffic of a step is lower
(three of the four source reads are served by L2); roofline.frac_hbm gives
the fraction from the measured HBM counters beside the algorithmic one.

The four conversions of a step run as one launch of the batch engine
(persistent kernels over a device table; tile shape, work-group count and
graph replay vs direct launch autotuned once, cached); the same
conversions as a per-conversion launch loop are timed beside it.  The
timed region is K steps back to back between two events; each step is one
launch of the batch dense kernel, so the region's mean step time is that
kernel's mean launch duration (the roofline).  A second pass with an event
pair around each of 50 launches gives the paper's statistic (mean of the
10 fastest, and the median).

Extra legs, outside the timed region: a single conversion per launch
(cold), the attainable HBM rate of a plain 16-byte copy kernel and the
launch floor, the plain round trip, jagged conversions, 512 heterogeneous
collections in one graph launch against the launch loop, a sweep at larger
object counts, host <-> device transfers with conversion (PCIe included),
the serving loop against a synchronous per-event loop, and the oracle timed
on one and on all host cores (cpu_baseline).
"""
import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_CELLS = 190_000
WIDTHS = (32, 64, 128)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--sets", type=int, default=32, help="rotating input/output copies")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serving-events", type=int, default=10_000,
                    help="events per rate in the serving leg (fewer for a traced run)")
    ap.add_argument("--leg", choices=sorted(LEGS),
                    help="run only this extra leg and print its JSON (for profiling one leg)")
    return ap.parse_args()


SERVING_EVENTS = [10_000]


def main():
    args = parse()
    SERVING_EVENTS[0] = args.serving_events
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding over several GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2511_04853_amd as P
    import workloads as Wk

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    P.lib()
    stream = torch.cuda.current_stream()
    sp = P.stream_ptr(stream)
    # calibration: one dispatch of the library's copy kernel moving 64 MiB
    # (untimed), for scaling the HBM byte counters of a profiled run
    calib = torch.zeros(64 << 20, dtype=torch.uint8, device="cuda")
    calib2 = torch.empty_like(calib)
    P.memcopy(calib2, "device", calib, "device", 64 << 20, stream)
    torch.cuda.synchronize()
    del calib, calib2
    if args.leg:
        print(json.dumps(LEGS[args.leg](P, Wk, torch, stream)), flush=True)
        return

    S = P.Schema(Wk.CELL)
    narrowed = ["f32" if f.type == "f64" else f.type for f in Wk.CELL.fields]
    aos = P.Layout(S, "aos")
    dsts = [P.Layout(S, "soa", storage=narrowed)] + [P.Layout(S, "aosoa", width=w, storage=narrowed)
                                                     for w in WIDTHS]
    n = N_CELLS
    v = Wk.cell_values(n)

    # source records built on the device from the generated columns
    def device_aos(values):
        cols = []
        for f in Wk.CELL.fields:
            cols.append(torch.from_numpy(np.ascontiguousarray(values.fields[f.name]).view(np.uint8)).cuda())
        soa64 = P.Layout(S, "soa")
        rec = torch.empty(aos.buffer_bytes(values.n)[0], dtype=torch.uint8, device="cuda")
        P.convert(P.View(soa64, values.n, cols), P.View(aos, values.n, [rec]), values.n)
        assert P.sync() == 0
        return rec

    rec0 = device_aos(v)
    tune_cache = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"rl_tune_{os.getpid()}.json")
    sets = []
    for r in range(args.sets):
        src = rec0 if r == 0 else rec0.clone()
        outs = []
        for L in dsts:
            bufs = [torch.empty(b, dtype=torch.uint8, device="cuda") for b in L.buffer_bytes(n)]
            outs.append(P.View(L, n, bufs))
        sv = P.View(aos, n, [src])
        # one batch per copy: the four conversions of a step in one graph launch
        b = Batch(P, autotune=1 if r == 0 else 0, cache=tune_cache)
        for d in outs:
            b.add(sv, d, n)
        b.finalize(sp)
        sets.append((sv, outs, b))
    torch.cuda.synchronize()
    shape = sets[0][2].shape()
    binfo = sets[0][2].info()
    fanned = binfo.fanout_steps == binfo.dense_steps and binfo.fanout_groups > 0
    step_kernel = (("rl::batch_fanout_db_kernel" if binfo.double_buffered else "rl::batch_fanout_kernel") if fanned else
                   "rl::batch_dense_db_kernel" if binfo.double_buffered else "rl::batch_dense_kernel")

    src_bytes = aos.buffer_bytes(n)[0]
    conv_bytes = [src_bytes + sum(L.buffer_bytes(n)) for L in dsts]
    step_bytes = sum(conv_bytes)
    min_bytes = src_bytes + sum(sum(L.buffer_bytes(n)) for L in dsts)

    def run(k, loop=False):
        b = sets[k % len(sets)][2]
        b.loop(sp) if loop else b.launch(sp)

    W = args.warmup
    for k in range(W):
        run(k)
    assert P.sync(stream) == 0, P.rl_last_error()

    # timed region: K steps back to back, bracketed by two events; the
    # steps use copies W, W + 1, ... (not touched by the warm-up while
    # W + K <= the number of copies)
    K = args.steps
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for k in range(K):
        run(W + k)
    t1.record(stream)
    torch.cuda.synchronize()
    ms_total = t0.elapsed_time(t1)
    assert P.sync(stream) == 0, P.rl_last_error()
    ms_per_step = ms_total / K
    value = step_bytes / (ms_per_step * 1e-3) / 1e9

    # A step is one launch of one batch kernel (the fan-out kernel when all
    # four conversions share each source tile, else the dense kernel; the
    # counts are host-known, so no other kernel runs), so its mean launch
    # duration in the timed region is ms_per_step.  An event pair around each of 50 launches
    # of a second pass gives the paper's statistic for isolated launches
    # (each includes its dispatch latency).
    mean_launch_ms = ms_per_step
    achieved = step_bytes / (mean_launch_ms * 1e-3) / 1e9
    iso = event_times(lambda k: run(W + K + k), stream, torch, 50)
    assert P.sync(stream) == 0, P.rl_last_error()

    # the same conversions as a launch loop (one kernel launch per conversion)
    for k in range(args.warmup):
        run(k, loop=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for k in range(K):
        run(k, loop=True)
    t1.record(stream)
    torch.cuda.synchronize()
    ms_loop = t0.elapsed_time(t1) / K

    out = {
        "metric": "conversion GB/s (read+write) vs HBM peak; batched speedup; p50/p99 event lat",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8 moves + f64->f32 RNE",
        "data": "synthetic",
        "config": {
            "workload": "cell collection, 190,000 objects, device AoS (32 B records) -> SoA with "
                        "energy_d f64->f32 and -> AoSoA W=32/64/128 (same narrowing), "
                        f"{args.sets} rotating copies ({args.sets * (step_bytes - 3 * src_bytes) / 1e6:.0f} MB "
                        "working set, beyond the 256 MB Infinity Cache)",
            "objects": n,
            "bytes_per_step": step_bytes,
            "conversions_per_step": len(dsts),
            "launch": f"one batch launch per step (the 4 conversions; {shape[3]}), "
                      f"tile {shape[0]} objects, {shape[1]} threads, {shape[2]} work-groups"
                      + (f", one source tile read per work-group for all {binfo.fanout_steps} conversions "
                         f"({binfo.fanout_threads} threads each)" if fanned else "")
                      + (", double-buffered" if binfo.double_buffered else "")
                      + (", non-temporal stores" if binfo.stream_stores else "") + " (autotuned)",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "kernel": step_kernel,
            "bytes_basis": "algorithmic: per conversion, source footprint read + destination footprint written",
            "mean_launch_us": round(mean_launch_ms * 1e3, 3),
            "isolated_launch_us": iso,
            "bytes_per_launch": int(step_bytes),
            # the least any kernel must move for the step: the shared source
            # read once and the four destinations written
            "bytes_min_per_launch": int(min_bytes),
            "frac_min_bytes": round(min_bytes / (mean_launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        },
        "step_launch_loop": {"ms_per_step": round(ms_loop, 5),
                             "GBps": round(step_bytes / (ms_loop * 1e-3) / 1e9, 2),
                             "batch_speedup": round(ms_loop / ms_per_step, 3)},
    }

    traffic = measured_traffic(out["roofline"]["kernel"], n)
    out["roofline"]["traffic"] = traffic
    if traffic:
        # the same launch time against the HBM bytes the counters saw
        out["roofline"]["frac_hbm"] = round(traffic / (mean_launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    del sets
    torch.cuda.empty_cache()
    if not args.no_extras:
        for name in EXTRA_ORDER:
            print(f"# leg {name}", file=sys.stderr, flush=True)
            out[name] = LEGS[name](P, Wk, torch, stream)
            torch.cuda.empty_cache()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(Wk, v, args.cpu_seconds, step_bytes)
    print(json.dumps(out), flush=True)


class Batch:
    """ctypes wrapper of an rl_batch."""

    def __init__(self, P, autotune=0, cache=None):
        self.P = P
        self.keep = []
        h = ctypes.c_void_p()
        opts = P.rl_batch_opts(autotune, cache.encode() if cache else None)
        P.check(P.lib().rl_batch_create(ctypes.byref(opts), ctypes.byref(h)), "rl_batch_create")
        self.h = h

    def add(self, sv, dv, n):
        self.keep += [sv, dv]
        self.P.check(self.P.lib().rl_batch_add(self.h, sv.ref(), dv.ref(), n), "rl_batch_add")

    def finalize(self, sp):
        self.P.check(self.P.lib().rl_batch_finalize(self.h, sp), "rl_batch_finalize")

    def launch(self, sp):
        self.P.check(self.P.lib().rl_batch_launch(self.h, sp), "rl_batch_launch")

    def loop(self, sp):
        self.P.check(self.P.lib().rl_batch_launch_loop(self.h, sp), "rl_batch_launch_loop")

    def width(self, k):
        w = ctypes.c_uint32()
        self.P.check(self.P.lib().rl_batch_item_width(self.h, k, ctypes.byref(w)), "width")
        return w.value

    def shape(self):
        a, b, c, g = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        self.P.check(self.P.lib().rl_batch_shape(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                                 ctypes.byref(g)), "shape")
        return a.value, b.value, c.value, "graph replay" if g.value else "direct launch"

    def info(self):
        i = self.P.rl_batch_info()
        self.P.check(self.P.lib().rl_batch_get_info(self.h, ctypes.byref(i)), "rl_batch_get_info")
        return i


def batched(P, W, torch, stream, tune_cache):
    """512 collections (three schemas, sizes log-uniform over 1k..200k,
    mixed kinds, auto block widths): one graph launch vs the launch loop.
    Sources are generated on the device (random field bits, Poisson(40)
    member counts) and laid out by the library."""
    sp = P.stream_ptr(stream)
    decls = {"plain8": W.PLAIN8, "cell": W.CELL, "cluster": W.CLUSTER}
    schemas = {k: P.Schema(d) for k, d in decls.items()}
    kinds = {"aos": ("aos", 0), "soa": ("soa", 0), "aosoa": ("aosoa", 64)}
    g = torch.Generator(device="cuda")
    g.manual_seed(1003)
    specs = W.batch_items()
    b = Batch(P, autotune=1, cache=tune_cache)
    keep = []
    item_bytes = []
    for it in specs:
        decl, S, n = decls[it["schema"]], schemas[it["schema"]], it["n"]
        narrow = ["f32" if f.type == "f64" else f.type for f in decl.fields if f.group < 0]
        narrow = narrow if it["schema"] == "cell" and it["dst"] != "aos" else None
        vals = P.Layout(S, "soa")
        mem = []
        bufs = []
        for f in decl.fields:
            if f.group < 0:
                bufs.append(torch.randint(0, 256, (n * W.TYPE_SIZE[f.type] * f.extent,), dtype=torch.uint8,
                                          device="cuda", generator=g))
        if decl.offset_types:
            lens = torch.poisson(torch.full((n,), 40.0, device="cuda"), generator=g).to(torch.int64)
            offs = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
            offs[1:] = torch.cumsum(lens, 0)
            tot = int(offs[-1].item())
            mem = [tot]
            bufs.append(offs.to(torch.int32).view(torch.uint8))
            for f in decl.fields:
                if f.group >= 0:
                    bufs.append(torch.randint(0, 256, (tot * W.TYPE_SIZE[f.type],), dtype=torch.uint8,
                                              device="cuda", generator=g))
        vview = P.View(vals, n, bufs, mem)
        sk = kinds[it["src"]]
        if sk[0] == "soa":
            sview, slay = vview, vals
        else:
            slay = P.Layout(S, sk[0], width=sk[1])
            sbufs = [torch.empty(x, dtype=torch.uint8, device="cuda") for x in slay.buffer_bytes(n, mem)]
            sview = P.View(slay, n, sbufs, mem)
            P.convert(vview, sview, n)
        dk = kinds[it["dst"]]
        dlay = P.Layout(S, dk[0], width=0 if dk[0] == "aosoa" else 0, storage=narrow)
        dbufs = [torch.empty(x, dtype=torch.uint8, device="cuda") for x in dlay.buffer_bytes(n, mem)]
        dview = P.View(dlay, n, dbufs, mem)
        b.add(sview, dview, n)
        keep += [vview, sview, dview, slay, dlay]
        item_bytes.append((slay, dlay, n, mem))
    assert P.sync(stream) == 0, P.rl_last_error()
    t = time.perf_counter()
    b.finalize(sp)
    tune_s = time.perf_counter() - t
    # algorithmic bytes: source and destination footprints at the chosen widths
    total = 0
    for k, (slay, dlay, n, mem) in enumerate(item_bytes):
        total += sum(slay.buffer_bytes(n, mem))
        if dlay.kind == "aosoa":
            w = b.width(k)
            dl2 = P.Layout(dlay.schema, "aosoa", width=w, storage=None if dlay.storage is None else dlay.storage)
            total += sum(dl2.buffer_bytes(n, mem))
        else:
            total += sum(dlay.buffer_bytes(n, mem))
    res = {"items": len(specs), "objects": int(sum(s["n"] for s in specs)), "bytes": total,
           "shape": b.shape(), "finalize_s": round(tune_s, 2)}
    for mode in ("graph", "loop"):
        fn = b.launch if mode == "graph" else b.loop
        for _ in range(3):
            fn(sp)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record(stream)
        for _ in range(reps):
            fn(sp)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[mode] = {"ms": round(ms, 4), "GBps": round(total / (ms * 1e-3) / 1e9, 1),
                     "frac_hbm": round(total / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    assert P.sync(stream) == 0, P.rl_last_error()
    res["speedup"] = round(res["loop"]["ms"] / res["graph"]["ms"], 3)
    del keep, b
    torch.cuda.empty_cache()
    return res


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "rl_internal.h", "plan.cpp", "batch.cpp"):
        h.update(open(os.path.join(ROOT, "paper_2511_04853_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, n):
    """HBM bytes per launch of the dominant kernel from the committed
    FETCH_SIZE / WRITE_SIZE counter summary, scaled by the same counters on
    a plain copy of known size; None when the kernel source changed since
    the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel.split('::')[-1]}_cell190k_step.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("kernel") != kernel or t.get("source_hash") != kernel_source_hash() or t.get("objects") != n:
        return None
    return int(t["hbm_bytes_per_launch"])


def _time(fn, stream, torch, reps=50, warm=5):
    """Mean ms of `reps` back-to-back calls fn(k) between two events."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(reps):
        fn(k)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def event_times(fn, stream, torch, count):
    """fn(k) for k < count, an event pair around each call: the paper's
    statistic over the durations (mean of the 10 fastest, median), in us."""
    evs = [[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(count)]
    torch.cuda.synchronize()
    for k in range(count):
        evs[k][0].record(stream)
        fn(k)
        evs[k][1].record(stream)
    torch.cuda.synchronize()
    return paper_stat([e[0].elapsed_time(e[1]) * 1e3 for e in evs])


def paper_stat(us):
    """Mean of the 10 fastest of the runs, and the median (the case study's
    statistic: mean of the 10 fastest of 50 executions)."""
    a = sorted(us)
    return {"runs": len(a), "mean10_fastest_us": round(float(np.mean(a[:10])), 3),
            "median_us": round(float(np.median(a)), 3)}


def single_conversion(P, W, torch, stream, sets=32):
    """One conversion per launch: the cell collection (190,000 objects) from
    AoS records into SoA (energy_d narrowed) and into AoSoA(64), rotating 32
    copies (334 MB per kind, beyond the Infinity Cache)."""
    S = P.Schema(W.CELL)
    narrowed = ["f32" if f.type == "f64" else f.type for f in W.CELL.fields]
    aos = P.Layout(S, "aos")
    n = 190_000
    lib, sp = P.lib(), P.stream_ptr(stream)
    res = {"objects": n, "copies": sets}
    for name, L in (("soa", P.Layout(S, "soa", storage=narrowed)),
                    ("aosoa64", P.Layout(S, "aosoa", width=64, storage=narrowed))):
        pairs = []
        for _ in range(sets):
            src = torch.randint(0, 255, (aos.buffer_bytes(n)[0],), dtype=torch.uint8, device="cuda")
            dst = [torch.empty(b, dtype=torch.uint8, device="cuda") for b in L.buffer_bytes(n)]
            pairs.append((P.View(aos, n, [src]), P.View(L, n, dst)))
        nbytes = aos.buffer_bytes(n)[0] + sum(L.buffer_bytes(n))
        fn = lambda k=0: lib.rl_convert(pairs[k % sets][0].ref(), pairs[k % sets][1].ref(), n, sp)
        ms = _time(fn, stream, torch, reps=64, warm=4)
        iso = event_times(fn, stream, torch, 50)
        assert P.sync(stream) == 0, P.rl_last_error()
        res[name] = {"bytes": nbytes, "us_back_to_back": round(ms * 1e3, 3),
                     "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1),
                     "frac_hbm_algorithmic": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "isolated": iso}
        del pairs
    return res


def copy_peak(P, W, torch, stream):
    """The attainable HBM rate: the library's plain 16-byte vector copy
    kernel (rl_memcopy, device to device) over 1 GiB buffers, three pairs
    rotating (cold); and back-to-back copies of 16 bytes from Python."""
    size = 1 << 30
    a = [torch.empty(size, dtype=torch.uint8, device="cuda") for _ in range(3)]
    b = [torch.empty(size, dtype=torch.uint8, device="cuda") for _ in range(3)]
    for t in a:
        t.fill_(7)
    fn = lambda k=0: P.memcopy(b[k % 3], "device", a[k % 3], "device", size, stream)
    ms = _time(fn, stream, torch, reps=12, warm=3)
    res = {"bytes_per_copy": 2 * size, "us": round(ms * 1e3, 1),
           "GBps_read_plus_write": round(2 * size / (ms * 1e-3) / 1e9, 1),
           "frac_of_spec": round(2 * size / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    assert torch.equal(b[0][:4096], a[0][:4096])
    # back-to-back 16-byte copies issued from Python: bound by the host's
    # submission rate (ctypes call + launch), an upper bound of the floor
    small = lambda k=0: P.memcopy(b[0], "device", a[0], "device", 16, stream)
    res["submit_floor_us"] = round(_time(small, stream, torch, reps=200, warm=10) * 1e3, 3)
    del a, b
    return res


def plain_round_trip(P, W, torch, stream, sets=64):
    """10,000 objects of 8 mixed scalars: AoS -> SoA -> AoS on the device
    (two launches), rotating copies."""
    S = P.Schema(W.PLAIN8)
    aos, soa = P.Layout(S, "aos"), P.Layout(S, "soa")
    n = 10_000
    lib, sp = P.lib(), P.stream_ptr(stream)
    A = [P.View(aos, n, [torch.randint(0, 256, (aos.buffer_bytes(n)[0],), dtype=torch.uint8, device="cuda")])
         for _ in range(sets)]
    B = [P.View(soa, n, [torch.empty(b, dtype=torch.uint8, device="cuda") for b in soa.buffer_bytes(n)])
         for _ in range(sets)]
    C = [P.View(aos, n, [torch.empty(aos.buffer_bytes(n)[0], dtype=torch.uint8, device="cuda")]) for _ in range(sets)]

    def rt(k=0):
        lib.rl_convert(A[k % sets].ref(), B[k % sets].ref(), n, sp)
        lib.rl_convert(B[k % sets].ref(), C[k % sets].ref(), n, sp)

    ms = _time(rt, stream, torch)
    by = 2 * (aos.buffer_bytes(n)[0] + sum(soa.buffer_bytes(n)))
    assert P.sync(stream) == 0
    return {"objects": n, "us_per_round_trip": round(ms * 1e3, 2), "GBps": round(by / (ms * 1e-3) / 1e9, 1)}


def _shuffle_pool(torch, rec, pool, offs, n, stride, g):
    """The same collection with its member blocks in a random order in the
    pool: records' byte pointers updated (the pointer field is found as the
    8-byte slot holding 8 * offsets of the canonical pool)."""
    lens = offs[1:] - offs[:-1]
    tot = int(offs[-1].item())
    r = rec.view(n, stride)
    ptr_off = None
    for o in range(0, stride - 7, 8):
        if torch.equal(r[:, o:o + 8].contiguous().view(torch.int64).view(-1), offs[:-1] * 8):
            ptr_off = o
            break
    assert ptr_off is not None, "no pointer field in the records"
    order = torch.randperm(n, device="cuda", generator=g)
    start = torch.zeros(n, dtype=torch.int64, device="cuda")
    start[order] = torch.cumsum(lens[order], 0) - lens[order]
    owner = torch.repeat_interleave(torch.arange(n, device="cuda"), lens)
    j = torch.arange(tot, device="cuda") - offs[:-1][owner]
    new_pool = torch.empty_like(pool)
    new_pool.view(-1, 8)[start[owner] + j] = pool.view(-1, 8)[:tot]
    new_rec = rec.clone()
    new_rec.view(n, stride)[:, ptr_off:ptr_off + 8] = (start * 8).view(torch.uint8).view(n, 8)
    return new_rec, new_pool


def jagged(P, W, torch, stream, sets=8):
    """50,000 clusters with Poisson(40) (index, weight) members: AoS records
    + pool -> SoA + offsets (scan + gather), and back.  Forward from pools
    whose member blocks are shuffled, and from pools in object order."""
    S = P.Schema(W.CLUSTER)
    aos, soa = P.Layout(S, "aos"), P.Layout(S, "soa")
    n = 50_000
    lib, sp = P.lib(), P.stream_ptr(stream)
    g = torch.Generator(device="cuda")
    g.manual_seed(1002)
    vals, back = [], []
    for r in range(sets):
        lens = torch.poisson(torch.full((n,), 40.0, device="cuda"), generator=g).to(torch.int64)
        offs = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
        offs[1:] = torch.cumsum(lens, 0)
        tot = int(offs[-1].item())
        bufs = [torch.randint(0, 256, (4 * n,), dtype=torch.uint8, device="cuda", generator=g) for _ in range(6)]
        bufs.append(offs.to(torch.int32).view(torch.uint8))
        bufs += [torch.randint(0, 256, (4 * tot,), dtype=torch.uint8, device="cuda", generator=g) for _ in range(2)]
        sv = P.View(soa, n, bufs, [tot])
        av = P.View(aos, n, [torch.empty(x, dtype=torch.uint8, device="cuda") for x in aos.buffer_bytes(n, [tot])],
                    [tot])
        P.convert(sv, av, n)
        assert P.sync(stream) == 0
        rec_s, pool_s = _shuffle_pool(torch, av.tensors[0], av.tensors[1], offs, n,
                                      aos.buffer_bytes(1, [0])[0], g)
        avs = P.View(aos, n, [rec_s, pool_s], [tot])
        dv = P.View(soa, n, [torch.empty(x, dtype=torch.uint8, device="cuda") for x in soa.buffer_bytes(n, [tot])],
                    [tot])
        if r == 0:   # both pools give the same columns
            dv2 = P.View(soa, n, [torch.empty(x, dtype=torch.uint8, device="cuda")
                                  for x in soa.buffer_bytes(n, [tot])], [tot])
            P.convert(av, dv, n)
            P.convert(avs, dv2, n)
            assert P.sync(stream) == 0
            assert all(torch.equal(a, b) for a, b in zip(dv.tensors, dv2.tensors)), "shuffled pool differs"
            del dv2
        vals.append((av, dv, tot, avs))
    assert P.sync(stream) == 0
    fwd_s = _time(lambda k=0: lib.rl_convert(vals[k % sets][3].ref(), vals[k % sets][1].ref(), n, sp), stream, torch)
    fwd = _time(lambda k=0: lib.rl_convert(vals[k % sets][0].ref(), vals[k % sets][1].ref(), n, sp), stream, torch)
    rev = _time(lambda k=0: lib.rl_convert(vals[k % sets][1].ref(), vals[k % sets][0].ref(), n, sp), stream, torch)
    fwd_iso = event_times(lambda k=0: lib.rl_convert(vals[k % sets][3].ref(), vals[k % sets][1].ref(), n, sp),
                          stream, torch, 50)
    rev_iso = event_times(lambda k=0: lib.rl_convert(vals[k % sets][1].ref(), vals[k % sets][0].ref(), n, sp),
                          stream, torch, 50)
    assert P.sync(stream) == 0
    tot = int(np.mean([v[2] for v in vals]))
    by = sum(aos.buffer_bytes(n, [tot])) + sum(soa.buffer_bytes(n, [tot]))
    return {"objects": n, "members": tot, "bytes_each_way": by,
            "forward_isolated": fwd_iso, "reverse_isolated": rev_iso,
            "forward_shuffled_pool_us": round(fwd_s * 1e3, 2),
            "forward_shuffled_pool_GBps": round(by / (fwd_s * 1e-3) / 1e9, 1),
            "forward_us": round(fwd * 1e3, 2), "forward_GBps": round(by / (fwd * 1e-3) / 1e9, 1),
            "reverse_us": round(rev * 1e3, 2), "reverse_GBps": round(by / (rev * 1e-3) / 1e9, 1)}


def serving(P, W, torch, stream, rates=(1000, 3000), n_events=10_000, hold=512, pool_events=64, warmup=1000):
    """Open-loop Poisson arrivals; each event one collection per schema
    (plain / cell / cluster, log-normal sizes with medians 10k / 100k / 20k,
    sigma 0.5) in pinned host AoS memory; converted into device SoA under a
    16 GB budget; results held until 512 newer events are done."""
    import threading
    sys.setswitchinterval(2e-4)
    decls = [W.PLAIN8, W.CELL, W.CLUSTER]
    schemas = [P.Schema(d) for d in decls]
    src_l = [P.Layout(S, "aos", space="pinned") for S in schemas]
    dev_aos = [P.Layout(S, "aos") for S in schemas]
    dst_l = [P.Layout(S, "soa", storage=["f32" if f.type == "f64" else f.type for f in d.fields if f.group < 0]
                      if d is W.CELL else None) for S, d in zip(schemas, decls)]
    sizes = W.serving_events(pool_events)
    g = torch.Generator(device="cuda")
    g.manual_seed(1004)
    events = []
    for row in sizes:
        items = []
        for j, (S, d) in enumerate(zip(schemas, decls)):
            n = int(row[j])
            vals = P.Layout(S, "soa")
            bufs = [torch.randint(0, 256, (n * W.TYPE_SIZE[f.type],), dtype=torch.uint8, device="cuda",
                                  generator=g) for f in d.fields if f.group < 0]
            mem = []
            if d.offset_types:
                lens = torch.poisson(torch.full((n,), 40.0, device="cuda"), generator=g).to(torch.int64)
                offs = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
                offs[1:] = torch.cumsum(lens, 0)
                tot = int(offs[-1].item())
                mem = [tot]
                bufs.append(offs.to(torch.int32).view(torch.uint8))
                bufs += [torch.randint(0, 256, (tot * W.TYPE_SIZE[f.type],), dtype=torch.uint8, device="cuda",
                                       generator=g) for f in d.fields if f.group >= 0]
            if d is W.CELL:   # valid doubles in the narrowed field
                bufs[6] = (torch.rand(n, dtype=torch.float64, device="cuda", generator=g) * 1e3).view(torch.uint8)
            daos = [torch.empty(x, dtype=torch.uint8, device="cuda") for x in dev_aos[j].buffer_bytes(n, mem)]
            P.convert(P.View(vals, n, bufs, mem), P.View(dev_aos[j], n, daos, mem), n)
            pinned = [torch.empty(t.numel(), dtype=torch.uint8, pin_memory=True) for t in daos]
            for h_, t in zip(pinned, daos):
                h_.copy_(t)
            items.append((P.View(src_l[j], n, pinned, mem), dst_l[j], n))
        events.append(items)
    assert P.sync(stream) == 0
    torch.cuda.synchronize()
    ev_bytes = [sum(sum(v.layout.buffer_bytes(n, list(v._mcap)[:1] if v.layout.schema.n_groups else []))
                    for v, _, n in items) for items in events]
    res = {"event_pool": pool_events, "mean_event_h2d_MB": round(float(np.mean(ev_bytes)) / 1e6, 2),
           "budget_GiB": 16, "hold": hold, "warmup_events": warmup}
    # one server for the whole leg; a warm-up run first takes the first-use
    # costs (per-stream staging buffers, pool pages) out of the measurement
    srv = P.Server(16 << 30, max_in_flight=32, n_streams=8)

    def run(rate, count, seed):
        arrivals = W.poisson_arrivals(count, rate, seed=seed)
        tickets = [None] * count
        late = np.zeros(count)
        lat_ms = np.zeros(count)
        done_t = np.zeros(count)
        lock = threading.Lock()

        def producer():
            for k in range(count):
                while True:
                    dt = arrivals[k] - (time.perf_counter() - t0)
                    if dt <= 0:
                        break
                    if dt > 3e-4:
                        time.sleep(dt - 2e-4)
                t = srv.submit(events[k % pool_events])
                late[k] = (time.perf_counter() - t0) - arrivals[k]   # submit behind schedule
                with lock:
                    tickets[k] = t

        th = threading.Thread(target=producer)
        t0 = time.perf_counter()
        th.start()
        released = 0
        for k in range(count):
            while True:
                with lock:
                    t = tickets[k]
                if t is not None:
                    break
                time.sleep(0.0001)
            r = srv.wait(t)
            assert r["status"] == 0
            # latency from the scheduled arrival (open loop: a late submit counts)
            lat_ms[k] = r["latency_ns"] / 1e6 + late[k] * 1e3
            done_t[k] = arrivals[k] + lat_ms[k] / 1e3
            while released <= k - hold:
                srv.release(tickets[released])
                released += 1
        th.join()
        while released < count:
            srv.release(tickets[released])
            released += 1
        span = done_t.max() - arrivals[0]
        return {"events": count,
                "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
                "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
                "max_ms": round(float(lat_ms.max()), 3),
                "submit_late_p99_ms": round(float(np.percentile(late, 99)) * 1e3, 3),
                "events_per_s": round(count / span, 1),
                "link_GBps": round(count * float(np.mean(ev_bytes)) / span / 1e9, 2)}

    run(1000, warmup, seed=2004)   # warm-up (1 s at 1,000 events/s)
    for rate in rates:
        res[f"{rate}/s"] = run(rate, n_events, seed=1004 + rate)
    # offered load above the host link's rate: throughput saturates there
    # (latency then grows with the queue, so only the rates are reported)
    sat = run(6000, n_events, seed=1004 + 6000)
    res["saturation_offered_6000/s"] = {"events_per_s": sat["events_per_s"], "link_GBps": sat["link_GBps"]}
    st = srv.stats()
    res["peak_resident_GB"] = round(st["peak_bytes"] / 1e9, 3)
    srv.close()
    del srv
    torch.cuda.synchronize()

    # the baseline: a synchronous per-event loop on one stream, each event's
    # transfers enqueued and waited for before the next event starts (same
    # events, same arrival processes; results into preallocated buffers)
    loop_dst = []
    for items in events:
        outs = []
        for view, layout, n in items:
            mem = list(view._mcap)[:1] if view.layout.schema.n_groups else []
            outs.append(P.View(layout, n, [torch.empty(x, dtype=torch.uint8, device="cuda")
                                           for x in layout.buffer_bytes(n, mem)], mem))
        loop_dst.append(outs)

    def serve_one(k):
        for (view, layout, n), dv in zip(events[k % pool_events], loop_dst[k % pool_events]):
            P.transfer(view, dv, n, stream)
        assert P.sync(stream) == 0, P.rl_last_error()

    def loop_run(rate, count, seed):
        arrivals = W.poisson_arrivals(count, rate, seed=seed)
        lat_ms = np.zeros(count)
        t0 = time.perf_counter()
        for k in range(count):
            while True:
                dt = arrivals[k] - (time.perf_counter() - t0)
                if dt <= 0:
                    break
                if dt > 3e-4:
                    time.sleep(dt - 2e-4)
            serve_one(k)
            lat_ms[k] = ((time.perf_counter() - t0) - arrivals[k]) * 1e3
        span = (time.perf_counter() - t0) - arrivals[0]
        return {"events": count, "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
                "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
                "events_per_s": round(count / span, 1)}

    for k in range(min(200, n_events)):   # warm-up
        serve_one(k)
    loop = {}
    for rate in rates:
        loop[f"{rate}/s"] = loop_run(rate, min(3000, n_events), seed=3004 + rate)
    nb = min(3000, n_events)
    t = time.perf_counter()
    for k in range(nb):
        serve_one(k)
    loop["back_to_back"] = {"events": nb, "events_per_s": round(nb / (time.perf_counter() - t), 1)}
    res["per_event_loop"] = loop
    res["server_over_loop_throughput"] = round(res["saturation_offered_6000/s"]["events_per_s"] /
                                               loop["back_to_back"]["events_per_s"], 3)
    del loop_dst
    return res


def _cluster_device_collection(P, W, torch, n, g, aos, soa):
    """A cluster collection built on the device: Poisson(40) member counts,
    random field and member bits, as AoS records + canonical pool (returns
    the records view and the member total)."""
    lens = torch.poisson(torch.full((n,), 40.0, device="cuda"), generator=g).to(torch.int64)
    offs = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    offs[1:] = torch.cumsum(lens, 0)
    tot = int(offs[-1].item())
    bufs = [torch.randint(0, 256, (4 * n,), dtype=torch.uint8, device="cuda", generator=g) for _ in range(6)]
    bufs.append(offs.to(torch.int32).view(torch.uint8))
    bufs += [torch.randint(0, 256, (4 * tot,), dtype=torch.uint8, device="cuda", generator=g) for _ in range(2)]
    av = P.View(aos, n, [torch.empty(x, dtype=torch.uint8, device="cuda") for x in aos.buffer_bytes(n, [tot])], [tot])
    P.convert(P.View(soa, n, bufs, [tot]), av, n)
    return av, tot


def sweep(P, W, torch, stream, copies=4, schemas=("plain8", "cell"), sizes=(1 << 20, 1 << 22, 1 << 24, 1 << 25),
          jagged=True):
    """AoS records -> SoA at larger object counts, `copies` copies rotating
    (cold at every size): the plain schema (8 scalars) and the cell schema
    (energy_d narrowed) at 2^20 .. 2^25 objects, the cluster schema (jagged,
    Poisson(40) members) at 2^21; the library's plain copy kernel over the
    same bytes (half read, half written) beside each row."""
    res = {}
    lib, sp = P.lib(), P.stream_ptr(stream)

    def copy_rate(nbytes):
        half = nbytes // 2 // 16 * 16
        a = [torch.empty(half, dtype=torch.uint8, device="cuda") for _ in range(copies)]
        b = [torch.empty(half, dtype=torch.uint8, device="cuda") for _ in range(copies)]
        ms = _time(lambda k=0: P.memcopy(b[k % copies], "device", a[k % copies], "device", half, stream),
                   stream, torch, reps=12, warm=copies)
        return round(2 * half / (ms * 1e-3) / 1e9, 1)

    for sname, decl in (("plain8", W.PLAIN8), ("cell", W.CELL)):
        if sname not in schemas:
            continue
        S = P.Schema(decl)
        narrowed = ["f32" if f.type == "f64" else f.type for f in decl.fields] if decl is W.CELL else None
        aos = P.Layout(S, "aos")
        soa = P.Layout(S, "soa", storage=narrowed)
        for n in sizes:
            pairs = []
            for _ in range(copies):
                src = torch.randint(0, 255, (aos.buffer_bytes(n)[0],), dtype=torch.uint8, device="cuda")
                dst = [torch.empty(x, dtype=torch.uint8, device="cuda") for x in soa.buffer_bytes(n)]
                pairs.append((P.View(aos, n, [src]), P.View(soa, n, dst)))
            nbytes = aos.buffer_bytes(n)[0] + sum(soa.buffer_bytes(n))
            ms = _time(lambda k=0: lib.rl_convert(pairs[k % copies][0].ref(), pairs[k % copies][1].ref(), n, sp),
                       stream, torch, reps=12, warm=copies)
            assert P.sync(stream) == 0, P.rl_last_error()
            del pairs
            torch.cuda.empty_cache()
            gbs = nbytes / (ms * 1e-3) / 1e9
            cp = copy_rate(nbytes)
            res[f"{sname}/{n}"] = {"us": round(ms * 1e3, 2), "GBps": round(gbs, 1),
                                   "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "copy_kernel_GBps": cp,
                                   "frac_of_copy": round(gbs / cp, 4)}
            torch.cuda.empty_cache()
    if not jagged:
        return res
    # jagged: cluster records + pool -> SoA + offsets + member columns
    S = P.Schema(W.CLUSTER)
    aos, soa = P.Layout(S, "aos"), P.Layout(S, "soa")
    n = 1 << 21
    g = torch.Generator(device="cuda")
    g.manual_seed(1002)
    sets = []
    for _ in range(copies):
        av, tot = _cluster_device_collection(P, W, torch, n, g, aos, soa)
        dv = P.View(soa, n, [torch.empty(x, dtype=torch.uint8, device="cuda") for x in soa.buffer_bytes(n, [tot])],
                    [tot])
        sets.append((av, dv, tot))
    assert P.sync(stream) == 0
    ms = _time(lambda k=0: lib.rl_convert(sets[k % copies][0].ref(), sets[k % copies][1].ref(), n, sp),
               stream, torch, reps=12, warm=copies)
    assert P.sync(stream) == 0, P.rl_last_error()
    tot = int(np.mean([x[2] for x in sets]))
    nbytes = sum(aos.buffer_bytes(n, [tot])) + sum(soa.buffer_bytes(n, [tot]))
    del sets
    torch.cuda.empty_cache()
    gbs = nbytes / (ms * 1e-3) / 1e9
    cp = copy_rate(nbytes)
    res[f"cluster/{n}"] = {"members": tot, "us": round(ms * 1e3, 2), "GBps": round(gbs, 1),
                           "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "copy_kernel_GBps": cp,
                           "frac_of_copy": round(gbs / cp, 4)}
    torch.cuda.empty_cache()
    return res


def _wall(fn, torch, reps=20, warm=3, rounds=3):
    """Wall seconds per fn() call: `rounds` rounds of `reps` back-to-back
    calls, the device drained before and after each round; the fastest
    round's mean (one host stall inside a round would otherwise double a
    transfer of a hundred microseconds)."""
    for _ in range(warm):
        fn()
    best = float("inf")
    for _ in range(rounds):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        best = min(best, (time.perf_counter() - t) / reps)
    return best


def h2d(P, W, torch, stream):
    """Pinned host collections -> device layouts with conversion, PCIe
    included (never the headline): the cell collection (190,000 objects,
    6.08 MB of records) into SoA and AoSoA 32/64/128 (energy_d narrowed),
    staged (DMA copy + conversion) and zero-copy (the kernel reads host
    memory); the jagged cluster collection (50,000 records + pool); a plain
    pinned copy of the same bytes for the link rate."""
    res = {}
    S = P.Schema(W.CELL)
    narrowed = ["f32" if f.type == "f64" else f.type for f in W.CELL.fields]
    aos_h = P.Layout(S, "aos", space="pinned")
    n = 190_000
    host = torch.randint(0, 255, (aos_h.buffer_bytes(n)[0],), dtype=torch.uint8).pin_memory()
    raw = torch.empty(host.numel(), dtype=torch.uint8, device="cuda")
    dt = _wall(lambda: raw.copy_(host, non_blocking=True), torch)
    res["cell_plain_copy"] = {"bytes": host.numel(), "us": round(dt * 1e6, 1),
                              "link_GBps": round(host.numel() / dt / 1e9, 2)}
    for name, L in (("soa", P.Layout(S, "soa", storage=narrowed)),) + tuple(
            (f"aosoa{w}", P.Layout(S, "aosoa", width=w, storage=narrowed)) for w in (32, 64, 128)):
        dst = [torch.empty(b, dtype=torch.uint8, device="cuda") for b in L.buffer_bytes(n)]
        sv, dv = P.View(aos_h, n, [host]), P.View(L, n, dst)
        for mode in ("staged", "zero_copy"):
            dt = _wall(lambda: P.transfer(sv, dv, n, stream, mode=mode), torch)
            res[f"cell_{name}_{mode}"] = {"us": round(dt * 1e6, 1), "link_GBps": round(host.numel() / dt / 1e9, 2)}
    assert P.sync(stream) == 0, P.rl_last_error()
    # jagged
    S = P.Schema(W.CLUSTER)
    aos, soa, aos_hj = P.Layout(S, "aos"), P.Layout(S, "soa"), P.Layout(S, "aos", space="pinned")
    g = torch.Generator(device="cuda")
    g.manual_seed(1002)
    m = 50_000
    av, tot = _cluster_device_collection(P, W, torch, m, g, aos, soa)
    assert P.sync(stream) == 0
    hbufs = [t.cpu().pin_memory() for t in av.tensors]
    hv = P.View(aos_hj, m, hbufs, [tot])
    dv = P.View(soa, m, [torch.empty(x, dtype=torch.uint8, device="cuda") for x in soa.buffer_bytes(m, [tot])], [tot])
    hb = sum(t.numel() for t in hbufs)
    for mode in ("staged", "zero_copy"):
        dt = _wall(lambda: P.transfer(hv, dv, m, stream, mode=mode), torch)
        res[f"cluster_soa_{mode}"] = {"host_bytes": hb, "us": round(dt * 1e6, 1), "link_GBps": round(hb / dt / 1e9, 2)}
    assert P.sync(stream) == 0, P.rl_last_error()
    return res


def d2h(P, W, torch, stream):
    """Device collections -> pinned host records with conversion, PCIe
    included: the cell collection from SoA (energy_d narrowed) back into
    the original AoS records (energy_d widened to f64), and the cluster
    collection from SoA + offsets into records + a canonical pool; staged
    (conversion into device staging + DMA copy) and zero-copy (the kernel
    writes host memory); a plain device -> pinned copy for the link rate."""
    res = {}
    S = P.Schema(W.CELL)
    narrowed = ["f32" if f.type == "f64" else f.type for f in W.CELL.fields]
    soa = P.Layout(S, "soa", storage=narrowed)
    aos_h = P.Layout(S, "aos", space="pinned")
    n = 190_000
    src = [torch.randint(0, 255, (b,), dtype=torch.uint8, device="cuda") for b in soa.buffer_bytes(n)]
    src[6] = (torch.rand(n, device="cuda") * 1e3).view(torch.uint8)   # valid floats to widen
    host = torch.empty(aos_h.buffer_bytes(n)[0], dtype=torch.uint8).pin_memory()
    raw = torch.empty(host.numel(), dtype=torch.uint8, device="cuda")
    dt = _wall(lambda: host.copy_(raw, non_blocking=True), torch)
    res["cell_plain_copy"] = {"bytes": host.numel(), "us": round(dt * 1e6, 1),
                              "link_GBps": round(host.numel() / dt / 1e9, 2)}
    sv, hv = P.View(soa, n, src), P.View(aos_h, n, [host])
    for mode in ("staged", "zero_copy"):
        dt = _wall(lambda: P.transfer(sv, hv, n, stream, mode=mode), torch)
        res[f"cell_aos_{mode}"] = {"us": round(dt * 1e6, 1), "link_GBps": round(host.numel() / dt / 1e9, 2)}
    assert P.sync(stream) == 0, P.rl_last_error()
    S = P.Schema(W.CLUSTER)
    aos, soa, aos_hj = P.Layout(S, "aos"), P.Layout(S, "soa"), P.Layout(S, "aos", space="pinned")
    g = torch.Generator(device="cuda")
    g.manual_seed(1002)
    m = 50_000
    av, tot = _cluster_device_collection(P, W, torch, m, g, aos, soa)
    dv = P.View(soa, m, [torch.empty(x, dtype=torch.uint8, device="cuda") for x in soa.buffer_bytes(m, [tot])], [tot])
    P.convert(av, dv, m)
    assert P.sync(stream) == 0
    hbufs = [torch.empty(x, dtype=torch.uint8).pin_memory() for x in aos_hj.buffer_bytes(m, [tot])]
    hv = P.View(aos_hj, m, hbufs, [tot])
    hb = sum(t.numel() for t in hbufs)
    for mode in ("staged", "zero_copy"):
        dt = _wall(lambda: P.transfer(dv, hv, m, stream, mode=mode), torch)
        res[f"cluster_aos_{mode}"] = {"host_bytes": hb, "us": round(dt * 1e6, 1), "link_GBps": round(hb / dt / 1e9, 2)}
    assert P.sync(stream) == 0, P.rl_last_error()
    return res


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    """Host threads to time the oracle on: the CPUs this process may use,
    at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(W, v, seconds, step_bytes):
    """The oracle (plain C per-object loop) on the benchmark step (the four
    conversions of the cell collection), buffers prepared once: on one host
    thread, and split into contiguous object ranges on all host threads
    (same loop body).  50 runs each (fewer if a run is long), the paper's
    statistic over them; value = algorithmic bytes / mean of the 10 fastest."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    S = oracle.Schema(W.CELL)
    narrowed = ["f32" if t == "f64" else t for t in S.leaf_types()]
    aos = oracle.make_layout(S, "aos")
    dsts = [oracle.make_layout(S, "soa", storage=narrowed)] + [
        oracle.make_layout(S, "aosoa", width=w, storage=narrowed) for w in WIDTHS]
    src = oracle.pack(S, v, aos)
    preps = [oracle.Prepared(aos, src, d, v.n) for d in dsts]
    threads = host_threads()
    pool = ThreadPoolExecutor(threads)
    out = {}
    for label, th in (("one_thread", 1), ("all_threads", threads)):
        times = []
        t_end = time.perf_counter() + seconds / 2
        while len(times) < 50 and (len(times) < 10 or time.perf_counter() < t_end):
            t = time.perf_counter()
            for p_ in preps:
                assert p_.run(th, pool) == 0
            times.append((time.perf_counter() - t) * 1e6)
        st = paper_stat(times)
        out[label] = {"threads": th, **st, "GBps": round(step_bytes / (st["mean10_fastest_us"] * 1e-6) / 1e9, 3)}
    pool.shutdown()
    best = out["all_threads"]
    return {"value": best["GBps"], "unit": "GB/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"the benchmark step (190,000 cell objects into SoA and AoSoA 32/64/128, energy_d narrowed), "
                      f"{best['runs']} runs on {threads} host threads (contiguous object ranges), "
                      f"mean of the 10 fastest {best['mean10_fastest_us'] / 1e3:.2f} ms per step; "
                      f"one thread: {out['one_thread']['GBps']} GB/s",
            "detail": out}


def cpu_events(P, W, torch, stream, seconds=8.0):
    """Serving workload on the host cores: the oracle converts whole events
    (one plain, one cell and one cluster collection of log-normal sizes,
    records -> SoA, energy_d narrowed), one event per host thread at a time,
    no transfer; events per second."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    decls = [W.PLAIN8, W.CELL, W.CLUSTER]
    schemas = [oracle.Schema(d) for d in decls]
    srcs = [oracle.make_layout(S, "aos") for S in schemas]
    dsts = [oracle.make_layout(S, "soa", storage=(["f32" if t == "f64" else t for t in S.leaf_types()]
                                                  if d is W.CELL else None)) for S, d in zip(schemas, decls)]
    sizes = W.serving_events(16)
    events = []
    for k, row in enumerate(sizes):
        items = []
        for j, (S, d) in enumerate(zip(schemas, decls)):
            n = int(row[j])
            vals = (W.plain_values(n, seed=5000 + k) if d is W.PLAIN8 else
                    W.cell_values(n, seed=5000 + k) if d is W.CELL else W.cluster_values(n, seed=5000 + k))
            items.append((srcs[j], oracle.pack(S, vals, srcs[j]), dsts[j], n,
                          [vals.total(0)] if d.offset_types else []))
        events.append(items)

    def convert_event(items):
        for sl, sb, dl, n, mem in items:
            st, _, _ = oracle.convert(sl, sb, dl, n, mem, mem)
            assert st == 0

    threads = host_threads()
    with ThreadPoolExecutor(threads) as pool:
        list(pool.map(convert_event, events[:threads]))   # warm-up
        done = 0
        t = time.perf_counter()
        while time.perf_counter() - t < seconds:
            list(pool.map(convert_event, [events[(done + i) % len(events)] for i in range(threads * 4)]))
            done += threads * 4
        dt = time.perf_counter() - t
    return {"events_per_s": round(done / dt, 1), "threads": threads, "cpu_model": cpu_model(), "events": done}


def pipeline(P, W, torch, stream):
    """The case study's two pipelines (stand-in arithmetic, the paper's
    statistic over the runs): sensors filled on the host, transferred into
    device SoA with the conversion and calibrated, against the grid size;
    particles reconstructed on a 5,000 x 5,000 grid and transferred back
    into the original records + member pool, against the particle count.
    Reported: each stage's time and the share of transfer + conversion."""
    import workloads.case_study as C
    res = {"sensors": {}, "particles": {}}
    # untimed warm-up of both pipelines (first calls load the stand-ins'
    # device code)
    C.sensor_pipeline(P, torch, 60, C.sensor_grid(60, seed=1), stream, reps=2)
    for side in (100, 300, 1000, 3000, 5000):
        v = C.sensor_grid(side, seed=side)
        reps = 10 if side <= 1000 else 4
        runs, host, cols, typed = C.sensor_pipeline(P, torch, side, v, stream, reps=reps)
        row = {k: paper_stat([r[k] * 1e3 for r in runs])["mean10_fastest_us"] for k in ("fill", "h2d_convert", "energy")}
        tot = sum(row.values())
        res["sensors"][f"{side}x{side}"] = {**{k + "_us": v_ for k, v_ in row.items()},
                                            "transfer_convert_share": round(row["h2d_convert"] / tot, 3)}
        if side != 5000:
            del host, cols, typed
            torch.cuda.empty_cache()
    C.particle_pipeline(P, torch, 5000, C.seed_sensors(5000, 50, seed=1), typed, stream, reps=2)
    for npart in (100, 1_000, 10_000, 100_000):
        seeds = C.seed_sensors(5000, npart, seed=npart)
        runs, dbufs, hbufs = C.particle_pipeline(P, torch, 5000, seeds, typed, stream, reps=6)
        row = {k: paper_stat([r[k] * 1e3 for r in runs])["mean10_fastest_us"] for k in ("reconstruct", "d2h_convert")}
        res["particles"][str(npart)] = {**{k + "_us": v_ for k, v_ in row.items()},
                                        "members": runs[-1]["members"],
                                        "transfer_convert_share": round(row["d2h_convert"] / sum(row.values()), 3)}
    assert P.sync(stream) == 0, P.rl_last_error()
    return res


def pairs(P, W, torch, stream, copies=4, n=1 << 24):
    """Every ordered pair of layout kinds (AoS, SoA, AoSoA(64)) for the plain
    and cell schemas at 2^24 objects, `copies` copies rotating (cold), each
    against the copy kernel over the same bytes."""
    res = {}
    lib, sp = P.lib(), P.stream_ptr(stream)
    kinds = (("aos", 0), ("soa", 0), ("aosoa", 64))
    for sname, decl in (("plain8", W.PLAIN8), ("cell", W.CELL)):
        S = P.Schema(decl)
        for sk in kinds:
            for dk in kinds:
                if sk == dk:
                    continue
                sl, dl = P.Layout(S, sk[0], width=sk[1]), P.Layout(S, dk[0], width=dk[1])
                views = []
                for _ in range(copies):
                    src = [torch.randint(0, 255, (b,), dtype=torch.uint8, device="cuda") for b in sl.buffer_bytes(n)]
                    dst = [torch.empty(b, dtype=torch.uint8, device="cuda") for b in dl.buffer_bytes(n)]
                    views.append((P.View(sl, n, src), P.View(dl, n, dst)))
                nbytes = sum(sl.buffer_bytes(n)) + sum(dl.buffer_bytes(n))
                ms = _time(lambda k=0: lib.rl_convert(views[k % copies][0].ref(), views[k % copies][1].ref(), n, sp),
                           stream, torch, reps=12, warm=copies)
                assert P.sync(stream) == 0, P.rl_last_error()
                del views
                torch.cuda.empty_cache()
                gbs = nbytes / (ms * 1e-3) / 1e9
                res[f"{sname}/{sk[0]}->{dk[0]}"] = {"us": round(ms * 1e3, 2), "GBps": round(gbs, 1),
                                                    "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    return res


LEGS = {
    "single_conversion": single_conversion,
    "pairs": pairs,
    "copy_peak": copy_peak,
    "round_trip": lambda P, W, torch, stream: plain_round_trip(P, W, torch, stream),
    "jagged": jagged,
    "batched": lambda P, W, torch, stream: batched(
        P, W, torch, stream, os.path.join(os.environ.get("TMPDIR", "/tmp"), f"rl_tune_{os.getpid()}.json")),
    "sweep": sweep,
    "h2d": h2d,
    "d2h": d2h,
    "serving": lambda P, W, torch, stream: serving(P, W, torch, stream, n_events=SERVING_EVENTS[0],
                                                   warmup=min(1000, SERVING_EVENTS[0])),
    "cpu_events": cpu_events,
    "pipeline": pipeline,
    # one sweep row alone (cell AoS -> SoA at 2^24 objects), for its counters
    "sweep_cell_2_24": lambda P, W, torch, stream: sweep(P, W, torch, stream, schemas=("cell",), sizes=(1 << 24,),
                                                         jagged=False),
}
EXTRA_ORDER = ["single_conversion", "copy_peak", "round_trip", "jagged", "batched", "sweep", "pairs", "h2d", "d2h",
               "pipeline", "serving", "cpu_events"]


if __name__ == "__main__":
    main()
