"""Benchmark: slice-based ray-casting volume illumination on one MI355X.

One step = the whole hot path for one light direction of the orbit: the
attenuation build (section 3.2.1) followed by a shell frame and a cone frame
(sections 3.2.2-3.2.3), 1920x1080, on the 512^3 u16 phantom with 512 slices
of 1024^2 (the light moves every step, so every step rebuilds the stack).
Inputs are resident in HBM before timing starts.

Prints ONE JSON line on stdout; progress goes to stderr.

    python bench.py [--steps 16] [--warmup 2] [--workload large]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

# Hardware counters of a kernel on a workload, from rocprofv3 --pmc runs of
# this bench (one counter set per run; commands and raw figures: profiles/).
# HBM bytes per launch are FETCH_SIZE and WRITE_SIZE (KiB per dispatch)
# scaled by what the same counters read for a plain 1 GiB device copy (bench.py
# --copy-probe 1024: FETCH_SIZE reads half the bytes copied, WRITE_SIZE all of
# them).  valu_insts (SQ_INSTS_VALU, wave instructions) and gui_cycles
# (GRBM_GUI_ACTIVE summed over the 8 XCDs) give the VALU issue fraction: a
# wave64 instruction occupies one of the 1024 SIMDs for 4 cycles (16 lanes per
# cycle; packed FP32 is not used).  ta_busy (TA_TA_BUSY_sum over the 256
# address units) gives the vector-memory address unit's busy fraction.  Each
# entry holds the sha256 of the sources the kernel is built from when the
# counters were taken; once those change the entry no longer applies and the
# bench reports the figures as null.
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
N_SIMDS, N_TAS, N_XCDS = 1024, 256, 8
# (vi_api.hip fixes the stack layout both kernels address)
KERNEL_SOURCES = {"render": ["vi_render.hip", "vi_device.h", "vi_internal.h", "vi_api.hip"],
                  "build": ["vi_build.hip", "vi_device.h", "vi_internal.h", "vi_api.hip"]}
MEASURED = {
    # large workload (512^3 u16 in the quad layout, 16^3 empty-space cells with occupancy bits, 512 x
    # 1024^2 f32 stack in rows, 1920x1080), mean of the three launches of bench --steps 2 --warmup 1
    # (lights 0, 0, 1); per launch: FETCH_SIZE / WRITE_SIZE in KiB, SQ_INSTS_VALU, GRBM_GUI_ACTIVE
    # (summed over the 8 XCDs), TA_TA_BUSY_sum and the other SQ counters of the same passes
    ("build", "large", "rows", 16, "quads"): {"sha256": "0980c39b73478c21f25a7a99b84b31e2b5d5b0ead1a7c3475945d33b70f10cbc", "fetch_kib": 292007.8, "write_kib": 2123952.4, "valu_insts": 164526486, "gui_cycles": 12876287, "ta_busy": 262863551, "vmem_rd": 1226619, "vmem_wr": 8487682, "waves": 16896, "wave_cycles": 2859996056, "busy_cycles": 49613123, "wait_inst_any": 632566836, "lds_insts": 15502698, "salu_insts": 107482245, "tcp_accesses": 66858631, "tcc_read_req": 14678032, "tcc_hit": 26952260, "tcc_miss": 21715285},
    ("render_shell", "large", "rows", 16, "quads"): {"sha256": "5a6bcb811cd3c707a1697f9d9ecf6e4f2ec0176bf83397d7ce1c9b0f1a9a7533", "fetch_kib": 108693.1, "write_kib": 33384.4, "valu_insts": 511498181, "gui_cycles": 20077457, "ta_busy": 366366152, "vmem_rd": 17659382, "vmem_wr": 148647, "waves": 130560, "wave_cycles": 2432241094, "busy_cycles": 71808189, "wait_inst_any": 363795259, "lds_insts": 16872411, "salu_insts": 116374954, "tcp_accesses": 448494575, "tcc_read_req": 26169923, "tcc_hit": 24717088, "tcc_miss": 2018113},
    ("render_cone", "large", "rows", 16, "quads"): {"sha256": "5a6bcb811cd3c707a1697f9d9ecf6e4f2ec0176bf83397d7ce1c9b0f1a9a7533", "fetch_kib": 120562.9, "write_kib": 33482.7, "valu_insts": 561198279, "gui_cycles": 22652654, "ta_busy": 448381787, "vmem_rd": 22669024, "vmem_wr": 148647, "waves": 130560, "wave_cycles": 2284903712, "busy_cycles": 78246335, "wait_inst_any": 533830761, "lds_insts": 16872411, "salu_insts": 138693131, "tcp_accesses": 579402332, "tcc_read_req": 40094574, "tcc_hit": 38450642, "tcc_miss": 2210050},
}


# The L2 probe (bench.py --l2-probe 2048: libvi_probe.so reads a 2 MiB buffer,
# resident in every XCD's L2, 4 GiB over): per launch TCP_TCC_READ_REQ_sum (L1
# to L2 read requests) and GRBM_GUI_ACTIVE from a rocprofv3 --pmc run, and the
# HIP-event read rate.  The frames' L1 -> L2 read requests per second are
# quoted against the probe's, counted the same way (requests, not bytes, so no
# request size is assumed).
L2_PROBE = {"buffer_bytes": 2097152, "bytes_read": 4294967296, "tcc_read_req": 19846548, "gui_cycles": 2447567,
            "gbs": 28312.1}
CLOCK_HZ = 2.4e9


def l2_roof(r, ms):
    """L1 -> L2 read requests of a recorded launch against the L2 probe's rate."""
    if not r or "tcc_read_req" not in r:
        return None
    probe_rate = L2_PROBE["tcc_read_req"] / (L2_PROBE["gui_cycles"] / N_XCDS / CLOCK_HZ)
    rate = r["tcc_read_req"] / (ms * 1e-3)
    return {"read_requests": r["tcc_read_req"], "achieved_greq_per_s": round(rate / 1e9, 2),
            "probe_greq_per_s": round(probe_rate / 1e9, 2), "frac": round(rate / probe_rate, 4),
            "hit_frac": round(r["tcc_hit"] / max(1, r["tcc_hit"] + r["tcc_miss"]), 4),
            "probe_read_gbs": L2_PROBE["gbs"]}


def source_sha(kind: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_2008_06134_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured(kernel: str, workload: str, layout: str, cell: int, vol_layout: str):
    """Recorded counters of `kernel` on `workload` for the current sources, or None."""
    m = MEASURED.get((kernel, workload, layout, cell, vol_layout))
    kind = "build" if kernel == "build" else "render"
    if not m or m["sha256"] != source_sha(kind):
        return None
    return m


def traffic_bytes(m) -> int | None:
    if not m:
        return None
    return int(m["fetch_kib"] * 1024 * FETCH_SCALE + m["write_kib"] * 1024 * WRITE_SCALE)


# Algorithmic FP32 operations of the method per composited segment (one with
# non-zero opacity; an FMA counts 2): its position (6), the trilinear fetch
# (8 normalisations, 7 lerps: 29), the transfer function (14), the Eq. 6
# opacity correction (4), the emission (21) and the front-to-back update (9)
# = 83, plus the coefficient gather: the sample's light-grid coordinates (6)
# and per tap its offset and a depth-linear bilinear lookup (24 for a shell
# or the shadow tap, 32 for a ring-cone tap, 30 for a lattice tap) and its
# weighting.  Skipped segments cost no arithmetic of the method.
FLOPS_PER_SAMPLE = {"none": 83, "shadow": 83 + 6 + 24, "shell": 83 + 6 + 6 * 24 + 12,
                    "cone": 83 + 6 + 8 * 32 + 9, "cone5": 83 + 6 + 25 * 30 + 26, "phong": 83 + 6 * 29 + 40}
FP32_PEAK_TFLOPS = 157.3   # MI355X vector FP32, published (packed FP32; 78.6 without packing)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, raw, tab, light, cam, modes, opts, stride, nthreads=0):
    """The FP64 oracle timed on the host cores on one step of the same workload:
    the full attenuation build, then the step's frames on a stratified pixel
    sample (every `stride`-th row and column); the frame time is scaled up by
    the sampled fraction.  Rate = step samples / step time.  Beside it, one
    thread on the small workload (its whole step) and on a sample of the
    medium one."""
    from oracle import oracle as O
    ovol, otf = O.Volume(raw), O.TF(tab)
    Wd, Hd = cam["width"], cam["height"]
    ys, xs = np.meshgrid(np.arange(stride // 2, Hd, stride), np.arange(stride // 2, Wd, stride), indexing="ij")
    pix = (ys * Wd + xs).ravel().astype(np.int64)
    frac = pix.size / (Wd * Hd)
    st = O.Stack(ovol, otf, light, w.n_slices, w.res)
    t0 = time.perf_counter()
    st.fill(nthreads)
    t_build = time.perf_counter() - t0
    samples = 0
    t0 = time.perf_counter()
    for m in modes:
        mm, extra = (m, {}) if m != "cone5" else ("cone", {"cone_grid": 5})
        _, _, nt, _ = O.render(ovol, otf, st, cam, mm, w.step_vox, {**opts, **extra}, pixels=pix,
                               want_full=False, nthreads=nthreads)
        samples += int(nt.sum())
    t_render = time.perf_counter() - t0
    step_time = t_build + t_render / frac
    return {"value": round(samples / frac / step_time, 1), "unit": "samples/s", "cores": O.threads(),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": (f"light 0 of the large workload: full FP64 build of {w.res}^2 columns x {w.n_slices} slabs "
                       f"in {t_build * 1e3:.0f} ms, then the {'+'.join(modes)} frames on {pix.size} of {Wd * Hd} "
                       f"pixels (every {stride}th row and column, {samples} samples) in {t_render * 1e3:.0f} ms; "
                       f"the frame time is scaled by 1/{frac:.3f}: {step_time * 1e3:.0f} ms per step"),
            "build_ms": round(t_build * 1e3, 1), "frames_ms_sampled": round(t_render * 1e3, 1),
            "single_thread": single_thread_baselines()}


def single_thread_baselines():
    """The oracle on one thread: the small workload's whole step (build + shell
    frame, 256^2) and the medium workload's build plus its cone 5x5 frame on
    every 8th row and column (scaled up)."""
    from oracle import oracle as O
    from paper_2008_06134_amd import workloads as W
    out = {}
    for name, stride in (("small", 1), ("medium", 8)):
        w = W.WORKLOADS[name]
        raw, tab = w.volume(), w.tf()
        ovol, otf = O.Volume(raw), O.TF(tab)
        cam = w.camera()
        Wd, Hd = cam["width"], cam["height"]
        ys, xs = np.meshgrid(np.arange(stride // 2, Hd, stride), np.arange(stride // 2, Wd, stride), indexing="ij")
        pix = (ys * Wd + xs).ravel().astype(np.int64)
        frac = pix.size / (Wd * Hd)
        st = O.Stack(ovol, otf, w.lights()[0], w.n_slices, w.res)
        t0 = time.perf_counter()
        st.fill(1)
        tb = time.perf_counter() - t0
        mode = w.modes[0]
        t0 = time.perf_counter()
        _, _, nt, _ = O.render(ovol, otf, st, cam, mode, w.step_vox, w.opts, pixels=pix, want_full=False, nthreads=1)
        tr = time.perf_counter() - t0
        n = int(nt.sum()) / frac
        step = tb + tr / frac
        out[name] = {"build_ms": round(tb * 1e3, 1), "frame_ms": round(tr / frac * 1e3, 1),
                     "samples_per_s": round(n / step, 1),
                     "frame_sample": f"{pix.size} of {Wd * Hd} pixels" + ("" if stride == 1 else ", scaled")}
    return out


# ---------------------------------------------------------------------------
# serving: continuous batching vs sequential plain renders, Poisson arrivals
# ---------------------------------------------------------------------------

# stack layout of every stack the bench builds (0 tiled, 1 rows; --stack-layout)
STACK_LAYOUT = 1


def _outputs(reqs, dev, per_size=8):
    """A small ring of output images per image size (the bench never reads them)."""
    import torch
    rings, outs = {}, []
    for r in reqs:
        key = (r["cam"]["height"], r["cam"]["width"])
        ring = rings.setdefault(key, {"bufs": [], "i": 0})
        if len(ring["bufs"]) < per_size:
            ring["bufs"].append(torch.empty((*key, 4), dtype=torch.float32, device=dev))
        outs.append(ring["bufs"][ring["i"] % len(ring["bufs"])])
        ring["i"] += 1
    return outs


def serve(vols, reqs, budget, max_inflight=16, tiles=8192, dev="cuda:0"):
    """Submit `reqs` at their arrival times to the continuous-batching server."""
    import torch
    from paper_2008_06134_amd import vi
    srv = vi.Server(budget, max_inflight, tiles)
    ids = [srv.register(v, tf) for v, tf in vols]
    outs = _outputs(reqs, dev)
    torch.cuda.synchronize()
    tickets = []
    t0 = time.perf_counter()
    for r, o in zip(reqs, outs):
        dt = t0 + r["arrival"] - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        t, _ = srv.submit(ids[r["vol"]], r["light"], r["n"], r["res"], r["cam"], r["mode"], 0.5, out=o,
                          layout=STACK_LAYOUT)
        tickets.append(t)
    for t in tickets:
        rc = srv.wait(t)
        if rc != 0:
            raise RuntimeError(f"request failed with {rc}")
    st = srv.stats()
    srv.close()
    return {"p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
            "frames_per_s": round(st["frames_per_s"], 2), "stack_hits": st["stack_hits"],
            "stack_builds": st["stack_builds"], "evictions": st["evictions"],
            "frames_per_launch": round(st["mean_frames_per_launch"], 2)}


def sequential(vols, reqs, budget, reuse=True, dev="cuda:0"):
    """The plain per-frame renderer, one request at a time in arrival order, with
    the same resident volumes and (if `reuse`) an LRU stack cache of `budget` bytes."""
    import collections
    import torch
    from paper_2008_06134_amd import vi
    outs = _outputs(reqs, dev)
    cache, used = collections.OrderedDict(), 0
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r, o in zip(reqs, outs):
        arrival = t0 + r["arrival"]
        dt = arrival - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        v, tf = vols[r["vol"]]
        key = (r["vol"], tuple(r["light"]), r["n"], r["res"])
        st = cache.get(key) if reuse else None
        if st is not None:
            cache.move_to_end(key)
        else:
            need = vi.slices_bytes(r["n"], r["res"], vi.VI_F32, STACK_LAYOUT)
            while reuse and cache and used + need > budget:
                _, old = cache.popitem(last=False)
                used -= vi.slices_bytes(old.n, old.res, vi.VI_F32, STACK_LAYOUT)
            st = vi.build_attenuation(v, tf, r["light"], r["n"], r["res"], layout=STACK_LAYOUT)
            if reuse:
                cache[key] = st
                used += need
        vi.render(v, tf, st, r["cam"], r["mode"], 0.5, out=o)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - arrival) * 1e3)
    span = time.perf_counter() - t0 - reqs[0]["arrival"]
    lat = np.array(lat)
    return {"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "frames_per_s": round(len(reqs) / span, 2)}


def serving_inputs(vol_sizes, dev, vessels=True):
    from paper_2008_06134_amd import vi
    from paper_2008_06134_amd import workloads as W
    tab = W.tf_ct()
    vols = []
    for i, N in enumerate(vol_sizes):
        raw = W.serving_volume(N, i, vessels=vessels)
        tf = vi.TF.from_numpy(tab, dev)
        vols.append((vi.Volume.from_numpy(raw, dev).to_quads().with_minmax(16).with_occupancy(tf), tf))
        if len(vol_sizes) > 16 and i % 8 == 7:
            log(f"{i + 1} of {len(vol_sizes)} serving volumes resident")
    return vols


def serving_capacity(vols, vol_sizes, budget, count=200, seed=99):
    """Sequential plain renders back to back (all requests present at t=0): frames/s."""
    from paper_2008_06134_amd import workloads as W
    reqs = W.serving_requests(count, vol_sizes, 1e9, seed=seed)
    for r in reqs:
        r["arrival"] = 0.0
    sequential(vols, reqs[:20], budget)          # warm-up
    return sequential(vols, reqs, budget)["frames_per_s"]


def serving_quick(dev, budget=24 << 30, count=300):
    """The default bench's serving leg, on inputs of the serving configuration:
    8 resident u16 phantoms 128^3-512^3 with vessels, images 512^2-1920x1080,
    shell/cone 50/50, lights changing every 1-10 frames; Poisson arrivals at
    0.9x and 1.2x the sequential capacity, against sequential plain renders."""
    from paper_2008_06134_amd import workloads as W
    sizes = [128, 192, 256, 320, 384, 448, 512, 256]
    vols = serving_inputs(sizes, dev, vessels=True)
    cap = serving_capacity(vols, sizes, budget)
    out = {"volumes": "8 resident u16 phantoms 128^3-512^3 with vessels (quad layout + empty-space map + "
                      "occupancy bits)", "requests_per_rate": count, "sequential_capacity_fps": cap, "rates": []}
    for f in (0.9, 1.2):
        reqs = W.serving_requests(count, sizes, f * cap, seed=5 + int(10 * f))
        serve(vols, reqs[:30], budget)                 # warm-up
        out["rates"].append({"rate_x": f, "rate_hz": round(f * cap, 2), "served": serve(vols, reqs, budget),
                             "sequential": sequential(vols, reqs, budget)})
    return out


def serving_sweep(dev, budget=48 << 30, count=2000, rates=(0.25, 0.5, 0.75, 0.9, 1.0, 1.2)):
    from paper_2008_06134_amd import workloads as W
    sizes = W.serving_volume_sizes(64)
    t0 = time.perf_counter()
    vols = serving_inputs(sizes, dev)
    log(f"64 serving volumes generated in {time.perf_counter() - t0:.0f} s")
    cap = serving_capacity(vols, sizes, budget)
    log(f"sequential capacity {cap:.1f} frames/s")
    rows = []
    for f in rates:
        reqs = W.serving_requests(count, sizes, f * cap, seed=int(100 * f))
        row = {"rate_x": f, "rate_hz": round(f * cap, 2), "served": serve(vols, reqs, budget),
               "sequential": sequential(vols, reqs, budget),
               "sequential_no_reuse": sequential(vols, reqs, budget, reuse=False)}
        log(json.dumps(row))
        rows.append(row)
    return {"volumes": 64, "volume_edges": sizes, "requests_per_rate": count, "capacity_fps": cap, "rows": rows}


def scaling_sweep(dev, slices=(64, 128, 256, 512), resolutions=(128, 256, 512, 1024), reps=5):
    """Build and frame times over slab count x slice resolution on the large workload
    (light 0, its camera), each the mean of `reps` HIP-event timed launches."""
    import torch
    from paper_2008_06134_amd import vi
    from paper_2008_06134_amd import workloads as W
    w = W.WORKLOADS["large"]
    raw, tab = w.volume(), w.tf()
    tf = vi.TF.from_numpy(tab, dev)
    vol = vi.Volume.from_numpy(raw, dev).to_quads().with_minmax(16).with_occupancy(tf)
    light, cam = w.lights()[0], w.camera(0)
    img = torch.empty((cam["height"], cam["width"], 4), dtype=torch.float32, device=dev)

    def timed(fn):
        fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    rows = []
    for n in slices:
        for res in resolutions:
            buf = vi.stack_buffer(n, res, vi.VI_F32, dev, STACK_LAYOUT)
            st = vi.build_attenuation(vol, tf, light, n, res, out=buf, layout=STACK_LAYOUT)
            row = {"n": n, "res": res,
                   "build_ms": round(timed(lambda: vi.build_attenuation(vol, tf, light, n, res, out=buf,
                                                                       layout=STACK_LAYOUT)), 4)}
            for m, extra in (("shell", {}), ("cone", {}), ("cone5", {"cone_grid": 5})):
                mm = "cone" if m == "cone5" else m
                row[f"{m}_ms"] = round(timed(lambda: vi.render(vol, tf, st, cam, mm, w.step_vox, extra, out=img)), 4)
            log(json.dumps(row))
            rows.append(row)
            del buf, st
    # the paper's flexibility claim: frame time nearly flat in the slab count
    flat = {}
    for res in resolutions:
        r = [x for x in rows if x["res"] == res]
        lo, hi = min(r, key=lambda x: x["n"]), max(r, key=lambda x: x["n"])
        flat[str(res)] = {m: round(hi[f"{m}_ms"] / lo[f"{m}_ms"], 3) for m in ("shell", "cone", "cone5")}
    return {"workload": "large 512^3 u16, light 0, 1920x1080", "layout": ["tiled", "rows"][STACK_LAYOUT],
            "rows": rows, f"frame_ms_ratio_n{max(slices)}_over_n{min(slices)}": flat}


def measure_steps(w, raw, scale, tab, lights, modes, stack_dtype, args, dev):
    """Time `args.steps` steps (build + every mode's frame for light i) after warm-up."""
    import torch
    from paper_2008_06134_amd import vi
    vol_lin = vi.Volume.from_numpy(raw, dev, scale)
    tf = vi.TF.from_numpy(tab, dev)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    # one-off per volume: brick or quad layout + empty-space map
    vol = (vol_lin.to_quads() if args.volume_layout == "quads" else vol_lin.to_bricks()).with_minmax(args.cell)
    if not args.no_occupancy:
        vol = vol.with_occupancy(tf)  # per (volume, TF): one bit per empty-space cell
    torch.cuda.synchronize()
    prep_ms = (time.perf_counter() - tb) * 1e3
    del vol_lin
    stack = vi.stack_buffer(w.n_slices, w.res, stack_dtype, dev, STACK_LAYOUT)
    cam0 = w.camera(0)
    imgs = {m: torch.empty((cam0["height"], cam0["width"], 4), dtype=torch.float32, device=dev) for m in modes}
    counters = {m: torch.zeros(2, dtype=torch.int64, device=dev) for m in modes}

    def mode_args(m):
        mm, extra = ("cone", {"cone_grid": 5}) if m == "cone5" else (m, {})
        if args.nearest_layer:
            extra = {**extra, "nearest_layer": 1}
        return mm, extra

    # point lights: each at args.point_light world units up-stream of the centre
    # along its direction
    positions = None
    if args.point_light:
        positions = [[0.5 - args.point_light * c for c in l] for l in lights]

    def step(i, events=None):
        li = i % len(lights)
        cam = w.camera(li)
        if events is not None:
            events[0].record()
        if positions is None:
            st = vi.build_attenuation(vol, tf, lights[li], w.n_slices, w.res, stack_dtype, out=stack,
                                      layout=STACK_LAYOUT)
        else:
            st = vi.build_attenuation(vol, tf, None, w.n_slices, w.res, stack_dtype, out=stack,
                                      layout=STACK_LAYOUT, position=positions[li])
        if events is not None:
            events[1].record()
        for k, m in enumerate(modes):
            mm, extra = mode_args(m)
            vi.render(vol, tf, st, cam, mm, w.step_vox, extra, out=imgs[m], samples=counters[m])
            if events is not None:
                events[2 + k].record()

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    for c in counters.values():
        c.zero_()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2 + len(modes))] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i, evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    out = {"build_ms": [e[0].elapsed_time(e[1]) for e in evs],
           "render_ms": {m: [e[1 + k].elapsed_time(e[2 + k]) for e in evs] for k, m in enumerate(modes)},
           "samples": {m: int(counters[m][0].item()) for m in modes},
           "opaque": {m: int(counters[m][1].item()) for m in modes}, "wall": wall, "prep_ms": prep_ms,
           "vol_bytes": raw.nbytes}
    del vol, stack, imgs
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=["small", "medium", "large", "precision"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=2)
    ap.add_argument("--no-serving", action="store_true", help="skip the short serving leg")
    ap.add_argument("--modes", default=None, help="comma-separated modes to time (none, shadow, shell, cone, cone5)")
    ap.add_argument("--scaling-sweep", action="store_true",
                    help="only run the slab-count x slice-resolution sweep (build and frame times)")
    ap.add_argument("--serving-sweep", action="store_true",
                    help="only run the full serving sweep (64 volumes, 6 arrival rates, 2000 requests each)")
    ap.add_argument("--cell", type=int, default=0, choices=[0, 4, 8, 16, 32],
                    help="edge in voxels of the empty-space map's cells; 0 = the smallest of 16 and 32 whose "
                         "occupancy bits fit in LDS (at most 65536 cells): 16 at 512^3, 32 at 1024^3")
    ap.add_argument("--stack-layout", default="rows", choices=["tiled", "rows"],
                    help="stack layout of every stack built (rows: one 8-byte load per bilinear row)")
    ap.add_argument("--volume-layout", default="auto", choices=["auto", "bricks", "quads"],
                    help="4x4x4 bricks, or quads (each slot its voxel's 2x2 x/y neighbourhood: 4x the bytes, "
                         "two loads per trilinear footprint); auto = quads, except bricks for the 1024^3 "
                         "precision workload (where quads measured slower)")
    ap.add_argument("--no-occupancy", action="store_true",
                    help="decide empty space from the min/max map and the TF per cell instead of occupancy bits")
    ap.add_argument("--point-light", type=float, default=0.0, metavar="DIST",
                    help="point lights DIST world units from the volume centre (against each light "
                         "direction) instead of directional lights")
    ap.add_argument("--nearest-layer", action="store_true",
                    help="stack lookups read the layer nearest each depth index instead of interpolating in depth")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates the HBM byte counters)")
    ap.add_argument("--store-probe", action="store_true",
                    help="only run the store-only probe of the build's write pattern (libvi_probe.so): 513 "
                         "layers of 1024 rows of 1024 floats, rows off and on the 128-byte line grid")
    ap.add_argument("--l2-probe", type=int, default=0, metavar="KIB",
                    help="only run the L2 probe (libvi_probe.so): 4 GiB of reads from one KIB KiB buffer, a "
                         "power of two of at least 8 KiB that fits in L2 (measures the L2 read rate the "
                         "gather roof is quoted against)")
    args = ap.parse_args()
    global STACK_LAYOUT
    STACK_LAYOUT = {"tiled": 0, "rows": 1}[args.stack_layout]
    if args.volume_layout == "auto":
        args.volume_layout = "bricks" if args.workload == "precision" else "quads"
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe * 2 ** 18, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 4, "launches": 3}), flush=True)
        return
    if args.store_probe:
        import ctypes
        import torch
        probe = ctypes.CDLL(os.path.join(ROOT, "paper_2008_06134_amd", "libvi_probe.so"))
        probe.vi_probe_store_rows.argtypes = [ctypes.c_void_p] + [ctypes.c_uint32] * 6 + [ctypes.c_void_p]
        res, layers = 1024, 513
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        rows_out = []
        # (name, first element, row pitch, layer stride): the row layout's pitch with its rows anywhere in a
        # line, and rows and layers on the line grid
        for name, org, pitch in (("rows off the line grid (pitch 1028)", 2 * 1028 + 2, 1028),
                                 ("rows on the line grid (pitch 1056)", 2 * 1056 + 32, 1056)):
            lstride = (res + 4) * pitch
            need = org + (layers - 1) * lstride + (res - 1) * pitch + res
            out = torch.empty(need, dtype=torch.float32, device="cuda:0")

            def launch():
                rc = probe.vi_probe_store_rows(ctypes.c_void_p(out.data_ptr()), res, res, layers, org, pitch,
                                               lstride, None)
                if rc:
                    raise RuntimeError(f"vi_probe_store_rows failed: {rc}")
            launch()
            ts = []
            for _ in range(5):
                e0.record()
                launch()
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            ms = sorted(ts)[2]
            nbytes = res * res * layers * 4
            rows_out.append({"pattern": name, "bytes": nbytes, "ms": round(ms, 4),
                             "gbs": round(nbytes / (ms * 1e-3) / 1e9, 1)})
            del out
        print(json.dumps({"store_probe": rows_out}), flush=True)
        return
    if args.l2_probe:
        import ctypes
        import torch
        probe = ctypes.CDLL(os.path.join(ROOT, "paper_2008_06134_amd", "libvi_probe.so"))
        probe.vi_probe_l2_read.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                           ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
        chunks, step, blocks = args.l2_probe // 4, 37, 4096       # 4 KiB chunks; 37 is coprime to a power of two
        iters = max(1, (1 << 32) // (blocks * 4096))               # 4 GiB read per launch
        buf = torch.ones(chunks * 1024, dtype=torch.float32, device="cuda:0")
        out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda:0")

        def launch():
            rc = probe.vi_probe_l2_read(ctypes.c_void_p(buf.data_ptr()), chunks, step, iters, blocks,
                                        ctypes.c_void_p(out.data_ptr()), None)
            if rc:
                raise RuntimeError(f"vi_probe_l2_read failed: {rc}")
        launch()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ts = []
        for _ in range(3):
            e0.record()
            launch()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = sorted(ts)[1]
        nbytes = blocks * 4096 * iters
        print(json.dumps({"l2_probe_buffer_bytes": chunks * 4096, "bytes_read": nbytes, "launches": 4,
                          "ms": round(ms, 4), "gbs": round(nbytes / (ms * 1e-3) / 1e9, 1)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding is a design, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2008_06134_amd import vi
    from paper_2008_06134_amd import workloads as W

    if args.serving_sweep:
        torch.cuda.set_device(0)
        print(json.dumps({"serving_sweep": serving_sweep("cuda:0")}), flush=True)
        return
    if args.scaling_sweep:
        torch.cuda.set_device(0)
        print(json.dumps({"scaling_sweep": scaling_sweep("cuda:0")}), flush=True)
        return

    w = W.WORKLOADS[args.workload]
    if args.cell == 0:
        args.cell = 16 if -(-w.N // 16) ** 3 <= 65536 else 32
    t0 = time.perf_counter()
    raw, tab = w.volume(), w.tf()
    log(f"workload {w.name}: {raw.shape} {raw.dtype} generated in {time.perf_counter() - t0:.1f} s")
    lights = w.lights()
    modes = w.modes if w.name != "medium" else ["cone5"]
    if args.modes:
        modes = args.modes.split(",")
    if args.point_light:
        if not args.point_light > 0.8661:
            ap.error("a point light must lie outside the sphere around the volume (DIST > 0.8661)")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cam0 = w.camera(0)
    Wd, Hd = cam0["width"], cam0["height"]
    precision = w.name == "precision"
    if precision:
        f16 = W.to_f16_normalised(raw)
        m = measure_steps(w, f16, 1.0, tab, lights, modes, vi.VI_BF16, args, dev)
        m_half = None
        if STACK_LAYOUT == vi.VI_STACK_ROWS:
            log("half-precision transmittance stack on the same FP16 volume ...")
            m_half = measure_steps(w, f16, 1.0, tab, lights, modes, vi.VI_F16, args, dev)
        del f16
        log("FP32 path on the same volume for comparison ...")
        m_fp32 = measure_steps(w, raw, None, tab, lights, modes, vi.VI_F32, args, dev)
    else:
        m = measure_steps(w, raw, None, tab, lights, modes, vi.VI_F32, args, dev)
    build_ms, render_ms, samples, wall = m["build_ms"], m["render_ms"], m["samples"], m["wall"]
    total_samples = sum(samples.values())
    frames = args.steps * len(modes)

    # Roofline of the dominant kernel (the most time per step).  A frame is
    # bound by vector-ALU instruction issue (the counters put its VALU issue
    # near the SIMDs' capacity while HBM moves a fraction of the compulsory
    # bytes), so its roof is the FP32 ALU: achieved = the method's algorithmic
    # FP32 operations per launch (FLOPS_PER_SAMPLE x composited segments) over
    # the launch's mean HIP-event time.  The HBM view (compulsory bytes, and
    # the bytes the counters saw) and the counters' VALU-issue and
    # address-unit fractions stand beside it.  The build is a write stream:
    # its roof is HBM.
    vol_bytes = m["vol_bytes"]
    stack_bytes = w.n_slices * w.res * w.res * (2 if precision else 4)
    img_bytes = Wd * Hd * 16
    opaque = m["opaque"]
    totals = {"build": sum(build_ms), **{f"render_{k}": sum(v) for k, v in render_ms.items()}}
    dom = max(totals, key=totals.get)
    rec = None if (args.point_light or args.no_occupancy or args.nearest_layer) else \
        measured(dom, w.name, args.stack_layout, args.cell, args.volume_layout)

    def counter_fracs(r, ms):
        if not r:
            return None, None
        cycles = r["gui_cycles"] / N_XCDS  # per XCD = per SIMD
        return (round(r["valu_insts"] * 4.0 / (N_SIMDS * cycles), 4),
                round(r["ta_busy"] / (N_TAS * cycles), 4))

    if dom == "build":
        per_launch, avg_ms = vol_bytes + stack_bytes, float(np.mean(build_ms))
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        tb = traffic_bytes(rec)
        roofline = {"bound": "hbm", "kernel": "build", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": tb,
                    "bytes_per_launch": per_launch, "avg_launch_ms": round(avg_ms, 4)}
    else:
        mode = dom[len("render_"):]
        avg_ms = float(np.mean(render_ms[mode]))
        flops = FLOPS_PER_SAMPLE[mode] * opaque[mode] / args.steps
        achieved = flops / (avg_ms * 1e-3) / 1e12
        tb = traffic_bytes(rec)
        valu, ta = counter_fracs(rec, avg_ms)
        ideal = vol_bytes + stack_bytes + img_bytes
        roofline = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 5), "traffic": tb,
                    "flops_per_launch": int(flops), "flops_per_composited_segment": FLOPS_PER_SAMPLE[mode],
                    "avg_launch_ms": round(avg_ms, 4),
                    "valu_issue_frac": valu, "address_unit_busy_frac": ta, "l2": l2_roof(rec, avg_ms),
                    "hbm": {"compulsory_bytes": ideal,
                            "compulsory_gbs": round(ideal / (avg_ms * 1e-3) / 1e9, 2),
                            "compulsory_frac": round(ideal / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                            "measured_gbs": None if tb is None else round(tb / (avg_ms * 1e-3) / 1e9, 2)}}
    build_ms_mean = float(np.mean(build_ms))
    brec = None if (args.point_light or args.no_occupancy or args.nearest_layer) else \
        measured("build", w.name, args.stack_layout, args.cell, args.volume_layout)
    btb = traffic_bytes(brec)
    kernels = {"volume_prepare_ms_once": round(m["prep_ms"], 3),
               "build_ms_mean": round(build_ms_mean, 4),
               "build_hbm_frac": round((vol_bytes + stack_bytes) / (build_ms_mean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "build_hbm_measured_gbs": None if btb is None else round(btb / (build_ms_mean * 1e-3) / 1e9, 2)}
    for k, v in render_ms.items():
        kernels[f"render_{k}_ms_mean"] = round(float(np.mean(v)), 4)
        kernels[f"render_{k}_samples_per_frame"] = samples[k] // args.steps
        kernels[f"render_{k}_composited_per_frame"] = opaque[k] // args.steps
        kernels[f"render_{k}_samples_per_s"] = round(samples[k] / (sum(v) * 1e-3), 1)
        kernels[f"render_{k}_composited_per_s"] = round(opaque[k] / (sum(v) * 1e-3), 1)
    # spread of the per-launch HIP-event times (each step renders a different light and camera)
    kernels["ms_p10_p50_p90"] = {name: [round(float(x), 4) for x in np.percentile(v, [10, 50, 90])]
                                 for name, v in [("build", build_ms)] + [(f"render_{k}", v)
                                                                         for k, v in render_ms.items()]}

    result = {
        "metric": "ray samples/s (build + shell + cone frames per light direction), 512^3 1080p",
        "value": round(total_samples / wall, 1),
        "composited_samples_per_s": round(sum(m["opaque"].values()) / wall, 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16 volume, bf16 optical depth, f32 math" if precision else "f32",
        "data": "synthetic",
        "fps": round(frames / wall, 3),
        "config": {"workload": (f"{w.name}: {w.N}^3 {'f16' if precision else raw.dtype} phantom "
                                f"({'4x4x4 bricks' if args.volume_layout == 'bricks' else '4x4x4 bricks of 2x2 quads'}, "
                                f"{args.cell}^3 empty-space cells{'' if args.no_occupancy else ' + occupancy bits'}), "
                                f"{w.n_slices} slices x {w.res}^2 {'bf16' if precision else 'f32'} "
                                f"({args.stack_layout}), "
                                f"{Wd}x{Hd}, step {w.step_vox} voxel, modes {'+'.join(modes)}, "
                                + (f"{len(lights)} point lights at {args.point_light} from the centre "
                                 if args.point_light else f"{len(lights)} light directions ")
                                + "(one rebuild per step)"
                                + (", nearest-layer lookups" if args.nearest_layer else "")),
                   "frames_per_step": len(modes)},
        "kernels": kernels,
        "roofline": roofline,
    }
    if precision:
        def leg(mm):
            return {"ms_per_step": round(mm["wall"] * 1e3 / args.steps, 4),
                    "build_ms_mean": round(float(np.mean(mm["build_ms"])), 4),
                    **{f"render_{k}_ms_mean": round(float(np.mean(v)), 4) for k, v in mm["render_ms"].items()}}
        result["fp32_path_same_volume"] = leg(m_fp32)
        if m_half is not None:
            # the same FP16 volume with a half-precision transmittance stack
            # (optical depth summed in float, stored as 2^-tau): no exponential per texel
            result["half_stack_same_volume"] = leg(m_half)
    if not args.no_serving and not precision:
        log("serving leg ...")
        torch.cuda.empty_cache()
        result["serving"] = serving_quick("cuda:0")
    if not args.no_cpu_baseline and not precision and not args.point_light and not args.nearest_layer:
        log("timing the oracle on a pixel sample ...")
        opts = {}
        result["cpu_baseline"] = cpu_baseline(w, raw, tab, lights[0], cam0, modes, opts, args.cpu_stride)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
