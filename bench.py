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


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(w, raw, tab, light, cam, modes, opts, stride, nthreads=0):
    """The FP64 oracle on a stratified pixel sample of the same frames (stack
    columns built on demand), timed on the host cores."""
    from oracle import oracle as O
    ovol, otf = O.Volume(raw), O.TF(tab)
    Wd, Hd = cam["width"], cam["height"]
    ys, xs = np.meshgrid(np.arange(stride // 2, Hd, stride), np.arange(stride // 2, Wd, stride), indexing="ij")
    pix = (ys * Wd + xs).ravel().astype(np.int64)
    t0 = time.perf_counter()
    st = O.Stack(ovol, otf, light, w.n_slices, w.res)
    samples = 0
    for m in modes:
        mm, extra = (m, {}) if m != "cone5" else ("cone", {"cone_grid": 5})
        _, _, nt, _ = O.render(ovol, otf, st, cam, mm, w.step_vox, {**opts, **extra}, pixels=pix,
                               want_full=False, nthreads=nthreads)
        samples += int(nt.sum())
    dt = time.perf_counter() - t0
    return {"value": samples / dt, "unit": "samples/s", "cores": O.threads(), "kind": "oracle",
            "sample": (f"{pix.size} of {Wd * Hd} pixels (every {stride}th row and column) of the "
                       f"{'+'.join(modes)} frames of light 0, {st.columns_built()} of {w.res ** 2} stack columns "
                       f"built on demand; {samples} samples in {dt:.1f} s")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=["small", "medium", "large"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=2)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe * 2 ** 18, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 4, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding is a design, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2008_06134_amd import vi
    from paper_2008_06134_amd import workloads as W

    w = W.WORKLOADS[args.workload]
    t0 = time.perf_counter()
    raw, tab = w.volume(), w.tf()
    log(f"workload {w.name}: {raw.shape} {raw.dtype} generated in {time.perf_counter() - t0:.1f} s")
    lights = w.lights()
    modes = w.modes if w.name != "medium" else ["cone5"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    vol_lin = vi.Volume.from_numpy(raw, dev)
    tf = vi.TF.from_numpy(tab, dev)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    vol = vol_lin.to_bricks().with_minmax(8)  # one-off per volume: bricks + empty-space map
    torch.cuda.synchronize()
    brick_ms = (time.perf_counter() - tb) * 1e3
    del vol_lin
    stack = vi.stack_buffer(w.n_slices, w.res, vi.VI_F32, dev)
    cam0 = w.camera(0)
    Wd, Hd = cam0["width"], cam0["height"]
    imgs = {m: torch.empty((Hd, Wd, 4), dtype=torch.float32, device=dev) for m in modes}
    counters = {m: torch.zeros(1, dtype=torch.int64, device=dev) for m in modes}

    def mode_args(m):
        return ("cone", {"cone_grid": 5}) if m == "cone5" else (m, {})

    def step(i, events=None):
        li = i % len(lights)
        cam = w.camera(li)
        if events is not None:
            events[0].record()
        st = vi.build_attenuation(vol, tf, lights[li], w.n_slices, w.res, out=stack)
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

    build_ms = [e[0].elapsed_time(e[1]) for e in evs]
    render_ms = {m: [e[1 + k].elapsed_time(e[2 + k]) for e in evs] for k, m in enumerate(modes)}
    samples = {m: int(counters[m].item()) for m in modes}
    total_samples = sum(samples.values())
    frames = args.steps * len(modes)

    # roofline of the dominant kernel, algorithmic (compulsory) bytes per launch
    vol_bytes = raw.nbytes
    stack_bytes = w.n_slices * w.res * w.res * 4
    img_bytes = Wd * Hd * 16
    totals = {"build": sum(build_ms), **{f"render_{m}": sum(v) for m, v in render_ms.items()}}
    dom = max(totals, key=totals.get)
    if dom == "build":
        per_launch, avg_ms = vol_bytes + stack_bytes, np.mean(build_ms)
    else:
        per_launch, avg_ms = vol_bytes + stack_bytes + img_bytes, np.mean(render_ms[dom[len("render_"):]])
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                "bytes_per_launch": per_launch, "avg_launch_ms": round(float(avg_ms), 4)}
    kernels = {"volume_prepare_ms_once": round(brick_ms, 3),
               "build_ms_mean": round(float(np.mean(build_ms)), 4),
               "build_hbm_frac": round((vol_bytes + stack_bytes) / (np.mean(build_ms) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    for m, v in render_ms.items():
        kernels[f"render_{m}_ms_mean"] = round(float(np.mean(v)), 4)
        kernels[f"render_{m}_samples_per_frame"] = samples[m] // args.steps
        kernels[f"render_{m}_samples_per_s"] = round(samples[m] / (sum(v) * 1e-3), 1)

    result = {
        "metric": "ray samples/s (build + shell + cone frames per light direction), 512^3 1080p",
        "value": round(total_samples / wall, 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "fps": round(frames / wall, 3),
        "config": {"workload": (f"{w.name}: {w.N}^3 {raw.dtype} phantom (4x4x4 bricks, 8^3 empty-space cells), "
                                f"{w.n_slices} slices x {w.res}^2 f32, "
                                f"{Wd}x{Hd}, step {w.step_vox} voxel, modes {'+'.join(modes)}, "
                                f"{len(lights)} light directions (one rebuild per step)"),
                   "frames_per_step": len(modes)},
        "kernels": kernels,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on a pixel sample ...")
        opts = {}
        result["cpu_baseline"] = cpu_baseline(w, raw, tab, lights[0], cam0, modes, opts, args.cpu_stride)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
