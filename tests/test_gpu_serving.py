"""Serving on the GPU: every frame served in a mix matches the FP64 oracle
(max-abs 1e-4 per RGBA channel) and equals the same frame rendered alone with
vi_render (bit for bit); stacks are reused while the light is unchanged,
eviction under a small pool keeps results right, and the server drains
cleanly."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2008_06134_amd import vi
from paper_2008_06134_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL_IMG = 1e-4


def _volumes():
    vols = []
    for k, N in enumerate([48, 64, 80, 96]):
        raw = W.ct_phantom_u16(N, seed=100 + k, vessels=(k % 2 == 1))
        v = vi.Volume.from_numpy(raw, DEV).to_quads().with_minmax(16)
        tf = vi.TF.from_numpy(W.tf_ct(), DEV)
        if k % 2 == 0:
            v = v.with_occupancy(tf)     # a launch mixes frames with and without occupancy bits
        vols.append((N, v, tf, raw))
    return vols


def _requests(vols, count, seed):
    rng = np.random.default_rng(seed)
    sizes = [(64, 48), (96, 96), (128, 72), (80, 112), (33, 17)]
    reqs = []
    for i in range(count):
        vi_ = int(rng.integers(len(vols)))
        N = vols[vi_][0]
        li = int(rng.integers(3))
        light = W.light_from_angles(2 * math.pi * li / 3 + 0.1 * vi_, math.radians(35))
        w, h = sizes[int(rng.integers(len(sizes)))]
        cam = W.camera_orbit(w, h, float(rng.uniform(0, 2 * math.pi)), math.radians(20))
        mode = ["shell", "cone", "cone5", "shadow", "phong"][int(rng.integers(5))]
        darken = 1.0 if li == 2 else 0.0          # the compensated build is part of a stack's identity
        # light 0 becomes a point light two units up-stream of the centre
        pos = None
        if li == 0:
            pos = [0.5 - 2.0 * c for c in light]
        reqs.append(dict(vol=vi_, light=light, n=N, res=min(2 * N, 1024), cam=cam, mode=mode, darken=darken,
                         pos=pos))
    return reqs


def _alone(vols, r, layout=vi.VI_STACK_TILED):
    _, v, tf, _ = vols[r["vol"]]
    st = vi.build_attenuation(v, tf, r["light"], r["n"], r["res"], layout=layout, darken=r["darken"],
                              position=r["pos"])
    m, extra = ("cone", {"cone_grid": 5}) if r["mode"] == "cone5" else (r["mode"], {})
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    img = vi.render(v, tf, st, r["cam"], m, 0.5, extra, samples=cnt)
    torch.cuda.synchronize()
    return img.clone(), int(cnt.item())


def _oracle(vols, r):
    """The FP64 oracle's frame for request r (terminated rays, as the GPU)."""
    raw = vols[r["vol"]][3]
    ovol, otf = O.Volume(raw), O.TF(W.tf_ct())
    light = None if r["pos"] is not None else r["light"]
    ost = O.Stack(ovol, otf, light, r["n"], r["res"], darken=r["darken"], position=r["pos"])
    m, extra = ("cone", {"cone_grid": 5}) if r["mode"] == "cone5" else (r["mode"], {})
    _, ref, nt, _ = O.render(ovol, otf, ost, r["cam"], m, 0.5, extra, want_full=False)
    return ref, int(nt.sum())


def _check_oracle(vols, reqs, imgs, counters=None):
    worst = 0.0
    for i, r in enumerate(reqs):
        ref, n_ref = _oracle(vols, r)
        err = float(np.abs(imgs[i].cpu().double().numpy() - ref).max())
        worst = max(worst, err)
        assert err <= TOL_IMG, f"request {i} ({r['mode']}, pos {r['pos']}): max-abs {err:.3e} vs the oracle"
        if counters is not None:
            n = int(counters[i].item())
            assert abs(n - n_ref) <= 1e-3 * n_ref + 16
    print(f"[serving] {len(reqs)} served frames vs the FP64 oracle: worst max-abs {worst:.3e}", flush=True)


def _submit(srv, ids, r, samples=None, layout=vi.VI_STACK_TILED):
    m, extra = ("cone", {"cone_grid": 5}) if r["mode"] == "cone5" else (r["mode"], {})
    return srv.submit(ids[r["vol"]], r["light"], r["n"], r["res"], r["cam"], m, 0.5, extra, samples=samples,
                      layout=layout, darken=r["darken"], position=r["pos"])


@pytest.mark.parametrize("layout", [vi.VI_STACK_TILED, vi.VI_STACK_ROWS])
def test_mixed_burst_equals_frames_rendered_alone(layout):
    vols = _volumes()
    reqs = _requests(vols, 40, seed=1)
    srv = vi.Server(stack_budget=256 << 20, max_inflight=12, tiles_per_launch=64)
    ids = [srv.register(v, tf) for _, v, tf, _ in vols]
    counters = [torch.zeros(1, dtype=torch.int64, device=DEV) for _ in reqs]
    subs = [_submit(srv, ids, r, counters[i], layout) for i, r in enumerate(reqs)]
    for t, _ in subs:
        assert srv.wait(t, 60000) == 0
    torch.cuda.synchronize()
    st = srv.stats()
    print(f"[serving] {st['completed']} frames, {st['launches']} launches, "
          f"{st['mean_frames_per_launch']:.2f} frames/launch, hits {st['stack_hits']} builds {st['stack_builds']}",
          flush=True)
    assert st["completed"] == len(reqs)
    assert st["mean_frames_per_launch"] > 1.0          # launches really mix frames
    assert st["stack_hits"] > 0                         # the light repeats: stacks are reused
    assert any(r["pos"] is not None for r in reqs) and any(r["pos"] is None for r in reqs)
    _check_oracle(vols, reqs, [img for _, img in subs], counters)
    for i, r in enumerate(reqs):
        ref, n_ref = _alone(vols, r, layout)
        assert torch.equal(subs[i][1], ref), f"request {i} differs from its standalone render"
        assert int(counters[i].item()) == n_ref
    srv.close()


def test_small_pool_evicts_and_stays_correct():
    vols = _volumes()
    reqs = _requests(vols, 16, seed=2)
    biggest = max(vi.slices_bytes(r["n"], r["res"]) for r in reqs)
    srv = vi.Server(stack_budget=biggest + 4096, max_inflight=4, tiles_per_launch=32)
    ids = [srv.register(v, tf) for _, v, tf, _ in vols]
    subs = [_submit(srv, ids, r) for r in reqs]
    for t, _ in subs:
        assert srv.wait(t, 60000) == 0
    st = srv.stats()
    assert st["evictions"] > 0 and st["pool_peak"] <= st["pool_bytes"]
    _check_oracle(vols, reqs, [img for _, img in subs])
    for i, r in enumerate(reqs):
        ref, _ = _alone(vols, r)
        assert torch.equal(subs[i][1], ref)
    srv.close()


def test_oversized_and_invalid_requests_are_refused():
    vols = _volumes()
    srv = vi.Server(stack_budget=1 << 20, max_inflight=2)
    ids = [srv.register(v, tf) for _, v, tf, _ in vols]
    cam = W.camera_orbit(32, 32, 0.3, 0.3)
    with pytest.raises(vi.VIError) as e:
        srv.submit(ids[0], [0, 0, 1], 64, 256, cam, "shell", 0.5)    # 16 MiB stack > 1 MiB pool
    assert e.value.code == -3
    with pytest.raises(vi.VIError):
        srv.submit(ids[0], [0, 0, 0], 8, 8, cam, "shell", 0.5)       # degenerate light
    t, img = srv.submit(ids[0], [0, 0, 1], 8, 16, cam, "shell", 0.5)
    assert srv.wait(t, 30000) == 0
    assert srv.stats()["rejected"] == 1
    srv.close()


def test_destroy_drains_queued_work():
    vols = _volumes()
    reqs = _requests(vols, 12, seed=3)
    srv = vi.Server(stack_budget=256 << 20, max_inflight=2, tiles_per_launch=16)
    ids = [srv.register(v, tf) for _, v, tf, _ in vols]
    subs = [_submit(srv, ids, r) for r in reqs]
    srv.close()                         # must finish every queued frame first
    torch.cuda.synchronize()
    _check_oracle(vols, reqs, [img for _, img in subs])
    for i in (0, len(reqs) - 1):
        ref, _ = _alone(vols, reqs[i])
        assert torch.equal(subs[i][1], ref)
