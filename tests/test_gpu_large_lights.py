"""GPU parity at the benchmarked large size, every light of the orbit.

512^3 u16 phantom with vessels, 512 slabs x 1024^2 row-layout stack,
1920 x 1080 pinhole camera, prepared as the benchmark prepares it (quads,
16^3-voxel empty-space cells, occupancy bits).  For each of the 16 seeded
light directions: sampled stack columns (<= 2e-5) and the FULL shell and
cone images (every pixel, max-abs <= 1e-4 per RGBA channel) against the FP64
oracle; the 5 x 5 cone lattice in full on four of the lights.  Plus the
cone's fallback basis when the view runs exactly along the light, and a
point light at the large size (sampled).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2008_06134_amd import vi
from paper_2008_06134_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL_IMG = 1e-4
TOL_STACK = 2e-5


@pytest.fixture(scope="module")
def large():
    w = W.WORKLOADS["large"]
    raw, tab = w.volume(), w.tf()
    tf = vi.TF.from_numpy(tab, DEV)
    vol = vi.Volume.from_numpy(raw, DEV).to_quads().with_minmax(16).with_occupancy(tf)
    torch.cuda.synchronize()
    return w, raw, tab, vol, tf, O.Volume(raw), O.TF(tab)


def _frame(vol, tf, st, cam, mode, step, opts):
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    img = vi.render(vol, tf, st, cam, mode, step, opts, samples=cnt)
    torch.cuda.synchronize()
    return img.cpu().double().numpy(), int(cnt.item())


def _compare(name, img, ref, ns, nt):
    diff = np.abs(img - ref).max(axis=-1)
    err = float(diff.max())
    wy, wx = np.unravel_index(int(np.argmax(diff)), diff.shape)
    print(f"[parity] {name}: full image max-abs {err:.3e} (worst pixel {wx},{wy}), "
          f"segments {ns} vs {int(nt.sum())}", flush=True)
    assert err <= TOL_IMG
    assert abs(ns - int(nt.sum())) <= 1e-3 * int(nt.sum()) + 16


LATTICE_LIGHTS = (0, 4, 8, 12)


@pytest.mark.parametrize("li", range(16))
def test_large_light_full_images(large, li):
    w, raw, tab, vol, tf, ovol, otf = large
    light = w.lights()[li]
    cam = w.camera(li)
    print(f"[parity] large light {li}: {np.round(light, 4).tolist()}", flush=True)
    st = vi.build_attenuation(vol, tf, light, w.n_slices, w.res, layout=vi.VI_STACK_ROWS)
    torch.cuda.synchronize()
    ost = O.Stack(ovol, otf, light, w.n_slices, w.res)
    rng = np.random.default_rng(500 + li)
    ij = rng.integers(0, w.res, size=(400, 2))
    want = np.stack([ost.column(i, j) for i, j in ij], axis=1)
    S = st.dense()
    got = S[:, torch.as_tensor(ij[:, 1], device=DEV), torch.as_tensor(ij[:, 0], device=DEV)]
    err_s = float(np.abs(got.cpu().double().numpy() - want).max())
    del S, got
    print(f"[parity] large light {li} stack columns: max-abs {err_s:.3e}", flush=True)
    assert err_s <= TOL_STACK
    modes = [("shell", {}), ("cone", {})]
    if li in LATTICE_LIGHTS:
        modes.append(("cone", {"cone_grid": 5}))
    for mode, opts in modes:
        img, ns = _frame(vol, tf, st, cam, mode, w.step_vox, opts)
        _, ref, nt, _ = O.render(ovol, otf, ost, cam, mode, w.step_vox, opts, want_full=False)
        _compare(f"large light {li} {mode}{' 5x5' if opts else ''}", img, ref, ns, nt)
    del st, ost


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_cone_fallback_when_view_runs_along_the_light(sign):
    """An orthographic view exactly along +L or -L: B (the direction toward the
    viewer with its L part removed) vanishes and the cone takes U instead, on
    both sides."""
    w = W.WORKLOADS["medium"]
    raw = W.ct_phantom_u16(96, seed=21)
    tab = W.tf_ct()
    tf = vi.TF.from_numpy(tab, DEV)
    vol = vi.Volume.from_numpy(raw, DEV).to_quads().with_minmax(16).with_occupancy(tf)
    light = np.array(W.DIAGONAL_LIGHT, dtype=np.float64)
    light /= np.linalg.norm(light)
    eye = (np.array([0.5, 0.5, 0.5]) - sign * 2.0 * light).tolist()
    cam = {"kind": "ortho", "eye": eye, "target": [0.5, 0.5, 0.5], "up": [0.0, 1.0, 0.0],
           "ortho_half_h": 0.8, "width": 96, "height": 80}
    ovol, otf = O.Volume(raw), O.TF(tab)
    ost = O.Stack(ovol, otf, light.tolist(), 96, 160)
    st = vi.build_attenuation(vol, tf, light.tolist(), 96, 160, layout=vi.VI_STACK_ROWS)
    for opts in ({}, {"cone_grid": 5}):
        img, ns = _frame(vol, tf, st, cam, "cone", 0.5, opts)
        _, ref, nt, _ = O.render(ovol, otf, ost, cam, "cone", 0.5, opts, want_full=False)
        _compare(f"cone along {'+' if sign > 0 else '-'}L{' 5x5' if opts else ''}", img, ref, ns, nt)
        assert float(np.abs(ref).max()) > 1e-2       # the view is not empty


def test_point_light_large_sampled(large):
    """A point light 2.0 from the centre at the large size: sampled frustum
    columns and shadow / shell / cone pixels against the oracle."""
    w, raw, tab, vol, tf, ovol, otf = large
    d = np.array(w.lights()[3])
    pos = (np.array([0.5, 0.5, 0.5]) - 2.0 * d).tolist()
    cam = w.camera(3)
    st = vi.build_attenuation(vol, tf, None, w.n_slices, w.res, layout=vi.VI_STACK_ROWS, position=pos)
    torch.cuda.synchronize()
    ost = O.Stack(ovol, otf, None, w.n_slices, w.res, position=pos)
    rng = np.random.default_rng(77)
    ij = rng.integers(0, w.res, size=(400, 2))
    want = np.stack([ost.column(i, j) for i, j in ij], axis=1)
    S = st.dense()
    got = S[:, torch.as_tensor(ij[:, 1], device=DEV), torch.as_tensor(ij[:, 0], device=DEV)]
    err_s = float(np.abs(got.cpu().double().numpy() - want).max())
    del S, got
    print(f"[parity] large point light stack columns: max-abs {err_s:.3e}", flush=True)
    assert err_s <= TOL_STACK
    pix = np.unique(np.concatenate([rng.choice(cam["width"] * cam["height"], 3000, replace=False),
                                    (cam["height"] // 2) * cam["width"] + np.arange(cam["width"])]))
    for mode in ("shadow", "shell", "cone"):
        img, _ = _frame(vol, tf, st, cam, mode, w.step_vox, {})
        _, ref, _, _ = O.render(ovol, otf, ost, cam, mode, w.step_vox, {}, pixels=pix, want_full=False)
        err = float(np.abs(img.reshape(-1, 4)[pix] - ref).max())
        print(f"[parity] large point light {mode} ({pix.size} px): max-abs {err:.3e}", flush=True)
        assert err <= TOL_IMG
