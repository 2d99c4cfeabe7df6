"""GPU parity of the point light (section 3.2.1's light projection L_p with a
light position, the light of Fig. 7): the stack is a set of frustum columns
from the light, slabs are planes of constant depth from it, and every stack
lookup projects through its own depth.  FP32 against the FP64 oracle, both
stack layouts; bfloat16 optical depth against the oracle's columns; Phong with
the light vector toward the light per sample; the cone (section 3.2.3, Eq. 11)
about the light's direction at each sample, rings and lattice."""
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
TOL_STACK = 2e-5
LAYOUTS = (vi.VI_STACK_TILED, vi.VI_STACK_ROWS)
LNAME = {vi.VI_STACK_TILED: "tiled", vi.VI_STACK_ROWS: "rows"}

# above the volume, off to one side, level with it and low, and over a
# corner (0.61 from it)
POSITIONS = [[0.5, 0.5, 2.5], [-1.1, 1.7, 1.4], [2.2, -0.4, 0.3], [1.35, 1.35, 1.35]]


def _inputs(raw, tab, cell=16):
    """As the benchmark prepares a volume: quads, empty-space map, occupancy bits."""
    tf = vi.TF.from_numpy(tab, DEV)
    vol = vi.Volume.from_numpy(raw, DEV).to_quads()
    if cell:
        vol = vol.with_minmax(cell).with_occupancy(tf)
    return vol, tf


def _render(vol, tf, st, cam, mode, step, opts=None):
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    img = vi.render(vol, tf, st, cam, mode, step, opts, samples=cnt)
    torch.cuda.synchronize()
    return img.cpu().double().numpy(), int(cnt.item())


def _report(name, err):
    print(f"[parity] {name}: max-abs {err:.3e}", flush=True)


@pytest.mark.parametrize("pos", POSITIONS)
def test_point_light_stack_and_images(pos):
    w = W.WORKLOADS["small"]
    raw, tab = w.volume(), w.tf()
    vol, tf = _inputs(raw, tab)
    ovol, otf = O.Volume(raw), O.TF(tab)
    ost = O.Stack(ovol, otf, None, w.n_slices, w.res, position=pos)
    S = ost.export()
    cam = w.camera(W=96, H=80)
    opts = {"bg": [0.1, 0.05, 0.02, 0.3], "ambient": 0.1}
    modes = {"shadow": ("shadow", {}), "shell": ("shell", {}), "cone": ("cone", {}),
             "cone5": ("cone", {"cone_grid": 5})}
    refs = {k: O.render(ovol, otf, ost, cam, m, w.step_vox, {**opts, **x}, want_full=False)
            for k, (m, x) in modes.items()}
    for lay in LAYOUTS:
        st = vi.build_attenuation(vol, tf, None, w.n_slices, w.res, layout=lay, position=pos)
        assert st.s.positional == 1 and list(st.s.P) == [float(c) for c in pos]
        err_s = np.abs(st.dense().cpu().double().numpy() - S).max()
        _report(f"point {pos} stack ({LNAME[lay]})", err_s)
        assert err_s <= TOL_STACK
        for m, (_, ref, nt, _) in refs.items():
            img, ns = _render(vol, tf, st, cam, modes[m][0], w.step_vox, {**opts, **modes[m][1]})
            err = np.abs(img - ref).max()
            _report(f"point {pos} {m} ({LNAME[lay]})", err)
            assert err <= TOL_IMG
            assert abs(ns - nt.sum()) <= 1e-3 * nt.sum() + 16


def test_point_light_differs_from_directional():
    """The point light is not the directional light along its axis: the
    shadows fan out; a far light converges to the directional one (their
    texel grids differ, so at a fine stack only)."""
    w = W.WORKLOADS["small"]
    raw, tab = w.volume(), w.tf()
    vol, tf = _inputs(raw, tab)
    n, res = 128, 256
    cam = w.camera(W=64, H=64)
    st_p = vi.build_attenuation(vol, tf, None, n, res, layout=vi.VI_STACK_ROWS, position=[0.5, 0.5, 1.6])
    st_d = vi.build_attenuation(vol, tf, [0.0, 0.0, -1.0], n, res, layout=vi.VI_STACK_ROWS)
    st_far = vi.build_attenuation(vol, tf, None, n, res, layout=vi.VI_STACK_ROWS, position=[0.5, 0.5, 2000.0])
    for m, x in (("shadow", {}), ("cone", {}), ("cone", {"cone_grid": 5})):
        a, _ = _render(vol, tf, st_p, cam, m, w.step_vox, x)
        b, _ = _render(vol, tf, st_d, cam, m, w.step_vox, x)
        c, _ = _render(vol, tf, st_far, cam, m, w.step_vox, x)
        print(f"[point] {m}{' 5x5' if x else ''}: near vs directional {np.abs(a - b).max():.3e}, "
              f"far vs directional {np.abs(c - b).max():.3e} (mean {np.abs(c - b).mean():.2e})", flush=True)
        assert np.abs(a - b).max() > 0.1
        assert np.abs(c - b).max() < 0.03 and np.abs(c - b).mean() < 1e-3


def test_point_light_uniform_medium_near_corner():
    """A uniform medium fills the cube and the light sits just outside the
    sphere around it, over a corner: shell taps near that corner fall at or
    behind the light's depth plane (the stack reads 1 there), and samples sit
    a few thousandths from the apex."""
    N = 32
    raw = W.constant_cube(N, 60)
    tab = W.tf_ramp()
    vol, tf = _inputs(raw, tab, cell=8)
    ovol, otf = O.Volume(raw), O.TF(tab)
    pos = [0.5 + 0.87 / math.sqrt(3.0)] * 3
    n, res = 24, 40
    ost = O.Stack(ovol, otf, None, n, res, position=pos)
    cam = W.camera_orbit(64, 56, math.radians(40), math.radians(30))
    opts = {"shell_count": 2, "shell_h_vox": 1.5, "cone_rings": 3, "cone_angles": 6, "cone_tan": 1.5}
    for m, x in (("shadow", {}), ("shell", {}), ("cone", {}), ("cone", {"cone_grid": 7})):
        _, ref, _, _ = O.render(ovol, otf, ost, cam, m, 0.5, {**opts, **x}, want_full=False)
        for lay in LAYOUTS:
            st = vi.build_attenuation(vol, tf, None, n, res, layout=lay, position=pos)
            err_s = np.abs(st.dense().cpu().double().numpy() - ost.export()).max()
            img, _ = _render(vol, tf, st, cam, m, 0.5, {**opts, **x})
            err = np.abs(img - ref).max()
            _report(f"point near corner {m}{' 7x7' if x else ''} ({LNAME[lay]}), stack {err_s:.2e}", err)
            assert err_s <= TOL_STACK and err <= TOL_IMG


def test_point_light_bf16_optical_depth():
    w = W.WORKLOADS["medium"]
    raw, tab = w.volume(), w.tf()
    vol, tf = _inputs(raw, tab)
    pos = [-0.8, 1.9, 1.2]
    st = vi.build_attenuation(vol, tf, None, 96, 160, vi.VI_BF16, layout=vi.VI_STACK_ROWS, position=pos)
    ost = O.Stack(O.Volume(raw), O.TF(tab), None, 96, 160, position=pos)
    rng = np.random.default_rng(8)
    ij = rng.integers(0, 160, size=(300, 2))
    tau = st.dense()[:, torch.as_tensor(ij[:, 1], device=DEV), torch.as_tensor(ij[:, 0], device=DEV)]
    got = np.exp2(-tau.float().cpu().double().numpy())
    want = np.stack([ost.column(i, j) for i, j in ij], axis=1)
    err = np.abs(got - want).max()
    _report("point bf16 stack columns", err)
    assert err < 4e-3


def test_point_light_medium_sampled():
    """256^3 u16 CT phantom at the medium workload's stack and image size."""
    w = W.WORKLOADS["medium"]
    raw, tab = w.volume(), w.tf()
    vol, tf = _inputs(raw, tab)
    ovol, otf = O.Volume(raw), O.TF(tab)
    pos = [1.9, -0.7, 1.6]
    ost = O.Stack(ovol, otf, None, w.n_slices, w.res, position=pos)
    cam = w.camera()
    rng = np.random.default_rng(21)
    pix = np.unique(np.concatenate([rng.choice(cam["width"] * cam["height"], 1200, replace=False),
                                    (cam["height"] // 2) * cam["width"] + np.arange(cam["width"])]))
    ij = rng.integers(0, w.res, size=(600, 2))
    want = np.stack([ost.column(i, j) for i, j in ij], axis=1)
    st = vi.build_attenuation(vol, tf, None, w.n_slices, w.res, layout=vi.VI_STACK_ROWS, position=pos)
    S = st.dense()
    got = S[:, torch.as_tensor(ij[:, 1], device=DEV), torch.as_tensor(ij[:, 0], device=DEV)]
    err_s = np.abs(got.cpu().double().numpy() - want).max()
    del S, got
    assert err_s <= TOL_STACK
    for m in ("shell", "cone"):
        _, ref, _, _ = O.render(ovol, otf, ost, cam, m, w.step_vox, {}, pixels=pix, want_full=False)
        img, _ = _render(vol, tf, st, cam, m, w.step_vox)
        err = np.abs(img.reshape(-1, 4)[pix] - ref).max()
        _report(f"point medium {m} ({pix.size} px), stack columns {err_s:.2e}", err)
        assert err <= TOL_IMG


def test_point_cone_view_along_the_light_ray():
    """An orthographic view along the line from the light through the cube's
    centre, with an odd image width and height so that the centre pixel's ray
    runs on that line: there the view vector is parallel to the light's
    direction at every sample, B vanishes and both sides take U's part across
    L_s; the pixels around it have B nearly at right angles to it."""
    N = 72
    raw = W.ct_phantom_u16(N, seed=31, vessels=True)
    tab = W.tf_ct()
    vol, tf = _inputs(raw, tab, cell=8)
    ovol, otf = O.Volume(raw), O.TF(tab)
    pos = [1.9, 1.4, -0.6]
    axis = np.array([0.5, 0.5, 0.5]) - np.array(pos)
    axis /= np.linalg.norm(axis)
    n, res = 64, 96
    ost = O.Stack(ovol, otf, None, n, res, position=pos)
    st = vi.build_attenuation(vol, tf, None, n, res, layout=vi.VI_STACK_ROWS, position=pos)
    for sign in (1.0, -1.0):
        eye = (np.array([0.5, 0.5, 0.5]) - sign * 1.5 * axis).tolist()
        cam = {"kind": "ortho", "eye": eye, "target": [0.5, 0.5, 0.5], "up": [0.0, 1.0, 0.0],
               "ortho_half_h": 0.7, "width": 63, "height": 47}
        for x in ({}, {"cone_grid": 5}):
            _, ref, _, _ = O.render(ovol, otf, ost, cam, "cone", 0.5, x, want_full=False)
            img, _ = _render(vol, tf, st, cam, "cone", 0.5, x)
            err = np.abs(img - ref).max()
            _report(f"point cone along {'+' if sign > 0 else '-'}L_s{' 5x5' if x else ''}", err)
            assert err <= TOL_IMG
            assert float(np.abs(ref[23, 31]).max()) > 1e-3      # the centre pixel is not empty


@pytest.mark.parametrize("pos", [[0.5, 0.5, 2.5], [2.2, -0.4, 0.3]])
def test_point_light_phong(pos):
    w = W.WORKLOADS["small"]
    raw, tab = w.volume(), w.tf()
    vol, tf = _inputs(raw, tab)
    lf = vi.light_frame(None, 1, 1, position=pos)
    cam = w.camera(W=96, H=80)
    opts = {"bg": [0.1, 0.05, 0.02, 0.3]}
    img, _ = _render(vol, tf, lf, cam, "phong", w.step_vox, opts)
    ost = O.Stack(O.Volume(raw), O.TF(tab), None, 1, 1, position=pos)
    _, ref, _, _ = O.render(O.Volume(raw), O.TF(tab), ost, cam, "phong", w.step_vox, opts, want_full=False)
    err = np.abs(img - ref).max()
    _report(f"point {pos} phong", err)
    assert err <= TOL_IMG
    # the directional light along the point light's axis gives another image
    ax = vi.light_frame(None, 1, 1, position=pos).frame()["L"]
    img_d, _ = _render(vol, tf, vi.light_frame(ax, 1, 1), cam, "phong", w.step_vox, opts)
    assert np.abs(img - img_d).max() > 1e-3
