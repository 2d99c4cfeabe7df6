"""GPU parity of the local Phong comparison mode (section 4, Fig. 7 (b)):
central-difference normals, no stack read, FP32 against the FP64 oracle."""
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


def _inputs(raw, tab, scale=None):
    """As the benchmark prepares a volume: quads, empty-space map, occupancy bits."""
    tf = vi.TF.from_numpy(tab, DEV)
    vol = vi.Volume.from_numpy(raw, DEV, scale).to_quads().with_minmax(16).with_occupancy(tf)
    return vol, tf


def _render(vol, tf, light, cam, opts=None, step=0.5):
    lf = vi.light_frame(light, 1, 1)
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    img = vi.render(vol, tf, lf, cam, "phong", step, opts, samples=cnt)
    torch.cuda.synchronize()
    return img.cpu().double().numpy(), int(cnt.item())


def test_phong_small_full_image():
    w = W.WORKLOADS["small"]
    raw, tab = w.volume(), w.tf()
    vol, tf = _inputs(raw, tab)
    light = w.lights()[0]
    cam = w.camera()
    opts = {"bg": [0.1, 0.05, 0.02, 0.3]}
    img, ns = _render(vol, tf, light, cam, opts)
    ost = O.Stack(O.Volume(raw), O.TF(tab), light, 1, 1)
    _, ref, nt, _ = O.render(O.Volume(raw), O.TF(tab), ost, cam, "phong", w.step_vox, opts, want_full=False)
    err = np.abs(img - ref).max()
    print(f"[parity] small phong: max-abs {err:.3e}", flush=True)
    assert err <= TOL_IMG
    assert abs(ns - nt.sum()) <= 1e-3 * nt.sum() + 16


@pytest.mark.parametrize("light_index", [0, 7])
def test_phong_large_sampled(light_index):
    """512^3 u16 CT phantom, 1920x1080, in the benchmark's launch configuration."""
    w = W.WORKLOADS["large"]
    raw, tab = w.volume(), w.tf()
    vol, tf = _inputs(raw, tab)
    light = w.lights()[light_index]
    cam = w.camera(light_index)
    img, _ = _render(vol, tf, light, cam)
    rng = np.random.default_rng(40 + light_index)
    pix = np.unique(np.concatenate([rng.choice(cam["width"] * cam["height"], 1500, replace=False),
                                    (cam["height"] // 2) * cam["width"] + np.arange(cam["width"])]))
    ost = O.Stack(O.Volume(raw), O.TF(tab), light, 1, 1)
    _, ref, _, _ = O.render(O.Volume(raw), O.TF(tab), ost, cam, "phong", w.step_vox, {}, pixels=pix,
                            want_full=False)
    err = np.abs(img.reshape(-1, 4)[pix] - ref).max()
    print(f"[parity] large phong[{light_index}] ({pix.size} px): max-abs {err:.3e}", flush=True)
    assert err <= TOL_IMG


@pytest.mark.parametrize("shin,ks,geps", [(1.0, 0.8, 0.02), (64.0, 0.5, 0.005), (0.0, 0.3, 0.1)])
def test_phong_options_and_ragged(shin, ks, geps):
    N = 37
    raw = W.sphere_u8(N, radius=N * 0.32, density=190, noise=25, seed=N)
    tab = W.tf_ramp()
    vol, tf = _inputs(raw, tab)
    light = [0.3, -0.8, 0.5]
    cam = W.camera_orbit(41, 29, 0.8, 0.4, distance=1.8)
    opts = {"phong_ks": ks, "phong_shininess": shin, "grad_eps": geps, "phong_ka": 0.05, "light_rgb": [1, 0.9, 0.7]}
    img, _ = _render(vol, tf, light, cam, opts)
    ost = O.Stack(O.Volume(raw), O.TF(tab), light, 1, 1)
    _, ref, _, _ = O.render(O.Volume(raw), O.TF(tab), ost, cam, "phong", 0.5, opts, want_full=False)
    err = np.abs(img - ref).max()
    print(f"[parity] ragged phong shin={shin} ks={ks} eps={geps}: max-abs {err:.3e}", flush=True)
    assert err <= TOL_IMG


def test_phong_unit_ambient_equals_unlit_bitwise():
    w = W.WORKLOADS["small"]
    vol, tf = _inputs(w.volume(), w.tf())
    cam = w.camera(W=64, H=48)
    a, na = _render(vol, tf, w.lights()[0], cam, {"phong_ka": 1.0, "phong_kd": 0.0, "phong_ks": 0.0})
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    b = vi.render(vol, tf, None, cam, "none", 0.5, samples=cnt)
    torch.cuda.synchronize()
    assert np.array_equal(a, b.cpu().double().numpy()) and na == int(cnt.item())
