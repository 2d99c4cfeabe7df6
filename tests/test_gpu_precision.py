"""Precision form on the GPU: FP16 normalised volume, bfloat16 optical-depth stack,
float accumulation -- error against the FP64 oracle stated as max-abs and PSNR.

Two references (both the plain FP64 method):
  (i)  the oracle on the original 12-bit u16 volume: the whole precision-form error;
  (ii) the oracle on the FP16-quantised volume: the bfloat16 stack and float error only.
PSNR = 10 log10(1 / MSE) over pixels x 4 channels (peak 1), target >= 50 dB.
"""
import functools
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2008_06134_amd import vi
from paper_2008_06134_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda"


def psnr(a, b):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return math.inf if mse == 0 else 10.0 * math.log10(1.0 / mse)


@functools.lru_cache(maxsize=1)
def _phantom(N):
    raw = W.ct_phantom_u16(N, seed=4, vessels=True)
    return raw, W.to_f16_normalised(raw)


def _precision_case(N, n, res, cam, light, mode, opts, pix, layout=vi.VI_STACK_ROWS, sdt=vi.VI_BF16):
    raw, f16 = _phantom(N)
    tab = W.tf_ct()
    # as the benchmark prepares the precision volume: bricks, the cell size whose occupancy bits fit in LDS
    tf = vi.TF.from_numpy(tab, DEV)
    cell = 16 if N <= 640 else 32
    vol = vi.Volume.from_numpy(f16, DEV, 1.0).to_bricks().with_minmax(cell).with_occupancy(tf)
    st = vi.build_attenuation(vol, tf, light, n, res, sdt, layout=layout)
    img = vi.render(vol, tf, st, cam, mode, 0.5, opts)
    torch.cuda.synchronize()
    got = img.cpu().double().numpy().reshape(-1, 4)
    rng = np.random.default_rng(7)
    ij = rng.integers(0, res, size=(400, 2))
    dense = st.dense()
    tau = dense[:, torch.as_tensor(ij[:, 1], device=DEV), torch.as_tensor(ij[:, 0], device=DEV)]
    tau = tau.float().cpu().double().numpy()
    del img, dense
    otf = O.TF(tab)
    o_u16, o_f16 = O.Volume(raw), O.Volume(f16, 1.0)
    s16 = O.Stack(o_f16, otf, light, n, res)
    # stack: 2^-tau (base-2 optical depth) against the oracle's transmittance, sampled columns
    T_gpu = np.exp2(-tau) if sdt == vi.VI_BF16 else tau      # (half stacks hold T itself)
    T_ref = np.stack([s16.column(i, j) for i, j in ij], axis=1)
    err_T = float(np.abs(T_gpu - T_ref).max())
    _, ref16, _, _ = O.render(o_f16, otf, s16, cam, mode, 0.5, opts, pixels=pix, want_full=False)
    su = O.Stack(o_u16, otf, light, n, res)
    _, refu, _, _ = O.render(o_u16, otf, su, cam, mode, 0.5, opts, pixels=pix, want_full=False)
    g = got[pix]
    return err_T, (np.abs(g - refu).max(), psnr(g, refu)), (np.abs(g - ref16).max(), psnr(g, ref16))


def _pixels(W_, H_, stride):
    ys, xs = np.meshgrid(np.arange(stride // 2, H_, stride), np.arange(stride // 2, W_, stride), indexing="ij")
    return (ys * W_ + xs).ravel().astype(np.int64)


@pytest.mark.parametrize("layout", [vi.VI_STACK_TILED, vi.VI_STACK_ROWS])
@pytest.mark.parametrize("mode", ["shell", "cone"])
def test_precision_form_medium(mode, layout):
    cam = W.camera_orbit(512, 384, 1.0, math.radians(20))
    light = W.light_from_angles(0.3, math.radians(35))
    err_T, (mu, pu), (m16, p16) = _precision_case(256, 256, 512, cam, light, mode, {}, _pixels(512, 384, 4), layout)
    print(f"[precision] 256^3 {mode} layout {layout}: stack |dT| {err_T:.2e}; vs u16 oracle max-abs {mu:.2e} PSNR {pu:.1f} dB; "
          f"vs f16 oracle max-abs {m16:.2e} PSNR {p16:.1f} dB", flush=True)
    assert err_T < 4e-3          # bfloat16 optical depth: |dT| <= T tau 2^-8
    assert p16 >= 50.0 and pu >= 50.0


@pytest.mark.parametrize("mode", ["shell", "cone"])
def test_precision_form_full_size_sampled(mode):
    """1024^3 FP16 volume, 512 slabs x 1024^2 bfloat16 (row layout, as benchmarked), 1920x1080 -- on a
    pixel sample."""
    w = W.WORKLOADS["precision"]
    cam = w.camera(0)
    light = w.lights()[0]
    err_T, (mu, pu), (m16, p16) = _precision_case(w.N, w.n_slices, w.res, cam, light, mode, {},
                                                  _pixels(cam["width"], cam["height"], 16))
    print(f"[precision] 1024^3 {mode}: stack |dT| {err_T:.2e}; vs u16 oracle max-abs {mu:.2e} PSNR {pu:.1f} dB; "
          f"vs f16 oracle max-abs {m16:.2e} PSNR {p16:.1f} dB", flush=True)
    assert err_T < 4e-3
    assert p16 >= 50.0 and pu >= 50.0


@pytest.mark.parametrize("mode", ["shell", "cone"])
def test_half_transmittance_stack(mode):
    """The half-precision transmittance stack (optical depth summed in float, stored as
    2^-tau in half precision): 256^3 in full on a pixel grid and 1024^3 sampled."""
    cam = W.camera_orbit(512, 384, 1.0, math.radians(20))
    light = W.light_from_angles(0.3, math.radians(35))
    err_T, (mu, pu), (m16, p16) = _precision_case(256, 256, 512, cam, light, mode, {}, _pixels(512, 384, 4),
                                                  sdt=vi.VI_F16)
    print(f"[precision] half stack 256^3 {mode}: stack |dT| {err_T:.2e}; vs u16 oracle max-abs {mu:.2e} "
          f"PSNR {pu:.1f} dB; vs f16 oracle max-abs {m16:.2e} PSNR {p16:.1f} dB", flush=True)
    assert err_T < 1e-3          # half precision: |dT| <= T 2^-11 (+ float optical depth)
    assert p16 >= 50.0 and pu >= 50.0
    w = W.WORKLOADS["precision"]
    cam = w.camera(0)
    err_T, (mu, pu), (m16, p16) = _precision_case(w.N, w.n_slices, w.res, cam, w.lights()[0], mode, {},
                                                  _pixels(cam["width"], cam["height"], 16), sdt=vi.VI_F16)
    print(f"[precision] half stack 1024^3 {mode}: stack |dT| {err_T:.2e}; vs u16 oracle max-abs {mu:.2e} "
          f"PSNR {pu:.1f} dB; vs f16 oracle max-abs {m16:.2e} PSNR {p16:.1f} dB", flush=True)
    assert err_T < 1e-3
    assert p16 >= 50.0 and pu >= 50.0
