"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

FP32 path: max-abs <= 1e-4 per RGBA channel, element by element, on the same
seeded inputs -- full images at the small size, sampled pixels and stack
columns (the oracle computes those one by one) at the medium and large sizes,
in the launch configuration the benchmark times.  Edge cases: empty volume,
ragged image and slice sizes, one slab, odd volume edges, rays that miss.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2008_06134_amd import vi
from paper_2008_06134_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_IMG = 1e-4      # per RGBA channel, FP32 path
TOL_STACK = 2e-5    # transmittance, FP32 product over <= 512 slabs

DEV = "cuda"
LAYOUTS = (vi.VI_STACK_TILED, vi.VI_STACK_ROWS)
LNAME = {vi.VI_STACK_TILED: "tiled", vi.VI_STACK_ROWS: "rows"}


def _mode(m):
    return ("cone", {"cone_grid": 5}) if m == "cone5" else (m, {})


def gpu_inputs(raw, tab, scale=None, quads=True, cell=16, bits=False):
    """Device volume -- with quads=True and bits=True as the benchmark runs it:
    the quad layout (4x4x4 bricks of 2x2 neighbourhoods) with an empty-space
    map of 16^3-voxel cells and its occupancy bits for the TF -- and TF."""
    vol = vi.Volume.from_numpy(raw, DEV, scale)
    if quads:
        vol = vol.to_quads()
    tf = vi.TF.from_numpy(tab, DEV)
    if cell:
        vol = vol.with_minmax(cell)
        if bits:
            vol = vol.with_occupancy(tf)
    return vol, tf


def gpu_render(vol, tf, st, cam, mode, step, opts=None):
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    img = vi.render(vol, tf, st, cam, mode, step, opts, samples=cnt)
    torch.cuda.synchronize()
    return img.cpu().double().numpy(), int(cnt.item())


def report(name, err):
    print(f"[parity] {name}: max-abs {err:.3e}", flush=True)


# ---------------------------------------------------------------- small workload, full images

@pytest.mark.parametrize("mode", ["shell", "shadow", "cone", "cone5", "none"])
def test_small_full_image(mode):
    w = W.WORKLOADS["small"]
    raw, tab = w.volume(), w.tf()
    light = w.lights()[0]
    vol, tf = gpu_inputs(raw, tab, bits=True)
    ost = O.Stack(O.Volume(raw), O.TF(tab), light, w.n_slices, w.res)
    S = ost.export()
    cam = w.camera()
    m, extra = _mode(mode)
    opts = {"bg": [0.1, 0.05, 0.02, 0.3], **extra}
    _, ref, nt, nf = O.render(O.Volume(raw), O.TF(tab), ost, cam, m, w.step_vox, opts, want_full=False)
    for lay in LAYOUTS:
        st = vi.build_attenuation(vol, tf, light, w.n_slices, w.res, layout=lay)
        err_s = np.abs(st.dense().cpu().double().numpy() - S).max()
        report(f"small stack ({LNAME[lay]})", err_s)
        assert err_s <= TOL_STACK
        img, ns = gpu_render(vol, tf, st, cam, m, w.step_vox, opts)
        err = np.abs(img - ref).max()
        report(f"small {mode} ({LNAME[lay]})", err)
        assert err <= TOL_IMG
        assert abs(ns - nt.sum()) <= 1e-3 * nt.sum() + 16
        # the second counter: segments composited with non-zero opacity (a
        # subset of those marched; the same count again in the same launch)
        cnt = torch.zeros(2, dtype=torch.int64, device=DEV)
        img2 = vi.render(vol, tf, st, cam, m, w.step_vox, opts, samples=cnt)
        torch.cuda.synchronize()
        n2, nop = int(cnt[0].item()), int(cnt[1].item())
        assert n2 == ns and 0 < nop <= n2
        assert torch.equal(img2.cpu().double(), torch.from_numpy(img))


# ---------------------------------------------------------------- medium / large, sampled

def _sample_pixels(W_, H_, count, seed):
    rng = np.random.default_rng(seed)
    pix = rng.choice(W_ * H_, size=count, replace=False)
    # plus a full middle row and column (ragged-tile edges included)
    row = (H_ // 2) * W_ + np.arange(W_)
    col = np.arange(H_) * W_ + W_ // 2
    return np.unique(np.concatenate([pix, row, col]))


def _sampled_parity(name, raw, tab, light, n, res, cam, mode, step, opts, npix, seed, cols=1500):
    """Both stack layouts against one oracle reference (sampled stack columns and pixels), with the
    volume as the benchmark prepares it (quads, map, occupancy bits)."""
    vol, tf = gpu_inputs(raw, tab, bits=True)
    ovol, otf = O.Volume(raw), O.TF(tab)
    ost = O.Stack(ovol, otf, light, n, res)
    rng = np.random.default_rng(seed + 1)
    ij = rng.integers(0, res, size=(cols, 2))
    want = np.stack([ost.column(i, j) for i, j in ij], axis=1)
    pix = _sample_pixels(cam["width"], cam["height"], npix, seed)
    _, ref, nt, _ = O.render(ovol, otf, ost, cam, mode, step, opts, pixels=pix, want_full=False)
    for lay in LAYOUTS:
        st = vi.build_attenuation(vol, tf, light, n, res, layout=lay)
        torch.cuda.synchronize()
        S = st.dense()
        got = S[:, torch.as_tensor(ij[:, 1], device=DEV), torch.as_tensor(ij[:, 0], device=DEV)]
        err_s = np.abs(got.cpu().double().numpy() - want).max()
        report(f"{name} stack columns ({LNAME[lay]})", err_s)
        assert err_s <= TOL_STACK
        del S, got
        img, ns = gpu_render(vol, tf, st, cam, mode, step, opts)
        del st
        got = img.reshape(-1, 4)[pix]
        err = np.abs(got - ref).max()
        worst = pix[np.argmax(np.abs(got - ref).max(axis=1))]
        report(f"{name} {mode} {LNAME[lay]} ({pix.size} px, worst pixel {worst % cam['width']},"
               f"{worst // cam['width']})", err)
        assert err <= TOL_IMG


@pytest.fixture(scope="module")
def medium():
    w = W.WORKLOADS["medium"]
    return w, w.volume(), w.tf()


def test_medium_cone5x5_sampled(medium):
    w, raw, tab = medium
    _sampled_parity("medium", raw, tab, w.lights()[0], w.n_slices, w.res, w.camera(), "cone", w.step_vox,
                    {"cone_grid": 5}, 3000, seed=11)


@pytest.mark.parametrize("mode", ["shell", "cone"])
def test_medium_other_modes_sampled(medium, mode):
    w, raw, tab = medium
    _sampled_parity("medium", raw, tab, w.lights()[0], w.n_slices, w.res, w.camera(), mode, w.step_vox,
                    {}, 1500, seed=12)


@pytest.fixture(scope="module")
def large():
    w = W.WORKLOADS["large"]
    return w, w.volume(), w.tf()


@pytest.mark.parametrize("light_index,mode", [(0, "shell"), (0, "cone"), (5, "shell"), (11, "cone")])
def test_large_sampled(large, light_index, mode):
    w, raw, tab = large
    light = w.lights()[light_index]
    _sampled_parity(f"large[{light_index}]", raw, tab, light, w.n_slices, w.res, w.camera(light_index), mode,
                    w.step_vox, {}, 1500, seed=20 + light_index, cols=800)


# ---------------------------------------------------------------- edge cases

def test_empty_volume_is_background_exactly():
    raw = np.zeros((24, 24, 24), np.uint8)
    tab = W.tf_ramp()
    vol, tf = gpu_inputs(raw, tab)
    st = vi.build_attenuation(vol, tf, [0.2, 0.5, -1], 7, 19)
    assert torch.all(st.dense() == 1.0)
    bg = [0.1, 0.2, 0.3, 0.4]
    for m in ["shadow", "shell", "cone", "cone5", "none"]:
        mm, extra = _mode(m)
        img, ns = gpu_render(vol, tf, st, W.camera_orbit(37, 23, 0.3, 0.2), mm, 0.5, {"bg": bg, **extra})
        assert np.all(img == np.asarray(bg, dtype=np.float32).astype(np.float64))
        assert ns > 0


def test_constant_cube_closed_form():
    """Unlit constant cube, orthographic chord 1: alpha = 1-(1-a0)^N, C = rgb alpha."""
    N, a0, rgb = 32, 0.03, [0.9, 0.6, 0.3]
    raw = np.full((N, N, N), 100, np.uint8)
    tab = np.tile(np.array(rgb + [a0]), (256, 1))
    vol, tf = gpu_inputs(raw, tab)
    cam = W.camera_ortho_front(40, 40, half_h=0.75)
    img, ns = gpu_render(vol, tf, None, cam, "none", 0.5)
    a_pix = 1 - (1 - a0) ** N
    xs = 0.5 + (2 * (np.arange(40) + 0.5) / 40 - 1) * 0.75
    inside = (xs > 0) & (xs < 1)
    sel = img[np.ix_(inside, inside)]
    np.testing.assert_allclose(sel[..., :3], np.broadcast_to(np.array(rgb) * a_pix, sel[..., :3].shape), atol=5e-6)
    np.testing.assert_allclose(sel[..., 3], a_pix, atol=5e-6)
    assert ns == int(inside.sum()) ** 2 * 2 * N


@pytest.mark.parametrize("N,n,res,W_,H_,light,kind", [
    (33, 1, 50, 37, 23, [0.3, -0.8, 0.5], "persp"),    # odd edge, one slab, ragged slices and image
    (20, 9, 17, 1, 1, [1, 1, -1], "persp"),            # a single pixel
    (16, 5, 3, 64, 17, [0, 0, -1], "ortho"),           # very coarse stack, axis light
    (48, 64, 96, 50, 70, [-1, 0.1, 0.2], "persp"),     # slab thinner than a voxel
])
@pytest.mark.parametrize("mode", ["shell", "cone", "cone5"])
def test_ragged_and_degenerate_shapes(N, n, res, W_, H_, light, kind, mode):
    raw = W.sphere_u8(N, radius=N * 0.3, density=190, noise=25, seed=N)
    tab = W.tf_ramp()
    vol, tf = gpu_inputs(raw, tab)
    ost = O.Stack(O.Volume(raw), O.TF(tab), light, n, res)
    cam = W.camera_orbit(W_, H_, 0.8, 0.4, distance=1.8) if kind == "persp" else W.camera_ortho_front(W_, H_)
    m, extra = _mode(mode)
    opts = {"bg": [0.2, 0.1, 0.0, 0.5], "ambient": 0.15, **extra}
    _, ref, nt, _ = O.render(O.Volume(raw), O.TF(tab), ost, cam, m, 0.5, opts, want_full=False)
    for lay in LAYOUTS:
        st = vi.build_attenuation(vol, tf, light, n, res, layout=lay)
        err_s = np.abs(st.dense().cpu().double().numpy() - ost.export()).max()
        assert err_s <= TOL_STACK
        img, ns = gpu_render(vol, tf, st, cam, m, 0.5, opts)
        err = np.abs(img - ref).max()
        report(f"ragged N={N} n={n} res={res} {W_}x{H_} {mode} {LNAME[lay]}", err)
        assert err <= TOL_IMG


@pytest.mark.parametrize("dtype", [np.uint16, np.float16, np.float32])
def test_volume_dtypes(dtype):
    N = 40
    base = W.ct_phantom_u16(N, seed=9)
    if dtype == np.uint16:
        raw, scale = base, None
    elif dtype == np.float16:
        raw, scale = W.to_f16_normalised(base), 1.0
    else:
        raw, scale = (base / 4095.0).astype(np.float32), 1.0
    tab = W.tf_ct()
    vol, tf = gpu_inputs(raw, tab, scale)
    light = [0.4, 0.3, -0.8]
    st = vi.build_attenuation(vol, tf, light, 40, 64)
    ovol = O.Volume(raw, scale)
    ost = O.Stack(ovol, O.TF(tab), light, 40, 64)
    assert np.abs(st.dense().cpu().double().numpy() - ost.export()).max() <= TOL_STACK
    cam = W.camera_orbit(48, 40, 1.0, 0.35)
    img, _ = gpu_render(vol, tf, st, cam, "shell", 0.5)
    _, ref, _, _ = O.render(ovol, O.TF(tab), ost, cam, "shell", 0.5, want_full=False)
    assert np.abs(img - ref).max() <= TOL_IMG


def test_termination_off_matches_full_oracle():
    w = W.WORKLOADS["small"]
    raw, tab = w.volume(), w.tf()
    vol, tf = gpu_inputs(raw, tab)
    light = w.lights()[0]
    st = vi.build_attenuation(vol, tf, light, w.n_slices, w.res)
    ost = O.Stack(O.Volume(raw), O.TF(tab), light, w.n_slices, w.res)
    cam = w.camera(W=96, H=96)
    img, ns = gpu_render(vol, tf, st, cam, "shell", 0.5, {"term_eps": 0.0})
    full, _, _, nf = O.render(O.Volume(raw), O.TF(tab), ost, cam, "shell", 0.5)
    assert np.abs(img - full).max() <= TOL_IMG
    # with term_eps = 0 a float32 ray still stops once its opacity rounds to 1
    assert 0.5 * nf.sum() < ns <= nf.sum()


@pytest.mark.parametrize("N", [64, 33, 6])
def test_brick_layout_matches_its_definition(N):
    rng = np.random.default_rng(N)
    raw = rng.integers(0, 4096, size=(N, N, N)).astype(np.uint16)
    lin = vi.Volume.from_numpy(raw, DEV)
    br = lin.to_bricks()
    torch.cuda.synchronize()
    NP = (N + 3) // 4 * 4
    nb = NP // 4
    got = br.data.cpu().numpy().view(np.uint16)
    assert got.size == NP ** 3
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    off = ((z // 4) * nb * nb + (y // 4) * nb + x // 4) * 64 + (z % 4) * 16 + (y % 4) * 4 + x % 4
    assert np.array_equal(got[off], raw)


@pytest.mark.parametrize("N", [64, 33, 6])
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16, np.float16, np.float32])
def test_quad_layout_matches_its_definition(N, dtype):
    """Slot (x,y,z) of the quad layout holds v(x,y,z), v(x+1,y,z), v(x,y+1,z),
    v(x+1,y+1,z) (indices clamped to N-1) at 4 * brick offset."""
    rng = np.random.default_rng(N + 7)
    raw = rng.integers(0, 4096 if dtype == np.uint16 else 256, size=(N, N, N)).astype(dtype)
    q = vi.Volume.from_numpy(raw, DEV).to_quads()
    torch.cuda.synchronize()
    NP = (N + 3) // 4 * 4
    nb = NP // 4
    got = q.data.cpu().numpy().view(raw.dtype)
    assert got.size == 4 * NP ** 3
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    off = 4 * (((z // 4) * nb * nb + (y // 4) * nb + x // 4) * 64 + (z % 4) * 16 + (y % 4) * 4 + x % 4)
    x1, y1 = np.minimum(x + 1, N - 1), np.minimum(y + 1, N - 1)
    for c, (yy, xx) in enumerate([(y, x), (y, x1), (y1, x), (y1, x1)]):
        assert np.array_equal(got[off + c], raw[z, yy, xx])


@pytest.mark.parametrize("N,n,res", [(64, 32, 64), (33, 7, 50)])
@pytest.mark.parametrize("mode", ["shell", "cone", "cone5", "phong"])
def test_bricked_volume_gives_bitwise_identical_results(N, n, res, mode):
    """Linear, brick and quad layouts: identical stacks, images and sample counts."""
    raw = W.sphere_u8(N, radius=N * 0.35, density=180, noise=30, seed=N + 1)
    tab = W.tf_ramp()
    lin, tf = gpu_inputs(raw, tab, quads=False, cell=0)
    light = [0.6, -0.3, -0.74]
    s1 = vi.build_attenuation(lin, tf, light, n, res)
    m, extra = _mode(mode)
    cam = W.camera_orbit(70, 50, 2.2, 0.5)
    a, na = gpu_render(lin, tf, s1, cam, m, 0.5, extra)
    for other in (lin.to_bricks(), lin.to_quads(), lin.to_quads().with_minmax(8)):
        s2 = vi.build_attenuation(other, tf, light, n, res)
        torch.cuda.synchronize()
        assert torch.equal(s1.dense(), s2.dense())   # padding texels of the tiles are never written
        s2.s.tag = 0  # stack built from the other copy, rendered with either
        b, nb = gpu_render(other, tf, s2, cam, m, 0.5, extra)
        assert np.array_equal(a, b) and na == nb


def test_quad_layout_point_light_and_map():
    """The quad layout under a point light and with its own empty-space map
    (which equals the linear volume's map)."""
    raw = W.ct_phantom_u16(40, seed=9, vessels=True)
    tab = W.tf_ct()
    lin, tf = gpu_inputs(raw, tab, quads=False, cell=0)
    q = lin.to_quads()
    ml, mq = lin.with_minmax(8), q.with_minmax(8)
    torch.cuda.synchronize()
    assert torch.equal(ml.minmax, mq.minmax)
    pos = [1.8, 0.2, 1.5]
    s1 = vi.build_attenuation(ml, tf, None, 30, 48, position=pos)
    s2 = vi.build_attenuation(mq, tf, None, 30, 48, position=pos)
    torch.cuda.synchronize()
    assert torch.equal(s1.dense(), s2.dense())
    cam = W.camera_orbit(64, 48, 0.9, 0.4)
    s1.s.tag = 0  # one stack, rendered with either copy of the volume
    for m in ("shadow", "shell"):
        a, na = gpu_render(ml, tf, s1, cam, m, 0.5)
        b, nb = gpu_render(mq, tf, s1, cam, m, 0.5)
        assert np.array_equal(a, b) and na == nb


@pytest.mark.parametrize("cell", [4, 8, 16, 32])
@pytest.mark.parametrize("mode", ["shell", "cone5", "none"])
def test_empty_space_map_changes_nothing(cell, mode):
    """Skipping zero-opacity cells must give bit-identical stacks, images and counts."""
    raw = W.ct_phantom_u16(48, seed=5, vessels=True)
    tab = W.tf_ct()
    plain, tf = gpu_inputs(raw, tab, cell=0)
    mapped = plain.with_minmax(cell)
    light = [0.3, 0.4, -0.86]
    s1 = vi.build_attenuation(plain, tf, light, 40, 72)
    s2 = vi.build_attenuation(mapped, tf, light, 40, 72)
    torch.cuda.synchronize()
    assert torch.equal(s1.dense(), s2.dense())
    m, extra = _mode(mode)
    cam = W.camera_orbit(90, 60, 0.7, 0.3)
    a, na = gpu_render(plain, tf, s1, cam, m, 0.5, extra)
    b, nb = gpu_render(mapped, tf, s1, cam, m, 0.5, extra)
    assert np.array_equal(a, b) and na == nb
    # with small cells the map does mark some cells empty (and others not)
    mm = mapped.minmax.view(-1, 2).cpu().numpy()
    assert (mm[:, 1] >= 0.2).any()
    if cell <= 8:
        assert (mm[:, 1] < 0.2).any()


def test_stack_is_camera_independent_and_deterministic():
    w = W.WORKLOADS["small"]
    raw, tab = w.volume(), w.tf()
    vol, tf = gpu_inputs(raw, tab)
    a = vi.build_attenuation(vol, tf, w.lights()[0], w.n_slices, w.res)
    b = vi.build_attenuation(vol, tf, w.lights()[0], w.n_slices, w.res)
    torch.cuda.synchronize()
    assert torch.equal(a.dense(), b.dense())
    S = a.dense()
    assert float(S.min()) >= 0.0 and float(S.max()) <= 1.0
    assert bool(torch.all(S[1:] <= S[:-1]))
    cam = w.camera()
    i1 = vi.render(vol, tf, a, cam, "shell", 0.5).clone()
    i2 = vi.render(vol, tf, a, cam, "shell", 0.5)
    torch.cuda.synchronize()
    assert torch.equal(i1, i2)


@pytest.mark.parametrize("res,n", [(1, 11), (6, 11), (19, 11), (64, 11), (64, 1), (64, 2), (45, 3)])
@pytest.mark.parametrize("dtype", [vi.VI_F32, vi.VI_BF16])
def test_row_layout_matches_its_definition(res, n, dtype):
    """Row layout: the grid row-major with a two-texel border and a leading
    layer that transmit fully (T = 1, optical depth 0) and a trailing layer
    equal to the last; interior bit for bit equal to the tiled stack.  The
    sizes span one and several workgroup runs per layer, and one, two and
    an odd number of slabs (the build pairs slabs and rotates every other
    layer by half a line)."""
    raw = W.sphere_u8(30, radius=10, density=200, noise=30, seed=res)
    vol, tf = gpu_inputs(raw, W.tf_ramp())
    light = [0.3, -0.5, 0.8]
    t = vi.build_attenuation(vol, tf, light, n, res, dtype, layout=vi.VI_STACK_TILED)
    r = vi.build_attenuation(vol, tf, light, n, res, dtype, layout=vi.VI_STACK_ROWS)
    torch.cuda.synchronize()
    D = t.dense()
    ring = 1.0 if dtype == vi.VI_F32 else 0.0
    want = torch.full((n + 2, res + 4, res + 4), ring, dtype=D.dtype, device=DEV)
    want[1:n + 1, 2:res + 2, 2:res + 2] = D
    want[n + 1] = want[n]      # the trailing layer repeats the last
    assert r.data.shape == (n + 2, res + 4, vi.row_pitch(res, dtype))
    assert torch.equal(r.padded(), want)
    assert torch.equal(r.dense(), D)
    # lookups from either layout, the first and last layers included, agree bit for bit
    cam = W.camera_orbit(40, 32, 0.7, 0.3)
    for mode, opts in (("shell", {}), ("cone", {}), ("shadow", {"nearest_layer": 1})):
        a = vi.render(vol, tf, t, cam, mode, 0.5, opts)
        b = vi.render(vol, tf, r, cam, mode, 0.5, opts)
        torch.cuda.synchronize()
        assert torch.equal(a, b), mode


@pytest.mark.parametrize("res", [1, 19, 64])
def test_half_stack_matches_its_definition(res):
    """Half-precision stack (row layout only): border and leading layer hold 1, every texel
    is the float stack's transmittance within half precision's rounding (relative 2^-11,
    plus the float optical depth's own rounding), and the tiled layout is refused."""
    raw = W.sphere_u8(30, radius=10, density=200, noise=30, seed=res)
    vol, tf = gpu_inputs(raw, W.tf_ramp())
    light, n = [0.3, -0.5, 0.8], 11
    f = vi.build_attenuation(vol, tf, light, n, res, vi.VI_F32, layout=vi.VI_STACK_ROWS)
    h = vi.build_attenuation(vol, tf, light, n, res, vi.VI_F16, layout=vi.VI_STACK_ROWS)
    torch.cuda.synchronize()
    assert h.data.dtype == torch.float16 and h.data.shape == (n + 2, res + 4, vi.row_pitch(res, vi.VI_F16))
    P = h.padded().float()
    ring = torch.ones_like(P)
    ring[1:, 2:res + 2, 2:res + 2] = 0.0
    assert torch.all(P[ring > 0] == 1.0)
    assert torch.equal(P[n + 1], P[n])      # the trailing layer repeats the last
    T32, T16 = f.dense().double(), h.dense().double()
    err = float(((T16 - T32).abs() - T32 * 2.0 ** -11).max())
    report(f"half stack res {res} vs float stack (beyond 2^-11 T)", err)
    assert err <= 2e-6
    with pytest.raises(vi.VIError) as e:
        vi.build_attenuation(vol, tf, light, n, res, vi.VI_F16, layout=vi.VI_STACK_TILED)
    assert e.value.code == -2


@pytest.mark.parametrize("dtype", [vi.VI_F32, vi.VI_BF16])
@pytest.mark.parametrize("mode", ["shadow", "shell", "cone", "cone5"])
def test_row_layout_gives_bitwise_identical_images(dtype, mode):
    raw = W.ct_phantom_u16(56, seed=6, vessels=True)
    vol, tf = gpu_inputs(raw, W.tf_ct())
    light = [-0.4, 0.7, 0.6]
    m, extra = _mode(mode)
    cam = W.camera_orbit(83, 61, 1.9, 0.45)
    out = []
    for lay in LAYOUTS:
        st = vi.build_attenuation(vol, tf, light, 45, 77, dtype, layout=lay)
        out.append(gpu_render(vol, tf, st, cam, m, 0.5, extra))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]


@pytest.mark.parametrize("darken", [0.5, 1.0, 2.5])
def test_darkening_compensation_parity(darken):
    """Section 4's (1+alpha)^m slab compensation in the build, both stack layouts."""
    w = W.WORKLOADS["small"]
    raw, tab = w.volume(), w.tf()
    vol, tf = gpu_inputs(raw, tab)
    light = w.lights()[0]
    ost = O.Stack(O.Volume(raw), O.TF(tab), light, w.n_slices, w.res, darken=darken)
    S = ost.export()
    cam = w.camera(W=96, H=80)
    _, ref, _, _ = O.render(O.Volume(raw), O.TF(tab), ost, cam, "shell", w.step_vox, want_full=False)
    plain = O.Stack(O.Volume(raw), O.TF(tab), light, w.n_slices, w.res)
    _, ref0, _, _ = O.render(O.Volume(raw), O.TF(tab), plain, cam, "shell", w.step_vox, want_full=False)
    assert np.abs(ref - ref0).max() > 1e-2            # the option visibly changes the image
    for lay in LAYOUTS:
        st = vi.build_attenuation(vol, tf, light, w.n_slices, w.res, layout=lay, darken=darken)
        assert st.s.darken == darken
        err_s = np.abs(st.dense().cpu().double().numpy() - S).max()
        img, _ = gpu_render(vol, tf, st, cam, "shell", w.step_vox)
        err = np.abs(img - ref).max()
        report(f"darken m={darken} {LNAME[lay]}: stack {err_s:.2e}", err)
        assert err_s <= TOL_STACK and err <= TOL_IMG


def test_darkening_bf16_optical_depth():
    """bfloat16 optical depth with the compensation: 2^-tau against the oracle's columns."""
    w = W.WORKLOADS["medium"]
    raw, tab = w.volume(), w.tf()
    vol, tf = gpu_inputs(raw, tab)
    light = w.lights()[0]
    st = vi.build_attenuation(vol, tf, light, 64, 128, vi.VI_BF16, layout=vi.VI_STACK_ROWS, darken=1.5)
    ost = O.Stack(O.Volume(raw), O.TF(tab), light, 64, 128, darken=1.5)
    rng = np.random.default_rng(3)
    ij = rng.integers(0, 128, size=(300, 2))
    tau = st.dense()[:, torch.as_tensor(ij[:, 1], device=DEV), torch.as_tensor(ij[:, 0], device=DEV)]
    got = np.exp2(-tau.float().cpu().double().numpy())
    want = np.stack([ost.column(i, j) for i, j in ij], axis=1)
    err = np.abs(got - want).max()
    report("darken bf16 stack columns", err)
    assert err < 4e-3


@pytest.mark.parametrize("shells,weights", [(2, [1, 0]), (2, [0.25, 1]), (3, [3, 2, 1]), (3, [])])
def test_weighted_shells_parity(shells, weights):
    w = W.WORKLOADS["small"]
    raw, tab = w.volume(), w.tf()
    vol, tf = gpu_inputs(raw, tab)
    light = w.lights()[0]
    ost = O.Stack(O.Volume(raw), O.TF(tab), light, w.n_slices, w.res)
    cam = w.camera(W=96, H=80)
    opts = {"shell_count": shells, "shell_w": weights}
    _, ref, _, _ = O.render(O.Volume(raw), O.TF(tab), ost, cam, "shell", w.step_vox, opts, want_full=False)
    _, ref1, _, _ = O.render(O.Volume(raw), O.TF(tab), ost, cam, "shell", w.step_vox, want_full=False)
    if weights != [1, 0]:                              # (1, 0) is the one-voxel shell itself
        assert np.abs(ref - ref1).max() > 1e-2
    for lay in LAYOUTS:
        st = vi.build_attenuation(vol, tf, light, w.n_slices, w.res, layout=lay)
        img, _ = gpu_render(vol, tf, st, cam, "shell", w.step_vox, opts)
        err = np.abs(img - ref).max()
        report(f"shells {shells} weights {weights} {LNAME[lay]}", err)
        assert err <= TOL_IMG


def test_coloured_light_parity():
    """Light colour (R17) scales the emission per channel, every gather mode."""
    w = W.WORKLOADS["small"]
    raw, tab = w.volume(), w.tf()
    vol, tf = gpu_inputs(raw, tab)
    light = w.lights()[0]
    ost = O.Stack(O.Volume(raw), O.TF(tab), light, w.n_slices, w.res)
    st = vi.build_attenuation(vol, tf, light, w.n_slices, w.res, layout=vi.VI_STACK_ROWS)
    cam = w.camera(W=80, H=64)
    opts = {"light_rgb": [1.0, 0.7, 0.35], "ambient": 0.2}
    for mode in ["shadow", "shell", "cone"]:
        _, ref, _, _ = O.render(O.Volume(raw), O.TF(tab), ost, cam, mode, w.step_vox, opts, want_full=False)
        img, _ = gpu_render(vol, tf, st, cam, mode, w.step_vox, opts)
        err = np.abs(img - ref).max()
        report(f"coloured light {mode}", err)
        assert err <= TOL_IMG


# ---------------------------------------------------------------- occupancy bits

def _occupancy_reference(mm, tab):
    """Bit per cell: some transfer-function entry the cell's value range can
    interpolate (widened by one entry each side) has non-zero opacity."""
    K = tab.shape[0]
    lo = np.maximum((mm[:, 0].astype(np.float32) * np.float32(K - 1)).astype(np.int64) - 1, 0)
    hi = np.minimum((mm[:, 1].astype(np.float32) * np.float32(K - 1)).astype(np.int64) + 2, K - 1)
    opaque = np.flatnonzero(tab[:, 3] > 0)
    occ = np.zeros(mm.shape[0], bool)
    for c in range(mm.shape[0]):
        occ[c] = np.any((opaque >= lo[c]) & (opaque <= hi[c]))
    return occ


@pytest.mark.parametrize("cell", [4, 8, 16])
def test_occupancy_bits_match_their_definition(cell):
    raw = W.ct_phantom_u16(48, seed=12, vessels=True)
    tab = W.tf_ct()
    vol, tf = gpu_inputs(raw, tab, cell=cell)
    occ = vol.with_occupancy(tf)
    torch.cuda.synchronize()
    mm = vol.minmax.view(-1, 2).cpu().numpy()
    words = occ.occ.cpu().numpy().view(np.uint32)
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1).reshape(-1)[:mm.shape[0]].astype(bool)
    want = _occupancy_reference(mm, tab)
    assert np.array_equal(bits, want)
    assert want.any()
    # super-cells: 4 x 4 x 4 cells each, set where any of their cells is
    nc = -(-48 // cell)
    snc = -(-nc // 4)
    ncw = -(-mm.shape[0] // 32)
    sw = words[ncw:]
    sbits = ((sw[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1).reshape(-1)[:snc ** 3].astype(bool)
    cells = want.reshape(nc, nc, nc)  # z, y, x
    swant = np.zeros((snc, snc, snc), dtype=bool)
    for Z in range(snc):
        for Y in range(snc):
            for X in range(snc):
                swant[Z, Y, X] = cells[4 * Z:4 * Z + 4, 4 * Y:4 * Y + 4, 4 * X:4 * X + 4].any()
    assert np.array_equal(sbits, swant.reshape(-1))
    if cell <= 8:                                  # 27 cells of 16^3 are all occupied here
        assert not want.all()


@pytest.mark.parametrize("N,cell", [(64, 8), (168, 4)])   # bits in LDS; 74088 cells: bits read from memory
@pytest.mark.parametrize("mode", ["none", "shadow", "shell", "cone", "cone5", "phong"])
def test_occupancy_bits_change_nothing(N, cell, mode):
    """Stacks, images and sample counts with the bits equal those with the map alone, bit for bit."""
    raw = W.ct_phantom_u16(N, seed=13, vessels=True)
    tab = W.tf_ct()
    mapped, tf = gpu_inputs(raw, tab, cell=cell)
    bits = mapped.with_occupancy(tf)
    light = [0.35, -0.5, -0.79]
    n, res = N // 2, N
    s1 = vi.build_attenuation(mapped, tf, light, n, res, layout=vi.VI_STACK_ROWS)
    s2 = vi.build_attenuation(bits, tf, light, n, res, layout=vi.VI_STACK_ROWS)
    torch.cuda.synchronize()
    assert torch.equal(s1.dense(), s2.dense())
    m, extra = _mode(mode)
    cam = W.camera_orbit(96, 72, 1.1, 0.35)
    a, na = gpu_render(mapped, tf, s1, cam, m, 0.5, extra)
    b, nb = gpu_render(bits, tf, s1, cam, m, 0.5, extra)
    assert np.array_equal(a, b) and na == nb


def test_occupancy_bits_point_light():
    raw = W.ct_phantom_u16(56, seed=14, vessels=True)
    tab = W.tf_ct()
    mapped, tf = gpu_inputs(raw, tab, cell=8)
    bits = mapped.with_occupancy(tf)
    pos = [-0.9, 1.6, 1.3]
    s1 = vi.build_attenuation(mapped, tf, None, 40, 64, position=pos)
    s2 = vi.build_attenuation(bits, tf, None, 40, 64, position=pos)
    torch.cuda.synchronize()
    assert torch.equal(s1.dense(), s2.dense())
    cam = W.camera_orbit(80, 64, 2.0, 0.3)
    for m in ("shadow", "shell", "phong"):
        a, na = gpu_render(mapped, tf, s1, cam, m, 0.5)
        b, nb = gpu_render(bits, tf, s1, cam, m, 0.5)
        assert np.array_equal(a, b) and na == nb


def test_occupancy_bits_refuse_another_transfer_function():
    raw = W.ct_phantom_u16(32, seed=15)
    vol, tf = gpu_inputs(raw, W.tf_ct(), cell=8)
    bits = vol.with_occupancy(tf)
    other = vi.TF.from_numpy(W.tf_ramp(), DEV)
    with pytest.raises(vi.VIError):
        vi.build_attenuation(bits, other, [0, 0, 1], 16, 32)


def test_rewritten_transfer_function_is_refused():
    """A table rewritten in place (same device address, new contents) names
    another identity: occupancy bits and stacks made with the old contents
    are refused, not silently reused."""
    raw = W.ct_phantom_u16(32, seed=16)
    vol, tf = gpu_inputs(raw, W.tf_ct(), cell=8)
    bits = vol.with_occupancy(tf)
    st = vi.build_attenuation(bits, tf, [0, 0, 1], 16, 32)
    torch.cuda.synchronize()
    tf.data.copy_(torch.from_numpy(W.tf_ramp()).to(DEV))   # same pointer, other table
    again = vi.TF(tf.data)
    assert again.data.data_ptr() == tf.data.data_ptr()
    with pytest.raises(vi.VIError):
        vi.build_attenuation(bits, again, [0, 0, 1], 16, 32)
    cam = {"kind": "ortho", "eye": [0.5, -2.0, 0.5], "target": [0.5, 0.5, 0.5], "up": [0, 0, 1],
           "ortho_half_h": 0.75, "width": 16, "height": 16}
    with pytest.raises(vi.VIError):
        vi.render(vol, again, st, cam, "shell", 0.5)


@pytest.mark.parametrize("dtype", [vi.VI_F32, vi.VI_BF16])
def test_out_of_range_tf_opacity_is_clamped(dtype):
    """A table whose opacity runs from -0.1 to 1.1: the build and the render both take the
    interpolated opacity clamped to [0, 1] (a <= 0 transmits, a >= 1 is opaque), as the oracle does;
    stack and image against the oracle, occupancy bits on."""
    raw = W.sphere_u8(48, radius=18, density=150, noise=60, seed=12)
    tab = W.tf_ramp().copy()
    tab[:, 3] = np.linspace(-0.1, 1.1, tab.shape[0])
    vol, tf = gpu_inputs(raw, tab, bits=True)
    light, n, res = [0.3, -0.4, 0.87], 40, 72
    ovol, otf = O.Volume(raw), O.TF(tab)
    ost = O.Stack(ovol, otf, light, n, res)
    st = vi.build_attenuation(vol, tf, light, n, res, dtype, layout=vi.VI_STACK_ROWS)
    torch.cuda.synchronize()
    S = st.dense().float().cpu().double().numpy()
    T = S if dtype == vi.VI_F32 else np.exp2(-S)
    err_s = float(np.abs(T - ost.export()).max())
    assert float(ost.export().min()) < 1e-3            # some columns are fully shadowed
    cam = W.camera_orbit(80, 64, 0.7, 0.35)
    _, ref, _, _ = O.render(ovol, otf, ost, cam, "shell", 0.5, want_full=False)
    img, _ = gpu_render(vol, tf, st, cam, "shell", 0.5)
    err = float(np.abs(img - ref).max())
    report(f"out-of-range TF opacity ({'f32' if dtype == vi.VI_F32 else 'bf16'}), stack {err_s:.2e}", err)
    if dtype == vi.VI_F32:
        assert err_s <= TOL_STACK and err <= TOL_IMG
    else:
        assert err_s < 4e-3 and err < 5e-3
