"""Closed forms, exact special cases and invariants that pin the oracle (CPU only).

P1 empty volume -> stack 1, image = background, exactly
P2 constant cube, no coefficient: textbook emission-absorption (Eq. 2/3) over the chord
P3 Beer-Lambert stack (Eq. 6): exact for an axis light, within one slab for an oblique one
P5 opaque box: exact shadow footprint for every gather mode
P6 light parallel to view: closed-form limit and convergence
P7 stack lookup vs a dense march toward the light: second-order convergence
P8 reductions (vanishing shell step == direct shadow)
P9 invariants (alpha <= 1, 0 <= C <= alpha, stack monotone, termination bound)
P11 local Phong (section 4's comparison mode): exact gradients of linear fields, closed-form
    ramp images for diffuse-only, specular-only, oblique and flat-field lighting, the unlit
    reduction, and the lit side of a sphere
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2008_06134_amd import workloads as W

SQ3 = math.sqrt(3.0)
MODES = ["shadow", "shell", "cone", "cone5"]


def _mode(m):
    return ("cone", {"cone_grid": 5}) if m == "cone5" else (m, {})


def _const_tf(rgba):
    return O.TF(np.tile(np.asarray(rgba, float), (256, 1)))


def _tf_zero_then(rgba):
    """alpha 0 at value 0, the given rgba for every other entry (value 0 stays empty)."""
    t = np.tile(np.asarray(rgba, float), (256, 1))
    t[0] = [0, 0, 0, 0]
    return O.TF(t)


# ------------------------------------------------------------------ P1

@pytest.mark.parametrize("mode", ["none"] + MODES)
@pytest.mark.parametrize("kind", ["ortho", "persp"])
def test_p1_empty_volume_gives_background(mode, kind):
    raw = np.zeros((12, 12, 12), np.uint8)
    vol, tf = O.Volume(raw), O.TF(W.tf_ramp())
    st = O.Stack(vol, tf, [1, 1, -1], 6, 10)
    assert np.all(st.export() == 1.0)
    bg = [0.1, 0.2, 0.3, 0.4]
    cam = W.camera_ortho_front(10, 8) if kind == "ortho" else W.camera_orbit(10, 8, 0.7, 0.3)
    m, extra = _mode(mode)
    full, term, nt, nf = O.render(vol, tf, st, cam, m, 0.5, {"bg": bg, **extra})
    assert np.all(full == np.asarray(bg)) and np.all(term == np.asarray(bg))
    assert nf.sum() > 0  # rays did hit the cube


# ------------------------------------------------------------------ P2

def test_p2_constant_cube_ortho_chord_one():
    N, a0, rgb = 16, 0.05, [0.9, 0.6, 0.3]
    raw = np.full((N, N, N), 100, np.uint8)
    vol, tf = O.Volume(raw), _const_tf(rgb + [a0])
    cam = W.camera_ortho_front(32, 32, half_h=0.75)
    full, term, nt, nf = O.render(vol, tf, None, cam, "none", 0.5)
    a_pix = 1 - (1 - a0) ** N            # chord 1 = N reference lengths
    hit = 0
    for py in range(32):
        for px in range(32):
            x = 0.5 + (2 * (px + 0.5) / 32 - 1) * 0.75
            z = 0.5 + (1 - 2 * (py + 0.5) / 32) * 0.75
            if 0 < x < 1 and 0 < z < 1:
                hit += 1
                np.testing.assert_allclose(full[py, px], np.array(rgb + [1.0]) * a_pix, rtol=1e-12)
                assert nf[py, px] == 2 * N   # chord / half-voxel step
            elif not (0 <= x <= 1 and 0 <= z <= 1):
                assert np.all(full[py, px] == 0)
    assert hit > 100


@pytest.mark.parametrize("step", [0.5, 0.37, 1.0])
def test_p2_constant_cube_perspective_chords(step):
    """Chord lengths from bisection on the inside indicator, independent of the slab test."""
    N, a0, rgb = 16, 0.08, [0.2, 0.7, 0.5]
    raw = np.full((N, N, N), 77, np.uint8)
    vol, tf = O.Volume(raw), _const_tf(rgb + [a0])
    cam = {"kind": "persp", "eye": [0.45, 0.55, -1.4], "target": [0.5, 0.5, 0.5], "up": [0, 1, 0],
           "fovy_deg": 40.0, "width": 20, "height": 20}
    full, term, nt, nf = O.render(vol, tf, None, cam, "none", step)
    inside = lambda p: bool(np.all((p >= 0) & (p <= 1)))  # noqa: E731
    checked = 0
    for py in range(0, 20, 3):
        for px in range(0, 20, 3):
            o, d = O.camera_ray(cam, px, py)
            ts = np.linspace(0, 5, 5001)
            ins = np.array([inside(o + t * d) for t in ts])
            if not ins.any():
                assert np.all(full[py, px] == 0)
                continue
            lo, hi = ts[ins][0], ts[ins][-1]

            def edge(a, b, enter):
                for _ in range(80):
                    m = 0.5 * (a + b)
                    if inside(o + m * d) == enter:
                        b = m
                    else:
                        a = m
                return b if enter else a
            t0 = edge(lo - 1e-3, lo, True)
            t1 = edge(hi, hi + 1e-3, False)
            D = t1 - t0
            a_pix = 1 - (1 - a0) ** (D * N)
            np.testing.assert_allclose(full[py, px], np.array(rgb + [1.0]) * a_pix, rtol=1e-9, atol=1e-12)
            checked += 1
    assert checked > 20


def test_p2_termination_bound():
    N = 16
    raw = np.full((N, N, N), 200, np.uint8)
    vol, tf = O.Volume(raw), _const_tf([1.0, 0.5, 0.25, 0.6])
    cam = W.camera_ortho_front(16, 16, half_h=0.6)
    full, term, nt, nf = O.render(vol, tf, None, cam, "none", 0.5)
    eps = 2.0 ** -15
    assert np.abs(full - term).max() <= eps
    assert (nt < nf).any()                         # termination did happen
    # terminated pixels keep at most eps of transmittance, and stopped at the first such sample
    a_step = 1 - (1 - 0.6) ** 0.5
    k_expect = math.ceil(math.log(eps) / math.log(1 - a_step))
    assert (nt[nt < nf] == k_expect).all()


# ------------------------------------------------------------------ P3

def test_p3_beer_lambert_axis_light_exact():
    N, n, res, a0 = 16, 16, 16, 0.07
    raw = np.full((N, N, N), 90, np.uint8)
    vol, tf = O.Volume(raw), _const_tf([1, 1, 1, a0])
    st = O.Stack(vol, tf, [0, 0, 1], n, res)
    S = st.export()
    f = st.frame
    u = -f["R"] + (np.arange(res) + 0.5) * 2 * f["R"] / res
    k = np.arange(n)
    expect = (1 - a0) ** ((k + 1) * (1.0 / n) * N)
    for j in range(res):
        for i in range(res):
            if abs(u[i]) < 0.5 and abs(u[j]) < 0.5:
                np.testing.assert_allclose(S[:, j, i], expect, rtol=1e-12)
            elif abs(u[i]) > 0.5 or abs(u[j]) > 0.5:
                assert np.all(S[:, j, i] == 1.0)


@pytest.mark.parametrize("light", [[1, 1, -1], [0.3, -0.8, 0.5], [-1, 0.2, 0.1]])
def test_p3_beer_lambert_oblique_within_one_slab(light):
    N, n, res, a0 = 16, 24, 20, 0.05
    raw = np.full((N, N, N), 90, np.uint8)
    vol, tf = O.Volume(raw), _const_tf([1, 1, 1, a0])
    st = O.Stack(vol, tf, light, n, res)
    S = st.export()
    f = st.frame
    sigma = -math.log(1 - a0) * N
    u = -f["R"] + (np.arange(res) + 0.5) * 2 * f["R"] / res
    for j in range(res):
        for i in range(res):
            base = f["c"] + u[i] * f["U"] + u[j] * f["V"] - (f["L"] @ f["c"]) * f["L"]
            # Liang-Barsky clip of the column line to the cube, parameter = distance along L
            lo, hi = -np.inf, np.inf
            for ax in range(3):
                if abs(f["L"][ax]) < 1e-15:
                    if not (0 <= base[ax] <= 1):
                        lo, hi = 1, 0
                    continue
                t1, t2 = (0 - base[ax]) / f["L"][ax], (1 - base[ax]) / f["L"][ax]
                lo, hi = max(lo, min(t1, t2)), min(hi, max(t1, t2))
            for k in range(n):
                face = f["dmin"] + (k + 1) * f["ds"]
                d_in = max(0.0, min(hi, face) - lo) if hi > lo else 0.0
                assert abs(S[k, j, i] - math.exp(-sigma * d_in)) <= sigma * f["ds"] + 1e-12


# ------------------------------------------------------------------ P5

def _p5_setup():
    N = 32
    plate = np.zeros((N, N, N), np.uint8)
    plate[4:8, 4:28, 4:28] = 100                    # z in [4,8) voxels, partially transparent
    both = plate.copy()
    both[18:26, 8:24, 8:24] = 255                    # opaque box above the plate
    tab = np.zeros((256, 4))
    tab[:, 0], tab[:, 1], tab[:, 2] = 0.9, 0.8, 0.7
    tab[:, 3] = np.linspace(0, 1, 256)               # value 255 -> alpha exactly 1
    return N, plate, both, tab


@pytest.mark.parametrize("mode", MODES)
def test_p5_opaque_box_exact_shadow_footprint(mode):
    N, plate, both, tab = _p5_setup()
    n, res = 64, 96
    light = np.array([0.3, 0.2, -1.0])
    tf = O.TF(tab)
    vplate, vboth = O.Volume(plate), O.Volume(both)
    st_plate = O.Stack(vplate, tf, light, n, res)
    st_box = O.Stack(vboth, tf, light, n, res)
    # view the plate from below, looking up (+z): the plate is composited first
    Wd = 40
    cam = {"kind": "ortho", "eye": [0.5, 0.5, -1.0], "target": [0.5, 0.5, 0.5], "up": [0, 1, 0],
           "ortho_half_h": 0.5, "width": Wd, "height": Wd}
    m, extra = _mode(mode)
    ref, _, _, _ = O.render(vplate, tf, st_plate, cam, m, 0.5, extra)
    img, _, _, _ = O.render(vplate, tf, st_box, cam, m, 0.5, extra)

    f = st_box.frame
    L = f["L"]
    texel = 2 * f["R"] / res
    tap = {"shadow": 0.0, "shell": 1.0 / N, "cone": 2 * f["ds"] * math.sqrt(2.0),
           "cone5": f["ds"] * math.sqrt(2.0)}[mode]
    margin = math.sqrt(2) * texel + f["ds"] + tap + 1.0 / N
    # fully opaque region of the box: where all 8 trilinear neighbours are box voxels
    core_lo = np.array([8.5, 8.5, 18.5]) / N
    core_hi = np.array([23.5, 23.5, 25.5]) / N
    supp_lo = np.array([7.5, 7.5, 17.5]) / N         # where the box changes the volume at all
    supp_hi = np.array([24.5, 24.5, 26.5]) / N

    def back_ray_hits(p, lo, hi):
        """Does p - s L, s > 0, meet the box [lo, hi]?"""
        a, b = 0.0, np.inf
        for ax in range(3):
            dl = -L[ax]
            if abs(dl) < 1e-15:
                if not (lo[ax] <= p[ax] <= hi[ax]):
                    return False
                continue
            t1, t2 = (lo[ax] - p[ax]) / dl, (hi[ax] - p[ax]) / dl
            a, b = max(a, min(t1, t2)), min(b, max(t1, t2))
        return b >= a

    n_in = n_out = 0
    for py in range(Wd):
        for px in range(Wd):
            o, d = O.camera_ray(cam, px, py)
            # plate support (alpha > 0) along this ray: z in (3.5, 8.5) voxels
            seg = [o + ((z / N) - o[2]) * d for z in np.linspace(3.5, 8.5, 21)]
            if all(back_ray_hits(p, core_lo + margin, core_hi - margin) for p in (seg[0], seg[-1])):
                n_in += 1
                assert np.all(img[py, px, :3] == 0.0), (py, px, img[py, px])
                assert img[py, px, 3] == ref[py, px, 3]
            elif not any(back_ray_hits(p, supp_lo - margin, supp_hi + margin) for p in seg):
                n_out += 1
                assert np.all(img[py, px] == ref[py, px]), (py, px)
    assert n_in >= 8 and n_out >= 100, (n_in, n_out)
    # the plate is lit somewhere, so the shadow is not vacuous
    assert ref[..., :3].max() > 0.05


# ------------------------------------------------------------------ P6

def test_p6_light_parallel_to_view_converges():
    """L = fwd = +z, constant cube, direct shadow: C -> rgb/2 (1 - exp(-2 sigma D)).

    When the ray steps coincide with the slabs the discrete sum telescopes to
    the limit exactly; otherwise it converges to it at second order."""
    N, a0, rgb = 8, 0.1, np.array([0.8, 0.4, 0.2])
    raw = np.full((N, N, N), 120, np.uint8)
    vol, tf = O.Volume(raw), _const_tf(list(rgb) + [a0])
    sigma = -math.log(1 - a0) * N
    limit = rgb / 2 * (1 - math.exp(-2 * sigma * 1.0))
    cam = {"kind": "ortho", "eye": [0.5, 0.5, -1.0], "target": [0.5, 0.5, 0.5], "up": [0, 1, 0],
           "ortho_half_h": 0.05, "width": 2, "height": 2}
    for n, step in [(8, 1.0), (16, 0.5), (32, 0.25)]:
        st = O.Stack(vol, tf, [0, 0, 1], n, 16)
        full, _, _, _ = O.render(vol, tf, st, cam, "shadow", step)
        assert np.abs(full[..., :3] - limit).max() < 1e-14
    errs = []
    for n, step in [(6, 0.9), (12, 0.45), (24, 0.225), (48, 0.1125)]:
        st = O.Stack(vol, tf, [0, 0, 1], n, 16)
        full, _, _, _ = O.render(vol, tf, st, cam, "shadow", step)
        errs.append(np.abs(full[..., :3] - limit).max())
    assert errs[-1] < 5e-6
    for e0, e1 in zip(errs, errs[1:]):
        assert e0 / e1 > 3.0, errs


# ------------------------------------------------------------------ P7

def test_p7_stack_lookup_converges_to_dense_light_march():
    """Transmittance from the stack vs exp(-integral of sigma) marched toward the light.

    With the midpoint slab rule, faces at the layer boundaries and bilinear
    texels, the error is second order in the slab and texel size; a half-slab
    or half-texel misregistration, an exclusive layer or nearest-layer lookup
    would each leave a first-order error."""
    N = 16
    g = (np.arange(N) + 0.5) / N
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    field = np.exp(-(((X - 0.45) ** 2 + (Y - 0.55) ** 2 + (Z - 0.5) ** 2) / (2 * 0.18 ** 2)))
    raw = (0.6 * field).astype(np.float32)
    vol = O.Volume(raw, scale=1.0)
    tab = np.zeros((256, 4))
    tab[:, 3] = 0.25 * np.linspace(0, 1, 256)        # smooth, kink-free alpha in value
    tf = O.TF(tab)
    light = np.array([0.4, -0.3, 0.85])
    L = light / np.linalg.norm(light)
    rng = np.random.default_rng(7)
    pts = rng.uniform(0.3, 0.7, size=(40, 3))

    def dense(p):
        # distance back to the cube along -L
        s_max = min(((0.0 - p[a]) / -L[a]) if -L[a] < 0 else ((1.0 - p[a]) / -L[a]) for a in range(3))
        M = 4000
        ds = s_max / M
        tau = 0.0
        for m in range(M):
            q = p - (m + 0.5) * ds * L
            a = O.tf_lookup(tf, O.volume_sample(vol, q))[3]
            tau += -math.log(1 - a) * N * ds
        return math.exp(-tau)

    ref = np.array([dense(p) for p in pts])
    errs = []
    for n in [12, 24, 48, 96]:
        st = O.Stack(vol, tf, light, n, n)
        got = np.array([st.lookup(p) for p in pts])
        errs.append(np.abs(got - ref).max())
    assert errs[-1] < 1.2e-3
    # convergence order ~2 (ratio ~4 per halving); first order would give ~2
    assert errs[-2] / errs[-1] > 3.0 and errs[-3] / errs[-2] > 3.0, errs


# ------------------------------------------------------------------ P8

def test_p8_vanishing_shell_equals_shadow():
    raw = W.sphere_u8(16, radius=6, density=180, noise=20, seed=3)
    vol, tf = O.Volume(raw), O.TF(W.tf_ramp())
    st = O.Stack(vol, tf, [1, 1, -1], 8, 16)
    cam = W.camera_orbit(12, 12, 0.4, 0.3)
    a, _, _, _ = O.render(vol, tf, st, cam, "shadow", 0.5)
    b, _, _, _ = O.render(vol, tf, st, cam, "shell", 0.5, {"shell_h_vox": 1e-9})
    assert np.abs(a - b).max() < 1e-8
    # a constant stack (no attenuation anywhere) gives A = 1: "none" equals every mode
    empty_tf = O.TF(np.zeros((256, 4)))
    st1 = O.Stack(vol, empty_tf, [1, 1, -1], 8, 16)
    ref, _, _, _ = O.render(vol, tf, None, cam, "none", 0.5)
    for m in MODES:
        mm, extra = _mode(m)
        img, _, _, _ = O.render(vol, tf, st1, cam, mm, 0.5, extra)
        assert np.abs(img - ref).max() < 1e-15


def test_p8_gather_weights_bounded_by_taps():
    """Equal weights summing to one: min over taps <= A <= max over taps."""
    raw = W.sphere_u8(16, radius=6, density=180, noise=20, seed=4)
    vol, tf = O.Volume(raw), O.TF(W.tf_ramp())
    st = O.Stack(vol, tf, [0.2, 1, -0.4], 12, 16)
    rng = np.random.default_rng(8)
    for _ in range(100):
        p = rng.uniform(0.2, 0.8, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        A = st.coefficient("shell", p, d)
        h = 1.0 / 16
        taps = [st.lookup(p + s * h * e) for e in np.eye(3) for s in (-1, 1)]
        assert min(taps) - 1e-15 <= A <= max(taps) + 1e-15
        assert A == pytest.approx(np.mean(taps), abs=1e-15)
        assert 0.0 <= st.coefficient("cone", p, d) <= 1.0


# ------------------------------------------------------------------ P9

@pytest.mark.parametrize("mode", MODES)
def test_p9_invariants_small_workload(mode):
    w = W.WORKLOADS["small"]
    raw = w.volume()
    vol, tf = O.Volume(raw), O.TF(w.tf())
    st = O.Stack(vol, tf, w.lights()[0], w.n_slices, w.res)
    S = st.export()
    assert S.min() >= 0.0 and S.max() <= 1.0
    assert np.all(np.diff(S, axis=0) <= 0.0)            # monotone along the light
    cam = w.camera(W=64, H=64)
    m, extra = _mode(mode)
    full, term, nt, nf = O.render(vol, tf, st, cam, m, 0.5, extra)
    for img in (full, term):
        a = img[..., 3]
        assert a.min() >= 0.0 and a.max() <= 1.0
        assert np.all(img[..., :3] >= 0.0)
        assert np.all(img[..., :3] <= a[..., None] + 1e-15)
    assert np.abs(full - term).max() <= 2.0 ** -15
    assert np.all(nt <= nf)


# ------------------------------------------------------------------ cone geometry (section 3.2.3, Eq. 11)

def _half_space_stack(n=16, res=16):
    """Light along +z; opaque for z >= 1/2: the stack is exactly 1 up to depth 1/2."""
    N = 16
    raw = np.zeros((N, N, N), np.uint8)
    raw[8:] = 255
    tab = np.zeros((256, 4))
    tab[:, 3] = np.linspace(0, 1, 256)
    return O.Stack(O.Volume(raw), O.TF(tab), [0, 0, 1], n, res)


@pytest.mark.parametrize("grid", [0, 5])
def test_cone_opens_toward_the_light(grid):
    st = _half_space_stack()
    opts = {"cone_grid": grid}
    d = np.array([1.0, 0.3, 0.2]) / np.linalg.norm([1.0, 0.3, 0.2])
    # lit side, within two slabs of the shadowing layer: every tap toward the light is lit
    assert st.coefficient("cone", [0.5, 0.5, 0.45], d, opts) == 1.0
    # the direct lookup there is lit too, a point beyond the layer is dark
    assert st.lookup([0.5, 0.5, 0.45]) == 1.0
    assert st.coefficient("cone", [0.5, 0.5, 0.9], d, opts) < 1e-6


@pytest.mark.parametrize("grid", [0, 5])
def test_cone_taps_invariant_under_quarter_turn_of_view(grid):
    """Four ring angles (and the square lattice) map onto themselves when the
    view turns by 90 degrees about L, so A must not change; a gather that
    spread along B only would."""
    N = 16
    raw = np.zeros((N, N, N), np.uint8)
    raw[2:14, 2:14, 10:14] = 255      # opaque wall, x in [10,14) voxels: the stack varies along x
    tab = np.zeros((256, 4))
    tab[:, 3] = np.linspace(0, 0.5, 256)
    st = O.Stack(O.Volume(raw), O.TF(tab), [0, 0, 1], 16, 32)
    opts = {"cone_grid": grid}
    p = [0.58, 0.5, 0.7]
    a_x = st.coefficient("cone", p, [-1.0, 0.0, 0.0], opts)   # B = +x
    a_y = st.coefficient("cone", p, [0.0, -1.0, 0.0], opts)   # B = +y
    a_xm = st.coefficient("cone", p, [1.0, 0.0, 0.0], opts)   # B = -x
    assert a_x == pytest.approx(a_y, abs=1e-14) and a_x == pytest.approx(a_xm, abs=1e-14)
    assert 0.0 < a_x < 1.0
    # the ring radius is c_m tan(phi): a narrower cone reads a different neighbourhood
    assert st.coefficient("cone", p, [-1.0, 0.0, 0.0], {"cone_grid": grid, "cone_tan": 0.2}) != pytest.approx(a_x)


# ------------------------------------------------------------------ P11 local Phong (comparison mode)

def _linear_volume(N, c0, grad):
    """f32 volume f = c0 + grad . (x, y, z) in voxel-index units (raw[z][y][x])."""
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    return (c0 + grad[0] * x + grad[1] * y + grad[2] * z).astype(np.float32)


def test_p11_gradient_of_a_linear_field_is_exact():
    """Central differences of the trilinear reconstruction of a linear field are
    the field's own gradient (per voxel) wherever no index is clamped; distinct
    per-axis slopes catch a swapped or mis-signed axis."""
    N, grad = 24, (2.0 ** -7, -(2.0 ** -8), 3 * 2.0 ** -10)   # dyadic: the f32 volume is exactly linear
    vol = O.Volume(_linear_volume(N, 0.5, grad), 1.0)
    rng = np.random.default_rng(3)
    for _ in range(50):
        g_vox = rng.uniform(1.0, N - 2.0, size=3)          # voxel coords: p +- 1 voxel stays unclamped
        p = (g_vox + 0.5) / N
        np.testing.assert_allclose(O.gradient(vol, p), grad, rtol=0, atol=1e-14)


PHONG = {"phong_ka": 0.1, "phong_kd": 0.7, "phong_ks": 0.4, "phong_shininess": 4.0, "grad_eps": 0.02}


@pytest.mark.parametrize("slope,L,sd_ss", [
    # unit normal n = -x: light along the normal -> full diffuse, reflection along -x is
    # perpendicular to the view -> no specular
    (2.0 ** -5, (1, 0, 0), lambda o: (o["phong_ka"] + o["phong_kd"], 0.0)),
    # light from behind the volume toward the camera: l = -v is perpendicular to n and
    # mirrors onto the view direction -> no diffuse, full specular
    (2.0 ** -5, (0, -1, 0), lambda o: (o["phong_ka"], o["phong_ks"])),
    # oblique light at 30 degrees from the normal in the x-y plane: diffuse cos 30,
    # mirror direction at 60 degrees from the view -> specular cos(60)^s... = sin(30)^s
    (2.0 ** -5, (math.cos(math.radians(30)), -math.sin(math.radians(30)), 0),
     lambda o: (o["phong_ka"] + o["phong_kd"] * math.cos(math.radians(30)),
                o["phong_ks"] * math.sin(math.radians(30)) ** o["phong_shininess"])),
    # flat field (|g| = 2^-8 < grad_eps): the normal shrinks to |g| / grad_eps;
    # diffuse scales with it, the mirror term with its square (r.v = 0 here)
    (2.0 ** -8, (1, 0, 0), lambda o: (o["phong_ka"] + o["phong_kd"] * 2.0 ** -8 / o["grad_eps"], 0.0)),
])
def test_p11_phong_closed_form_ramp(slope, L, sd_ss):
    """Ortho view along +y through a field linear in x with a constant TF: every
    segment of a ray has the same normal, so a pixel is (sd rgb + ss) times the
    chord opacity 1 - (1 - a0)^N, for rays whose samples never clamp in x."""
    N, a0, rgb = 24, 0.04, [0.9, 0.6, 0.3]
    raw = _linear_volume(N, 0.125, (slope, 0.0, 0.0))   # dyadic: exactly linear in f32
    vol, tf = O.Volume(raw, 1.0), _const_tf(rgb + [a0])
    st = O.Stack(vol, tf, L, 4, 4)                       # the light frame only (no column is built)
    cam = W.camera_ortho_front(48, 8, half_h=0.5 * 8 / 48)   # half width 0.5: the cube spans the image
    full, _, _, _ = O.render(vol, tf, st, cam, "phong", 0.5, PHONG)
    sd, ss = sd_ss(PHONG)
    a_pix = 1 - (1 - a0) ** N
    want = np.array([(sd * c + ss) * a_pix for c in rgb] + [a_pix])
    checked = 0
    for px in range(48):
        x = 0.5 + (2 * (px + 0.5) / 48 - 1) * 0.5        # world x of the column (aspect 6, half width 0.5)
        gx = x * N - 0.5
        if 1.0 <= gx <= N - 2.0:
            for py in range(8):
                np.testing.assert_allclose(full[py, px], want, rtol=1e-12, atol=1e-15)
            checked += 1
    assert checked > 30
    # the direct terms agree with the render
    p = [0.5, 0.5, 0.5]
    assert O.phong(vol, np.asarray(L, float) / np.linalg.norm(L), p, [0, 1, 0], PHONG) == pytest.approx((sd, ss), abs=1e-14)


def test_p11_phong_reduces_to_unlit():
    """k_a = 1, k_d = k_s = 0 gives exactly the unlit (A = 1) image."""
    w = W.WORKLOADS["small"]
    vol, tf = O.Volume(w.volume()), O.TF(w.tf())
    st = O.Stack(vol, tf, w.lights()[0], w.n_slices, w.res)
    cam = w.camera(W=24, H=24)
    a, _, na, _ = O.render(vol, tf, st, cam, "phong", 0.5,
                           {"phong_ka": 1.0, "phong_kd": 0.0, "phong_ks": 0.0}, want_full=False)
    b, _, nb, _ = O.render(vol, tf, None, cam, "none", 0.5, want_full=False)
    assert np.array_equal(a, b) and np.array_equal(na, nb)


def test_p11_phong_sphere_lit_side_brighter():
    """A lit sphere: rays hitting the side facing the light are brighter than those
    on the far side (normal orientation -g points out of a dense object)."""
    N = 40
    raw = W.sphere_u8(N, radius=14, density=200, noise=0, seed=1)
    vol, tf = O.Volume(raw), O.TF(W.tf_ramp())
    st = O.Stack(vol, tf, [1, 0, 0], 4, 4)               # light travels +x: lit side is x < 0.5
    cam = W.camera_ortho_front(32, 32, half_h=0.5)
    full, _, _, _ = O.render(vol, tf, st, cam, "phong", 0.5, {"phong_ks": 0.0}, want_full=True)
    lum = full[..., :3].sum(-1)
    assert lum[12:20, 7:11].mean() > 1.5 * lum[12:20, 21:25].mean()


# ------------------------------------------------------------------ P12 slab compensation (1+alpha)^m (section 4)

def _slab_medium(N=16, value=100):
    raw = np.zeros((N, N, N), np.uint8)
    raw[2:N - 2, 2:N - 2, 2:N - 2] = value
    return raw


def test_p12_darkening_m1_is_one_minus_alpha_squared():
    """m = 1: every slab passes (1-alpha)(1+alpha) = 1 - alpha^2 of the light, so along an axis
    light through a constant medium the column is (1 - alpha_s^2)^k (alpha_s the slab opacity)."""
    N, a0 = 16, 0.1
    vol, tf = O.Volume(_slab_medium(N)), _tf_zero_then([1, 1, 1, a0])
    n, res = 32, 16                                   # ds = half a voxel along z
    st = O.Stack(vol, tf, [0, 0, 1], n, res, darken=1.0)
    plain = O.Stack(vol, tf, [0, 0, 1], n, res)
    a_s = 1 - (1 - a0) ** 0.5
    col, ref = st.column(res // 2, res // 2), plain.column(res // 2, res // 2)
    # slabs whose midpoints sample the interior plateau (voxel centres 2.5 .. N-3.5 away from edges)
    inside = [k for k in range(n) if 3.0 <= (k + 0.5) * N / n <= N - 3.0]
    for k0, k1 in zip(inside[:-1], inside[1:]):
        np.testing.assert_allclose(col[k1] / col[k0], 1 - a_s ** 2, rtol=1e-12)
        np.testing.assert_allclose(ref[k1] / ref[k0], 1 - a_s, rtol=1e-12)


def test_p12_darkening_large_m_caps_every_slab_at_one():
    """(1-alpha)(1+alpha)^3 > 1 for alpha < 0.5...: with the cap no slab attenuates, stack == 1."""
    vol, tf = O.Volume(_slab_medium()), _tf_zero_then([1, 1, 1, 0.05])
    st = O.Stack(vol, tf, [0.3, -0.2, 1], 12, 10, darken=3.0)
    assert np.all(st.export() == 1.0)


def test_p12_darkening_is_monotone_in_m():
    w = W.WORKLOADS["small"]
    vol, tf = O.Volume(w.volume()), O.TF(w.tf())
    cols = []
    for m in (0.0, 0.5, 1.0, 2.0):
        st = O.Stack(vol, tf, w.lights()[0], 16, 24, darken=m)
        cols.append(st.export())
    for a, b in zip(cols[:-1], cols[1:]):
        assert np.all(b >= a)                          # more compensation never darkens
        assert np.all(np.diff(b, axis=0) <= 0)         # and the stack stays monotone along the light


# ------------------------------------------------------------------ P13 weighted shells (section 3.2.3)

def test_p13_shell_weights_reduce_to_single_shells():
    """Two shells with weights (1, 0) are the one-voxel shell; (0, 1) is the two-voxel shell,
    i.e. one shell at twice the step; (1, 1) equals the default equal weights exactly."""
    w = W.WORKLOADS["small"]
    vol, tf = O.Volume(w.volume()), O.TF(w.tf())
    st = O.Stack(vol, tf, w.lights()[0], w.n_slices, w.res)
    rng = np.random.default_rng(5)
    for _ in range(40):
        p = rng.uniform(0.2, 0.8, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        one = st.coefficient("shell", p, d, {"shell_count": 1})
        two = st.coefficient("shell", p, d, {"shell_count": 1, "shell_h_vox": 2.0})
        assert st.coefficient("shell", p, d, {"shell_count": 2, "shell_w": [1, 0]}) == one
        assert st.coefficient("shell", p, d, {"shell_count": 2, "shell_w": [0, 1]}) == two
        eq = st.coefficient("shell", p, d, {"shell_count": 2})
        assert st.coefficient("shell", p, d, {"shell_count": 2, "shell_w": [1, 1]}) == eq
        assert st.coefficient("shell", p, d, {"shell_count": 2, "shell_w": [3, 1]}) == pytest.approx(
            (3 * one + two) / 4, abs=1e-15)


# ------------------------------------------------------------------ P14 point light (perspective light frusta)

def _ray_box(o, d):
    """Parameter interval where o + t d lies in the unit cube (slab method)."""
    t0, t1 = -np.inf, np.inf
    for a in range(3):
        if d[a] == 0:
            if not 0 <= o[a] <= 1:
                return 1.0, 0.0
            continue
        ta, tb = (0 - o[a]) / d[a], (1 - o[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return t0, t1


def test_p14_point_light_frame_covers_the_cube():
    """Every cube vertex projects inside the texel square and lies between the first and last slab
    planes; one vertex touches the square's edge (the square is the smallest)."""
    for pos in ([0.5, 0.5, -3.0], [2.0, -1.5, 2.5], [-0.9, 1.7, 0.3]):
        f = O.light_frame(None, 16, 32, position=pos)
        P, L, U, V, R = np.asarray(pos), f["L"], f["U"], f["V"], f["R"]
        np.testing.assert_allclose(L, (0.5 - P) / np.linalg.norm(0.5 - P), atol=1e-15)
        uv = []
        for vtx in range(8):
            w = np.array([vtx & 1, (vtx >> 1) & 1, (vtx >> 2) & 1], float) - P
            d = L @ w
            assert f["dmin"] - 1e-12 <= d <= f["dmax"] + 1e-12
            uv.append(max(abs(U @ w), abs(V @ w)) / d)
        assert max(uv) == pytest.approx(R, abs=1e-15)


def test_p14_point_light_constant_medium_closed_form():
    """A constant medium filling the cube: the column of texel (i, j) is the ray from the light
    through the texel; its layer k is (1-a)^(m_k ds |D| / dref), m_k = slabs up to k whose mid-plane
    crossing lies in the cube -- counted here from an independent ray/box clip."""
    N, a0 = 16, 0.03
    raw = np.full((N, N, N), 100, np.uint8)
    vol, tf = O.Volume(raw), _const_tf([1, 1, 1, a0])
    pos = np.array([1.7, -0.6, 2.4])
    n, res = 24, 12
    st = O.Stack(vol, tf, None, n, res, position=pos)
    f = st.frame
    for i, j in [(0, 0), (5, 7), (11, 3), (6, 6)]:
        u = -f["R"] + (i + 0.5) * 2 * f["R"] / res
        v = -f["R"] + (j + 0.5) * 2 * f["R"] / res
        D = f["L"] + u * f["U"] + v * f["V"]
        t0, t1 = _ray_box(pos, D)                       # L.D = 1: the ray parameter is the depth
        dk = f["dmin"] + (np.arange(n) + 0.5) * f["ds"]
        m = np.cumsum((dk >= t0) & (dk <= t1))
        want = (1 - a0) ** (m * f["ds"] * np.linalg.norm(D) * N)
        np.testing.assert_allclose(st.column(i, j), want, rtol=1e-12, atol=1e-15)


def test_p14_point_light_lookup_registers_with_the_columns():
    """A point on a column's ray reads that column, interpolated in depth only."""
    w = W.WORKLOADS["small"]
    vol, tf = O.Volume(w.volume()), O.TF(w.tf())
    pos = np.array([-1.2, 1.9, 2.2])
    n, res = 20, 24
    st = O.Stack(vol, tf, None, n, res, position=pos)
    f = st.frame
    rng = np.random.default_rng(2)
    for _ in range(30):
        i, j = rng.integers(0, res, 2)
        u = -f["R"] + (i + 0.5) * 2 * f["R"] / res
        v = -f["R"] + (j + 0.5) * 2 * f["R"] / res
        D = f["L"] + u * f["U"] + v * f["V"]
        d = rng.uniform(f["dmin"] + 1.5 * f["ds"], f["dmax"] - 1.5 * f["ds"])
        p = pos + d * D
        z = (d - f["dmin"]) / f["ds"] - 1.0                # layer coordinate (face q holds layer q-1)
        col = st.column(int(i), int(j))
        k0 = int(np.floor(z))
        want = col[k0] + (z - k0) * (col[k0 + 1] - col[k0])
        assert st.lookup(p) == pytest.approx(want, abs=1e-12)


def test_p14_point_light_on_the_axis_keeps_the_sphere_symmetry():
    """Light on the z axis over a centred sphere: the stack is invariant under a quarter turn of the
    texel grid about the axis."""
    N = 24
    raw = W.sphere_u8(N, radius=8, density=180, noise=0, seed=1)
    vol, tf = O.Volume(raw), O.TF(W.tf_ramp())
    st = O.Stack(vol, tf, None, 12, 16, position=[0.5, 0.5, -2.5])
    S = st.export()
    np.testing.assert_allclose(S, np.rot90(S, k=1, axes=(1, 2)), atol=1e-12)
    assert S.min() < 0.5                                  # the sphere does cast a shadow


# ------------------------------------------------------------------ P15 cone under a point light (R39)

def test_p15_point_cone_taps_geometry():
    """Cone under a point light: ring m of the default cone (2 rings x 4 angles) is centred on the
    line from the light through the sample, at t_m = m ds / (L . L_s) toward the light (m slabs of
    depth), in the plane across L_s, radius t_m tan(phi), the first tap along the view direction
    with its L_s part removed and the four taps a quarter turn apart about L_s.  Catches
    the axis direction L taken for L_s, t_m without the obliquity, a radial axis not
    perpendicular to L_s, a misrotated ring."""
    w = W.WORKLOADS["small"]
    vol, tf = O.Volume(w.volume()), O.TF(w.tf())
    pos = np.array([-1.4, 2.1, 1.9])
    st = O.Stack(vol, tf, None, 20, 24, position=pos)
    f = st.frame
    L = np.asarray(f["L"])
    rng = np.random.default_rng(7)
    for _ in range(12):
        p = rng.uniform(0.2, 0.8, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        taps = st.cone_taps(p, d)
        assert taps.shape == (8, 3)
        Ls = (p - pos) / np.linalg.norm(p - pos)
        wv = -d - (-d @ Ls) * Ls
        Bp = wv / np.linalg.norm(wv)
        for m in (1, 2):
            ring = taps[4 * (m - 1):4 * m]
            tm = m * f["ds"] / (L @ Ls)
            centre = p - tm * Ls
            # the ring's centre lies on the light ray through p, exactly m slabs of depth nearer the light
            np.testing.assert_allclose(ring.mean(axis=0), centre, atol=1e-12)
            np.testing.assert_allclose(L @ (centre - pos), L @ (p - pos) - m * f["ds"], atol=1e-12)
            off = ring - centre
            np.testing.assert_allclose(off @ Ls, 0.0, atol=1e-12)
            np.testing.assert_allclose(np.linalg.norm(off, axis=1), tm, rtol=1e-12)   # tan(phi) = 1
            np.testing.assert_allclose(off[0] / tm, Bp, atol=1e-12)
            np.testing.assert_allclose(off[1] / tm, np.cross(Ls, Bp), atol=1e-12)
            np.testing.assert_allclose(off[2], -off[0], atol=1e-12)
            np.testing.assert_allclose(off[3], -off[1], atol=1e-12)
    # directional light: t_m = m ds along L exactly (the rings of section 3.2.3)
    sd = O.Stack(vol, tf, w.lights()[0], 20, 24)
    p, d = np.array([0.5, 0.45, 0.55]), np.array([0.0, 1.0, 0.0])
    taps = sd.cone_taps(p, d)
    Ld = np.asarray(sd.frame["L"])
    np.testing.assert_allclose((taps - p) @ Ld, np.repeat([-1, -2], 4) * sd.frame["ds"], atol=1e-14)


def test_p15_point_cone_tends_to_the_directional_cone():
    """A point light receding along -L gives the directional cone in the limit: tap positions
    approach the directional cone's about as 1/distance, so the coefficient, read from one stack,
    does too (ring and lattice); and the coefficient is the mean stack value over its taps (Eq. 11).
    Two stacks are not compared with each other: their grids differ, and so do their bilinear
    reconstructions near sharp shadow edges."""
    w = W.WORKLOADS["small"]
    vol, tf = O.Volume(w.volume()), O.TF(w.tf())
    L = np.array([1.0, 1.0, -1.0]) / np.sqrt(3.0)
    n, res = 24, 32
    sd = O.Stack(vol, tf, L, n, res)
    rng = np.random.default_rng(11)
    pts = [(rng.uniform(0.3, 0.7, 3), rng.normal(size=3)) for _ in range(16)]
    pts = [(p, d / np.linalg.norm(d)) for p, d in pts]
    for opts in ({}, {"cone_grid": 5}):
        geo, coef = [], []
        for D in (40.0, 400.0, 4000.0):
            sp = O.Stack(vol, tf, None, n, res, position=0.5 - D * L)
            g = c = 0.0
            for p, d in pts:
                tp, td = sp.cone_taps(p, d, opts), sd.cone_taps(p, d, opts)
                g = max(g, float(np.abs(tp - td).max()))
                cp = sp.coefficient("cone", p, d, opts)
                assert abs(cp - np.mean([sp.lookup(t) for t in tp])) < 1e-14
                c = max(c, abs(cp - np.mean([sp.lookup(t) for t in td])))
            geo.append(g)
            coef.append(c)
        assert geo[2] < 1e-4 and geo[1] < geo[0] / 6 and geo[2] < geo[1] / 6, geo
        assert coef[2] < 1e-4 and coef[2] < coef[0] / 6, coef


# ------------------------------------------------------------------ P16 nearest-layer lookup (R25)

def _face_point(st, p, f, frame):
    """p moved to depth index q = f without changing its texel coordinates: along L for a
    directional light, along the ray from the light for a point light."""
    L = np.asarray(frame["L"])
    span = frame["dmax"] - frame["dmin"]
    if frame.get("positional"):
        P = np.asarray(frame["P"])
        d = L @ (p - P)
        df = frame["dmin"] + f * span / frame["n"]
        return P + (df / d) * (p - P)
    q = frame["n"] * (L @ p - frame["dmin"]) / span
    return p + (f - q) * span / frame["n"] * L


def test_p16_nearest_layer_reads_the_nearest_face():
    """Nearest-layer lookup (R25): at any point it equals the continuous lookup (R11) at the
    same texel coordinates on face f = floor(q + 1/2 + shift), clamped to 0..n (face 0 reads 1),
    for a directional and a point light.  Catches rounding down instead of to nearest, the
    face/layer offset (face f holds layer f - 1), a missing clamp."""
    w = W.WORKLOADS["small"]
    vol, tf = O.Volume(w.volume()), O.TF(w.tf())
    rng = np.random.default_rng(5)
    for light, pos in (([0.3, -0.5, 0.81], None), (None, [1.9, -0.6, 1.3])):
        st = O.Stack(vol, tf, light, 20, 28, position=pos)
        f = st.frame
        L = np.asarray(f["L"])
        differs = 0
        for _ in range(300):
            p = rng.uniform(-0.05, 1.05, 3)
            shift = 0.0 if rng.random() < 0.5 else float(rng.uniform(-0.45, 0.45))
            if f.get("positional"):
                q = f["n"] * (L @ (p - np.asarray(f["P"])) - f["dmin"]) / (f["dmax"] - f["dmin"])
            else:
                q = f["n"] * (L @ p - f["dmin"]) / (f["dmax"] - f["dmin"])
            face = int(min(max(math.floor(q + 0.5 + shift), 0), f["n"]))
            got = st.lookup(p, nearest=True, shift=shift)
            want = 1.0 if face == 0 else st.lookup(_face_point(st, p, face, f))
            assert abs(got - want) < 1e-12, (p, q, shift, got, want)
            differs += abs(got - st.lookup(p)) > 1e-6
        assert differs >= 20          # the two readings really differ (where the stack is not 1)


def test_p16_nearest_layer_converges_at_first_order():
    """Against the dense light march of P7: the nearest layer's error falls in proportion to
    the slab thickness (first order), the continuous reading's with its square."""
    N = 16
    g = (np.arange(N) + 0.5) / N
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    field = np.exp(-(((X - 0.45) ** 2 + (Y - 0.55) ** 2 + (Z - 0.5) ** 2) / (2 * 0.18 ** 2)))
    vol = O.Volume((0.6 * field).astype(np.float32), scale=1.0)
    tab = np.zeros((256, 4))
    tab[:, 3] = 0.25 * np.linspace(0, 1, 256)
    tf = O.TF(tab)
    light = np.array([0.4, -0.3, 0.85])
    L = light / np.linalg.norm(light)
    rng = np.random.default_rng(7)
    pts = rng.uniform(0.3, 0.7, size=(40, 3))

    def dense(p):
        s_max = min(((0.0 - p[a]) / -L[a]) if -L[a] < 0 else ((1.0 - p[a]) / -L[a]) for a in range(3))
        M = 4000
        ds = s_max / M
        tau = 0.0
        for m in range(M):
            q = p - (m + 0.5) * ds * L
            a = O.tf_lookup(tf, O.volume_sample(vol, q))[3]
            tau += -math.log(1 - a) * N * ds
        return math.exp(-tau)

    ref = np.array([dense(p) for p in pts])
    near, cont = [], []
    for n in [12, 24, 48, 96]:
        st = O.Stack(vol, tf, light, n, 4 * n)
        near.append(np.abs(np.array([st.lookup(p, nearest=True) for p in pts]) - ref).max())
        cont.append(np.abs(np.array([st.lookup(p) for p in pts]) - ref).max())
    # over an 8x refinement first order gains ~8 (the max over points is noisy per step),
    # second order ~64
    assert 4.0 < near[0] / near[-1] < 14.0, near
    assert cont[0] / cont[-1] > 25.0 and near[-1] > 5 * cont[-1], (near, cont)
