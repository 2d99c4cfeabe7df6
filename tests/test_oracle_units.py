"""Pins of the oracle's building blocks (CPU only).

Each test fixes a step by something other than the oracle itself: a value
derived by hand from the paper's definitions, a textbook construction, an
exact property of the interpolants, or a library routine the step reduces to.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O

SQ3 = math.sqrt(3.0)


# ---------------------------------------------------------------- light frame (Eq. 8, readings R9/R10)

def test_light_frame_diagonal_worked_example():
    # L = (1,1,-1)/sqrt3 : hand-derived basis and distances (Eq. 8 over the cube vertices)
    f = O.light_frame([1, 1, -1], 32, 64)
    np.testing.assert_allclose(f["L"], np.array([1, 1, -1]) / SQ3, atol=1e-15)
    np.testing.assert_allclose(f["U"], np.array([2, -1, 1]) / math.sqrt(6), atol=1e-15)
    np.testing.assert_allclose(f["V"], np.array([0, -1, -1]) / math.sqrt(2), atol=1e-15)
    assert f["dmin"] == pytest.approx(-1 / SQ3, abs=1e-15)   # vertex (0,0,1)
    assert f["dmax"] == pytest.approx(2 / SQ3, abs=1e-15)    # vertex (1,1,0)
    assert f["ds"] == pytest.approx(SQ3 / 32, abs=1e-15)
    assert f["R"] == pytest.approx(SQ3 / 2, abs=1e-15)


@pytest.mark.parametrize("l,U,V,dmin,dmax", [
    ([0, 0, 1], [1, 0, 0], [0, 1, 0], 0.0, 1.0),
    ([0, 0, -1], [1, 0, 0], [0, -1, 0], -1.0, 0.0),
    ([3, 0, 0], [0, 1, 0], [0, 0, 1], 0.0, 1.0),
    ([0, -2, 0], [1, 0, 0], [0, 0, 1], -1.0, 0.0),
])
def test_light_frame_axis_aligned(l, U, V, dmin, dmax):
    f = O.light_frame(l, 8, 8)
    np.testing.assert_allclose(f["U"], U, atol=1e-15)
    np.testing.assert_allclose(f["V"], V, atol=1e-15)
    assert f["dmin"] == pytest.approx(dmin, abs=1e-15)
    assert f["dmax"] == pytest.approx(dmax, abs=1e-15)


def test_light_frame_orthonormal_random():
    rng = np.random.default_rng(0)
    for _ in range(50):
        l = rng.normal(size=3)
        f = O.light_frame(l, 7, 9)
        B = np.stack([f["U"], f["V"], f["L"]])
        np.testing.assert_allclose(B @ B.T, np.eye(3), atol=1e-14)
        assert np.linalg.det(B) == pytest.approx(1.0, abs=1e-14)   # U x V = L
        # the square of half-width R about the centre covers every cube vertex
        for v in np.array(np.meshgrid([0, 1], [0, 1], [0, 1])).reshape(3, -1).T:
            r = v - 0.5
            assert abs(r @ f["U"]) <= f["R"] + 1e-15 and abs(r @ f["V"]) <= f["R"] + 1e-15


@pytest.mark.parametrize("bad", [[0, 0, 0], [float("nan"), 1, 0], [float("inf"), 0, 0]])
def test_light_frame_rejects_degenerate(bad):
    with pytest.raises(ValueError):
        O.light_frame(bad, 4, 4)


# ---------------------------------------------------------------- volume sampling (readings R2, R22)

def test_volume_sample_voxel_centres_exact():
    rng = np.random.default_rng(1)
    raw = rng.integers(0, 256, size=(6, 6, 6), dtype=np.uint8)
    vol = O.Volume(raw)
    for z, y, x in [(0, 0, 0), (5, 5, 5), (2, 3, 4), (5, 0, 3)]:
        p = [(x + 0.5) / 6, (y + 0.5) / 6, (z + 0.5) / 6]
        assert O.volume_sample(vol, p) == pytest.approx(raw[z, y, x] / 255.0, abs=1e-15)


def test_volume_sample_reproduces_linear_field():
    N = 8
    g = np.arange(N) + 0.0
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    raw = (0.1 + 0.02 * X + 0.03 * Y + 0.01 * Z).astype(np.float32)
    vol = O.Volume(raw, scale=1.0)
    rng = np.random.default_rng(2)
    for _ in range(200):
        gi = rng.uniform(0, N - 1, 3)            # between first and last voxel centres
        p = (gi + 0.5) / N
        expect = 0.1 + 0.02 * gi[0] + 0.03 * gi[1] + 0.01 * gi[2]
        # the float32 table holds the field rounded; allow its rounding
        assert O.volume_sample(vol, p) == pytest.approx(expect, abs=2e-8)


def test_volume_sample_clamps_to_edge():
    raw = np.zeros((4, 4, 4), dtype=np.uint8)
    raw[:, :, 0] = 200
    vol = O.Volume(raw)
    # within half a voxel of the x=0 face the sample equals the first voxel column
    assert O.volume_sample(vol, [0.0, 0.5, 0.5]) == pytest.approx(200 / 255, abs=1e-15)
    assert O.volume_sample(vol, [0.1, 0.5, 0.5]) == pytest.approx(200 / 255, abs=1e-15)
    # midway between the first two voxel centres
    assert O.volume_sample(vol, [1.0 / 4, 0.5, 0.5]) == pytest.approx(100 / 255, abs=1e-15)


def test_volume_normalisation_and_clamp():
    raw = np.full((2, 2, 2), 5000, dtype=np.uint16)
    assert O.volume_sample(O.Volume(raw), [0.5, 0.5, 0.5]) == 1.0
    raw = np.full((2, 2, 2), 4095, dtype=np.uint16)
    assert O.volume_sample(O.Volume(raw), [0.5, 0.5, 0.5]) == 1.0
    raw = np.full((2, 2, 2), 255, dtype=np.uint8)
    assert O.volume_sample(O.Volume(raw), [0.5, 0.5, 0.5]) == 1.0


def test_half_conversion_matches_numpy_for_all_finite_bit_patterns():
    bits = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    halves = bits.view(np.float16)
    finite = np.isfinite(halves)
    vals = halves[finite].astype(np.float64)
    # one voxel per bit pattern, read back through the trilinear sampler at the voxel centre
    sel = bits[finite]
    for chunk in np.array_split(np.arange(sel.size), 8):
        for idx in chunk[::97]:
            raw = np.full((2, 2, 2), sel[idx], dtype=np.uint16).view(np.float16)
            got = O.volume_sample(O.Volume(raw, scale=1.0), [0.5, 0.5, 0.5])
            assert got == pytest.approx(min(max(vals[idx], 0.0), 1.0), abs=0.0, rel=0.0)


# ---------------------------------------------------------------- transfer function (reading R21)

def test_tf_lookup_entries_and_interpolation():
    rng = np.random.default_rng(3)
    tab = rng.uniform(0, 1, size=(256, 4))
    tf = O.TF(tab)
    for i in [0, 1, 100, 254, 255]:
        np.testing.assert_allclose(O.tf_lookup(tf, i / 255.0), tab[i], atol=1e-13)
    np.testing.assert_allclose(O.tf_lookup(tf, (10.5) / 255.0), 0.5 * (tab[10] + tab[11]), atol=1e-13)
    np.testing.assert_allclose(O.tf_lookup(tf, 1.0), tab[255], atol=1e-15)


# ---------------------------------------------------------------- opacity correction (Eq. 6, reading R8)

def test_segment_alpha_properties():
    dref = 1.0 / 64
    for a in [0.0, 0.01, 0.3, 0.9, 0.999]:
        assert O.segment_alpha(a, 0.0, dref) == 0.0
        assert O.segment_alpha(a, dref, dref) == pytest.approx(a, abs=1e-15)
        for l1, l2 in [(0.3 * dref, 0.7 * dref), (dref, 2.5 * dref), (0.01 * dref, 0.02 * dref)]:
            lhs = (1 - O.segment_alpha(a, l1, dref)) * (1 - O.segment_alpha(a, l2, dref))
            assert lhs == pytest.approx(1 - O.segment_alpha(a, l1 + l2, dref), abs=1e-15)
    assert O.segment_alpha(1.0, 1e-9, dref) == 1.0
    # half a voxel: 1 - sqrt(1 - a)
    assert O.segment_alpha(0.75, 0.5 * dref, dref) == pytest.approx(0.5, abs=1e-15)


# ---------------------------------------------------------------- cameras (textbook look-at / projection)

def _lookat(cam):
    eye = np.asarray(cam["eye"], float)
    f = np.asarray(cam["target"], float) - eye
    f /= np.linalg.norm(f)
    s = np.cross(f, cam["up"])
    s /= np.linalg.norm(s)
    u = np.cross(s, f)
    return eye, np.stack([s, u, -f])


@pytest.mark.parametrize("W,H", [(16, 16), (32, 18)])
def test_perspective_rays_project_to_pixel_centres(W, H):
    cam = {"kind": "persp", "eye": [1.7, -0.9, 1.3], "target": [0.5, 0.5, 0.5], "up": [0, 0, 1],
           "fovy_deg": 37.0, "width": W, "height": H}
    eye, M = _lookat(cam)
    th = math.tan(math.radians(37.0) / 2)
    for py in range(0, H, 3):
        for px in range(0, W, 5):
            o, d = O.camera_ray(cam, px, py)
            np.testing.assert_allclose(o, eye, atol=1e-15)
            assert np.linalg.norm(d) == pytest.approx(1.0, abs=1e-15)
            Xv = M @ (o + 2.0 * d - eye)
            xn = Xv[0] / -Xv[2] / (th * W / H)
            yn = Xv[1] / -Xv[2] / th
            assert xn == pytest.approx(2 * (px + 0.5) / W - 1, abs=1e-13)
            assert yn == pytest.approx(1 - 2 * (py + 0.5) / H, abs=1e-13)   # y = 0 on top


def test_orthographic_rays():
    cam = {"kind": "ortho", "eye": [0.5, -1.0, 0.5], "target": [0.5, 0.5, 0.5], "up": [0, 0, 1],
           "ortho_half_h": 0.75, "width": 8, "height": 4}
    for py in range(4):
        for px in range(8):
            o, d = O.camera_ray(cam, px, py)
            np.testing.assert_allclose(d, [0, 1, 0], atol=1e-15)
            xn = 2 * (px + 0.5) / 8 - 1
            yn = 1 - 2 * (py + 0.5) / 4
            np.testing.assert_allclose(o, [0.5 + xn * 0.75 * 2, -1.0, 0.5 + yn * 0.75], atol=1e-15)


def test_cube_hit_against_bisection():
    rng = np.random.default_rng(4)
    inside = lambda p: bool(np.all((p >= 0) & (p <= 1)))  # noqa: E731
    for _ in range(300):
        o = rng.uniform(-1.5, 2.5, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        hit, ti, tf = O.cube_hit(o, d)
        ts = np.linspace(0, 6, 6001)
        ins = np.array([inside(o + t * d) for t in ts])
        if not ins.any():
            assert not hit or tf - ti < 2e-3
            continue
        assert hit
        lo, hi = ts[ins][0], ts[ins][-1]
        assert abs(ti - lo) <= 1.001e-3 and abs(tf - hi) <= 1.001e-3
        # sharpen with bisection on both ends
        if ti > 0:
            a, b = lo - 1e-3, lo
            for _ in range(60):
                m = 0.5 * (a + b)
                a, b = (a, m) if inside(o + m * d) else (m, b)
            assert ti == pytest.approx(b, abs=1e-12)


def test_stack_lookup_registration_with_build():
    """A point at the far face of slab k above texel (i,j) reads S[k][j][i]
    exactly (Eq. 9 index k+1 there); halfway through slab k it reads the mean
    of the two faces (continuous depth, reading R11)."""
    rng = np.random.default_rng(5)
    raw = rng.integers(0, 256, size=(10, 10, 10), dtype=np.uint8)
    vol, tf = O.Volume(raw), O.TF(np.stack([np.linspace(0, 1, 256)] * 3 + [np.linspace(0, 0.6, 256)], 1))
    st = O.Stack(vol, tf, [0.3, -0.5, 0.8], 9, 11)
    S = st.export()
    f = st.frame
    for (k, j, i) in [(0, 0, 0), (3, 5, 7), (8, 10, 10), (4, 2, 9)]:
        ui = -f["R"] + (i + 0.5) * 2 * f["R"] / 11
        vj = -f["R"] + (j + 0.5) * 2 * f["R"] / 11
        base = f["c"] + ui * f["U"] + vj * f["V"] - (f["L"] @ f["c"]) * f["L"]
        p_face = base + (f["dmin"] + (k + 1) * f["ds"]) * f["L"]
        assert st.lookup(p_face) == pytest.approx(S[k, j, i], abs=1e-12)
        p_mid = base + (f["dmin"] + (k + 0.5) * f["ds"]) * f["L"]
        prev = S[k - 1, j, i] if k > 0 else 1.0
        assert st.lookup(p_mid) == pytest.approx(0.5 * (prev + S[k, j, i]), abs=1e-12)
    # before the first face: fully transmitting; beyond the last: last layer (reading R12)
    p = f["c"] + (f["dmin"] - 0.1 - f["L"] @ f["c"]) * f["L"]
    assert st.lookup(p) == 1.0
    far = f["c"] + (f["dmax"] + 0.3 - f["L"] @ f["c"]) * f["L"]
    i = j = 5
    ui = -f["R"] + (i + 0.5) * 2 * f["R"] / 11
    far = far + ui * f["U"] + ui * f["V"]
    assert st.lookup(far) == pytest.approx(S[-1, j, i], abs=1e-12)
    # far outside the light square: border transmits fully
    assert st.lookup(f["c"] + 3.0 * f["U"]) == 1.0
