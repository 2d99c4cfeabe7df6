"""The C-ABI library on the CPU: it loads, exports every declared symbol, and its
host-side logic (light frame, validation, sizes) behaves -- no kernel launches."""
import ctypes as C
import math
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2008_06134_amd import vi


def test_library_exports_every_header_symbol():
    declared = vi.header_symbols()
    assert {"vi_build_attenuation", "vi_render", "vi_light_frame", "vi_last_error"} <= set(declared)
    out = subprocess.run(["nm", "-D", "--defined-only", vi.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(re.findall(r"\bT (vi_\w+)", out.stdout))
    missing = set(declared) - exported
    assert not missing, missing
    # and the binding binds exactly those
    assert set(vi.SIGNATURES) == set(declared)
    lib = vi.lib()
    for name in declared:
        assert getattr(lib, name) is not None


def test_version_and_defaults():
    assert "gfx950" in vi.version()
    d = vi.default_opts()
    assert d["term_eps"] == 2.0 ** -15 and d["shell_count"] == 1 and d["cone_rings"] == 2
    assert d["cone_angles"] == 4 and d["cone_grid"] == 0 and d["cone_tan"] == 1.0
    assert d["ambient"] == 0.0 and d["bg"] == [0, 0, 0, 0] and d["light_rgb"] == [1, 1, 1]
    # the oracle's defaults are the same readings
    od = O.default_opts()
    for k in ("term_eps", "shell_count", "shell_h_vox", "cone_rings", "cone_angles", "cone_grid", "cone_tan",
              "ambient"):
        assert od[k] == pytest.approx(d[k], rel=0, abs=0)


@pytest.mark.parametrize("light", [[1, 1, -1], [0, 0, 1], [0.3, -0.8, 0.5], [-1e-3, 2.0, 1e-7], [5, -5, 0]])
def test_light_frame_matches_oracle(light):
    f = vi.light_frame(light, 17, 33).frame()
    g = O.light_frame(light, 17, 33)
    for k in ("L", "U", "V", "c"):
        np.testing.assert_allclose(f[k], g[k], atol=2e-16)
    for k in ("dmin", "dmax", "ds", "R"):
        assert f[k] == pytest.approx(g[k], abs=4e-16)


@pytest.mark.parametrize("pos", [[0.5, 0.5, 2.5], [-1.2, 0.3, 1.9], [3.0, -2.0, -1.0], [0.5, 1.37, 0.5]])
def test_point_light_frame_matches_oracle(pos):
    """Point light (section 3.2.1's L_p with a light position): the descriptor
    the library computes equals the oracle's frame."""
    f = vi.light_frame(None, 17, 33, position=pos).frame()
    g = O.light_frame(None, 17, 33, position=pos)
    assert f["positional"] == 1 and g["positional"] == 1
    for k in ("L", "U", "V", "c", "P"):
        np.testing.assert_allclose(f[k], g[k], atol=4e-16)
    for k in ("dmin", "dmax", "ds", "R"):
        assert f[k] == pytest.approx(g[k], rel=1e-14, abs=1e-15)


@pytest.mark.parametrize("pos", [[0.5, 0.5, 0.5], [0.5, 0.5, 1.3], [1.0, 1.0, 1.0], [math.nan, 0, 3],
                                 [math.inf, 0, 0]])
def test_point_light_inside_or_invalid_rejected(pos):
    assert _err(lambda: vi.light_frame(None, 8, 8, position=pos)) == -1


def test_slices_bytes():
    assert vi.slices_bytes(512, 1024, vi.VI_F32) == 512 * 1024 * 1024 * 4
    assert vi.slices_bytes(512, 1024, vi.VI_BF16) == 512 * 1024 * 1024 * 2
    assert vi.slices_bytes(0, 10, vi.VI_F32) == 0
    assert vi.slices_bytes(4, 4, vi.VI_U8) == 0


def _err(fn):
    with pytest.raises(vi.VIError) as e:
        fn()
    return e.value.code


@pytest.mark.parametrize("light,n,res,dt,code", [
    ([0, 0, 0], 8, 8, vi.VI_F32, -1),
    ([math.nan, 0, 1], 8, 8, vi.VI_F32, -1),
    ([math.inf, 0, 1], 8, 8, vi.VI_F32, -1),
    ([0, 0, 1], 0, 8, vi.VI_F32, -1),
    ([0, 0, 1], 4097, 8, vi.VI_F32, -1),
    ([0, 0, 1], 8, 0, vi.VI_F32, -1),
    ([0, 0, 1], 8, 8193, vi.VI_F32, -1),
    ([0, 0, 1], 8, 8, vi.VI_U8, -2),
])
def test_light_frame_validation(light, n, res, dt, code):
    assert _err(lambda: vi.light_frame(light, n, res, dt)) == code
    assert vi.lib().vi_last_error().decode() != ""


class _Fake:
    """Host-side structs pointing at fake (never dereferenced) device addresses:
    every call below is rejected during validation, before any launch."""

    def __init__(self, n=16, dtype=vi.VI_U8, K=256):
        self.vol = vi.Volume_t(0x10000, dtype, n, 1.0 / 255)
        self.tf = vi.TF_t(0x20000, K)


def _build(f, light=(0, 0, 1), n=8, res=8, dt=vi.VI_F32, buf=0x30000, desc=True, layout=vi.VI_STACK_TILED,
           darken=None):
    lib = vi.lib()
    s = vi.Slices_t()
    opts = C.byref(vi.BuildOpts_t(darken)) if darken is not None else None
    return lib.vi_build_attenuation(C.byref(f.vol) if f.vol else None, C.byref(f.tf) if f.tf else None,
                                    vi._vec3(light), n, res, dt, layout, opts, C.c_void_p(buf),
                                    C.byref(s) if desc else None, C.c_void_p(0))


def test_build_validation_errors():
    f = _Fake()
    f.vol.data = None
    assert _build(f) == -1
    f = _Fake(dtype=7)
    assert _build(f) == -2
    f = _Fake(n=1)
    assert _build(f) == -1
    f = _Fake(K=1)
    assert _build(f) == -1
    f = _Fake(K=2000)
    assert _build(f) == -1
    assert _build(_Fake(), buf=0) == -1
    assert _build(_Fake(), buf=0x30002) == -1        # misaligned stack
    assert _build(_Fake(), buf=0x30008) == -1        # stacks are 16-byte aligned
    assert _build(_Fake(), layout=2) == -2           # unknown stack layout
    assert _build(_Fake(), darken=-1.0) == -1        # compensation exponent out of range
    assert _build(_Fake(), darken=math.nan) == -1
    assert _build(_Fake(), darken=65.0) == -1
    assert _build(_Fake(), light=(0, 0, 0)) == -1
    lib, s = vi.lib(), vi.Slices_t()
    inside = vi.build_opts(0.0, (0.5, 0.5, 1.2))              # point light inside the cube's sphere
    assert lib.vi_build_attenuation(C.byref(f.vol), C.byref(f.tf), None, 8, 8, vi.VI_F32, vi.VI_STACK_ROWS,
                                    C.byref(inside), C.c_void_p(0x30000), C.byref(s), C.c_void_p(0)) == -1
    bad = vi.build_opts(0.0, (0.5, 0.5, 3.0))
    bad.positional = 2
    assert lib.vi_build_attenuation(C.byref(f.vol), C.byref(f.tf), None, 8, 8, vi.VI_F32, vi.VI_STACK_ROWS,
                                    C.byref(bad), C.c_void_p(0x30000), C.byref(s), C.c_void_p(0)) == -1
    assert _build(_Fake(), dt=vi.VI_U16) == -2
    assert _build(_Fake(), desc=False) == -1
    assert _build(_Fake(), n=4096, res=8192) == -2   # tiled stack >= 4 GiB
    assert _build(_Fake(), n=4096, res=8192, layout=vi.VI_STACK_ROWS) == -2
    f = _Fake(n=1700, dtype=vi.VI_U8)                 # volume >= 4 GiB
    assert _build(f) == -2
    f = _Fake(dtype=vi.VI_U16)
    f.vol.data = 0x10001                              # misaligned 16-bit volume
    assert _build(f) == -1


def _render(f, sl=None, cam=None, mode=1, step=0.5, out=0x40000, opts=None):
    lib = vi.lib()
    if cam is None:
        cam = {"kind": "persp", "eye": [2, 2, 2], "target": [0.5, 0.5, 0.5], "up": [0, 0, 1], "fovy_deg": 40,
               "width": 8, "height": 8}
    o = vi.render_opts(opts)
    return lib.vi_render(C.byref(f.vol), C.byref(f.tf), C.byref(sl) if sl is not None else None,
                         C.byref(vi.camera(cam)), mode, C.c_float(step), C.byref(o), C.c_void_p(out), None,
                         C.c_void_p(0))


def _desc(f, n=8, res=8):
    s = vi.light_frame([0, 0, 1], n, res).s
    s.data = 0x50000
    s.vol_n = f.vol.n
    s.tag = vi.lib().vi_tag(C.byref(f.vol), C.byref(f.tf))
    return s


def test_render_validation_errors():
    f = _Fake()
    good = _desc(f)
    assert _render(f, None, mode=1) == -1                      # shading mode without a stack
    assert _render(f, good, mode=9) == -2
    assert _render(f, good, step=0.0) == -1
    assert _render(f, good, step=math.nan) == -1
    assert _render(f, good, out=0) == -1
    assert _render(f, good, out=0x40004) == -1                 # rgba not 16-byte aligned
    bad = _desc(f)
    bad.vol_n = 32
    assert _render(f, bad) == -1                               # stack from another volume size
    bad = _desc(f)
    bad.tag = 12345
    assert _render(f, bad) == -1                               # stack from another volume
    bad = _desc(f)
    bad.layout = 3
    assert _render(f, bad) == -2                               # unknown stack layout
    bad = _desc(f)
    bad.data = 0x50008
    assert _render(f, bad) == -1                               # stack not 16-byte aligned
    cam = {"kind": "persp", "eye": [0.5, 0.5, 0.5], "target": [0.5, 0.5, 0.5], "up": [0, 0, 1], "fovy_deg": 40,
           "width": 8, "height": 8}
    assert _render(f, good, cam=cam) == -1                     # eye == target
    cam = dict(cam, eye=[0.5, 0.5, 3.0])
    assert _render(f, good, cam=cam) == -1                     # up parallel to view
    cam = dict(cam, up=[0, 1, 0], fovy_deg=0.0)
    assert _render(f, good, cam=cam) == -1
    cam = dict(cam, fovy_deg=40.0, width=0)
    assert _render(f, good, cam=cam) == -1
    assert _render(f, good, mode=2, opts={"shell_count": 9}) == -1
    assert _render(f, good, mode=3, opts={"cone_grid": 8}) == -1
    assert _render(f, good, mode=3, opts={"cone_rings": 0}) == -1
    assert _render(f, good, mode=3, opts={"cone_angles": 17}) == -1
    assert _render(f, good, mode=2, opts={"shell_w": [1, -1]}) == -1
    assert _render(f, good, mode=2, opts={"shell_w": [math.inf]}) == -1
    assert _render(f, good, opts={"ambient": 1.5}) == -1
    assert "ambient" in vi.lib().vi_last_error().decode()
    # Phong: needs a light frame (not a stack), sane coefficients
    assert _render(f, None, mode=4) == -1
    assert _render(f, good, mode=5) == -2
    assert _render(f, good, mode=4, opts={"grad_eps": 0.0}) == -1
    assert _render(f, good, mode=4, opts={"phong_shininess": -1.0}) == -1
    assert _render(f, good, mode=4, opts={"phong_kd": math.nan}) == -1
    assert _render(f, good, mode=4, opts={"phong_ks": -0.1}) == -1
    nolight = _desc(f)
    nolight.L = (C.c_double * 3)(0, 0, 0)
    assert _render(f, nolight, mode=4) == -1
    # point light: the cone is accepted (its axis follows the light per sample) and its options checked
    pt = vi.light_frame(None, 8, 8, position=[0.5, 0.5, 3.0]).s
    pt.data, pt.vol_n, pt.tag = 0x50000, f.vol.n, 0
    assert _render(f, pt, mode=3, opts={"cone_tan": -1.0}) == -1
    assert "cone_tan" in vi.lib().vi_last_error().decode()
    assert _render(f, pt, mode=3, opts={"cone_grid": 9}) == -1
    bad = vi.light_frame(None, 8, 8, position=[0.5, 0.5, 3.0]).s
    bad.data, bad.vol_n, bad.tag = 0x50000, f.vol.n, 0
    bad.P = (C.c_double * 3)(math.nan, 0, 0)
    assert _render(f, bad, mode=1) == -1
    bad.P = (C.c_double * 3)(0.5, 0.5, 3.0)
    bad.dmin = 0.0
    assert _render(f, bad, mode=2) == -1


def test_tag_distinguishes_inputs():
    a, b = _Fake(), _Fake()
    b.vol.data = 0x11000
    lib = vi.lib()
    ta = lib.vi_tag(C.byref(a.vol), C.byref(a.tf))
    tb = lib.vi_tag(C.byref(b.vol), C.byref(b.tf))
    assert ta != tb and ta != 0
    assert ta == lib.vi_tag(C.byref(a.vol), C.byref(a.tf))


def test_volume_bytes_and_brick_validation():
    assert vi.volume_bytes(512, vi.VI_U16, vi.VI_LAYOUT_LINEAR) == 512 ** 3 * 2
    assert vi.volume_bytes(33, vi.VI_U8, vi.VI_LAYOUT_BRICK4) == 36 ** 3
    assert vi.volume_bytes(33, vi.VI_F32, vi.VI_LAYOUT_BRICK4) == 36 ** 3 * 4
    assert vi.volume_bytes(1, vi.VI_U8, 0) == 0 and vi.volume_bytes(8, vi.VI_BF16, 0) == 0
    assert vi.volume_bytes(8, vi.VI_U8, 5) == 0
    lib = vi.lib()
    src = vi.Volume_t(0x10000, vi.VI_U16, 16, 1 / 4095, vi.VI_LAYOUT_BRICK4)
    out = vi.Volume_t()
    assert lib.vi_volume_to_bricks(C.byref(src), C.c_void_p(0x20000), C.byref(out), None) == -1  # not linear
    src.layout = vi.VI_LAYOUT_LINEAR
    assert lib.vi_volume_to_bricks(C.byref(src), None, C.byref(out), None) == -1
    assert lib.vi_volume_to_bricks(C.byref(src), C.c_void_p(0x20001), C.byref(out), None) == -1
    src.layout = 7
    assert lib.vi_volume_to_bricks(C.byref(src), C.c_void_p(0x20000), C.byref(out), None) == -2
    # quads: four values per slot, aligned to a whole slot
    assert vi.volume_bytes(33, vi.VI_U16, vi.VI_LAYOUT_QUAD4) == 4 * 36 ** 3 * 2
    assert vi.volume_bytes(16, vi.VI_F32, vi.VI_LAYOUT_QUAD4) == 4 * 16 ** 3 * 4
    src.layout = vi.VI_LAYOUT_QUAD4
    assert lib.vi_volume_to_quads(C.byref(src), C.c_void_p(0x20000), C.byref(out), None) == -1  # not linear
    src.layout = vi.VI_LAYOUT_LINEAR
    assert lib.vi_volume_to_quads(C.byref(src), C.c_void_p(0x20004), C.byref(out), None) == -1  # 8-byte slots
    assert lib.vi_volume_to_quads(C.byref(src), None, C.byref(out), None) == -1
    big = vi.Volume_t(0x10000, vi.VI_U8, 1700, 1 / 255, vi.VI_LAYOUT_LINEAR)
    assert lib.vi_volume_to_quads(C.byref(big), C.c_void_p(0x20000), C.byref(out), None) == -2  # >= 4 GiB of slots
    # a quad volume whose pointer is not slot-aligned is rejected by the passes
    f = _Fake(dtype=vi.VI_U16)
    f.vol.layout = vi.VI_LAYOUT_QUAD4
    f.vol.data = 0x10004
    assert _build(f) == -1
    # stack buffers are padded to whole 8 x 4 tiles
    assert vi.slices_bytes(3, 10, vi.VI_F32) == 3 * 16 * 12 * 4
    # rows: n+2 layers of res+4 rows of pitch res+4 rounded up to 4, a layer's
    # size the least odd multiple of half a 128-byte line from there up
    assert vi.slices_bytes(3, 10, vi.VI_F32, vi.VI_STACK_ROWS) == 5 * 240 * 4  # 14 x 16 = 224 -> 15 x 16
    assert vi.slices_bytes(3, 10, vi.VI_BF16, vi.VI_STACK_ROWS) == 5 * 224 * 2  # 7 x 32
    assert vi.slices_bytes(2, 1024, vi.VI_BF16, vi.VI_STACK_ROWS) == 4 * 1056800 * 2  # 1028^2 -> 33025 x 32
    assert vi.slices_bytes(2, 1024, vi.VI_F16, vi.VI_STACK_ROWS) == 4 * 1056800 * 2
    assert vi.slices_bytes(2, 1024, vi.VI_F16, vi.VI_STACK_TILED) == 0
    assert vi.slices_bytes(2, 1024, vi.VI_F32, vi.VI_STACK_ROWS) == 4 * 1028 * 1028 * 4  # 66049 x 16
    assert vi.slices_bytes(2, 8, vi.VI_F32, 5) == 0


def test_row_layer_rule():
    """Row layout: pitch res + 4 rounded up to 4; a layer's size in bytes the
    least odd multiple of 64 from (res + 4) x pitch elements up, so the same
    texel of neighbouring layers lies half a 128-byte line apart and every
    other layer starts on a line; the library's stack size and the binding's
    pitch and layer agree for every res and dtype."""
    for res in list(range(1, 300)) + [511, 512, 1000, 1023, 1024, 2048, 4091]:
        w, p = res + 4, vi.row_pitch(res)
        assert p % 4 == 0 and w <= p < w + 4
        for dt, es in ((vi.VI_F32, 4), (vi.VI_BF16, 2), (vi.VI_F16, 2)):
            ls = vi.row_layer(res, dt)
            assert (ls * es) % 128 == 64 and w * p <= ls < w * p + 2 * 128 // es
            assert not any((q * es) % 128 == 64 for q in range(w * p, ls))  # the least such
            assert vi.slices_bytes(5, res, dt, vi.VI_STACK_ROWS) == 7 * ls * es


def test_occupancy_validation():
    lib = vi.lib()
    # cell bits, then the bits of the 4 x 4 x 4-cell super-cells
    assert lib.vi_volume_occupancy_bytes(512, 16) == 32 ** 3 // 32 * 4 + 8 ** 3 // 32 * 4
    assert lib.vi_volume_occupancy_bytes(33, 8) == (5 ** 3 + 31) // 32 * 4 + 4
    assert lib.vi_volume_occupancy_bytes(33, 5) == 0 and lib.vi_volume_occupancy_bytes(1, 8) == 0
    f = _Fake()
    out = vi.Volume_t()
    assert lib.vi_volume_occupancy(C.byref(f.vol), C.byref(f.tf), C.c_void_p(0x60000), C.byref(out), None) == -1
    assert "map" in lib.vi_last_error().decode()                 # no empty-space map
    f.vol.minmax, f.vol.cell = 0x70000, 8
    assert lib.vi_volume_occupancy(C.byref(f.vol), C.byref(f.tf), C.c_void_p(0x60002), C.byref(out), None) == -1
    assert lib.vi_volume_occupancy(C.byref(f.vol), C.byref(f.tf), None, C.byref(out), None) == -1
    # the passes take bits only with the transfer function (and map) they were made for
    f.vol.occ, f.vol.occ_tag = 0x60000, 12345
    assert _build(f) == -1
    assert "occupancy" in lib.vi_last_error().decode()
    assert _render(f, _desc(f), mode=2) == -1
    f.vol.minmax = None                                            # bits without a map
    assert _build(f) == -1


def test_minmax_validation():
    lib = vi.lib()
    assert lib.vi_volume_minmax_bytes(512, 8) == 64 ** 3 * 8
    assert lib.vi_volume_minmax_bytes(33, 8) == 5 ** 3 * 8
    assert lib.vi_volume_minmax_bytes(33, 5) == 0
    v = vi.Volume_t(0x10000, vi.VI_U16, 16, 1 / 4095, 0, None, 0)
    out = vi.Volume_t()
    assert lib.vi_volume_minmax(C.byref(v), 6, C.c_void_p(0x20000), C.byref(out), None) == -1
    assert lib.vi_volume_minmax(C.byref(v), 8, None, C.byref(out), None) == -1
    assert lib.vi_volume_minmax(C.byref(v), 8, C.c_void_p(0x20004), C.byref(out), None) == -1
    # a volume that claims a map with a bad cell size is rejected by every call
    v.minmax, v.cell = 0x30000, 12
    f = _Fake()
    f.vol = v
    assert _build(f) == -1


def test_tf_identity_is_its_contents():
    """Two tables at the same device address (a freed table's address reused
    by the allocator) with different contents name different stacks and
    occupancy bits; the same contents name the same."""
    import numpy as np
    import torch
    lib = vi.lib()
    ramp = np.linspace(0, 1, 256 * 4, dtype=np.float32).reshape(256, 4)
    other = ramp.copy()
    other[100, 3] = 0.5
    ta = vi.tf_tag(torch.from_numpy(ramp))
    tb = vi.tf_tag(torch.from_numpy(other))
    assert ta != 0 and tb != 0 and ta != tb
    assert ta == vi.tf_tag(torch.from_numpy(ramp.copy()))
    assert lib.vi_tf_tag(None, 4) == 0
    a, b = _Fake(), _Fake()
    a.tf.tag, b.tf.tag = ta, tb                       # same pointer 0x20000, other contents
    assert lib.vi_tag(C.byref(a.vol), C.byref(a.tf)) != lib.vi_tag(C.byref(b.vol), C.byref(b.tf))
    # a stack built with table a is refused with table b
    sa = _desc(a)
    assert _render(b, sa, mode=2) == -1
    assert "another volume or transfer function" in lib.vi_last_error().decode()
    # (occupancy bits carry the same identity: tests/test_gpu_parity.py makes
    # bits with one table and has them refused with a rewritten one)


def test_samples_opaque_flag_validated():
    f = _Fake()
    assert _render(f, _desc(f), mode=2, opts={"samples_opaque": 2}) == -1
    assert "samples_opaque" in vi.lib().vi_last_error().decode()


def test_step_bound_keeps_segments_below_2_24():
    """step_vox so small that a chord of sqrt(3) N voxels would hold more than
    2^24 segments is refused before any launch."""
    f = _Fake(n=16)
    good = _desc(f)
    assert _render(f, good, step=1e-6) == -1
    assert "2^24" in vi.lib().vi_last_error().decode()


def test_l2_probe_library_exports_its_entry_point():
    """The benchmark's probes are built beside libvi (their own library, loaded only
    by bench.py --l2-probe and --store-probe) and export their C entry points."""
    import subprocess
    path = os.path.join(os.path.dirname(vi.LIB_PATH), "libvi_probe.so")
    assert os.path.exists(path), "build the libraries first (paper_2008_06134_amd.build)"
    syms = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True, check=True).stdout
    assert " vi_probe_l2_read" in syms and " vi_probe_store_rows" in syms
