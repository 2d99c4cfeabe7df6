"""Thin ctypes binding of libvi (the C ABI in ``include/vi.h``).

Argument marshalling only: every step of both passes runs in the HIP kernels
of ``libvi.so``.  PyTorch is used for device memory and streams.  If the
library has not been built this module raises on first use -- there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvi.so")

VI_U8, VI_U16, VI_F16, VI_F32, VI_BF16 = 0, 1, 2, 3, 4
MODES = {"none": 0, "shadow": 1, "shell": 2, "cone": 3, "phong": 4}
_PHONG_KEYS = ("phong_ka", "phong_kd", "phong_ks", "phong_shininess", "grad_eps")
ERRORS = {-1: "VI_E_INVALID_ARG", -2: "VI_E_UNSUPPORTED", -3: "VI_E_NO_MEMORY", -4: "VI_E_DEVICE",
          -5: "VI_E_BUSY", -6: "VI_E_CANCELLED"}


class VIError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


VI_LAYOUT_LINEAR, VI_LAYOUT_BRICK4, VI_LAYOUT_QUAD4 = 0, 1, 2
VI_STACK_TILED, VI_STACK_ROWS = 0, 1


class Volume_t(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int), ("n", C.c_int), ("scale", C.c_float),
                ("layout", C.c_int), ("minmax", C.c_void_p), ("cell", C.c_int), ("occ", C.c_void_p),
                ("occ_tag", C.c_uint64)]


class TF_t(C.Structure):
    _fields_ = [("rgba", C.c_void_p), ("n_entries", C.c_int), ("tag", C.c_uint64)]


class Slices_t(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int), ("layout", C.c_int), ("n", C.c_int), ("res", C.c_int),
                ("L", C.c_double * 3), ("U", C.c_double * 3), ("V", C.c_double * 3), ("c", C.c_double * 3),
                ("dmin", C.c_double), ("dmax", C.c_double), ("ds", C.c_double), ("R", C.c_double),
                ("vol_n", C.c_int), ("tag", C.c_uint64), ("darken", C.c_float), ("positional", C.c_int),
                ("P", C.c_double * 3)]


class BuildOpts_t(C.Structure):
    _fields_ = [("darken", C.c_float), ("positional", C.c_int), ("position", C.c_double * 3)]


def build_opts(darken: float = 0.0, position=None) -> BuildOpts_t:
    """Build options: `position` (world xyz) makes the light a point light."""
    o = BuildOpts_t()
    o.darken = float(darken)
    if position is not None:
        o.positional = 1
        o.position = _vec3(position)
    return o


class Camera_t(C.Structure):
    _fields_ = [("kind", C.c_int), ("eye", C.c_double * 3), ("target", C.c_double * 3), ("up", C.c_double * 3),
                ("fovy_deg", C.c_double), ("ortho_half_h", C.c_double), ("width", C.c_int), ("height", C.c_int)]


class RenderOpts_t(C.Structure):
    _fields_ = [("ambient", C.c_float), ("light_rgb", C.c_float * 3), ("bg", C.c_float * 4),
                ("term_eps", C.c_float), ("shell_count", C.c_int), ("shell_w", C.c_float * 8),
                ("shell_h_vox", C.c_float),
                ("cone_rings", C.c_int), ("cone_angles", C.c_int), ("cone_grid", C.c_int), ("cone_tan", C.c_float),
                ("phong_ka", C.c_float), ("phong_kd", C.c_float), ("phong_ks", C.c_float),
                ("phong_shininess", C.c_float), ("grad_eps", C.c_float), ("samples_opaque", C.c_int),
                ("nearest_layer", C.c_int)]


class ServerCfg_t(C.Structure):
    _fields_ = [("stack_budget", C.c_size_t), ("max_inflight", C.c_int), ("tiles_per_launch", C.c_int),
                ("device", C.c_int)]


class Request_t(C.Structure):
    _fields_ = [("vol_id", C.c_int), ("light_dir", C.c_double * 3), ("n_slices", C.c_int), ("slice_res", C.c_int),
                ("slice_dtype", C.c_int), ("slice_layout", C.c_int), ("build", BuildOpts_t), ("camera", Camera_t), ("mode", C.c_int), ("step_vox", C.c_float),
                ("opts", RenderOpts_t), ("d_rgba", C.c_void_p), ("d_samples", C.c_void_p)]


class Stats_t(C.Structure):
    _fields_ = [(k, C.c_uint64) for k in ("submitted", "completed", "rejected", "cancelled", "stack_hits",
                                          "stack_builds", "evictions", "launches", "tiles")] + \
               [(k, C.c_double) for k in ("mean_frames_per_launch", "p50_ms", "p99_ms", "mean_ms", "max_ms",
                                          "frames_per_s")] + \
               [(k, C.c_size_t) for k in ("pool_bytes", "pool_in_use", "pool_peak")]


# every symbol declared in include/vi.h, with its ctypes signature
SIGNATURES = {
    "vi_version": ([], C.c_char_p),
    "vi_last_error": ([], C.c_char_p),
    "vi_default_render_opts": ([C.POINTER(RenderOpts_t)], C.c_int),
    "vi_slices_bytes": ([C.c_int, C.c_int, C.c_int, C.c_int], C.c_size_t),
    "vi_volume_bytes": ([C.c_int, C.c_int, C.c_int], C.c_size_t),
    "vi_volume_to_bricks": ([C.POINTER(Volume_t), C.c_void_p, C.POINTER(Volume_t), C.c_void_p], C.c_int),
    "vi_volume_to_quads": ([C.POINTER(Volume_t), C.c_void_p, C.POINTER(Volume_t), C.c_void_p], C.c_int),
    "vi_volume_minmax_bytes": ([C.c_int, C.c_int], C.c_size_t),
    "vi_volume_minmax": ([C.POINTER(Volume_t), C.c_int, C.c_void_p, C.POINTER(Volume_t), C.c_void_p], C.c_int),
    "vi_volume_occupancy_bytes": ([C.c_int, C.c_int], C.c_size_t),
    "vi_volume_occupancy": ([C.POINTER(Volume_t), C.POINTER(TF_t), C.c_void_p, C.POINTER(Volume_t), C.c_void_p],
                            C.c_int),
    "vi_light_frame": ([C.POINTER(C.c_double), C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(BuildOpts_t),
                        C.POINTER(Slices_t)], C.c_int),
    "vi_build_attenuation": ([C.POINTER(Volume_t), C.POINTER(TF_t), C.POINTER(C.c_double), C.c_int, C.c_int,
                              C.c_int, C.c_int, C.POINTER(BuildOpts_t), C.c_void_p, C.POINTER(Slices_t),
                              C.c_void_p], C.c_int),
    "vi_render": ([C.POINTER(Volume_t), C.POINTER(TF_t), C.POINTER(Slices_t), C.POINTER(Camera_t), C.c_int,
                   C.c_float, C.POINTER(RenderOpts_t), C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "vi_tag": ([C.POINTER(Volume_t), C.POINTER(TF_t)], C.c_uint64),
    "vi_tf_tag": ([C.c_void_p, C.c_int], C.c_uint64),
    "vi_server_create": ([C.POINTER(ServerCfg_t), C.POINTER(C.c_void_p)], C.c_int),
    "vi_server_register_volume": ([C.c_void_p, C.POINTER(Volume_t), C.POINTER(TF_t), C.POINTER(C.c_int)], C.c_int),
    "vi_server_submit": ([C.c_void_p, C.POINTER(Request_t), C.POINTER(C.c_uint64)], C.c_int),
    "vi_server_poll": ([C.c_void_p, C.c_uint64, C.POINTER(C.c_int)], C.c_int),
    "vi_server_wait": ([C.c_void_p, C.c_uint64, C.c_int], C.c_int),
    "vi_server_cancel": ([C.c_void_p, C.c_uint64], C.c_int),
    "vi_server_stats": ([C.c_void_p, C.POINTER(Stats_t)], C.c_int),
    "vi_server_reset_stats": ([C.c_void_p], C.c_int),
    "vi_server_destroy": ([C.c_void_p], None),
}

_lib = None


def lib():
    """Load libvi.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2008_06134_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise VIError(rc, lib().vi_last_error().decode())


def _stream(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _vec3(x):
    return (C.c_double * 3)(*[float(t) for t in x])


# ---------------------------------------------------------------------------
# inputs
# ---------------------------------------------------------------------------

_VOL_DT = {torch.uint8: VI_U8, torch.uint16: VI_U16, torch.int16: VI_U16, torch.float16: VI_F16,
           torch.float32: VI_F32}
_DEFAULT_SCALE = {VI_U8: 1.0 / 255.0, VI_U16: 1.0 / 4095.0, VI_F16: 1.0, VI_F32: 1.0}


class Volume:
    """A device-resident cubic volume (u8, u16 -- stored as uint16 or its int16 bit
    pattern --, f16 or f32) and the scale mapping raw values to [0,1].  `data` is
    raw[z][y][x] (linear layout), the 4x4x4 brick layout of `to_bricks()` or the quad
    layout of `to_quads()`."""

    def __init__(self, data: torch.Tensor, scale: float | None = None, n: int | None = None,
                 layout: int = VI_LAYOUT_LINEAR):
        if data.dtype not in _VOL_DT:
            raise TypeError(f"unsupported volume dtype {data.dtype}")
        if layout == VI_LAYOUT_LINEAR:
            if data.dim() != 3 or not (data.shape[0] == data.shape[1] == data.shape[2]):
                raise ValueError("volume must be a cubic N x N x N tensor")
            n = int(data.shape[0])
        elif n is None:
            raise ValueError("a bricked volume needs its edge n")
        self.data = data.contiguous()
        self.dtype = _VOL_DT[data.dtype]
        self.n = int(n)
        self.layout = layout
        self.scale = float(_DEFAULT_SCALE[self.dtype] if scale is None else scale)
        self.minmax = None
        self.s = Volume_t(self.data.data_ptr(), self.dtype, self.n, self.scale, layout, None, 0)

    @staticmethod
    def from_numpy(raw, device="cuda", scale=None) -> "Volume":
        import numpy as np
        if raw.dtype == np.uint16:
            t = torch.from_numpy(raw.view(np.int16)).to(device)
        else:
            t = torch.from_numpy(raw).to(device)
        return Volume(t, scale)

    def _relayout(self, layout: int, fn: str, out: torch.Tensor | None, stream) -> "Volume":
        nbytes = int(lib().vi_volume_bytes(self.n, self.dtype, layout))
        if out is None:
            out = torch.empty(nbytes // self.data.element_size(), dtype=self.data.dtype, device=self.data.device)
        if out.numel() * out.element_size() < nbytes:
            raise ValueError("layout buffer too small")
        res = Volume_t()
        _check(getattr(lib(), fn)(C.byref(self.s), C.c_void_p(out.data_ptr()), C.byref(res), _stream(stream)))
        return Volume(out, self.scale, self.n, layout)

    def to_bricks(self, out: torch.Tensor | None = None, stream=None) -> "Volume":
        """Copy into the 4x4x4 brick layout (vi_volume_to_bricks)."""
        return self._relayout(VI_LAYOUT_BRICK4, "vi_volume_to_bricks", out, stream)

    def to_quads(self, out: torch.Tensor | None = None, stream=None) -> "Volume":
        """Copy into the quad layout: brick order, each slot its voxel's 2x2 x/y
        neighbourhood (vi_volume_to_quads); 4x the bytes, two loads per trilinear
        footprint."""
        return self._relayout(VI_LAYOUT_QUAD4, "vi_volume_to_quads", out, stream)

    def with_minmax(self, cell: int = 16, out: torch.Tensor | None = None, stream=None) -> "Volume":
        """The same volume with an empty-space map of `cell`^3-voxel cells (vi_volume_minmax)."""
        nbytes = int(lib().vi_volume_minmax_bytes(self.n, cell))
        if nbytes == 0:
            raise ValueError("invalid cell size")
        if out is None:
            out = torch.empty(nbytes // 4, dtype=torch.float32, device=self.data.device)
        res = Volume_t()
        _check(lib().vi_volume_minmax(C.byref(self.s), int(cell), C.c_void_p(out.data_ptr()), C.byref(res),
                                      _stream(stream)))
        v = Volume(self.data, self.scale, self.n, self.layout)
        v.minmax = out
        v.s = res
        return v

    def with_occupancy(self, tf: "TF", out: torch.Tensor | None = None, stream=None) -> "Volume":
        """The same volume with occupancy bits for `tf` (vi_volume_occupancy): one
        bit per empty-space cell, which the passes read instead of the map.  The
        volume must have a map (with_minmax) and is then rendered with `tf` only."""
        if self.minmax is None:
            raise ValueError("occupancy bits need an empty-space map (with_minmax)")
        nbytes = int(lib().vi_volume_occupancy_bytes(self.n, int(self.s.cell)))
        if out is None:
            out = torch.empty(max(nbytes // 4, 1), dtype=torch.int32, device=self.data.device)
        res = Volume_t()
        _check(lib().vi_volume_occupancy(C.byref(self.s), C.byref(tf.s), C.c_void_p(out.data_ptr()), C.byref(res),
                                         _stream(stream)))
        v = Volume(self.data, self.scale, self.n, self.layout)
        v.minmax = self.minmax
        v.occ = out
        v.s = res
        return v


class TF:
    """A K x 4 float32 RGBA transfer-function table on the device."""

    def __init__(self, rgba: torch.Tensor):
        if rgba.dim() != 2 or rgba.shape[1] != 4:
            raise ValueError("transfer function must be K x 4")
        self.data = rgba.to(torch.float32).contiguous()
        # the table's content tag, from a host copy taken once here
        host = self.data.detach().to("cpu").contiguous()
        self.s = TF_t(self.data.data_ptr(), int(self.data.shape[0]), tf_tag(host))

    @staticmethod
    def from_numpy(tab, device="cuda") -> "TF":
        return TF(torch.from_numpy(tab).to(device=device, dtype=torch.float32))


def row_origin(dtype: int = VI_F32) -> int:
    """Column of texel 0 in a row of the row layout (two border texels precede it)."""
    return 2


def row_pitch(res: int, dtype: int = VI_F32) -> int:
    """Row pitch of the row layout: res + 4 rounded up to 4 (every stack dtype)."""
    return (res + 4 + 3) // 4 * 4


def row_layer(res: int, dtype: int = VI_F32) -> int:
    """Elements per layer of the row layout: the least odd multiple of half a
    128-byte line (16 floats, 32 two-byte texels) from (res + 4) x pitch up."""
    half = 16 if dtype == VI_F32 else 32
    m = -(-(res + 4) * row_pitch(res, dtype) // half)
    return (m | 1) * half


@dataclass
class Slices:
    """An attenuation stack: the device buffer and its descriptor.  Tiled:
    8 x 4 texel tiles per layer, shaped n x R4/4 x R8/8 x 4 x 8.  Rows:
    (n+2) x (res+4) x P with layer stride row_layer(res, dtype), texel (k, j, i) at
    [k+1, j+2, i+2]: a leading layer and a two-texel border around the
    res x res grid, all fully transmitting, and a trailing layer equal to
    the last."""
    data: torch.Tensor | None
    s: Slices_t

    def dense(self) -> torch.Tensor:
        """The stack as an n x res x res tensor (a device view/copy, for inspection)."""
        n, r = self.s.n, self.s.res
        t = self.data
        if self.s.layout == VI_STACK_ROWS:
            e = row_origin(self.s.dtype)
            return t[1:n + 1, 2:r + 2, e:e + r]
        return t.permute(0, 1, 3, 2, 4).reshape(n, t.shape[1] * 4, t.shape[2] * 8)[:, :r, :r]

    def padded(self) -> torch.Tensor:
        """Row layout only: (n+2) x (res+4) x (res+4), the grid with its border,
        the leading layer and the trailing layer."""
        r, e = self.s.res, row_origin(self.s.dtype)
        return self.data[:, :, e - 2:e + r + 2]

    @property
    def n(self):
        return self.s.n

    @property
    def res(self):
        return self.s.res

    def frame(self) -> dict:
        s = self.s
        return {"L": list(s.L), "U": list(s.U), "V": list(s.V), "c": list(s.c), "dmin": s.dmin, "dmax": s.dmax,
                "ds": s.ds, "R": s.R, "n": s.n, "res": s.res, "positional": s.positional, "P": list(s.P)}


def camera(cam: dict) -> Camera_t:
    c = Camera_t()
    c.kind = 1 if cam["kind"] in ("persp", 1) else 0
    c.eye = _vec3(cam["eye"])
    c.target = _vec3(cam["target"])
    c.up = _vec3(cam["up"])
    c.fovy_deg = float(cam.get("fovy_deg", 40.0))
    c.ortho_half_h = float(cam.get("ortho_half_h", 0.5))
    c.width = int(cam["width"])
    c.height = int(cam["height"])
    return c


def default_opts() -> dict:
    o = RenderOpts_t()
    _check(lib().vi_default_render_opts(C.byref(o)))
    return {"ambient": o.ambient, "light_rgb": list(o.light_rgb), "bg": list(o.bg), "term_eps": o.term_eps,
            "shell_count": o.shell_count, "shell_w": list(o.shell_w), "shell_h_vox": o.shell_h_vox,
            "cone_rings": o.cone_rings,
            "cone_angles": o.cone_angles, "cone_grid": o.cone_grid, "cone_tan": o.cone_tan,
            **{k: getattr(o, k) for k in _PHONG_KEYS}, "samples_opaque": o.samples_opaque,
            "nearest_layer": o.nearest_layer}


def render_opts(opts: dict | None) -> RenderOpts_t:
    d = default_opts()
    if opts:
        d.update(opts)
    o = RenderOpts_t()
    o.ambient = d["ambient"]
    o.light_rgb = (C.c_float * 3)(*d["light_rgb"])
    o.bg = (C.c_float * 4)(*d["bg"])
    o.term_eps = d["term_eps"]
    o.shell_count = int(d["shell_count"])
    w = [float(x) for x in d["shell_w"]] + [0.0] * 8
    o.shell_w = (C.c_float * 8)(*w[:8])
    o.shell_h_vox = d["shell_h_vox"]
    o.cone_rings = int(d["cone_rings"])
    o.cone_angles = int(d["cone_angles"])
    o.cone_grid = int(d["cone_grid"])
    o.cone_tan = d["cone_tan"]
    for k in _PHONG_KEYS:
        setattr(o, k, float(d[k]))
    o.samples_opaque = int(d["samples_opaque"])
    o.nearest_layer = int(d["nearest_layer"])
    return o


# ---------------------------------------------------------------------------
# calls
# ---------------------------------------------------------------------------

def slices_bytes(n: int, res: int, dtype: int = VI_F32, layout: int = VI_STACK_TILED) -> int:
    return int(lib().vi_slices_bytes(n, res, dtype, layout))


def stack_buffer(n: int, res: int, dtype: int = VI_F32, device="cuda", layout: int = VI_STACK_TILED) -> torch.Tensor:
    """An uninitialised device buffer in a stack layout (shapes as in Slices)."""
    tdt = {VI_F32: torch.float32, VI_BF16: torch.bfloat16, VI_F16: torch.float16}[dtype]
    if layout == VI_STACK_ROWS:
        # (n+2) x (res+4) x P over layers of row_layer elements
        ls, p = row_layer(res, dtype), row_pitch(res, dtype)
        flat = torch.empty((n + 2) * ls, dtype=tdt, device=device)
        return flat.as_strided((n + 2, res + 4, p), (ls, p, 1))
    r8, r4 = (res + 7) // 8 * 8, (res + 3) // 4 * 4
    return torch.empty((n, r4 // 4, r8 // 8, 4, 8), dtype=tdt, device=device)


def volume_bytes(n: int, dtype: int, layout: int) -> int:
    return int(lib().vi_volume_bytes(n, dtype, layout))


def light_frame(light_dir, n: int, res: int, dtype: int = VI_F32, layout: int = VI_STACK_TILED,
                position=None) -> Slices:
    s = Slices_t()
    ld = _vec3(light_dir) if light_dir is not None else None
    _check(lib().vi_light_frame(ld, int(n), int(res), int(dtype), int(layout), C.byref(build_opts(0.0, position)),
                                C.byref(s)))
    return Slices(None, s)


def build_attenuation(vol: Volume, tf: TF, light_dir, n_slices: int, slice_res: int, dtype: int = VI_F32,
                      out: torch.Tensor | None = None, stream=None, layout: int = VI_STACK_TILED,
                      darken: float = 0.0, position=None) -> Slices:
    """Attenuation stack for `light_dir` (section 3.2.1, Alg. 1); returns the stack
    (float32 transmittance, bfloat16 optical depth -log2 T, or float16 transmittance) and its descriptor.  `darken`
    is the exponent m of section 4's (1+alpha)^m slab compensation (0 = off);
    `position` (world xyz) builds for a point light there instead (`light_dir`
    is then ignored and may be None)."""
    if out is None:
        out = stack_buffer(n_slices, slice_res, dtype, vol.data.device, layout)
    # (a row-layout stack is a strided view whose layers may end in padding:
    # count the bytes of its storage from the view's first element)
    avail = out.untyped_storage().nbytes() - out.storage_offset() * out.element_size()
    if avail < slices_bytes(n_slices, slice_res, dtype, layout):
        raise ValueError("stack buffer too small")
    s = Slices_t()
    ld = _vec3(light_dir) if light_dir is not None else None
    _check(lib().vi_build_attenuation(C.byref(vol.s), C.byref(tf.s), ld, int(n_slices),
                                      int(slice_res), int(dtype), int(layout), C.byref(build_opts(darken, position)),
                                      C.c_void_p(out.data_ptr()), C.byref(s), _stream(stream)))
    return Slices(out, s)


def render(vol: Volume, tf: TF, slices: Slices | None, cam: dict, mode: str, step_vox: float,
           opts: dict | None = None, out: torch.Tensor | None = None, samples: torch.Tensor | None = None,
           stream=None) -> torch.Tensor:
    """Ray-cast one frame (sections 3.2.2-3.2.3, 4); returns H x W x 4 float32
    premultiplied RGBA.  Mode "phong" needs only the light frame of `slices`
    (``light_frame(...)`` serves).  `samples` (int64 device tensor of one element, or two: the
    second then gets the segments composited with non-zero opacity) gets the
    number of composited segments added to it."""
    W, H = int(cam["width"]), int(cam["height"])
    if out is None:
        out = torch.empty((H, W, 4), dtype=torch.float32, device=vol.data.device)
    if out.numel() < W * H * 4 or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("output must be a contiguous float32 tensor of H*W*4 elements")
    o = render_opts(opts)
    if samples is not None and samples.numel() >= 2:
        o.samples_opaque = 1
    sp = C.byref(slices.s) if slices is not None else None
    _check(lib().vi_render(C.byref(vol.s), C.byref(tf.s), sp, C.byref(camera(cam)), MODES[mode],
                           C.c_float(step_vox), C.byref(o), C.c_void_p(out.data_ptr()),
                           C.c_void_p(samples.data_ptr() if samples is not None else 0), _stream(stream)))
    return out


def tag(vol: Volume, tf: TF) -> int:
    return int(lib().vi_tag(C.byref(vol.s), C.byref(tf.s)))


def tf_tag(host_rgba: torch.Tensor) -> int:
    """Content tag of a K x 4 float32 table held in host memory."""
    t = host_rgba.to(torch.float32).contiguous()
    return int(lib().vi_tf_tag(C.c_void_p(t.data_ptr()), int(t.shape[0])))


def version() -> str:
    return lib().vi_version().decode()


def header_symbols() -> list:
    """Function names declared in include/vi.h."""
    import re
    hdr = os.path.join(os.path.dirname(HERE), "include", "vi.h")
    text = open(hdr).read()
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(vi_\w+)\s*\(", text, flags=re.M)))



# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------

REQ_PENDING, REQ_ADMITTED, REQ_DONE = 0, 1, 2


class Server:
    """The continuous-batching request loop of libvi (vi_server_*).

    Volumes and transfer functions are registered once and stay resident;
    each request names a volume, a light (n, res) and a camera/mode, and
    renders into its own device image.  Stacks are cached in a device pool of
    `stack_budget` bytes and reused while the light is unchanged."""

    def __init__(self, stack_budget: int, max_inflight: int = 16, tiles_per_launch: int = 8192, device: int = 0):
        cfg = ServerCfg_t(int(stack_budget), int(max_inflight), int(tiles_per_launch), int(device))
        h = C.c_void_p()
        _check(lib().vi_server_create(C.byref(cfg), C.byref(h)))
        self.h = h
        self._keep = {}     # ticket -> tensors that must outlive the request
        self._vols = []

    def register(self, vol: Volume, tf: TF) -> int:
        vid = C.c_int()
        _check(lib().vi_server_register_volume(self.h, C.byref(vol.s), C.byref(tf.s), C.byref(vid)))
        self._vols.append((vol, tf))
        return vid.value

    def submit(self, vol_id: int, light_dir, n_slices: int, slice_res: int, cam: dict, mode: str,
               step_vox: float, opts: dict | None = None, out: torch.Tensor | None = None,
               samples: torch.Tensor | None = None, dtype: int = VI_F32, device="cuda",
               layout: int = VI_STACK_TILED, darken: float = 0.0, position=None) -> tuple:
        W, H = int(cam["width"]), int(cam["height"])
        if out is None:
            out = torch.empty((H, W, 4), dtype=torch.float32, device=device)
        r = Request_t()
        r.vol_id = int(vol_id)
        r.light_dir = _vec3(light_dir if light_dir is not None else (0.0, 0.0, 1.0))
        r.n_slices, r.slice_res, r.slice_dtype = int(n_slices), int(slice_res), int(dtype)
        r.slice_layout = int(layout)
        r.build = build_opts(darken, position)
        r.camera = camera(cam)
        r.mode = MODES[mode]
        r.step_vox = float(step_vox)
        r.opts = render_opts(opts)
        r.d_rgba = out.data_ptr()
        r.d_samples = samples.data_ptr() if samples is not None else None
        t = C.c_uint64()
        _check(lib().vi_server_submit(self.h, C.byref(r), C.byref(t)))
        self._keep[t.value] = (out, samples)
        return t.value, out

    def poll(self, ticket: int) -> int:
        st = C.c_int()
        _check(lib().vi_server_poll(self.h, int(ticket), C.byref(st)))
        return st.value

    def wait(self, ticket: int, timeout_ms: int = -1) -> int:
        rc = lib().vi_server_wait(self.h, int(ticket), int(timeout_ms))
        if rc != -5:
            self._keep.pop(ticket, None)
        return rc

    def cancel(self, ticket: int) -> int:
        return lib().vi_server_cancel(self.h, int(ticket))

    def stats(self) -> dict:
        s = Stats_t()
        _check(lib().vi_server_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats_t._fields_}

    def reset_stats(self):
        _check(lib().vi_server_reset_stats(self.h))

    def close(self):
        if self.h:
            lib().vi_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
