"""FP64 CPU oracle -- Python wrapper (ctypes) over ``vi_oracle.c``.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It builds and loads
``libvi_oracle.so`` from the C source beside it and shares nothing with the
HIP library: inputs are plain NumPy arrays and dicts produced by the seeded
workload generators.

What the oracle computes (paper sections in brackets):
  * ``light_frame``      -- Eq. 8 min/max distances, slab thickness, light basis
  * ``Stack``            -- Alg. 1 attenuation stack, layer k = transmittance
                            after slab k; ``lookup`` is Eq. 9 index + Eq. 10 UV
  * ``render``           -- single-pass ray casting, Eq. 3 compositing with the
                            Eq. 7 coefficient (direct shadow, shell, cone), or
                            the local Phong model of the comparison in section 4
                            (``gradient``, ``phong``)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vi_oracle.c")
_LIB = os.path.join(_HERE, "libvi_oracle.so")

MODES = {"none": 0, "shadow": 1, "shell": 2, "cone": 3, "phong": 4}
_PHONG_KEYS = ("phong_ka", "phong_kd", "phong_ks", "phong_shininess", "grad_eps")
DTYPES = {np.dtype(np.uint8): 0, np.dtype(np.uint16): 1, np.dtype(np.float16): 2, np.dtype(np.float32): 3}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Volume(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int), ("N", C.c_int), ("scale", C.c_double)]


class _TF(C.Structure):
    _fields_ = [("rgba", C.POINTER(C.c_double)), ("K", C.c_int)]


class _Frame(C.Structure):
    _fields_ = [("L", C.c_double * 3), ("U", C.c_double * 3), ("V", C.c_double * 3), ("c", C.c_double * 3),
                ("dmin", C.c_double), ("dmax", C.c_double), ("ds", C.c_double), ("R", C.c_double),
                ("n", C.c_int), ("res", C.c_int), ("darken", C.c_double), ("positional", C.c_int),
                ("P", C.c_double * 3)]


class _Camera(C.Structure):
    _fields_ = [("kind", C.c_int), ("eye", C.c_double * 3), ("target", C.c_double * 3), ("up", C.c_double * 3),
                ("fovy_deg", C.c_double), ("ortho_half_h", C.c_double), ("width", C.c_int), ("height", C.c_int)]


class _Opts(C.Structure):
    _fields_ = [("ambient", C.c_double), ("light_rgb", C.c_double * 3), ("bg", C.c_double * 4),
                ("term_eps", C.c_double), ("shell_count", C.c_int), ("shell_w", C.c_double * 8),
                ("shell_h_vox", C.c_double),
                ("cone_rings", C.c_int), ("cone_angles", C.c_int), ("cone_grid", C.c_int), ("cone_tan", C.c_double),
                ("phong_ka", C.c_double), ("phong_kd", C.c_double), ("phong_ks", C.c_double),
                ("phong_shininess", C.c_double), ("grad_eps", C.c_double),
                ("nearest_layer", C.c_int), ("nearest_shift", C.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = C.CDLL(_LIB)
        P = C.POINTER
        lib.vio_default_opts.argtypes = [P(_Opts)]
        lib.vio_threads.restype = C.c_int
        lib.vio_light_frame.argtypes = [P(C.c_double), C.c_int, C.c_int, P(_Frame)]
        lib.vio_light_frame_point.argtypes = [P(C.c_double), C.c_int, C.c_int, P(_Frame)]
        lib.vio_volume_sample.argtypes = [P(_Volume), P(C.c_double)]
        lib.vio_volume_sample.restype = C.c_double
        lib.vio_tf_lookup.argtypes = [P(_TF), C.c_double, P(C.c_double)]
        lib.vio_segment_alpha.argtypes = [C.c_double, C.c_double, C.c_double]
        lib.vio_segment_alpha.restype = C.c_double
        lib.vio_stack_create.argtypes = [P(_Volume), P(_TF), P(_Frame)]
        lib.vio_stack_create.restype = C.c_void_p
        lib.vio_stack_destroy.argtypes = [C.c_void_p]
        lib.vio_stack_fill.argtypes = [C.c_void_p, C.c_int]
        lib.vio_stack_export.argtypes = [C.c_void_p, P(C.c_double), C.c_int]
        lib.vio_stack_column.argtypes = [C.c_void_p, C.c_int, C.c_int]
        lib.vio_stack_column.restype = P(C.c_double)
        lib.vio_stack_lookup.argtypes = [C.c_void_p, P(C.c_double)]
        lib.vio_stack_lookup.restype = C.c_double
        lib.vio_stack_lookup_layer.argtypes = [C.c_void_p, P(C.c_double), C.c_int, C.c_double]
        lib.vio_stack_lookup_layer.restype = C.c_double
        lib.vio_stack_columns_built.argtypes = [C.c_void_p]
        lib.vio_stack_columns_built.restype = C.c_int64
        lib.vio_camera_ray.argtypes = [P(_Camera), C.c_int, C.c_int, P(C.c_double), P(C.c_double)]
        lib.vio_cube_hit.argtypes = [P(C.c_double), P(C.c_double), P(C.c_double), P(C.c_double)]
        lib.vio_coefficient.argtypes = [C.c_void_p, C.c_int, P(_Opts), C.c_int, P(C.c_double), P(C.c_double)]
        lib.vio_coefficient.restype = C.c_double
        lib.vio_cone_taps.argtypes = [C.c_void_p, P(_Opts), P(C.c_double), P(C.c_double), P(C.c_double)]
        lib.vio_cone_taps.restype = C.c_int
        lib.vio_gradient.argtypes = [P(_Volume), P(C.c_double), P(C.c_double)]
        lib.vio_phong.argtypes = [P(_Volume), P(_Opts), P(C.c_double), P(C.c_double), P(C.c_double),
                                  P(C.c_double), P(C.c_double)]
        lib.vio_render.argtypes = [P(_Volume), P(_TF), C.c_void_p, P(_Camera), C.c_int, C.c_double, P(_Opts),
                                   P(C.c_int64), C.c_int64, P(C.c_double), P(C.c_double), P(C.c_int64),
                                   P(C.c_int64), C.c_int]
        lib.vio_render.restype = C.c_int
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _vec(x):
    return (C.c_double * 3)(*[float(t) for t in x])


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().vio_threads())


def default_opts() -> dict:
    o = _Opts()
    _load().vio_default_opts(C.byref(o))
    return {"ambient": o.ambient, "light_rgb": list(o.light_rgb), "bg": list(o.bg), "term_eps": o.term_eps,
            "shell_count": o.shell_count, "shell_w": list(o.shell_w), "shell_h_vox": o.shell_h_vox,
            "cone_rings": o.cone_rings,
            "cone_angles": o.cone_angles, "cone_grid": o.cone_grid, "cone_tan": o.cone_tan,
            "nearest_layer": o.nearest_layer, "nearest_shift": o.nearest_shift,
            **{k: getattr(o, k) for k in _PHONG_KEYS}}


def _opts(opts: dict | None) -> _Opts:
    d = default_opts()
    if opts:
        d.update(opts)
    o = _Opts()
    o.ambient = d["ambient"]
    o.light_rgb = (C.c_double * 3)(*d["light_rgb"])
    o.bg = (C.c_double * 4)(*d["bg"])
    o.term_eps = d["term_eps"]
    o.shell_count = int(d["shell_count"])
    w = list(d["shell_w"]) + [0.0] * 8
    o.shell_w = (C.c_double * 8)(*[float(x) for x in w[:8]])
    o.shell_h_vox = d["shell_h_vox"]
    for k in _PHONG_KEYS:
        setattr(o, k, float(d[k]))
    o.cone_rings = int(d["cone_rings"])
    o.cone_angles = int(d["cone_angles"])
    o.cone_grid = int(d["cone_grid"])
    o.cone_tan = d["cone_tan"]
    o.nearest_layer = int(d["nearest_layer"])
    o.nearest_shift = float(d["nearest_shift"])
    return o


class Volume:
    """A cubic volume raw[z][y][x] with its normalisation scale."""

    def __init__(self, raw: np.ndarray, scale: float | None = None):
        raw = np.ascontiguousarray(raw)
        assert raw.ndim == 3 and raw.shape[0] == raw.shape[1] == raw.shape[2], "cubic volumes only"
        if raw.dtype not in DTYPES:
            raise TypeError(f"unsupported volume dtype {raw.dtype}")
        if scale is None:
            scale = {np.dtype(np.uint8): 1.0 / 255.0, np.dtype(np.uint16): 1.0 / 4095.0}.get(raw.dtype, 1.0)
        self.raw = raw
        self.N = raw.shape[0]
        self.scale = float(scale)
        self._s = _Volume(raw.ctypes.data, DTYPES[raw.dtype], self.N, self.scale)


class TF:
    def __init__(self, rgba: np.ndarray):
        self.rgba = np.ascontiguousarray(rgba, dtype=np.float64)
        assert self.rgba.ndim == 2 and self.rgba.shape[1] == 4 and self.rgba.shape[0] >= 2
        self._s = _TF(_dptr(self.rgba), self.rgba.shape[0])


def light_frame(l, n: int, res: int, position=None) -> dict:
    """Light frame of a directional light `l` (propagation direction), or of a
    point light at `position` (then `l` is ignored)."""
    f = _Frame()
    if position is None:
        rc = _load().vio_light_frame((C.c_double * 3)(*[float(t) for t in l]), n, res, C.byref(f))
    else:
        rc = _load().vio_light_frame_point((C.c_double * 3)(*[float(t) for t in position]), n, res, C.byref(f))
    if rc != 0:
        raise ValueError("invalid light frame arguments")
    return {"L": np.array(f.L), "U": np.array(f.U), "V": np.array(f.V), "c": np.array(f.c), "dmin": f.dmin,
            "dmax": f.dmax, "ds": f.ds, "R": f.R, "n": f.n, "res": f.res, "positional": f.positional,
            "P": np.array(f.P), "_s": f}


def volume_sample(vol: Volume, p) -> float:
    return _load().vio_volume_sample(C.byref(vol._s), _vec(p))


def gradient(vol: Volume, p) -> np.ndarray:
    """Central differences of the reconstructed field at p, value per voxel (R29)."""
    g = (C.c_double * 3)()
    _load().vio_gradient(C.byref(vol._s), _vec(p), g)
    return np.array(g)


def phong(vol: Volume, L, p, d, opts: dict | None = None):
    """Local Phong terms (sd, ss) at p for ray direction d, light propagation direction L."""
    sd, ss = C.c_double(), C.c_double()
    _load().vio_phong(C.byref(vol._s), C.byref(_opts(opts)), _vec(L), _vec(p), _vec(d), C.byref(sd), C.byref(ss))
    return sd.value, ss.value


def tf_lookup(tf: TF, v: float) -> np.ndarray:
    out = (C.c_double * 4)()
    _load().vio_tf_lookup(C.byref(tf._s), float(v), out)
    return np.array(out)


def segment_alpha(a: float, length: float, dref: float) -> float:
    return _load().vio_segment_alpha(float(a), float(length), float(dref))


class Stack:
    """Attenuation stack S[k][j][i] (Alg. 1), columns built on first use."""

    def __init__(self, vol: Volume, tf: TF, light, n: int, res: int, darken: float = 0.0, position=None):
        self.vol, self.tf = vol, tf  # keep the buffers alive
        self.frame = light_frame(light, n, res, position)
        self.frame["_s"].darken = float(darken)
        self.n, self.res = n, res
        self._p = _load().vio_stack_create(C.byref(vol._s), C.byref(tf._s), C.byref(self.frame["_s"]))
        if not self._p:
            raise MemoryError("oracle stack allocation failed")

    def __del__(self):
        if getattr(self, "_p", None):
            _load().vio_stack_destroy(self._p)
            self._p = None

    def fill(self, nthreads: int = 0):
        _load().vio_stack_fill(self._p, nthreads)

    def export(self, nthreads: int = 0) -> np.ndarray:
        out = np.empty((self.n, self.res, self.res), dtype=np.float64)
        _load().vio_stack_export(self._p, _dptr(out), nthreads)
        return out

    def column(self, i: int, j: int) -> np.ndarray:
        ptr = _load().vio_stack_column(self._p, int(i), int(j))
        return np.ctypeslib.as_array(ptr, shape=(self.n,)).copy()

    def lookup(self, p, nearest: bool = False, shift: float = 0.0) -> float:
        """Transmittance at world point p: continuous in depth, or the nearest layer."""
        if nearest:
            return _load().vio_stack_lookup_layer(self._p, _vec(p), 1, float(shift))
        return _load().vio_stack_lookup(self._p, _vec(p))

    def columns_built(self) -> int:
        return int(_load().vio_stack_columns_built(self._p))

    def coefficient(self, mode: str, p, d, opts: dict | None = None) -> float:
        o = _opts(opts)
        return _load().vio_coefficient(self._p, MODES[mode], C.byref(o), self.vol.N, _vec(p), _vec(d))

    def cone_taps(self, p, d, opts: dict | None = None) -> np.ndarray:
        """World positions of the cone's taps at sample p for view direction d."""
        o = _opts(opts)
        out = np.zeros((128, 3))
        n = _load().vio_cone_taps(self._p, C.byref(o), _vec(p), _vec(d), _dptr(out))
        return out[:n].copy()


def _camera(cam: dict) -> _Camera:
    c = _Camera()
    c.kind = 1 if cam["kind"] in ("persp", 1) else 0
    c.eye = _vec(cam["eye"])
    c.target = _vec(cam["target"])
    c.up = _vec(cam["up"])
    c.fovy_deg = float(cam.get("fovy_deg", 40.0))
    c.ortho_half_h = float(cam.get("ortho_half_h", 0.5))
    c.width = int(cam["width"])
    c.height = int(cam["height"])
    return c


def camera_ray(cam: dict, px: int, py: int):
    o = (C.c_double * 3)()
    d = (C.c_double * 3)()
    _load().vio_camera_ray(C.byref(_camera(cam)), int(px), int(py), o, d)
    return np.array(o), np.array(d)


def cube_hit(o, d):
    ti, tf = C.c_double(), C.c_double()
    hit = _load().vio_cube_hit(_vec(o), _vec(d), C.byref(ti), C.byref(tf))
    return bool(hit), ti.value, tf.value


def render(vol: Volume, tf: TF, stack: Stack | None, cam: dict, mode: str, step_vox: float,
           opts: dict | None = None, pixels: np.ndarray | None = None, want_full: bool = True,
           nthreads: int = 0):
    """Render all pixels (image H x W x 4) or the listed pixel ids (npix x 4).

    Returns (full, term, samples_term, samples_full); ``full`` is None when
    ``want_full`` is False (rays then stop at termination)."""
    W, H = int(cam["width"]), int(cam["height"])
    if pixels is None:
        npix, pix_p, shape = W * H, None, (H, W)
    else:
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        npix, pix_p, shape = pixels.size, pixels.ctypes.data_as(C.POINTER(C.c_int64)), (pixels.size,)
    full = np.zeros((npix, 4)) if want_full else None
    term = np.zeros((npix, 4))
    nt = np.zeros(npix, dtype=np.int64)
    nf = np.zeros(npix, dtype=np.int64)
    o = _opts(opts)
    rc = _load().vio_render(C.byref(vol._s), C.byref(tf._s), stack._p if stack is not None else None,
                            C.byref(_camera(cam)), MODES[mode], float(step_vox), C.byref(o), pix_p, npix,
                            _dptr(full) if want_full else None, _dptr(term),
                            nt.ctypes.data_as(C.POINTER(C.c_int64)), nf.ctypes.data_as(C.POINTER(C.c_int64)),
                            int(nthreads))
    if rc != 0:
        raise ValueError("oracle render rejected its arguments")
    rs = lambda a: a.reshape(shape + (4,))  # noqa: E731
    return (rs(full) if want_full else None), rs(term), nt.reshape(shape), nf.reshape(shape)
