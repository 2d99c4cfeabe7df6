"""Seeded synthetic workloads: volumes, transfer-function tables, lights and cameras.

This module only *generates inputs*.  It holds none of the method's
arithmetic (no sampling, opacity, attenuation or compositing) and imports
neither the HIP binding nor the oracle, so both sides can consume the same
arrays.

The paper measures on CT scans (Engine and Foot, 256^3) that are not
available here; these phantoms stand in for them with the same shapes, value
ranges and structure: a soft-tissue body, a thin dense shell, an interior,
dense inserts and, at the large sizes, thin vessel-like tubes.  Every
generator is ``numpy.random.default_rng(seed)``-driven and C-ordered
``raw[z][y][x]``, and keeps a margin of at least two voxels that the
transfer functions map to zero opacity next to every cube face.

Named configurations (edge N, slab count n, slice resolution res, image):

=========  =====================  =====  ======  ==============  =========
name       volume                 n      res     image           mode
=========  =====================  =====  ======  ==============  =========
small      64^3 u8 noisy sphere   32     64      256^2 ortho     shell
medium     256^3 u16 CT phantom   256    512     1024^2 persp    cone 5x5
large      512^3 u16 + vessels    512    1024    1920x1080       shell,cone
precision  1024^3 u16 -> f16      512    1024    1920x1080       shell,cone
=========  =====================  =====  ======  ==============  =========
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# transfer-function tables (256 entries, RGBA, non-premultiplied, alpha per voxel)
# --------------------------------------------------------------------------


def tf_ramp(K: int = 256) -> np.ndarray:
    """Entry i: (i/(K-1), 1 - i/(K-1), 0.5, i/(K-1)); channels differ so swizzles show."""
    t = np.arange(K, dtype=np.float64) / (K - 1)
    return np.stack([t, 1.0 - t, np.full_like(t, 0.5), t], axis=1)


# control points of the CT table: value -> (r, g, b, a)
_CT_POINTS = [
    (0.00, (0.0, 0.0, 0.0, 0.0)),
    (0.20, (0.8, 0.5, 0.4, 0.0)),
    (0.25, (0.8, 0.5, 0.4, 0.02)),
    (0.35, (0.9, 0.6, 0.5, 0.05)),
    (0.60, (1.0, 0.9, 0.8, 0.30)),
    (0.75, (1.0, 1.0, 1.0, 0.90)),
    (1.00, (1.0, 1.0, 1.0, 1.00)),
]


def tf_ct(K: int = 256) -> np.ndarray:
    """Piecewise-linear CT table sampled at value i/(K-1); alpha 0 below 0.20."""
    xs = np.array([p for p, _ in _CT_POINTS])
    ys = np.array([c for _, c in _CT_POINTS])
    v = np.arange(K, dtype=np.float64) / (K - 1)
    return np.stack([np.interp(v, xs, ys[:, c]) for c in range(4)], axis=1)


# --------------------------------------------------------------------------
# volumes
# --------------------------------------------------------------------------


def _centres(N: int) -> np.ndarray:
    return (np.arange(N, dtype=np.float32) + 0.5)


def sphere_u8(N: int = 64, radius: float = 24.0, density: int = 200, noise: int = 20, seed: int = 1) -> np.ndarray:
    """A sphere of the given radius (voxels) about the centre: density + U{-noise..noise}
    inside, 0 outside (noise on the sphere only)."""
    rng = np.random.default_rng(seed)
    c = _centres(N) - N / 2.0
    r2 = c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2
    inside = r2 <= radius * radius
    vals = density + rng.integers(-noise, noise + 1, size=(N, N, N))
    return np.where(inside, vals, 0).astype(np.uint8)


def constant_cube(N: int, value, dtype=np.uint8, margin: int = 0) -> np.ndarray:
    vol = np.zeros((N, N, N), dtype=dtype)
    vol[margin:N - margin, margin:N - margin, margin:N - margin] = value
    return vol


@dataclass
class _Ellipsoid:
    centre: np.ndarray   # normalised [0,1]^3 coordinates (x, y, z)
    axes: np.ndarray     # semi-axes, normalised
    value: float


def _phantom_ellipsoids(rng: np.random.Generator) -> list:
    """Body, shell (outer/inner surfaces), interior and three inserts."""
    c = 0.5 + rng.uniform(-0.01, 0.01, 3)
    body = np.array([0.40, 0.34, 0.42]) * rng.uniform(0.97, 1.03, 3)
    shell_out = body * 0.86
    ells = [_Ellipsoid(c, body, 1000.0 + rng.uniform(-30, 30)),
            _Ellipsoid(c, shell_out, 3000.0 + rng.uniform(-100, 100))]
    ells.append(_Ellipsoid(c, None, 1100.0 + rng.uniform(-30, 30)))  # interior: axes set per N (shell thickness)
    for _ in range(3):
        off = rng.uniform(-0.5, 0.5, 3) * shell_out * 0.8
        ax = rng.uniform(0.04, 0.10, 3)
        ells.append(_Ellipsoid(c + off, ax, rng.uniform(1500.0, 4000.0)))
    return ells


def _ellipsoid_cover(z: np.ndarray, y: np.ndarray, x: np.ndarray, N: int, e: _Ellipsoid):
    """Soft indicator (about one voxel of partial-volume blur) of an ellipsoid on a
    z-chunk; returns (cover, (y-slice, x-slice)) restricted to the ellipsoid's box."""
    pad = 2.0 / N
    ys = slice(int(max(0, np.floor((e.centre[1] - e.axes[1] - pad) * N))),
               int(min(N, np.ceil((e.centre[1] + e.axes[1] + pad) * N))))
    xs = slice(int(max(0, np.floor((e.centre[0] - e.axes[0] - pad) * N))),
               int(min(N, np.ceil((e.centre[0] + e.axes[0] + pad) * N))))
    qz = ((z - e.centre[2]) / e.axes[2]) ** 2
    qy = ((y[ys] - e.centre[1]) / e.axes[1]) ** 2
    qx = ((x[xs] - e.centre[0]) / e.axes[0]) ** 2
    q = np.sqrt(qz[:, None, None] + qy[None, :, None] + qx[None, None, :])
    # approximate signed distance to the surface in voxels
    dist_vox = (q - 1.0) * float(e.axes.min()) * N
    return np.clip(0.5 - dist_vox, 0.0, 1.0).astype(np.float32), (ys, xs)


def _value_noise_axis_weights(N: int, spacing: float, G: int) -> np.ndarray:
    x = _centres(N) / spacing
    cell = np.floor(x).astype(np.int64)
    t = x - cell
    s = t * t * (3.0 - 2.0 * t)  # smoothstep
    W = np.zeros((N, G), dtype=np.float32)
    W[np.arange(N), cell] = 1.0 - s
    W[np.arange(N), cell + 1] = s
    return W


class ValueNoise:
    """3-octave value noise in [0,1] on an N^3 voxel grid: uniform lattice values
    (lattice spacing halves per octave, amplitude halves), smoothstep-interpolated.
    The (y, x) contractions are done once; ``chunk(z0, z1)`` finishes slices."""

    def __init__(self, N: int, rng: np.random.Generator, spacing: float = 32.0, octaves: int = 3):
        self.N = N
        self.parts = []
        amp_sum = 0.0
        for o in range(octaves):
            sp = spacing / 2 ** o
            G = int(math.ceil(N / sp)) + 2
            lat = rng.random((G, G, G), dtype=np.float32)      # lattice index order (z, y, x)
            W = _value_noise_axis_weights(N, sp, G)
            t = np.tensordot(lat, W, axes=([2], [1]))          # (a, b, x)
            t = np.tensordot(t, W, axes=([1], [1]))            # (a, x, y)
            amp = 0.5 ** o
            self.parts.append((amp, W, np.ascontiguousarray(np.transpose(t, (0, 2, 1)))))  # (a, y, x)
            amp_sum += amp
        self.amp_sum = amp_sum

    def chunk(self, z0: int, z1: int) -> np.ndarray:
        out = np.zeros((z1 - z0, self.N, self.N), dtype=np.float32)
        for amp, W, t in self.parts:
            out += amp * np.tensordot(W[z0:z1], t, axes=([1], [0]))
        return out / self.amp_sum


def ct_phantom_u16(N: int, seed: int, vessels: bool = False, noise_sigma: float = 30.0,
                   chunk: int = 64) -> np.ndarray:
    """Nested-ellipsoid CT phantom with 12-bit values (0..4095) plus N(0, sigma^2) noise.

    Body ~1000, a dense shell ~3000 about 6 voxels thick at N=256 (scaled with N),
    interior ~1100, three inserts 1500-4000.  With ``vessels``: tubes where two
    thin iso-bands of independent value noise intersect (value 3500), inside the
    body only."""
    rng = np.random.default_rng(seed)
    ells = _phantom_ellipsoids(rng)
    thick = 6.0 / 256.0  # shell thickness, normalised
    ells[2].axes = ells[1].axes - thick
    if vessels:
        noise1 = ValueNoise(N, rng)
        noise2 = ValueNoise(N, rng)
    noise_rng = np.random.default_rng(seed + 1000)
    out = np.empty((N, N, N), dtype=np.uint16)
    y = _centres(N) / N
    x = _centres(N) / N
    for z0 in range(0, N, chunk):
        z1 = min(N, z0 + chunk)
        z = _centres(N)[z0:z1] / N
        val = np.zeros((z1 - z0, N, N), dtype=np.float32)
        body = np.zeros_like(val)
        cov, (ys, xs) = _ellipsoid_cover(z, y, x, N, ells[0])
        body[:, ys, xs] = cov
        val += body * ells[0].value
        for e in ells[1:]:
            cov, (ys, xs) = _ellipsoid_cover(z, y, x, N, e)
            sub = val[:, ys, xs]
            val[:, ys, xs] = sub * (1.0 - cov) + cov * e.value
        if vessels:
            n1 = noise1.chunk(z0, z1)
            n2 = noise2.chunk(z0, z1)
            w, edge = 0.035, 0.015
            m = np.clip((w - np.abs(n1 - 0.5)) / edge, 0.0, 1.0) * np.clip((w - np.abs(n2 - 0.5)) / edge, 0.0, 1.0)
            m *= body  # vessels only inside the body
            val = val * (1.0 - m) + m * 3500.0
        val += noise_rng.normal(0.0, noise_sigma, size=val.shape).astype(np.float32)
        out[z0:z1] = np.clip(np.rint(val), 0, 4095).astype(np.uint16)
    return out


def to_f16_normalised(raw_u16: np.ndarray, chunk: int = 64) -> np.ndarray:
    """FP16 storage of raw/4095, rounded to nearest even by NumPy's float16 cast."""
    out = np.empty(raw_u16.shape, dtype=np.float16)
    for z0 in range(0, raw_u16.shape[0], chunk):
        out[z0:z0 + chunk] = (raw_u16[z0:z0 + chunk].astype(np.float64) / 4095.0).astype(np.float16)
    return out


# --------------------------------------------------------------------------
# cameras and lights
# --------------------------------------------------------------------------


def camera_ortho_front(W: int, H: int, half_h: float = 0.75) -> dict:
    """Orthographic view along +y, up +z, centred on the cube."""
    return {"kind": "ortho", "eye": [0.5, -1.0, 0.5], "target": [0.5, 0.5, 0.5], "up": [0.0, 0.0, 1.0],
            "fovy_deg": 0.0, "ortho_half_h": half_h, "width": W, "height": H}


def camera_orbit(W: int, H: int, azimuth: float, elevation: float, distance: float = 2.0,
                 fovy_deg: float = 40.0) -> dict:
    """Pinhole camera on a sphere about the cube centre, looking at it, up +z."""
    ce, se = math.cos(elevation), math.sin(elevation)
    eye = [0.5 + distance * ce * math.cos(azimuth), 0.5 + distance * ce * math.sin(azimuth), 0.5 + distance * se]
    return {"kind": "persp", "eye": eye, "target": [0.5, 0.5, 0.5], "up": [0.0, 0.0, 1.0],
            "fovy_deg": fovy_deg, "ortho_half_h": 0.0, "width": W, "height": H}


def light_from_angles(azimuth: float, elevation: float) -> list:
    """Propagation direction of a light placed at (azimuth, elevation) as seen
    from the cube centre (the light shines toward the centre)."""
    ce, se = math.cos(elevation), math.sin(elevation)
    return [-ce * math.cos(azimuth), -ce * math.sin(azimuth), -se]


DIAGONAL_LIGHT = [1.0 / math.sqrt(3.0), 1.0 / math.sqrt(3.0), -1.0 / math.sqrt(3.0)]


def orbit_lights(count: int = 16, seed: int = 3):
    """Seeded light orbit: azimuth 2 pi i / count + U(-0.1, 0.1), elevation
    35 deg + U(-5, 5) deg, shining downward.  Returns (light, azimuth) pairs."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        az = 2.0 * math.pi * i / count + rng.uniform(-0.1, 0.1)
        el = math.radians(35.0 + rng.uniform(-5.0, 5.0))
        out.append((light_from_angles(az, el), az))
    return out


# --------------------------------------------------------------------------
# named configurations
# --------------------------------------------------------------------------


@dataclass
class Workload:
    name: str
    N: int
    n_slices: int
    res: int
    step_vox: float
    modes: list
    opts: dict = field(default_factory=dict)
    seed: int = 0

    def volume(self) -> np.ndarray:
        if self.name == "small":
            return sphere_u8(self.N, seed=self.seed)
        return ct_phantom_u16(self.N, self.seed, vessels=self.name in ("large", "precision"))

    def tf(self) -> np.ndarray:
        return tf_ramp() if self.name == "small" else tf_ct()

    def lights(self):
        if self.name in ("large", "precision"):
            return [l for l, _ in orbit_lights(16, self.seed)]
        return [DIAGONAL_LIGHT]

    def camera(self, light_index: int = 0, W: int | None = None, H: int | None = None) -> dict:
        if self.name == "small":
            return camera_ortho_front(W or 256, H or 256)
        if self.name == "medium":
            return camera_orbit(W or 1024, H or 1024, 1.0, math.radians(20.0))
        _, az = orbit_lights(16, self.seed)[light_index]
        return camera_orbit(W or 1920, H or 1080, az + math.pi / 3.0, math.radians(20.0))


WORKLOADS = {
    "small": Workload("small", 64, 32, 64, 0.5, ["shell"], seed=1),
    "medium": Workload("medium", 256, 256, 512, 0.5, ["cone"], {"cone_grid": 5}, seed=2),
    "large": Workload("large", 512, 512, 1024, 0.5, ["shell", "cone"], seed=3),
    "precision": Workload("precision", 1024, 512, 1024, 0.5, ["shell", "cone"], seed=4),
}


# --------------------------------------------------------------------------
# serving workload: a Poisson stream over many resident volumes
# --------------------------------------------------------------------------

SERVING_IMAGE_SIZES = [(512, 512), (1024, 768), (1280, 720), (1024, 1024), (1920, 1080)]


def serving_volume_sizes(count: int = 64, seed: int = 5, sizes=(128, 192, 256, 320, 384, 448, 512)) -> list:
    rng = np.random.default_rng(seed)
    return [int(s) for s in rng.choice(sizes, size=count)]


def serving_volume(N: int, index: int, seed: int = 5, vessels: bool = True) -> np.ndarray:
    """Volume `index` of the serving set: the CT phantom generator with its own seed."""
    return ct_phantom_u16(N, seed=seed * 1000 + index, vessels=vessels)


def serving_requests(count: int, vol_sizes: list, rate_hz: float, seed: int = 5,
                     image_sizes=SERVING_IMAGE_SIZES) -> list:
    """`count` requests with exponential inter-arrival times of mean 1/rate_hz.

    Each request picks a volume uniformly; every volume keeps a session whose
    camera orbits 2 degrees per frame and whose light moves to a new seeded
    direction every U{1..10} of its frames; image size uniform over
    `image_sizes`; shell / cone 50/50.  Slab count n = N, slice resolution
    min(2N, 1024)."""
    rng = np.random.default_rng(seed)
    nv = len(vol_sizes)
    sess = [{"frame": 0, "az": float(rng.uniform(0, 2 * math.pi)), "left": int(rng.integers(1, 11)),
             "light": light_from_angles(float(rng.uniform(0, 2 * math.pi)), math.radians(35 + rng.uniform(-5, 5)))}
            for _ in range(nv)]
    t = 0.0
    out = []
    for _ in range(count):
        t += float(rng.exponential(1.0 / rate_hz))
        v = int(rng.integers(nv))
        s = sess[v]
        if s["left"] == 0:
            s["light"] = light_from_angles(float(rng.uniform(0, 2 * math.pi)), math.radians(35 + rng.uniform(-5, 5)))
            s["left"] = int(rng.integers(1, 11))
        s["left"] -= 1
        W_, H_ = image_sizes[int(rng.integers(len(image_sizes)))]
        cam = camera_orbit(W_, H_, s["az"] + math.radians(2.0) * s["frame"], math.radians(20.0))
        s["frame"] += 1
        N = vol_sizes[v]
        out.append({"arrival": t, "vol": v, "light": list(s["light"]), "n": N, "res": min(2 * N, 1024),
                    "cam": cam, "mode": "shell" if rng.random() < 0.5 else "cone"})
    return out
