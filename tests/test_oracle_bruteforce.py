"""P10: the C oracle against the independent NumPy statement on tiny inputs (CPU only)."""
import numpy as np
import pytest

import mini_oracle as M
from oracle import oracle as O
from paper_2008_06134_amd import workloads as W

CASES = [
    # N, n, res, light, dtype
    (4, 3, 5, [1, 1, -1], np.uint8),
    (6, 5, 7, [0.3, -0.9, 0.2], np.uint16),
    (8, 6, 9, [-0.5, 0.1, -0.7], np.uint8),
    (7, 4, 6, [0, 0, 1], np.float16),
]


def _case(N, dtype, seed):
    rng = np.random.default_rng(seed)
    if dtype == np.uint8:
        raw, scale = rng.integers(0, 256, (N, N, N)).astype(np.uint8), 1 / 255
    elif dtype == np.uint16:
        raw, scale = rng.integers(0, 4400, (N, N, N)).astype(np.uint16), 1 / 4095
    else:
        raw, scale = rng.uniform(0, 1, (N, N, N)).astype(np.float16), 1.0
    tab = rng.uniform(0, 1, (256, 4))
    tab[:, 3] *= 0.5
    return raw, scale, tab


@pytest.mark.parametrize("case", range(len(CASES)))
def test_p10_stack_matches_numpy(case):
    N, n, res, light, dtype = CASES[case]
    raw, scale, tab = _case(N, dtype, case)
    st = O.Stack(O.Volume(raw, scale), O.TF(tab), light, n, res)
    S = st.export()
    fr = M.frame(light, n, res)
    S2 = M.build(M.normalise(raw, scale), tab, fr)
    assert np.abs(S - S2).max() < 1e-13
    # lookups at random points inside and outside the cube
    rng = np.random.default_rng(100 + case)
    P = rng.uniform(-0.3, 1.3, (200, 3))
    a = np.array([st.lookup(p) for p in P])
    b = M.lookup(S2, fr, P)
    assert np.abs(a - b).max() < 1e-13


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("mode", ["none", "shadow", "shell", "cone", "cone5"])
@pytest.mark.parametrize("kind", ["ortho", "persp"])
def test_p10_render_matches_numpy(case, mode, kind):
    N, n, res, light, dtype = CASES[case]
    raw, scale, tab = _case(N, dtype, case)
    vol, tf = O.Volume(raw, scale), O.TF(tab)
    st = O.Stack(vol, tf, light, n, res)
    opts = O.default_opts()
    opts["bg"] = [0.05, 0.1, 0.15, 0.2]
    opts["ambient"] = 0.1
    opts["term_eps"] = 0.02          # make termination happen on tiny volumes
    m = mode
    if mode == "cone5":
        m, opts["cone_grid"] = "cone", 5
    if kind == "ortho":
        cam = W.camera_ortho_front(8, 8, half_h=0.6)
    else:
        cam = W.camera_orbit(8, 8, 0.3 + case, 0.25, distance=1.6, fovy_deg=45.0)
    full, term, nt, nf = O.render(vol, tf, st, cam, m, 0.5, opts)
    fr = M.frame(light, n, res)
    S2 = M.build(M.normalise(raw, scale), tab, fr)
    f2, t2 = M.render(raw, scale, tab, S2, fr, cam, m, 0.5, opts)
    assert np.abs(full - f2).max() < 1e-12
    assert np.abs(term - t2).max() < 1e-12
