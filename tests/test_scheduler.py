"""The serving scheduler on the CPU, with a recording executor (no GPU, no images).

Covers admission by pool footprint, LRU eviction of unpinned stacks, stack
reuse while the light is unchanged, continuous batching of tiles from several
frames into one launch, the launch tile budget, in-flight limits, cancellation,
failure isolation and the latency statistics; plus a multi-threaded stress
run of the same code under ThreadSanitizer and AddressSanitizer.
"""
import ctypes as C
import os
import subprocess
import time

import pytest

from paper_2008_06134_amd import vi

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "sched_harness.cpp"), os.path.join(ROOT, "paper_2008_06134_amd", "csrc", "vi_sched.cpp")]
BUILD = os.path.join(ROOT, "_build")

PENDING, ADMITTED, DONE = 0, 1, 2


def _compile(out, extra):
    os.makedirs(BUILD, exist_ok=True)
    if os.path.exists(out) and all(os.path.getmtime(out) > os.path.getmtime(s) for s in SRC):
        return out
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-pthread", "-I", os.path.join(ROOT, "include"),
                           *extra, *SRC, "-o", out])
    return out


@pytest.fixture(scope="module")
def H():
    so = _compile(os.path.join(BUILD, "sched_harness.so"), ["-fPIC", "-shared"])
    L = C.CDLL(so)
    L.h_new.restype = C.c_void_p
    L.h_new.argtypes = [C.c_size_t, C.c_int, C.c_int, C.c_int]
    L.h_register.argtypes = [C.c_void_p]
    L.h_submit.restype = C.c_longlong
    L.h_submit.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                           C.c_int, C.c_longlong, C.c_int, C.c_int]
    for f in ("h_poll", "h_wait", "h_cancel"):
        getattr(L, f).argtypes = [C.c_void_p, C.c_longlong] + ([C.c_int] if f == "h_wait" else [])
    L.h_stats.argtypes = [C.c_void_p, C.POINTER(vi.Stats_t)]
    L.h_finish.argtypes = [C.c_void_p, C.c_int]
    L.h_fail_builds_of.argtypes = [C.c_void_p, C.c_int]
    L.h_log.argtypes = [C.c_void_p, C.c_char_p, C.c_int]
    L.h_free.argtypes = [C.c_void_p]
    return L


class Sched:
    def __init__(self, L, pool=1 << 30, inflight=16, tiles=8192, manual=False, vols=4):
        self.L = L
        self.h = L.h_new(pool, inflight, tiles, int(manual))
        for _ in range(vols):
            L.h_register(self.h)

    def submit(self, vol, light=(0, 0, 1), n=8, res=16, w=32, h=32, tag=1, mode=2, dtype=vi.VI_F32):
        return self.L.h_submit(self.h, vol, *light, n, res, w, h, tag, mode, dtype)

    def poll(self, t):
        return self.L.h_poll(self.h, t)

    def wait(self, t, ms=2000):
        return self.L.h_wait(self.h, t, ms)

    def until(self, pred, timeout=3.0):
        t0 = time.time()
        while time.time() - t0 < timeout:
            if pred():
                return True
            time.sleep(0.002)
        return False

    def log(self):
        n = self.L.h_log(self.h, None, 0)
        buf = C.create_string_buffer(n + 1)
        self.L.h_log(self.h, buf, n + 1)
        return buf.value.decode().splitlines()

    def stats(self):
        s = vi.Stats_t()
        self.L.h_stats(self.h, C.byref(s))
        return s

    def close(self):
        self.L.h_free(self.h)


def test_frames_complete_and_stacks_are_reused(H):
    s = Sched(H)
    a = s.submit(0, tag=11)
    b = s.submit(0, tag=12)                      # same volume, light, n, res: reuse
    c = s.submit(0, light=(1, 0, 0), tag=13)     # light changed: rebuild
    d = s.submit(1, tag=14)                      # other volume
    for t in (a, b, c, d):
        assert s.wait(t) == 0 and s.poll(t) == DONE
    st = s.stats()
    assert st.completed == 4 and st.stack_builds == 3 and st.stack_hits == 1
    builds = [l for l in s.log() if l.startswith("B")]
    assert [int(l.split()[1]) for l in builds] == [0, 0, 1]
    assert st.p50_ms > 0 and st.p99_ms >= st.p50_ms and st.max_ms >= st.p99_ms
    s.close()


def test_continuous_batching_mixes_frames_in_one_launch(H):
    s = Sched(H, manual=True, tiles=10)
    a = s.submit(0, w=48, h=48, tag=21)          # 9 tiles
    assert s.until(lambda: any(l.startswith("L") for l in s.log()))
    b = s.submit(1, w=32, h=32, tag=22)          # 4 tiles, arrives while a is on the "GPU"
    assert s.until(lambda: sum(l.startswith("L") for l in s.log()) >= 2)
    launches = [l for l in s.log() if l.startswith("L")]
    assert launches[0] == "L 21 | 9"             # all of a fits one launch
    assert launches[1] == "L 22 | 4"             # b starts at once, a second launch in flight
    assert s.poll(a) == ADMITTED and s.poll(b) == ADMITTED
    H.h_finish(s.h, 2)
    assert s.wait(a) == 0 and s.wait(b) == 0
    s.close()
    # a request admitted while others still have tiles left shares their launch
    s = Sched(H, manual=True, tiles=6)
    a = s.submit(0, w=64, h=64, tag=31)          # 16 tiles -> 6 + 6 + 4
    assert s.until(lambda: sum(l.startswith("L") for l in s.log()) >= 2)   # two launches in flight
    b = s.submit(1, w=32, h=32, tag=32)
    H.h_finish(s.h, 1)
    assert s.until(lambda: sum(l.startswith("L") for l in s.log()) >= 3)
    launches = [l for l in s.log() if l.startswith("L")]
    assert launches[:3] == ["L 31 | 6", "L 31 | 6", "L 31 32 | 4 2"]
    H.h_finish(s.h, 10)
    assert s.wait(a) == 0 and s.wait(b) == 0
    s.close()


def test_frame_completes_only_after_its_last_tile(H):
    s = Sched(H, manual=True, tiles=5)
    a = s.submit(0, w=64, h=64, tag=41)          # 16 tiles: 5 5 5 1
    assert s.until(lambda: sum(l.startswith("L") for l in s.log()) >= 2)
    for _ in range(3):
        H.h_finish(s.h, 1)
        time.sleep(0.02)
        assert s.poll(a) == ADMITTED
    H.h_finish(s.h, 1)
    assert s.wait(a) == 0
    assert [l for l in s.log() if l.startswith("L")] == ["L 41 | 5"] * 3 + ["L 41 | 1"]
    s.close()


def test_admission_by_pool_footprint_and_lru_eviction(H):
    one = 8 * 16 * 16 * 4                        # bytes of one stack (n=8, res=16, f32)
    s = Sched(H, pool=one + 256, manual=True)
    a = s.submit(0, tag=51)
    assert s.until(lambda: s.poll(a) == ADMITTED)
    b = s.submit(1, tag=52)                      # its stack does not fit while a's is pinned
    time.sleep(0.05)
    assert s.poll(b) == PENDING
    H.h_finish(s.h, 1)                           # a completes -> its stack unpinned -> evicted for b
    assert s.wait(a) == 0
    assert s.until(lambda: s.poll(b) == ADMITTED)
    log = s.log()
    assert log.index("E 0") < max(i for i, l in enumerate(log) if l.startswith("B 1"))
    H.h_finish(s.h, 1)
    assert s.wait(b) == 0
    st = s.stats()
    assert st.evictions == 1 and st.pool_peak <= st.pool_bytes
    # a stack larger than the whole pool is refused at submit
    assert s.submit(0, n=64, res=64) == -3
    assert s.stats().rejected == 1
    s.close()


def test_inflight_limit_and_cancel(H):
    s = Sched(H, inflight=2, manual=True)
    t = [s.submit(i % 4, tag=60 + i) for i in range(4)]
    assert s.until(lambda: s.poll(t[0]) == ADMITTED and s.poll(t[1]) == ADMITTED)
    time.sleep(0.03)
    assert s.poll(t[2]) == PENDING and s.poll(t[3]) == PENDING
    assert H.h_cancel(s.h, t[3]) == 0 and s.poll(t[3]) == -6
    assert H.h_cancel(s.h, t[0]) == -5           # already admitted
    H.h_finish(s.h, 100)
    for x in t[:3]:
        assert s.wait(x) == 0
    assert s.wait(t[3]) == -6
    st = s.stats()
    assert st.completed == 3 and st.cancelled == 1
    s.close()


def test_invalid_requests_and_failed_builds_do_not_stop_the_server(H):
    s = Sched(H)
    assert s.submit(0, mode=7) == -1             # rejected by validation
    assert s.submit(9) == -1                     # unknown volume
    H.h_fail_builds_of(s.h, 2)
    bad = s.submit(2, tag=71)
    good = s.submit(1, tag=72)
    assert s.wait(bad) == -4 and s.poll(bad) == -4
    assert s.wait(good) == 0
    s.close()


def test_stack_dtype_classes_never_share_a_launch(H):
    s = Sched(H, manual=True, tiles=100)
    a = s.submit(0, tag=81, dtype=vi.VI_F32)
    b = s.submit(1, tag=82, dtype=vi.VI_BF16)
    assert s.until(lambda: sum(l.startswith("L") for l in s.log()) >= 2)
    assert [l for l in s.log() if l.startswith("L")] == ["L 81 | 4", "L 82 | 4"]
    H.h_finish(s.h, 10)
    assert s.wait(a) == 0 and s.wait(b) == 0
    s.close()


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_scheduler_stress_under_sanitizers(san):
    exe = _compile(os.path.join(BUILD, f"sched_stress_{san.split(',')[0]}"),
                   [f"-fsanitize={san}", "-fno-omit-frame-pointer", "-DVI_SCHED_STRESS"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ThreadSanitizer" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert "completed" in r.stdout
