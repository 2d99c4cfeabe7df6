// sched_harness.cpp -- CPU harness for the serving scheduler (test only).
//
// Links the scheduler core (paper_2008_06134_amd/csrc/vi_sched.cpp) with a
// recording executor that computes nothing: builds and launches are logged,
// and launches finish either at once or when the test says so.  The C entry
// points below are what tests/test_scheduler.py drives through ctypes; with
// -DVI_SCHED_STRESS the file also has a main() that hammers the scheduler
// from several threads (built with ThreadSanitizer / AddressSanitizer).
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "../paper_2008_06134_amd/csrc/vi_sched.h"

using namespace vi::sched;

namespace {

struct FakeExec : Executor {
    size_t pool;
    bool manual;
    std::mutex mu;
    std::string log;
    std::vector<int> done;  // per launch handle: 1 finished
    int finish_budget = 0;  // manual mode: launches allowed to finish
    int fail_build_vol = -1;

    FakeExec(size_t p, bool m) : pool(p), manual(m) {}
    size_t pool_bytes() const override { return pool; }
    int max_frames_per_launch() const override { return 8; }
    int validate(const vi_request& r, const VolumeRec&) override
    {
        if (r.mode < 0 || r.mode > 3 || r.camera.width < 1 || r.camera.height < 1) return VI_E_INVALID_ARG;
        return VI_OK;
    }
    size_t stack_bytes(const vi_request& r) override
    {
        return (size_t)r.n_slices * r.slice_res * r.slice_res * (r.slice_dtype == VI_BF16 ? 2 : 4);
    }
    int frame_class(const vi_request& r, const VolumeRec&) override { return r.slice_dtype; }
    int build(const vi_request& r, const VolumeRec&, StackRef* st) override
    {
        std::lock_guard<std::mutex> lk(mu);
        if (r.vol_id == fail_build_vol) return VI_E_DEVICE;
        char b[160];
        snprintf(b, sizeof b, "B %d %zu %zu\n", r.vol_id, st->offset, st->bytes);
        log += b;
        st->build_handle = 0;
        return VI_OK;
    }
    void drop_stack(StackRef* st) override
    {
        std::lock_guard<std::mutex> lk(mu);
        char b[80];
        snprintf(b, sizeof b, "E %zu\n", st->offset);
        log += b;
    }
    int launch(const std::vector<LaunchFrame>& frames, const std::vector<uint32_t>& tiles) override
    {
        std::lock_guard<std::mutex> lk(mu);
        std::string s = "L";
        for (const auto& f : frames) s += " " + std::to_string((long long)(uintptr_t)f.req->d_rgba);
        // tiles per frame, in order
        std::vector<int> cnt(frames.size(), 0);
        for (uint32_t t : tiles) cnt[t >> 22]++;
        s += " |";
        for (int c : cnt) s += " " + std::to_string(c);
        log += s + "\n";
        done.push_back(manual ? 0 : 1);
        return (int)done.size() - 1;
    }
    bool query(int h) override
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!done[h] && finish_budget > 0) {
            done[h] = 1;
            --finish_budget;
        }
        return done[h] != 0;
    }
    int wait(int h) override { return query(h) ? VI_OK : VI_E_BUSY; }
    void release(int) override {}
};

struct Harness {
    FakeExec* ex;
    Scheduler* s;
};

}  // namespace

extern "C" {

void* h_new(size_t pool, int max_inflight, int tiles_per_launch, int manual)
{
    auto* h = new Harness;
    h->ex = new FakeExec(pool, manual != 0);
    Config c;
    c.max_inflight = max_inflight;
    c.tiles_per_launch = tiles_per_launch;
    h->s = new Scheduler(c, std::unique_ptr<Executor>(h->ex));
    return h;
}

int h_register(void* hp)
{
    auto* h = (Harness*)hp;
    vi_volume v{};
    vi_tf t{};
    int id = -1;
    h->s->register_volume(&v, &t, &id);
    return id;
}

long long h_submit(void* hp, int vol, double lx, double ly, double lz, int n, int res, int w, int hgt, long long tag,
                   int mode, int dtype)
{
    auto* h = (Harness*)hp;
    vi_request r{};
    r.vol_id = vol;
    r.light_dir[0] = lx;
    r.light_dir[1] = ly;
    r.light_dir[2] = lz;
    r.n_slices = n;
    r.slice_res = res;
    r.slice_dtype = dtype;
    r.camera.width = w;
    r.camera.height = hgt;
    r.mode = mode;
    r.d_rgba = (float*)(uintptr_t)tag;
    uint64_t t = 0;
    int rc = h->s->submit(&r, &t);
    return rc == VI_OK ? (long long)t : (long long)rc;
}

int h_poll(void* hp, long long t)
{
    int st = -100;
    int rc = ((Harness*)hp)->s->poll((uint64_t)t, &st);
    return rc == VI_OK ? st : rc;
}
int h_wait(void* hp, long long t, int ms) { return ((Harness*)hp)->s->wait((uint64_t)t, ms); }
int h_cancel(void* hp, long long t) { return ((Harness*)hp)->s->cancel((uint64_t)t); }
void h_stats(void* hp, vi_stats* o) { ((Harness*)hp)->s->stats(o); }
void h_finish(void* hp, int n)
{
    auto* h = (Harness*)hp;
    std::lock_guard<std::mutex> lk(h->ex->mu);
    h->ex->finish_budget += n;
}
void h_fail_builds_of(void* hp, int vol)
{
    auto* h = (Harness*)hp;
    std::lock_guard<std::mutex> lk(h->ex->mu);
    h->ex->fail_build_vol = vol;
}
int h_log(void* hp, char* buf, int cap)
{
    auto* h = (Harness*)hp;
    std::lock_guard<std::mutex> lk(h->ex->mu);
    const int n = (int)h->ex->log.size();
    if (buf && cap > 0) {
        const int m = n < cap - 1 ? n : cap - 1;
        memcpy(buf, h->ex->log.data(), m);
        buf[m] = 0;
    }
    return n;
}
void h_free(void* hp)
{
    auto* h = (Harness*)hp;
    h_finish(hp, 1 << 30);  // let everything drain
    delete h->s;            // joins the scheduler thread, deletes the executor
    delete h;
}

}  // extern "C"

#ifdef VI_SCHED_STRESS
// Several producer threads submit, poll, wait and cancel while the
// scheduler admits, evicts and completes; run under TSan / ASan.
#include <thread>
int main()
{
    void* h = h_new(64ull << 20, 8, 64, 0);
    for (int v = 0; v < 6; ++v) h_register(h);
    std::atomic<int> bad{0};
    auto producer = [&](int id) {
        for (int i = 0; i < 300; ++i) {
            const int vol = (i + id) % 6;
            const double lx = (double)((i / 7) % 3), ly = 1.0, lz = -1.0;
            long long t = h_submit(h, vol, lx, ly, lz, 16 + 8 * (i % 3), 64 + 32 * (i % 4), 64 + 16 * (i % 5),
                                   48 + 16 * (i % 3), 1000 * id + i, 2, VI_F32);
            if (t < 0) {
                bad++;
                continue;
            }
            if (i % 17 == 0) h_cancel(h, t);
            int st = h_poll(h, t);
            if (st == -100) bad++;
            int rc = h_wait(h, t, 5000);
            if (rc != VI_OK && rc != VI_E_CANCELLED) bad++;
        }
    };
    std::vector<std::thread> th;
    for (int p = 0; p < 4; ++p) th.emplace_back(producer, p);
    for (auto& t : th) t.join();
    vi_stats s;
    h_stats(h, &s);
    h_free(h);
    printf("completed %llu cancelled %llu hits %llu builds %llu evictions %llu bad %d\n",
           (unsigned long long)s.completed, (unsigned long long)s.cancelled, (unsigned long long)s.stack_hits,
           (unsigned long long)s.stack_builds, (unsigned long long)s.evictions, bad.load());
    return bad.load() == 0 && s.completed + s.cancelled == 1200 ? 0 : 1;
}
#endif
