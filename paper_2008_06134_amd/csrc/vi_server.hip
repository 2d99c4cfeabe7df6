// vi_server.hip -- the HIP executor of the serving scheduler and the
// vi_server_* C ABI.  The executor owns the stack pool (one allocation at
// creation), a render stream and a build stream (default priority), and a
// ring of staging slots (pinned host + device copies of the frame
// parameters and tile list of one launch).
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "vi_internal.h"
#include "vi_sched.h"

namespace vi {

namespace {

constexpr int kSlots = 4;           // staging slots (> launches in flight)
constexpr int kMaxLaunchFrames = 64;

int slice_elem(int dt) { return dt == VI_F32 ? 4 : 2; }

class HipExecutor final : public sched::Executor {
public:
    HipExecutor(int device, size_t pool_bytes, int max_tiles) : dev_(device), max_tiles_(max_tiles) {}

    int init(size_t pool_bytes)
    {
        if (hipSetDevice(dev_) != hipSuccess) return fail_msg(VI_E_DEVICE, "cannot select the device");
        if (hipMalloc(&pool_, pool_bytes) != hipSuccess) {
            pool_ = nullptr;
            hipGetLastError();
            return fail_msg(VI_E_NO_MEMORY, "cannot allocate the stack pool");
        }
        pool_bytes_ = pool_bytes;
        if (hipStreamCreateWithFlags(&rs_, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&bs_, hipStreamNonBlocking) != hipSuccess)
            return fail_msg(VI_E_DEVICE, "cannot create streams");
        // per slot one staging area: the launch's frames, then its tiles,
        // copied to the device with one transfer
        const size_t stage = sizeof(RenderFrame) * kMaxLaunchFrames + 16 + sizeof(uint32_t) * (size_t)max_tiles_;
        for (auto& s : slots_) {
            if (hipMalloc(&s.d_stage, stage) != hipSuccess ||
                hipHostMalloc(&s.h_stage, stage, hipHostMallocDefault) != hipSuccess ||
                hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
                return fail_msg(VI_E_NO_MEMORY, "cannot allocate staging buffers");
        }
        return VI_OK;
    }

    ~HipExecutor() override
    {
        hipSetDevice(dev_);
        if (rs_) hipStreamSynchronize(rs_);
        if (bs_) hipStreamSynchronize(bs_);
        for (auto& s : slots_) {
            if (s.d_stage) hipFree(s.d_stage);
            if (s.h_stage) hipHostFree(s.h_stage);
            if (s.done) hipEventDestroy(s.done);
        }
        for (hipEvent_t e : build_events_)
            if (e) hipEventDestroy(e);
        if (rs_) hipStreamDestroy(rs_);
        if (bs_) hipStreamDestroy(bs_);
        if (pool_) hipFree(pool_);
    }

    void thread_init() override { hipSetDevice(dev_); }
    size_t pool_bytes() const override { return pool_bytes_; }
    int max_frames_per_launch() const override { return kMaxLaunchFrames; }

    int validate(const vi_request& r, const sched::VolumeRec& v) override
    {
        vi_slices sl;
        int rc = vi_light_frame(r.light_dir, r.n_slices, r.slice_res, r.slice_dtype, r.slice_layout, &r.build, &sl);
        if (rc != VI_OK) return rc;
        if (!(r.build.darken >= 0.0f && r.build.darken <= 64.0f))
            return fail_msg(VI_E_INVALID_ARG, "darken must be in [0, 64]");
        sl.data = pool_;  // stands in for the cached stack
        sl.vol_n = v.vol.n;
        sl.tag = 0;
        RenderFrame F;
        return make_frame(&v.vol, &v.tf, &sl, &r.camera, r.mode, r.step_vox, &r.opts, r.d_rgba, r.d_samples, &F);
    }

    size_t stack_bytes(const vi_request& r) override
    {
        return vi_slices_bytes(r.n_slices, r.slice_res, r.slice_dtype, r.slice_layout);
    }

    int frame_class(const vi_request& r, const sched::VolumeRec& v) override
    {
        return ((v.vol.dtype * 4 + v.vol.layout) * 8 + r.slice_dtype) * 2 + r.slice_layout;
    }

    int build(const vi_request& r, const sched::VolumeRec& v, sched::StackRef* st) override
    {
        void* dst = (char*)pool_ + st->offset;
        int rc = vi_build_attenuation(&v.vol, &v.tf, r.light_dir, r.n_slices, r.slice_res, r.slice_dtype,
                                      r.slice_layout, &r.build, dst, &st->desc, bs_);
        if (rc != VI_OK) return rc;
        int h = -1;
        for (size_t i = 0; i < build_events_.size(); ++i)
            if (!event_used_[i]) {
                h = (int)i;
                break;
            }
        if (h < 0) {
            hipEvent_t e;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
                return fail_msg(VI_E_DEVICE, "cannot create an event");
            build_events_.push_back(e);
            event_used_.push_back(false);
            h = (int)build_events_.size() - 1;
        }
        if (hipEventRecord(build_events_[h], bs_) != hipSuccess) return fail_msg(VI_E_DEVICE, "event record failed");
        event_used_[h] = true;
        st->build_handle = h;
        return VI_OK;
    }

    void drop_stack(sched::StackRef* st) override
    {
        if (st->build_handle >= 0) event_used_[st->build_handle] = false;
        st->build_handle = -1;
    }

    int launch(const std::vector<sched::LaunchFrame>& frames, const std::vector<uint32_t>& tiles) override
    {
        int slot = -1;
        for (int i = 0; i < kSlots; ++i)
            if (!slots_[i].busy) {
                slot = i;
                break;
            }
        if (slot < 0 || (int)frames.size() > kMaxLaunchFrames || (int)tiles.size() > max_tiles_)
            return fail_msg(VI_E_BUSY, "no staging slot free");
        Slot& S = slots_[slot];
        // staging: this launch's frames, then its tiles (16-byte aligned)
        RenderFrame* h_frames = (RenderFrame*)S.h_stage;
        const size_t frames_bytes = (frames.size() * sizeof(RenderFrame) + 15) / 16 * 16;
        uint32_t* h_tiles = (uint32_t*)((char*)S.h_stage + frames_bytes);
        const RenderFrame* d_frames = (const RenderFrame*)S.d_stage;
        const uint32_t* d_tiles = (const uint32_t*)((const char*)S.d_stage + frames_bytes);
        int maxK = 2;
        uint32_t occ_words = 0;  // LDS occupancy bits of the largest frame
        for (size_t f = 0; f < frames.size(); ++f) {
            const vi_request& r = *frames[f].req;
            const sched::VolumeRec& v = *frames[f].vol;
            int rc = make_frame(&v.vol, &v.tf, &frames[f].stack->desc, &r.camera, r.mode, r.step_vox, &r.opts,
                                r.d_rgba, r.d_samples, &h_frames[f]);
            if (rc != VI_OK) return rc;
            maxK = std::max(maxK, v.tf.n_entries);
            if (h_frames[f].occ.bits)
                occ_words = std::max(occ_words, h_frames[f].occ.words + h_frames[f].occ.swords);
        }
        // tiles grouped by kernel mode (stable), one kernel per mode present
        constexpr int kModes = kKernelModes;
        uint32_t count[kModes] = {0}, start[kModes + 1] = {0};
        for (uint32_t t : tiles) count[kernel_mode(h_frames[t >> 22])]++;
        for (int m = 0; m < kModes; ++m) start[m + 1] = start[m] + count[m];
        {
            uint32_t at[kModes];
            for (int m = 0; m < kModes; ++m) at[m] = start[m];
            for (uint32_t t : tiles) h_tiles[at[kernel_mode(h_frames[t >> 22])]++] = t;
        }
        hipError_t e = hipMemcpyAsync(S.d_stage, S.h_stage, frames_bytes + tiles.size() * sizeof(uint32_t),
                                      hipMemcpyHostToDevice, rs_);
        // device-side waits on the builds of the stacks this launch reads
        for (const auto& f : frames)
            if (e == hipSuccess && f.stack->build_handle >= 0)
                e = hipStreamWaitEvent(rs_, build_events_[f.stack->build_handle], 0);
        const vi_volume& v0 = frames[0].vol->vol;
        for (int m = 0; m < kModes && e == hipSuccess; ++m)
            if (count[m])
                e = launch_render_batch(v0.dtype, v0.layout, frames[0].req->slice_dtype, frames[0].req->slice_layout,
                                        m, d_frames, d_tiles + start[m], count[m], maxK, occ_words, rs_);
        if (e == hipSuccess) e = hipEventRecord(S.done, rs_);
        if (e != hipSuccess) return fail_msg(VI_E_DEVICE, hipGetErrorString(e));
        S.busy = true;
        return slot;
    }

    bool query(int h) override { return hipEventQuery(slots_[h].done) != hipErrorNotReady; }

    int wait(int h) override
    {
        hipError_t e = hipEventSynchronize(slots_[h].done);
        return e == hipSuccess ? VI_OK : VI_E_DEVICE;
    }

    void release(int h) override { slots_[h].busy = false; }

private:
    struct Slot {
        void* d_stage = nullptr;  // device: frames, then tiles
        void* h_stage = nullptr;  // pinned host mirror
        hipEvent_t done = nullptr;
        bool busy = false;
    };
    int dev_;
    int max_tiles_;
    void* pool_ = nullptr;
    size_t pool_bytes_ = 0;
    hipStream_t rs_ = nullptr, bs_ = nullptr;
    Slot slots_[kSlots];
    std::vector<hipEvent_t> build_events_;
    std::vector<bool> event_used_;
};

}  // namespace
}  // namespace vi

struct vi_server {
    vi::sched::Scheduler* sched;
};

extern "C" {

int vi_server_create(const vi_server_cfg* cfg, vi_server** out)
{
    if (!cfg || !out) return vi::fail_msg(VI_E_INVALID_ARG, "NULL config or output");
    if (cfg->stack_budget < 256) return vi::fail_msg(VI_E_INVALID_ARG, "stack_budget too small");
    if (cfg->max_inflight < 1 || cfg->max_inflight > 256)
        return vi::fail_msg(VI_E_INVALID_ARG, "max_inflight must be 1..256");
    const int tiles = cfg->tiles_per_launch > 0 ? cfg->tiles_per_launch : 8192;
    if (tiles > (1 << 22)) return vi::fail_msg(VI_E_INVALID_ARG, "tiles_per_launch too large");
    auto* ex = new (std::nothrow) vi::HipExecutor(cfg->device, cfg->stack_budget, tiles);
    if (!ex) return vi::fail_msg(VI_E_NO_MEMORY, "out of host memory");
    int rc = ex->init(cfg->stack_budget);
    if (rc != VI_OK) {
        delete ex;
        return rc;
    }
    vi::sched::Config sc;
    sc.max_inflight = cfg->max_inflight;
    sc.tiles_per_launch = tiles;
    sc.max_launches_in_flight = 2;
    auto* s = new (std::nothrow) vi_server;
    if (!s) {
        delete ex;
        return vi::fail_msg(VI_E_NO_MEMORY, "out of host memory");
    }
    s->sched = new vi::sched::Scheduler(sc, std::unique_ptr<vi::sched::Executor>(ex));
    *out = s;
    return VI_OK;
}

int vi_server_register_volume(vi_server* srv, const vi_volume* vol, const vi_tf* tf, int* vol_id)
{
    if (!srv) return vi::fail_msg(VI_E_INVALID_ARG, "NULL server");
    return srv->sched->register_volume(vol, tf, vol_id);
}

int vi_server_submit(vi_server* srv, const vi_request* req, uint64_t* ticket)
{
    if (!srv) return vi::fail_msg(VI_E_INVALID_ARG, "NULL server");
    return srv->sched->submit(req, ticket);
}

int vi_server_poll(vi_server* srv, uint64_t ticket, int* state)
{
    if (!srv) return vi::fail_msg(VI_E_INVALID_ARG, "NULL server");
    return srv->sched->poll(ticket, state);
}

int vi_server_wait(vi_server* srv, uint64_t ticket, int timeout_ms)
{
    if (!srv) return vi::fail_msg(VI_E_INVALID_ARG, "NULL server");
    return srv->sched->wait(ticket, timeout_ms);
}

int vi_server_cancel(vi_server* srv, uint64_t ticket)
{
    if (!srv) return vi::fail_msg(VI_E_INVALID_ARG, "NULL server");
    return srv->sched->cancel(ticket);
}

int vi_server_stats(vi_server* srv, vi_stats* out)
{
    if (!srv || !out) return vi::fail_msg(VI_E_INVALID_ARG, "NULL server or output");
    srv->sched->stats(out);
    return VI_OK;
}

int vi_server_reset_stats(vi_server* srv)
{
    if (!srv) return vi::fail_msg(VI_E_INVALID_ARG, "NULL server");
    srv->sched->reset_stats();
    return VI_OK;
}

void vi_server_destroy(vi_server* srv)
{
    if (!srv) return;
    delete srv->sched;  // drains queued and admitted work, then the executor frees its memory
    delete srv;
}

}  // extern "C"
