// vi_sched.h -- the serving scheduler of libvi (plain C++17, no HIP): request
// admission by pool footprint, the stack cache, continuous batching of
// frame tiles into render launches, and completion/latency bookkeeping.
// Device work goes through the Executor interface; libvi's executor drives
// HIP streams and kernels, the CPU tests plug in a recording executor.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/vi.h"

namespace vi {
namespace sched {

struct VolumeRec {
    vi_volume vol;
    vi_tf tf;
};

// A cached attenuation stack as handed to the executor.
struct StackRef {
    size_t offset = 0;       // byte offset in the pool
    size_t bytes = 0;
    vi_slices desc{};        // filled by Executor::build
    int build_handle = -1;   // executor's handle of the build (for device-side waits)
};

struct LaunchFrame {
    const vi_request* req;
    const VolumeRec* vol;
    const StackRef* stack;
};

// Tiles are 16 x 16 pixels; a tile entry packs x | y << 11 | frame << 22.
constexpr int kTile = 16;
inline uint32_t pack_tile(uint32_t tx, uint32_t ty, uint32_t f) { return tx | (ty << 11) | (f << 22); }
// Tile i of a W x H tile grid in launch order: 2 x 2 blocks of tiles
// (32 x 32 pixels), row pairs top to bottom; an odd last column or row is
// taken in order.  Consecutive tiles then cover square patches, which keeps
// the volume and stack footprint of a group of workgroups compact.
inline void tile_of(int i, int W, int H, uint32_t* tx, uint32_t* ty)
{
    const int pairs = H / 2, p = i / (2 * W);
    if (p >= pairs) {
        *tx = (uint32_t)(i - pairs * 2 * W);
        *ty = (uint32_t)(H - 1);
        return;
    }
    const int j = i - p * 2 * W, full = 4 * (W / 2);
    if (j < full) {
        *tx = (uint32_t)(2 * (j / 4) + (j & 1));
        *ty = (uint32_t)(2 * p + ((j >> 1) & 1));
    } else {
        *tx = (uint32_t)(W - 1);
        *ty = (uint32_t)(2 * p + (j - full));
    }
}

class Executor {
public:
    virtual ~Executor() = default;
    virtual void thread_init() {}  // called first on the scheduler thread
    virtual size_t pool_bytes() const = 0;
    virtual int max_frames_per_launch() const = 0;
    // submit-time checks of a request against its volume (VI_OK or an error code)
    virtual int validate(const vi_request& r, const VolumeRec& v) = 0;
    virtual size_t stack_bytes(const vi_request& r) = 0;
    // frames of one launch must share a class (the kernel instantiation)
    virtual int frame_class(const vi_request& r, const VolumeRec& v) = 0;
    // enqueue the build of a stack at st->offset; fills st->desc and st->build_handle
    virtual int build(const vi_request& r, const VolumeRec& v, StackRef* st) = 0;
    // the stack at st is no longer cached (its memory may be reused)
    virtual void drop_stack(StackRef* st) = 0;
    // enqueue one render launch over `tiles`; returns a handle >= 0 or an error code
    virtual int launch(const std::vector<LaunchFrame>& frames, const std::vector<uint32_t>& tiles) = 0;
    virtual bool query(int handle) = 0;  // launch finished?
    virtual int wait(int handle) = 0;    // block until finished; VI_OK or an error code
    virtual void release(int handle) = 0;
};

struct Config {
    int max_inflight = 16;
    int tiles_per_launch = 8192;
    int max_launches_in_flight = 2;
};

// First-fit allocator of byte ranges of the stack pool (256-byte aligned).
class Pool {
public:
    explicit Pool(size_t bytes);
    bool alloc(size_t bytes, size_t* off);
    void free(size_t off, size_t bytes);
    size_t capacity() const { return cap_; }
    size_t in_use() const { return used_; }

private:
    size_t cap_, used_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
};

class Scheduler {
public:
    Scheduler(const Config& cfg, std::unique_ptr<Executor> ex);
    ~Scheduler();
    int register_volume(const vi_volume* vol, const vi_tf* tf, int* id);
    int submit(const vi_request* r, uint64_t* ticket);
    int poll(uint64_t ticket, int* state);
    int wait(uint64_t ticket, int timeout_ms);
    int cancel(uint64_t ticket);
    void stats(vi_stats* out);
    void reset_stats();
    void shutdown();

private:
    using clock = std::chrono::steady_clock;
    struct Key {
        int vol_id, n, res, dtype, layout;
        uint32_t darken;  // build option bits
        int positional;   // lx, ly, lz: direction bits, or position bits when set
        uint64_t lx, ly, lz;
        bool operator==(const Key& o) const
        {
            return vol_id == o.vol_id && n == o.n && res == o.res && dtype == o.dtype && layout == o.layout &&
                   darken == o.darken && positional == o.positional && lx == o.lx && ly == o.ly && lz == o.lz;
        }
    };
    struct Stack {
        Key key;
        StackRef ref;
        int pins = 0;
        uint64_t last_use = 0;
        bool live = false;
    };
    struct Req {
        vi_request r;
        int state = VI_REQ_PENDING;
        int cls = 0;
        size_t stack_bytes = 0;
        int stack = -1;
        int tiles_x = 0, tiles_y = 0, ntiles = 0, next_tile = 0;
        clock::time_point submitted;
    };
    struct Launch {
        int handle;
        std::vector<uint64_t> finishing;  // frames whose last tile is in this launch
        std::vector<uint64_t> members;
    };

    void loop();
    bool admit();
    bool launch_next();
    void finish(Launch& L, int status);
    bool evict_one();
    int find_stack(const Key& k) const;
    Key key_of(const vi_request& r) const;

    Config cfg_;
    std::unique_ptr<Executor> ex_;
    Pool pool_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::vector<VolumeRec> vols_;
    std::unordered_map<uint64_t, Req> reqs_;
    std::deque<uint64_t> pending_;
    std::vector<uint64_t> active_;
    std::vector<Stack> stacks_;
    std::deque<Launch> launches_;
    uint64_t next_ticket_ = 1, use_clock_ = 0;
    bool stop_ = false;
    // statistics
    uint64_t n_sub_ = 0, n_done_ = 0, n_rej_ = 0, n_can_ = 0, n_hit_ = 0, n_build_ = 0, n_evict_ = 0;
    uint64_t n_launch_ = 0, n_tiles_ = 0, n_launch_frames_ = 0;
    size_t pool_peak_ = 0;
    std::vector<double> lat_ms_;
    bool have_first_ = false;
    clock::time_point first_sub_, last_done_;
    std::thread th_;
};

}  // namespace sched
}  // namespace vi
