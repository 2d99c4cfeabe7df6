// vi_sched.cpp -- serving scheduler (see vi_sched.h).
#include "vi_sched.h"

#include <string.h>

#include <algorithm>

namespace vi {
namespace sched {

// ---------------------------------------------------------------------------
// pool
// ---------------------------------------------------------------------------
Pool::Pool(size_t bytes) : cap_(bytes & ~(size_t)255)
{
    if (cap_) free_[0] = cap_;
}

bool Pool::alloc(size_t bytes, size_t* off)
{
    const size_t need = (bytes + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second >= need) {
            *off = it->first;
            const size_t rest = it->second - need, at = it->first + need;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += need;
            return true;
        }
    }
    return false;
}

void Pool::free(size_t off, size_t bytes)
{
    const size_t len = (bytes + 255) & ~(size_t)255;
    used_ -= len;
    auto it = free_.emplace(off, len).first;
    // merge with the following block
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        free_.erase(nx);
    }
    // and with the preceding one
    if (it != free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            free_.erase(it);
        }
    }
}

// ---------------------------------------------------------------------------
// scheduler
// ---------------------------------------------------------------------------
Scheduler::Scheduler(const Config& cfg, std::unique_ptr<Executor> ex)
    : cfg_(cfg), ex_(std::move(ex)), pool_(ex_->pool_bytes())
{
    th_ = std::thread([this] { loop(); });
}

Scheduler::~Scheduler() { shutdown(); }

void Scheduler::shutdown()
{
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (stop_ && !th_.joinable()) return;
        stop_ = true;
    }
    cv_work_.notify_all();
    if (th_.joinable()) th_.join();
}

int Scheduler::register_volume(const vi_volume* vol, const vi_tf* tf, int* id)
{
    if (!vol || !tf || !id) return VI_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(mu_);
    vols_.push_back(VolumeRec{*vol, *tf});
    *id = (int)vols_.size() - 1;
    return VI_OK;
}

Scheduler::Key Scheduler::key_of(const vi_request& r) const
{
    Key k;
    k.vol_id = r.vol_id;
    k.n = r.n_slices;
    k.res = r.slice_res;
    k.dtype = r.slice_dtype;
    k.layout = r.slice_layout;
    memcpy(&k.darken, &r.build.darken, 4);
    // the light is part of the identity bit for bit: its direction, or for
    // a point light its position
    k.positional = r.build.positional ? 1 : 0;
    const double* l = k.positional ? r.build.position : r.light_dir;
    memcpy(&k.lx, &l[0], 8);
    memcpy(&k.ly, &l[1], 8);
    memcpy(&k.lz, &l[2], 8);
    return k;
}

int Scheduler::find_stack(const Key& k) const
{
    for (size_t i = 0; i < stacks_.size(); ++i)
        if (stacks_[i].live && stacks_[i].key == k) return (int)i;
    return -1;
}

int Scheduler::submit(const vi_request* r, uint64_t* ticket)
{
    if (!r || !ticket) return VI_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(mu_);
    if (stop_) return VI_E_CANCELLED;
    if (r->vol_id < 0 || r->vol_id >= (int)vols_.size()) return VI_E_INVALID_ARG;
    const VolumeRec& v = vols_[r->vol_id];
    int rc = ex_->validate(*r, v);
    if (rc != VI_OK) return rc;
    Req q;
    q.r = *r;
    q.cls = ex_->frame_class(*r, v);
    q.stack_bytes = ex_->stack_bytes(*r);
    if (q.stack_bytes > pool_.capacity()) {
        ++n_rej_;
        return VI_E_NO_MEMORY;
    }
    q.tiles_x = (r->camera.width + kTile - 1) / kTile;
    q.tiles_y = (r->camera.height + kTile - 1) / kTile;
    q.ntiles = q.tiles_x * q.tiles_y;
    q.submitted = clock::now();
    if (!have_first_) {
        have_first_ = true;
        first_sub_ = q.submitted;
    }
    const uint64_t t = next_ticket_++;
    reqs_.emplace(t, q);
    pending_.push_back(t);
    ++n_sub_;
    *ticket = t;
    lk.unlock();
    cv_work_.notify_all();
    return VI_OK;
}

int Scheduler::poll(uint64_t ticket, int* state)
{
    if (!state) return VI_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return VI_E_INVALID_ARG;
    *state = it->second.state;
    return VI_OK;
}

int Scheduler::wait(uint64_t ticket, int timeout_ms)
{
    std::unique_lock<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return VI_E_INVALID_ARG;
    auto finished = [&] {
        const int s = reqs_.at(ticket).state;
        return s == VI_REQ_DONE || s < 0;
    };
    if (timeout_ms < 0) {
        cv_done_.wait(lk, finished);
    } else if (!cv_done_.wait_until(lk, std::chrono::system_clock::now() + std::chrono::milliseconds(timeout_ms),
                                    finished)) {
        return VI_E_BUSY;
    }
    const int s = reqs_.at(ticket).state;
    return s == VI_REQ_DONE ? VI_OK : s;
}

int Scheduler::cancel(uint64_t ticket)
{
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return VI_E_INVALID_ARG;
    if (it->second.state != VI_REQ_PENDING) return VI_E_BUSY;
    pending_.erase(std::remove(pending_.begin(), pending_.end(), ticket), pending_.end());
    it->second.state = VI_E_CANCELLED;
    ++n_can_;
    cv_done_.notify_all();
    return VI_OK;
}

bool Scheduler::evict_one()
{
    int victim = -1;
    for (size_t i = 0; i < stacks_.size(); ++i) {
        const Stack& s = stacks_[i];
        if (s.live && s.pins == 0 && (victim < 0 || s.last_use < stacks_[victim].last_use)) victim = (int)i;
    }
    if (victim < 0) return false;
    Stack& s = stacks_[victim];
    ex_->drop_stack(&s.ref);
    pool_.free(s.ref.offset, s.ref.bytes);
    s.live = false;
    ++n_evict_;
    return true;
}

bool Scheduler::admit()
{
    bool progress = false;
    while (!pending_.empty() && (int)active_.size() < cfg_.max_inflight) {
        const uint64_t t = pending_.front();
        Req& q = reqs_.at(t);
        const Key k = key_of(q.r);
        int sid = find_stack(k);
        if (sid >= 0) {
            ++n_hit_;
        } else {
            size_t off = 0;
            bool ok = pool_.alloc(q.stack_bytes, &off);
            while (!ok && evict_one()) ok = pool_.alloc(q.stack_bytes, &off);
            if (!ok) break;  // first come, first served: wait for pool memory
            pool_peak_ = std::max(pool_peak_, pool_.in_use());
            sid = -1;
            for (size_t i = 0; i < stacks_.size(); ++i)
                if (!stacks_[i].live) {
                    sid = (int)i;
                    break;
                }
            if (sid < 0) {
                stacks_.emplace_back();
                sid = (int)stacks_.size() - 1;
            }
            Stack& s = stacks_[sid];
            s = Stack();
            s.key = k;
            s.ref.offset = off;
            s.ref.bytes = q.stack_bytes;
            const int rc = ex_->build(q.r, vols_[q.r.vol_id], &s.ref);
            if (rc != VI_OK) {
                pool_.free(off, q.stack_bytes);
                q.state = rc;
                pending_.pop_front();
                cv_done_.notify_all();
                progress = true;
                continue;
            }
            s.live = true;
            ++n_build_;
        }
        Stack& s = stacks_[sid];
        s.pins++;
        s.last_use = ++use_clock_;
        q.stack = sid;
        q.state = VI_REQ_ADMITTED;
        active_.push_back(t);
        pending_.pop_front();
        progress = true;
    }
    return progress;
}

bool Scheduler::launch_next()
{
    std::vector<LaunchFrame> frames;
    std::vector<uint32_t> tiles;
    Launch L;
    int cls = -1, budget = cfg_.tiles_per_launch;
    const int max_frames = std::min(ex_->max_frames_per_launch(), 1023);
    for (uint64_t t : active_) {
        Req& q = reqs_.at(t);
        if (q.next_tile >= q.ntiles) continue;
        if (cls >= 0 && q.cls != cls) continue;
        cls = q.cls;
        const int take = std::min(budget, q.ntiles - q.next_tile);
        const uint32_t f = (uint32_t)frames.size();
        frames.push_back(LaunchFrame{&q.r, &vols_[q.r.vol_id], &stacks_[q.stack].ref});
        for (int i = q.next_tile; i < q.next_tile + take; ++i) {
            uint32_t tx, ty;
            tile_of(i, q.tiles_x, q.tiles_y, &tx, &ty);
            tiles.push_back(pack_tile(tx, ty, f));
        }
        q.next_tile += take;
        budget -= take;
        L.members.push_back(t);
        if (q.next_tile == q.ntiles) L.finishing.push_back(t);
        if (budget == 0 || (int)frames.size() == max_frames) break;
    }
    if (tiles.empty()) return false;
    const int h = ex_->launch(frames, tiles);
    ++n_launch_;
    n_tiles_ += tiles.size();
    n_launch_frames_ += frames.size();
    if (h < 0) {
        // the launch never ran: fail its frames
        for (uint64_t t : L.members) {
            Req& q = reqs_.at(t);
            q.state = h;
            stacks_[q.stack].pins--;
            active_.erase(std::remove(active_.begin(), active_.end(), t), active_.end());
        }
        cv_done_.notify_all();
        return true;
    }
    L.handle = h;
    launches_.push_back(std::move(L));
    return true;
}

void Scheduler::finish(Launch& L, int status)
{
    const auto now = clock::now();
    for (uint64_t t : L.finishing) {
        Req& q = reqs_.at(t);
        if (q.state < 0) continue;
        q.state = status == VI_OK ? VI_REQ_DONE : status;
        stacks_[q.stack].pins--;
        active_.erase(std::remove(active_.begin(), active_.end(), t), active_.end());
        if (status == VI_OK) {
            ++n_done_;
            lat_ms_.push_back(std::chrono::duration<double, std::milli>(now - q.submitted).count());
            last_done_ = now;
        }
    }
    if (status != VI_OK) {
        // a failed launch fails every frame that had tiles in it
        for (uint64_t t : L.members) {
            Req& q = reqs_.at(t);
            if (q.state == VI_REQ_ADMITTED) {
                q.state = status;
                stacks_[q.stack].pins--;
                active_.erase(std::remove(active_.begin(), active_.end(), t), active_.end());
            }
        }
    }
    ex_->release(L.handle);
    cv_done_.notify_all();
}

void Scheduler::loop()
{
    ex_->thread_init();
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
        bool progress = false;
        while (!launches_.empty() && ex_->query(launches_.front().handle)) {
            Launch L = std::move(launches_.front());
            launches_.pop_front();
            finish(L, ex_->wait(L.handle));
            progress = true;
        }
        progress |= admit();
        while ((int)launches_.size() < cfg_.max_launches_in_flight && launch_next()) progress = true;
        if (stop_ && pending_.empty() && active_.empty() && launches_.empty()) break;
        if (!progress) {
            // nothing to do until a launch finishes or a request arrives (timed
            // against the system clock: a plain timed wait on the mutex)
            cv_work_.wait_until(lk, std::chrono::system_clock::now() +
                                        std::chrono::microseconds(launches_.empty() ? 2000 : 10));
        }
    }
}

void Scheduler::stats(vi_stats* o)
{
    std::lock_guard<std::mutex> lk(mu_);
    memset(o, 0, sizeof *o);
    o->submitted = n_sub_;
    o->completed = n_done_;
    o->rejected = n_rej_;
    o->cancelled = n_can_;
    o->stack_hits = n_hit_;
    o->stack_builds = n_build_;
    o->evictions = n_evict_;
    o->launches = n_launch_;
    o->tiles = n_tiles_;
    o->mean_frames_per_launch = n_launch_ ? (double)n_launch_frames_ / n_launch_ : 0.0;
    if (!lat_ms_.empty()) {
        std::vector<double> v = lat_ms_;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const double x = p * (v.size() - 1);
            const size_t i = (size_t)x;
            const double f = x - i;
            return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
        };
        o->p50_ms = pct(0.50);
        o->p99_ms = pct(0.99);
        double s = 0;
        for (double x : v) s += x;
        o->mean_ms = s / v.size();
        o->max_ms = v.back();
        const double span = std::chrono::duration<double>(last_done_ - first_sub_).count();
        o->frames_per_s = span > 0 ? n_done_ / span : 0.0;
    }
    o->pool_bytes = pool_.capacity();
    o->pool_in_use = pool_.in_use();
    o->pool_peak = pool_peak_;
}

void Scheduler::reset_stats()
{
    std::lock_guard<std::mutex> lk(mu_);
    n_sub_ = n_done_ = n_rej_ = n_can_ = n_hit_ = n_build_ = n_evict_ = 0;
    n_launch_ = n_tiles_ = n_launch_frames_ = 0;
    pool_peak_ = pool_.in_use();
    lat_ms_.clear();
    have_first_ = false;
}

}  // namespace sched
}  // namespace vi
