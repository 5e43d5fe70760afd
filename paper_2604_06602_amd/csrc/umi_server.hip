// Native serving loop of the UMI library (include/umi_serve.h): continuous
// batching of detrending requests on one device.  Not a step of the method
// (arXiv 2604.06602, Section 2): it feeds the method's batched kernels
// through a replayable plan.
//
// Threads.  Callers submit and poll from any thread.  One scheduler thread
// admits waiting requests, stages and uploads them and launches steps; one
// waiter thread blocks on each in-flight step's completion event in launch
// order, then finishes the step (copies every result into its request's
// output, releases the step's memory, reports the completions) and wakes the
// scheduler, so result copies never hold up admission and launches.  `mu`
// guards the waiting queue, the shutdown flags and the statistics; `rmu` the
// arena, the staging rings, the event pool, upload bookkeeping and the
// in-flight count (taken after `mu` where both are held); `cmu` the
// completion queue; `wmu` the waiter's queue.
//
// Device work per step, on three streams: uploads (the copy kernel reads the
// pinned staging ring), the step itself (the plan's graph on the compute
// stream, after the uploads' events), and the download of every group's trend
// into the pinned result ring (after the step's event).  A request's staging
// block is released once its step has completed (its upload finished before
// the step started); its arena range once its result is in `out`.
#include <hip/hip_runtime.h>

#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "umi.h"
#include "umi_internal.h"
#include "umi_serve.h"

namespace umi {

umi_status report_error(umi_status s, const std::string& msg);
hipError_t enqueue_copy_list(uint8_t* const* dst, const uint8_t* const* src, const int64_t* bytes,
                             int64_t n, hipStream_t stream);
umi_status host_copy_many(int which, void* const* dst, const void* const* src,
                          const int64_t* bytes, int64_t n, int32_t threads);

namespace srv {

// Deadline `sec` seconds from now for condition-variable waits.  The waits
// here are short and re-check their condition, so the wall clock serves;
// (a steady-clock wait compiles to pthread_cond_clockwait, which the thread
// sanitizer the host code is tested under does not see as releasing the lock).
std::chrono::system_clock::time_point deadline(double sec)
{
    return std::chrono::system_clock::now() +
           std::chrono::duration_cast<std::chrono::system_clock::duration>(
               std::chrono::duration<double>(sec));
}

double now_s()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

// First-fit allocation of sample ranges of the arena.
class Arena {
  public:
    explicit Arena(int64_t capacity) : capacity_(capacity)
    {
        if (capacity > 0) free_[0] = capacity;
    }
    // start of a free range of n > 0 samples, or -1
    int64_t alloc(int64_t n)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const int64_t start = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[start + n] = len - n;
            used_ += n;
            return start;
        }
        return -1;
    }
    void release(int64_t start, int64_t n)
    {
        auto it = free_.emplace(start, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && start + n == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
        used_ -= n;
    }
    int64_t capacity() const { return capacity_; }
    int64_t used() const { return used_; }

  private:
    int64_t capacity_;
    std::map<int64_t, int64_t> free_;  // start -> length, coalesced
    int64_t used_ = 0;
};

// A pinned buffer handed out as a ring: blocks are allocated at the head and
// released in any order; space comes back when the oldest blocks are
// released.
class Ring {
  public:
    static constexpr int64_t kAlign = 256;
    uint8_t* base = nullptr;
    uint8_t* dev = nullptr;  // base's device address
    int64_t size = 0;

    // a block of at least n bytes as (id, offset); false when it does not fit now
    bool alloc(int64_t n, uint64_t* id, int64_t* off)
    {
        n = (n + kAlign - 1) / kAlign * kAlign;
        if (n > size) return false;
        reclaim();
        int64_t start = head_;
        if (live_.empty()) {
            start = head_ + n > size ? 0 : head_;
        } else {
            const int64_t tail = live_.front().start;
            if (head_ >= tail) {  // free: [head, size) and [0, tail)
                if (head_ + n > size) {
                    if (n >= tail) return false;
                    start = 0;
                }
            } else if (head_ + n >= tail) {  // free: [head, tail)
                return false;
            }
        }
        live_.push_back(Blk{start, false});
        head_ = start + n;
        *id = first_id_ + live_.size() - 1;
        *off = start;
        return true;
    }
    void release(uint64_t id)
    {
        live_[(size_t)(id - first_id_)].released = true;
        reclaim();
    }

  private:
    struct Blk {
        int64_t start;
        bool released;
    };
    void reclaim()
    {
        while (!live_.empty() && live_.front().released) {
            live_.pop_front();
            ++first_id_;
        }
    }
    std::deque<Blk> live_;
    uint64_t first_id_ = 0;
    int64_t head_ = 0;
};

struct Req {
    uint64_t tag;
    const float* flux;
    const double* time;
    float* out;
    int64_t n;
    int32_t W;
    float alpha, c;
    int32_t iters;
    double arrival, admitted = 0.0, launched = 0.0;
    int64_t offset = -1;
};

// The staging of the groups uploaded together: one block (a ring block, or a
// one-off pinned block for a group too large for the ring) and one event.
struct Upload {
    hipEvent_t ev = nullptr;
    bool in_ring = false;
    uint64_t ring_id = 0;
    uint8_t* oneoff = nullptr;
    uint8_t* oneoff_dev = nullptr;
    bool staging_freed = false;
    int groups_left = 0;  // groups not yet finished
};

struct Group {
    int32_t iters;
    int64_t offset, size;
    std::vector<Req> reqs;
    Upload* up = nullptr;
};

struct Step {
    std::vector<Group*> groups;
    hipEvent_t computed = nullptr, done = nullptr;
    bool out_in_ring = false;
    uint64_t out_id = 0;
    uint8_t* out_base = nullptr;   // the result block (ring or one-off)
    uint8_t* out_oneoff = nullptr;
    std::vector<int64_t> out_pos;  // byte offset of each group's trend in the block
    int64_t samples = 0, curves = 0;
    double launched = 0.0;
};

}  // namespace srv
}  // namespace umi

struct umi_server {
    using Req = umi::srv::Req;
    using Group = umi::srv::Group;
    using Step = umi::srv::Step;
    using Upload = umi::srv::Upload;

    umi_server_config cfg{};
    int device = 0;
    float* flux = nullptr;
    double* time = nullptr;
    float* trend = nullptr;
    umi_plan* plan = nullptr;
    hipStream_t up_stream = nullptr, compute = nullptr, down_stream = nullptr;
    // guarded by rmu
    std::mutex rmu;
    umi::srv::Ring ring_in, ring_out;
    umi::srv::Arena arena{0};
    std::vector<hipEvent_t> event_pool;
    int inflight = 0;  // launched steps not yet finished

    // guarded by mu
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req> waiting;
    bool closing = false, failed = false;
    uint64_t wake = 0;  // bumped by submits and completions
    umi_server_stats st{};

    // completions, guarded by cmu
    std::mutex cmu;
    std::condition_variable ccv;
    std::deque<umi_server_completion> completions;

    // in-flight steps for the waiter, guarded by wmu
    std::mutex wmu;
    std::condition_variable wcv;
    std::deque<Step*> wait_q;
    bool waiter_stop = false;

    // scheduler-owned state
    std::deque<Group*> to_upload;  // admitted, not uploaded
    std::deque<Group*> uploaded;   // uploaded, not launched

    std::thread scheduler, waiter;
    bool shut = false;
    std::mutex shut_mu;

    // ---------------------------------------------------------------------
    static umi_server_completion completion(const Req& r, umi_status status, double done)
    {
        umi_server_completion c{};
        c.tag = r.tag;
        c.status = (int32_t)status;
        c.admitted = r.admitted;
        c.launched = r.launched;
        c.done = done;
        return c;
    }
    void publish(const std::vector<umi_server_completion>& cs)
    {
        if (cs.empty()) return;
        {
            std::lock_guard<std::mutex> lk(cmu);
            completions.insert(completions.end(), cs.begin(), cs.end());
        }
        ccv.notify_all();
    }

    // The helpers below are called with rmu held.
    hipEvent_t take_event()
    {
        if (!event_pool.empty()) {
            hipEvent_t e = event_pool.back();
            event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            throw std::runtime_error("hipEventCreateWithFlags failed");
        return e;
    }
    void put_event(hipEvent_t e)
    {
        if (e) event_pool.push_back(e);
    }

    void free_staging(Upload* u)
    {
        if (u->staging_freed) return;
        u->staging_freed = true;
        if (u->in_ring) ring_in.release(u->ring_id);
        if (u->oneoff) (void)hipHostFree(u->oneoff);
        u->oneoff = nullptr;
    }
    // a group is done with its upload (its step completed or never ran)
    void group_done(Group* g)
    {
        Upload* u = g->up;
        g->up = nullptr;
        if (!u) return;
        free_staging(u);
        if (--u->groups_left == 0) {
            put_event(u->ev);
            delete u;
        }
    }

    // -- admission --------------------------------------------------------
    // Called with mu held: waiting requests FIFO into contiguous arena ranges;
    // requests admitted together with the same iteration count, in adjacent
    // ranges, form one group within the step limits.
    bool admit(double now)
    {
        bool any = false;
        Group* g = nullptr;
        std::lock_guard<std::mutex> rk(rmu);
        while (!waiting.empty()) {
            Req& r = waiting.front();
            const int64_t off = arena.alloc(r.n);
            if (off < 0) break;  // the head waits for memory: FIFO admission
            r.offset = off;
            r.admitted = now;
            if (g && g->iters == r.iters && g->offset + g->size == off &&
                (int64_t)g->reqs.size() < cfg.max_curves && g->size + r.n <= cfg.max_step_samples) {
                g->size += r.n;
            } else {
                g = new Group();
                g->iters = r.iters;
                g->offset = off;
                g->size = r.n;
                to_upload.push_back(g);
            }
            g->reqs.push_back(r);
            waiting.pop_front();
            any = true;
        }
        st.arena_used = arena.used();
        st.arena_high_water = std::max(st.arena_high_water, arena.used());
        return any;
    }

    // -- upload -------------------------------------------------------------
    // Stage the groups at the head of to_upload (at most two steps' worth
    // ahead of launch) into one block: each group's times, then its fluxes;
    // one batched host copy fills it, one copy-kernel call uploads it.
    bool upload(double* t_copy, double* t_enq)
    {
        int64_t staged = 0;
        for (Group* g : uploaded) staged += g->size;
        std::vector<Group*> gs;
        int64_t bytes = 0;
        const int64_t align = umi::srv::Ring::kAlign;
        for (Group* g : to_upload) {
            if (!(gs.empty() && uploaded.empty()) && staged >= 2 * cfg.max_step_samples) break;
            gs.push_back(g);
            staged += g->size;
            bytes += (12 * g->size + align - 1) / align * align;
        }
        if (gs.empty()) return false;
        Upload* u = new Upload();
        int64_t off = 0;
        uint8_t* base = nullptr;
        {
            std::lock_guard<std::mutex> rk(rmu);
            if (gs.size() > 1 && !ring_in.alloc(bytes, &u->ring_id, &off)) {
                // not all of them fit now: the first alone
                gs.resize(1);
                bytes = (12 * gs[0]->size + align - 1) / align * align;
            } else if (gs.size() > 1) {
                u->in_ring = true;
            }
            if (!u->in_ring && ring_in.alloc(bytes, &u->ring_id, &off)) u->in_ring = true;
        }
        if (u->in_ring) {
            base = ring_in.base + off;
        } else if (bytes > ring_in.size) {
            // larger than the whole ring (a lone oversize request): a one-off block
            void* p = nullptr;
            if (hipHostMalloc(&p, (size_t)bytes, hipHostMallocDefault) != hipSuccess) {
                delete u;
                throw std::runtime_error("pinned staging allocation failed");
            }
            u->oneoff = static_cast<uint8_t*>(p);
            base = u->oneoff;
            if (hipHostGetDevicePointer(reinterpret_cast<void**>(&u->oneoff_dev), p, 0) !=
                hipSuccess) {
                (void)hipHostFree(p);
                delete u;
                throw std::runtime_error("pinned staging has no device address");
            }
            std::lock_guard<std::mutex> lk(mu);
            ++st.staging_fallbacks;
        } else {
            delete u;  // the ring is full: wait for steps to complete
            return false;
        }
        const double t0 = umi::srv::now_s();
        std::vector<void*> dst;
        std::vector<const void*> src;
        std::vector<int64_t> nb;
        std::vector<uint8_t*> hd;
        std::vector<const uint8_t*> hs;
        std::vector<int64_t> hn;
        // the copy kernel reads the block at its device address
        uint8_t* const dbase = u->in_ring ? ring_in.dev + off : u->oneoff_dev;
        int64_t gbase = 0;
        for (Group* g : gs) {
            uint8_t* b = base + gbase;
            const uint8_t* db = dbase + gbase;
            int64_t pos = 0;
            for (const Req& r : g->reqs) {
                if (r.time) {
                    dst.push_back(b + 8 * pos);
                    src.push_back(r.time);
                    nb.push_back(8 * r.n);
                } else {
                    std::memset(b + 8 * pos, 0, (size_t)(8 * r.n));  // no gap information
                }
                dst.push_back(b + 8 * g->size + 4 * pos);
                src.push_back(r.flux);
                nb.push_back(4 * r.n);
                pos += r.n;
            }
            hd.push_back(reinterpret_cast<uint8_t*>(time + g->offset));
            hs.push_back(db);
            hn.push_back(8 * g->size);
            hd.push_back(reinterpret_cast<uint8_t*>(flux + g->offset));
            hs.push_back(db + 8 * g->size);
            hn.push_back(4 * g->size);
            gbase += (12 * g->size + align - 1) / align * align;
        }
        if (umi_host_copy_many(dst.data(), src.data(), nb.data(), (int64_t)dst.size(),
                               cfg.copy_threads) != UMI_OK) {
            std::lock_guard<std::mutex> rk(rmu);
            free_staging(u);
            delete u;
            throw std::runtime_error("staging copy failed");
        }
        const double t1 = umi::srv::now_s();
        {
            std::lock_guard<std::mutex> rk(rmu);
            u->ev = take_event();
        }
        if (umi::enqueue_copy_list(hd.data(), hs.data(), hn.data(), (int64_t)hd.size(),
                                   up_stream) != hipSuccess ||
            hipEventRecord(u->ev, up_stream) != hipSuccess) {
            (void)hipStreamSynchronize(up_stream);
            std::lock_guard<std::mutex> rk(rmu);
            put_event(u->ev);
            free_staging(u);
            delete u;
            throw std::runtime_error("upload enqueue failed");
        }
        *t_copy += t1 - t0;
        *t_enq += umi::srv::now_s() - t1;
        u->groups_left = (int)gs.size();
        for (Group* g : gs) {
            g->up = u;
            uploaded.push_back(g);
            to_upload.pop_front();
        }
        return true;
    }

    // -- launch -------------------------------------------------------------
    // The oldest uploaded group's iteration count, and every uploaded group
    // with it, up to the step limits.
    Step* next_step()
    {
        if (uploaded.empty()) return nullptr;
        const int32_t iters = uploaded.front()->iters;
        Step* s = new Step();
        std::deque<Group*> rest;
        for (Group* g : uploaded) {
            if (g->iters == iters && s->curves + (int64_t)g->reqs.size() <= cfg.max_curves &&
                (s->groups.empty() || s->samples + g->size <= cfg.max_step_samples)) {
                s->groups.push_back(g);
                s->curves += (int64_t)g->reqs.size();
                s->samples += g->size;
            } else {
                rest.push_back(g);
            }
        }
        uploaded.swap(rest);
        return s;
    }

    // Fail a step that did not (completely) run: its requests complete with
    // `status` once the device is done with their memory.
    void fail_step(Step* s, umi_status status)
    {
        (void)hipStreamSynchronize(up_stream);
        (void)hipStreamSynchronize(compute);
        (void)hipStreamSynchronize(down_stream);
        const double now = umi::srv::now_s();
        std::vector<umi_server_completion> cs;
        int64_t used;
        {
            std::lock_guard<std::mutex> rk(rmu);
            for (Group* g : s->groups) {
                for (const Req& r : g->reqs) cs.push_back(completion(r, status, now));
                arena.release(g->offset, g->size);
                group_done(g);
                delete g;
            }
            if (s->out_in_ring) ring_out.release(s->out_id);
            if (s->out_oneoff) (void)hipHostFree(s->out_oneoff);
            put_event(s->computed);
            put_event(s->done);
            used = arena.used();
        }
        publish(cs);
        std::lock_guard<std::mutex> lk(mu);
        st.failed += s->curves;
        st.arena_used = used;
        delete s;
    }

    void launch(Step* s, double* t_plan)
    {
        const double t0 = umi::srv::now_s();
        std::vector<int64_t> offs, lens;
        std::vector<int32_t> Ws;
        std::vector<float> al, cs;
        offs.reserve((size_t)s->curves);
        for (Group* g : s->groups) {
            for (Req& r : g->reqs) {
                r.launched = t0;
                offs.push_back(r.offset);
                lens.push_back(r.n);
                Ws.push_back(r.W);
                al.push_back(r.alpha);
                cs.push_back(r.c);
            }
        }
        s->launched = t0;
        hipEvent_t last = nullptr;
        for (Group* g : s->groups) {  // groups uploaded together share one event
            if (g->up->ev != last && hipStreamWaitEvent(compute, g->up->ev, 0) != hipSuccess) {
                fail_step(s, UMI_ERR_DEVICE);
                return;
            }
            last = g->up->ev;
        }
        umi_options o;
        std::memset(&o, 0, sizeof o);
        o.alpha = al.data();
        o.c = cs.data();
        umi_status stt = umi_plan_run_ex(plan, offs.data(), lens.data(), Ws.data(),
                                         (int64_t)offs.size(), al[0], cs[0],
                                         s->groups[0]->iters, &o);
        if (stt != UMI_OK) {
            fail_step(s, stt);
            return;
        }
        // the result block, and the download of every group's trend into it
        const int64_t bytes = 4 * s->samples;
        int64_t off = 0;
        uint8_t* out_dev = nullptr;  // the result block's device address
        {
            std::lock_guard<std::mutex> rk(rmu);
            s->out_in_ring = ring_out.alloc(bytes, &s->out_id, &off);
        }
        if (s->out_in_ring) {
            s->out_base = ring_out.base + off;
            out_dev = ring_out.dev + off;
        } else {
            void* p = nullptr;  // larger than the free ring: a one-off block
            if (hipHostMalloc(&p, (size_t)std::max<int64_t>(bytes, 1), hipHostMallocDefault) !=
                hipSuccess) {
                fail_step(s, UMI_ERR_NO_MEMORY);
                return;
            }
            s->out_oneoff = static_cast<uint8_t*>(p);
            s->out_base = s->out_oneoff;
            if (hipHostGetDevicePointer(reinterpret_cast<void**>(&out_dev), p, 0) != hipSuccess) {
                fail_step(s, UMI_ERR_DEVICE);
                return;
            }
            std::lock_guard<std::mutex> lk(mu);
            ++st.staging_fallbacks;
        }
        std::vector<uint8_t*> d;
        std::vector<const uint8_t*> src;
        std::vector<int64_t> nb;
        int64_t pos = 0;
        for (Group* g : s->groups) {
            s->out_pos.push_back(pos);
            d.push_back(out_dev + pos);
            src.push_back(reinterpret_cast<const uint8_t*>(trend + g->offset));
            nb.push_back(4 * g->size);
            pos += 4 * g->size;
        }
        try {
            std::lock_guard<std::mutex> rk(rmu);
            s->computed = take_event();
            s->done = take_event();
        } catch (...) {
            fail_step(s, UMI_ERR_DEVICE);
            return;
        }
        if (hipEventRecord(s->computed, compute) != hipSuccess ||
            hipStreamWaitEvent(down_stream, s->computed, 0) != hipSuccess ||
            umi::enqueue_copy_list(d.data(), src.data(), nb.data(), (int64_t)d.size(),
                                   down_stream) != hipSuccess ||
            hipEventRecord(s->done, down_stream) != hipSuccess) {
            fail_step(s, UMI_ERR_DEVICE);
            return;
        }
        *t_plan += umi::srv::now_s() - t0;
        {
            std::lock_guard<std::mutex> lk(mu);
            st.steps += 1;
            st.step_curves += s->curves;
            st.largest_step_samples = std::max(st.largest_step_samples, s->samples);
        }
        {
            std::lock_guard<std::mutex> rk(rmu);
            ++inflight;
        }
        {
            std::lock_guard<std::mutex> lk(wmu);
            wait_q.push_back(s);  // the waiter owns the step from here on
        }
        wcv.notify_one();
    }

    int inflight_count()
    {
        std::lock_guard<std::mutex> rk(rmu);
        return inflight;
    }

    // -- completion (waiter thread) -------------------------------------------
    // The step's device work is done (`device` is its completion event's
    // status): copy every result into its request's output (on a copy pool of
    // its own, so these copies never wait for the scheduler's staging copies),
    // release the step's memory, report its completions.
    void finish(Step* s, umi_status device)
    {
        const double t0 = umi::srv::now_s();
        std::vector<void*> d;
        std::vector<const void*> src;
        std::vector<int64_t> nb;
        for (size_t gi = 0; gi < s->groups.size(); ++gi) {
            const uint8_t* b = s->out_base + s->out_pos[gi];
            int64_t pos = 0;
            for (const Req& r : s->groups[gi]->reqs) {
                d.push_back(r.out);
                src.push_back(b + 4 * pos);
                nb.push_back(4 * r.n);
                pos += r.n;
            }
        }
        const umi_status cs =
            device != UMI_OK ? device
                             : umi::host_copy_many(1, d.data(), src.data(), nb.data(),
                                                   (int64_t)d.size(), cfg.copy_threads);
        const double now = umi::srv::now_s();
        int64_t samples = 0, used;
        std::vector<umi_server_completion> done;
        done.reserve((size_t)s->curves);
        {
            std::lock_guard<std::mutex> rk(rmu);
            for (Group* g : s->groups) {
                for (const Req& r : g->reqs) {
                    done.push_back(completion(r, cs, now));
                    samples += r.n;
                }
                arena.release(g->offset, g->size);
                group_done(g);
                delete g;
            }
            if (s->out_in_ring) ring_out.release(s->out_id);
            if (s->out_oneoff) (void)hipHostFree(s->out_oneoff);
            put_event(s->computed);
            put_event(s->done);
            --inflight;
            used = arena.used();
        }
        publish(done);
        const double t1 = umi::srv::now_s();
        {
            std::lock_guard<std::mutex> lk(mu);
            if (cs == UMI_OK) {
                st.completed += s->curves;
                st.samples += samples;
            } else {
                st.failed += s->curves;
            }
            st.arena_used = used;
            st.exec_s[3] += t1 - t0;
            st.loop_s[0] += t1 - t0;
            ++wake;
        }
        cv.notify_all();
        delete s;
    }

    // Everything waiting, admitted or uploaded and not yet launched fails
    // with `status` (called on a scheduler error, after which the scheduler
    // stops); launched steps are finished by the waiter as usual.
    void fail_all(umi_status status)
    {
        (void)hipStreamSynchronize(up_stream);
        const double now = umi::srv::now_s();
        std::deque<Req> w;
        {
            std::lock_guard<std::mutex> lk(mu);
            failed = true;
            w.swap(waiting);
            st.failed += (int64_t)w.size();
        }
        std::vector<umi_server_completion> cs;
        for (const Req& r : w) cs.push_back(completion(r, status, now));
        int64_t n = 0, used;
        {
            std::lock_guard<std::mutex> rk(rmu);
            auto drop = [&](Group* g) {
                for (const Req& r : g->reqs) cs.push_back(completion(r, status, now));
                n += (int64_t)g->reqs.size();
                arena.release(g->offset, g->size);
                group_done(g);
                delete g;
            };
            for (Group* g : to_upload) drop(g);
            for (Group* g : uploaded) drop(g);
            used = arena.used();
        }
        to_upload.clear();
        uploaded.clear();
        publish(cs);
        std::lock_guard<std::mutex> lk(mu);
        st.failed += n;
        st.arena_used = used;
    }

    // -- threads ------------------------------------------------------------
    void waiter_loop()
    {
        (void)hipSetDevice(device);
        for (;;) {
            Step* s = nullptr;
            {
                std::unique_lock<std::mutex> lk(wmu);
                wcv.wait(lk, [&] { return waiter_stop || !wait_q.empty(); });
                if (wait_q.empty()) return;  // stopping, nothing left
                s = wait_q.front();
                wait_q.pop_front();
            }
            const hipError_t e = hipEventSynchronize(s->done);
            finish(s, e == hipSuccess ? UMI_OK : UMI_ERR_DEVICE);
        }
    }

    void scheduler_loop()
    {
        (void)hipSetDevice(device);
        using umi::srv::now_s;
        try {
            for (;;) {
                const double t1 = now_s();
                double tc = 0.0, te = 0.0, tp = 0.0;
                bool progress = false;
                uint64_t seen;
                bool stop = false;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    seen = wake;
                    progress |= admit(t1);
                    stop = closing && waiting.empty();
                }
                const double t2 = now_s();
                while (upload(&tc, &te)) progress = true;
                const double t3 = now_s();
                while (!uploaded.empty() && inflight_count() < cfg.max_inflight) {
                    launch(next_step(), &tp);
                    progress = true;
                }
                const double t4 = now_s();
                {
                    std::lock_guard<std::mutex> lk(mu);
                    st.loop_s[1] += t2 - t1;
                    st.loop_s[2] += t3 - t2;
                    st.loop_s[3] += t4 - t3;
                    st.exec_s[0] += tc;
                    st.exec_s[1] += te;
                    st.exec_s[2] += tp;
                    if (t4 - t1 > st.longest_iteration_s) {
                        st.longest_iteration_s = t4 - t1;
                        st.longest_iteration_loop_s[0] = 0.0;
                        st.longest_iteration_loop_s[1] = t2 - t1;
                        st.longest_iteration_loop_s[2] = t3 - t2;
                        st.longest_iteration_loop_s[3] = t4 - t3;
                    }
                }
                const bool idle =
                    uploaded.empty() && to_upload.empty() && inflight_count() == 0;
                if (stop && idle) break;
                if (progress) continue;
                std::unique_lock<std::mutex> lk(mu);
                cv.wait_until(lk, umi::srv::deadline(idle ? 0.05 : 0.002),
                              [&] { return wake != seen; });
            }
        } catch (const std::exception&) {
            fail_all(UMI_ERR_DEVICE);
        }
    }

    void release_all()
    {
        if (plan) (void)umi_plan_destroy(plan);
        plan = nullptr;
        for (hipStream_t* s : {&up_stream, &compute, &down_stream})
            if (*s) {
                (void)hipStreamSynchronize(*s);
                (void)hipStreamDestroy(*s);
                *s = nullptr;
            }
        for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
        event_pool.clear();
        if (ring_in.base) (void)hipHostFree(ring_in.base);
        if (ring_out.base) (void)hipHostFree(ring_out.base);
        ring_in.base = ring_out.base = nullptr;
        if (flux) (void)hipFree(flux);
        if (time) (void)hipFree(time);
        if (trend) (void)hipFree(trend);
        flux = nullptr;
        time = nullptr;
        trend = nullptr;
    }

    void shutdown()
    {
        std::lock_guard<std::mutex> one(shut_mu);
        if (shut) return;
        shut = true;
        {
            std::lock_guard<std::mutex> lk(mu);
            closing = true;
            ++wake;
        }
        cv.notify_all();
        if (scheduler.joinable()) scheduler.join();
        {
            std::lock_guard<std::mutex> lk(wmu);
            waiter_stop = true;
        }
        wcv.notify_all();
        if (waiter.joinable()) waiter.join();
        int prev = 0;
        const bool restore = hipGetDevice(&prev) == hipSuccess;
        (void)hipSetDevice(device);
        release_all();
        if (restore) (void)hipSetDevice(prev);
    }
};

static_assert(sizeof(umi_server_config) == 48, "umi_server_config layout");
static_assert(sizeof(umi_server_completion) == 40, "umi_server_completion layout");
static_assert(sizeof(umi_server_stats) == 200, "umi_server_stats layout");

extern "C" {

umi_status umi_server_create(const umi_server_config* config, umi_server** out)
{
    using umi::report_error;
    if (!out) return report_error(UMI_ERR_INVALID_ARG, "umi_server_create: out is NULL");
    *out = nullptr;
    if (!config) return report_error(UMI_ERR_INVALID_ARG, "umi_server_create: config is NULL");
    umi_server_config c = *config;
    if (c.max_step_samples == 0) c.max_step_samples = int64_t(1) << 22;
    if (c.staging_bytes == 0) c.staging_bytes = int64_t(4) << 30;
    if (c.max_curves == 0) c.max_curves = 4096;
    if (c.max_W == 0) c.max_W = 721;
    if (c.max_inflight == 0) c.max_inflight = 2;
    if (c.copy_threads == 0) c.copy_threads = 4;
    if (c.capacity <= 0 || c.max_step_samples < 1 || c.staging_bytes < 1 << 20 ||
        c.max_curves < 1 || c.max_W < 1 || (c.max_W & 1) == 0 || c.max_W > UMI_MAX_WINDOW ||
        c.max_inflight < 1 || c.max_inflight > 8 || c.copy_threads < 1 ||
        c.copy_threads > UMI_HOST_COPY_MAX_THREADS || c.device < 0 || c.reserved != 0)
        return report_error(UMI_ERR_INVALID_ARG, "umi_server_create: config field out of range");
    umi_server* s = new umi_server();
    s->cfg = c;
    s->device = c.device;
    s->arena = umi::srv::Arena(c.capacity);
    s->st.arena_capacity = c.capacity;
    int prev = 0;
    const bool restore = hipGetDevice(&prev) == hipSuccess;
    hipError_t e = hipSetDevice(c.device);
    umi_status r = UMI_OK;
    auto hip_fail = [&](hipError_t he, const char* what) {
        r = report_error(he == hipErrorOutOfMemory ? UMI_ERR_NO_MEMORY : UMI_ERR_DEVICE,
                         std::string("umi_server_create: ") + what + ": " + hipGetErrorString(he));
    };
    void* p = nullptr;
    if (e != hipSuccess) {
        hip_fail(e, "hipSetDevice");
    } else if ((e = hipMalloc(&p, sizeof(float) * (size_t)c.capacity)) != hipSuccess) {
        hip_fail(e, "arena");
    } else {
        s->flux = static_cast<float*>(p);
        if ((e = hipMalloc(&p, sizeof(double) * (size_t)c.capacity)) != hipSuccess) {
            hip_fail(e, "arena");
        } else {
            s->time = static_cast<double*>(p);
            if ((e = hipMalloc(&p, sizeof(float) * (size_t)c.capacity)) != hipSuccess) {
                hip_fail(e, "arena");
            } else {
                s->trend = static_cast<float*>(p);
            }
        }
    }
    if (r == UMI_OK) {
        const int64_t out_bytes = std::max<int64_t>(c.staging_bytes / 3, 1 << 20);
        if ((e = hipHostMalloc(&p, (size_t)c.staging_bytes, hipHostMallocDefault)) != hipSuccess) {
            hip_fail(e, "pinned staging");
        } else {
            s->ring_in.base = static_cast<uint8_t*>(p);
            s->ring_in.size = c.staging_bytes;
            if ((e = hipHostGetDevicePointer(reinterpret_cast<void**>(&s->ring_in.dev), p, 0)) !=
                hipSuccess) {
                hip_fail(e, "pinned staging device address");
            } else if ((e = hipHostMalloc(&p, (size_t)out_bytes, hipHostMallocDefault)) !=
                       hipSuccess) {
                hip_fail(e, "pinned results");
            } else {
                s->ring_out.base = static_cast<uint8_t*>(p);
                s->ring_out.size = out_bytes;
                if ((e = hipHostGetDevicePointer(reinterpret_cast<void**>(&s->ring_out.dev), p,
                                                 0)) != hipSuccess)
                    hip_fail(e, "pinned results device address");
            }
        }
    }
    for (hipStream_t* st : {&s->up_stream, &s->compute, &s->down_stream}) {
        if (r != UMI_OK) break;
        if ((e = hipStreamCreateWithFlags(st, hipStreamNonBlocking)) != hipSuccess)
            hip_fail(e, "stream");
    }
    if (r == UMI_OK)
        r = umi_plan_create(&s->plan, c.capacity, c.max_curves, c.max_W, s->flux, s->time,
                            s->trend, nullptr, s->compute);
    if (r == UMI_OK) {
        try {
            s->scheduler = std::thread(&umi_server::scheduler_loop, s);
            s->waiter = std::thread(&umi_server::waiter_loop, s);
        } catch (...) {
            r = report_error(UMI_ERR_NO_MEMORY, "umi_server_create: cannot start threads");
        }
    }
    if (r != UMI_OK) {
        s->shutdown();
        delete s;
    } else {
        *out = s;
    }
    if (restore) (void)hipSetDevice(prev);
    return r;
}

umi_status umi_server_submit(umi_server* s, const float* flux, const double* time, int64_t n,
                             int32_t W, float alpha, float c, int32_t iters, double arrival,
                             float* out, uint64_t tag)
{
    using umi::report_error;
    if (!s) return report_error(UMI_ERR_INVALID_ARG, "umi_server_submit: server is NULL");
    if (W < 1 || (W & 1) == 0 || W > s->cfg.max_W)
        return report_error(UMI_ERR_INVALID_ARG, "umi_server_submit: W must be odd, 1 <= W <= " +
                                                     std::to_string(s->cfg.max_W));
    if (!(std::isfinite(alpha) && alpha > 0.0f && std::isfinite(c) && c > 0.0f))
        return report_error(UMI_ERR_INVALID_ARG,
                            "umi_server_submit: alpha and c must be finite and > 0");
    if (iters < 0) return report_error(UMI_ERR_INVALID_ARG, "umi_server_submit: iters < 0");
    if (n < 0 || n > s->cfg.capacity)
        return report_error(UMI_ERR_INVALID_ARG,
                            "umi_server_submit: n must be in [0, capacity]");
    if (n > 0 && (!flux || !out))
        return report_error(UMI_ERR_INVALID_ARG, "umi_server_submit: flux and out must not be NULL");
    umi::srv::Req r;
    r.tag = tag;
    r.flux = flux;
    r.time = time;
    r.out = out;
    r.n = n;
    r.W = W;
    r.alpha = alpha;
    r.c = c;
    r.iters = iters;
    const double now = umi::srv::now_s();
    r.arrival = arrival < 0.0 ? now : arrival;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->closing || s->failed)
            return report_error(UMI_ERR_INVALID_ARG, "umi_server_submit: server is shutting down");
        ++s->st.submitted;
        if (n > 0) {
            s->waiting.push_back(r);
            ++s->wake;
        }
    }
    if (n == 0) {
        r.admitted = r.launched = now;
        s->publish({umi_server::completion(r, UMI_OK, now)});
        std::lock_guard<std::mutex> lk(s->mu);
        ++s->st.completed;
        return UMI_OK;
    }
    s->cv.notify_all();
    return UMI_OK;
}

umi_status umi_server_poll(umi_server* s, umi_server_completion* out, int32_t max,
                           double timeout_s, int32_t* n_out)
{
    using umi::report_error;
    if (!s || !n_out || max < 0 || (max > 0 && !out) || !(timeout_s >= 0.0))
        return report_error(UMI_ERR_INVALID_ARG, "umi_server_poll: bad argument");
    *n_out = 0;
    std::unique_lock<std::mutex> lk(s->cmu);
    if (s->completions.empty() && timeout_s > 0.0)
        s->ccv.wait_until(lk, umi::srv::deadline(std::min(timeout_s, 1e6)),
                          [&] { return !s->completions.empty(); });
    int32_t k = 0;
    while (k < max && !s->completions.empty()) {
        out[k++] = s->completions.front();
        s->completions.pop_front();
    }
    *n_out = k;
    return UMI_OK;
}

umi_status umi_server_stats_get(umi_server* s, umi_server_stats* out)
{
    if (!s || !out) return umi::report_error(UMI_ERR_INVALID_ARG, "umi_server_stats_get: NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    return UMI_OK;
}

umi_status umi_server_reset_stats(umi_server* s)
{
    if (!s) return umi::report_error(UMI_ERR_INVALID_ARG, "umi_server_reset_stats: NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    umi_server_stats z{};
    z.arena_capacity = s->st.arena_capacity;
    z.arena_used = s->st.arena_used;
    z.arena_high_water = s->st.arena_used;
    s->st = z;
    return UMI_OK;
}

umi_status umi_server_shutdown(umi_server* s)
{
    if (!s) return umi::report_error(UMI_ERR_INVALID_ARG, "umi_server_shutdown: NULL");
    s->shutdown();
    return UMI_OK;
}

umi_status umi_server_destroy(umi_server* s)
{
    if (!s) return UMI_OK;
    s->shutdown();
    delete s;
    return UMI_OK;
}

}  // extern "C"
