// fd_serve.cpp -- continuous-batching shot server of libfd.
//
// The server owns a device arena of hbm_budget_bytes and two host threads.
// Submitted requests wait in FIFO order.  The admission thread admits the
// head request as soon as a slot is free and a first-fit block of the arena
// can hold its footprint (its grid workspace, velocity, wavelets and
// traces), uploads its inputs and creates its grid on the request's own
// stream, and hands it to the scheduler; it also finishes completed
// requests (traces copied out, block returned to the arena, ticket
// signalled), which may admit the next one.  The scheduler thread only
// enqueues: each round it enqueues the next chunk of steps of every resident
// request whose previous chunk has completed (an event per request), so the
// device interleaves the kernels of all resident shots, and neither an
// admission (host-to-device copies, grid set-up, which synchronises the new
// request's stream) nor a completion stalls the shots already running.
// With the shortest-work policy the scheduler keeps at most two chunks on
// the device, both for the resident request with the fewest remaining
// point-steps (preemptive shortest remaining work first, at chunk
// granularity): a shot large enough to fill the GPU gains nothing from
// sharing it, equal shares delay every shot, and this order lets short
// shots pass long ones.  The response-ratio policy orders the same way by
// (age + remaining time) / remaining time instead (highest response ratio
// next, preemptive at chunk granularity; the remaining time is the remaining
// point-steps over the device's measured rate): a short request still goes
// first, but a long one that has waited long enough is no longer passed, so
// the tail does not grow.  Each request runs the same kernels with the same
// launch geometry as a lone fd_forward, so its result does not depend on the
// mix it ran in or the policy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fd.h"
#include "fd_api_internal.h"

namespace {

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// First-fit allocator over [0, size) with coalescing of free blocks.
class Arena {
  public:
    explicit Arena(size_t size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align_up(bytes, 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(bytes, 256);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
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
    }
    size_t used() const { return used_; }

  private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

struct Footprint {
    size_t grid, vp, wav, rec, total;
};

Footprint footprint(const fd_request *r) {
    Footprint f{};
    size_t gb = 0;
    if (fd_grid_workspace_bytes(&r->grid, &gb) != FD_OK) return f;
    long long phys = 1;
    for (int a = 0; a < r->grid.ndim; ++a) phys *= r->grid.shape[a];
    f.grid = align_up(gb, 256);
    f.vp = align_up(sizeof(float) * (size_t)phys, 256);
    f.wav = align_up(sizeof(float) * (size_t)r->nt * r->nsrc, 256);
    f.rec = align_up(sizeof(float) * (size_t)r->nt * r->nrec, 256);
    f.total = f.grid + f.vp + f.wav + f.rec;
    return f;
}

struct Req {
    uint64_t ticket = 0;
    fd_grid_desc desc{};
    std::vector<float> vp, wav;
    std::vector<double> src, rec;
    int nsrc = 0, nrec = 0, nt = 0;
    double dt = 0;
    float *rec_out_host = nullptr;
    Footprint fp{};
    // resident state
    size_t off = 0;
    int slot = -1;
    fd_grid *grid = nullptr;
    float *d_wav = nullptr, *d_rec = nullptr;
    double pts = 0;      // padded points of the grid (remaining work = pts * (nt - next_step))
    int next_step = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};   // completion of the chunks in flight, oldest at ev_head
    int ev_steps[2] = {0, 0};                // steps of those chunks
    int ev_head = 0, ev_count = 0;
    fd_result res{};
    std::string msg;   // error message of a failed request
};

}  // namespace

struct fd_server {
    fd_server_desc d{};
    char *arena_base = nullptr;
    Arena *arena = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<bool> slot_busy;
    std::thread scheduler, admitter;
    std::mutex mu;
    std::condition_variable cv_admit, cv_sched, cv_done;
    std::deque<Req *> pending;     // submitted, not admitted (FIFO)
    std::deque<Req *> ready;       // admitted and set up, not yet picked up by the scheduler
    std::deque<Req *> finishing;   // last chunk completed (or failed), to be finished
    int inflight = 0;              // admitted and not yet finished
    std::map<uint64_t, Req *> done;
    std::set<uint64_t> live;   // tickets submitted and not yet collected by fd_wait
    bool stopping = false;
    uint64_t next_ticket = 1;
    size_t peak_bytes = 0;
    int peak_slots = 0;
    std::chrono::steady_clock::time_point t0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    bool drained() const { return stopping && pending.empty() && inflight == 0; }
    void run_scheduler();
    void run_admitter();
    int admit(Req *r);
    void finish(Req *r, int status);
    void to_finishing(Req *r, int status);
};

int fd_server::admit(Req *r) {
    hipStream_t s = streams[r->slot];
    char *base = arena_base + r->off;
    float *d_vp = (float *)(base + r->fp.grid);
    r->d_wav = (float *)(base + r->fp.grid + r->fp.vp);
    r->d_rec = (float *)(base + r->fp.grid + r->fp.vp + r->fp.wav);
    if (hipMemcpyAsync(d_vp, r->vp.data(), sizeof(float) * r->vp.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(r->d_wav, r->wav.data(), sizeof(float) * r->wav.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        return fdi_fail(FD_ERR_DEVICE, "request upload failed");
    int rc = fd_grid_create(&r->desc, base, r->fp.grid, d_vp, s, &r->grid);
    if (rc) return rc;
    fd_shot sh{r->nsrc, r->src.data(), r->d_wav, r->nrec, r->rec.data()};
    if ((rc = fdi_forward_prepare(r->grid, &sh, r->nt, r->dt, s))) return rc;
    if ((rc = fdi_forward_zero_state(r->grid, s))) return rc;
    for (hipEvent_t &e : r->ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return fdi_fail(FD_ERR_DEVICE, "event creation failed");
    fd_grid_info info;
    fd_grid_get_info(r->grid, &info);
    r->pts = (double)info.padded_points;
    r->next_step = 0;
    return FD_OK;
}

void fd_server::finish(Req *r, int status) {
    // (a failure reported by the scheduler thread carries its message already;
    // the error text is thread-local)
    if (status != FD_OK && r->msg.empty()) r->msg = fd_last_error();
    if (r->grid && status == FD_OK) {
        hipStream_t s = streams[r->slot];
        if (hipMemcpyAsync(r->rec_out_host, r->d_rec, sizeof(float) * (size_t)r->nt * r->nrec,
                           hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            status = FD_ERR_DEVICE;
    } else if (r->slot >= 0) {
        (void)hipStreamSynchronize(streams[r->slot]);
    }
    if (r->grid) fd_grid_destroy(r->grid);
    r->grid = nullptr;
    for (hipEvent_t &e : r->ev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (r->slot >= 0) {
        arena->release(r->off, r->fp.total);
        slot_busy[r->slot] = false;
        r->slot = -1;
        --inflight;
        cv_sched.notify_all();   // (drain check of a stopping scheduler)
    }
    r->res.status = status;
    r->res.t_done = now();
    r->res.bytes_reserved = r->fp.total;
    r->vp.clear();
    r->vp.shrink_to_fit();
    r->wav.clear();
    r->wav.shrink_to_fit();
    done[r->ticket] = r;
    cv_done.notify_all();
}

// Hand a request whose run ended (status FD_OK after its last chunk, or an
// error) to the admission thread, which finishes it.
void fd_server::to_finishing(Req *r, int status) {
    if (status != FD_OK) r->msg = fd_last_error();
    r->res.status = status;
    std::lock_guard<std::mutex> lk(mu);
    finishing.push_back(r);
    cv_admit.notify_all();
}

void fd_server::run_admitter() {
    (void)hipSetDevice(d.device);
    for (;;) {
        Req *fin = nullptr, *adm = nullptr, *rej = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (!finishing.empty()) {
                    fin = finishing.front();
                    finishing.pop_front();
                    break;
                }
                if (!pending.empty()) {
                    Req *r = pending.front();
                    if (r->fp.total > d.hbm_budget_bytes || r->fp.total == 0) {
                        pending.pop_front();
                        rej = r;
                        break;
                    }
                    // FIFO: the head waits for a slot and for arena space
                    size_t off = 0;
                    if (inflight < d.max_slots && arena->alloc(r->fp.total, &off)) {
                        int slot = -1;
                        for (int i = 0; i < d.max_slots; ++i)
                            if (!slot_busy[i]) {
                                slot = i;
                                break;
                            }
                        slot_busy[slot] = true;
                        r->off = off;
                        r->slot = slot;
                        r->res.t_start = now();
                        pending.pop_front();
                        ++inflight;
                        peak_bytes = std::max(peak_bytes, arena->used());
                        peak_slots = std::max(peak_slots, inflight);
                        adm = r;
                        break;
                    }
                }
                if (drained()) {
                    cv_sched.notify_all();
                    return;
                }
                cv_admit.wait(lk);
            }
        }
        if (fin) {
            finish(fin, fin->res.status);
        } else if (rej) {
            finish(rej, fdi_fail(FD_ERR_NOMEM, "request needs %zu bytes > budget", rej->fp.total));
        } else if (adm) {
            const int rc = admit(adm);
            if (rc) {
                finish(adm, rc);
            } else {
                std::lock_guard<std::mutex> lk(mu);
                ready.push_back(adm);
                cv_sched.notify_all();
            }
        }
    }
}

void fd_server::run_scheduler() {
    (void)hipSetDevice(d.device);
    const int chunk = d.steps_per_round > 0 ? d.steps_per_round : 50;
    std::vector<Req *> active;
    // device rate in point-steps per second, from the completion times of
    // chunks while the device is busy (the first chunk after an idle period
    // is timed from its enqueue)
    double rate = 0.0, t_prev = -1.0;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            if (active.empty()) cv_sched.wait(lk, [&] { return !ready.empty() || drained(); });
            if (active.empty() && ready.empty() && drained()) return;
            while (!ready.empty()) {
                active.push_back(ready.front());
                ready.pop_front();
            }
        }
        // one round.  Poll the chunks in flight; a request past its last
        // step (or failed) goes to finishing.  Then enqueue: with equal
        // shares, the next chunk of every request whose previous chunk is
        // done; with the shortest-work policy, chunks for the requests with
        // the least remaining point-steps, shortest first, up to two chunks
        // on the device (the shortest request gets both, queued back to back
        // on its stream, so it runs alone but for the tail of its last chunk)
        bool progressed = false;
        for (size_t i = 0; i < active.size();) {
            Req *r = active[i];
            int status = FD_OK;
            while (r->ev_count > 0) {
                const hipError_t q = hipEventQuery(r->ev[r->ev_head]);
                if (q == hipErrorNotReady) break;
                const double t = now();
                if (q == hipSuccess && t_prev >= 0.0 && t > t_prev) {
                    const double sample = r->pts * r->ev_steps[r->ev_head] / (t - t_prev);
                    rate = rate > 0.0 ? 0.8 * rate + 0.2 * sample : sample;
                }
                t_prev = t;
                r->ev_head ^= 1;
                --r->ev_count;
                progressed = true;
                if (q != hipSuccess) {
                    status = fdi_fail(FD_ERR_DEVICE, "request %llu: %s", (unsigned long long)r->ticket,
                                      hipGetErrorString(q));
                    break;
                }
            }
            if (status != FD_OK || (r->ev_count == 0 && r->next_step >= r->nt)) {
                active.erase(active.begin() + (long)i);
                to_finishing(r, status);
                progressed = true;
            } else {
                ++i;
            }
        }
        int on_device = 0;
        for (const Req *r : active) on_device += r->ev_count;
        if (on_device == 0) t_prev = -1.0;   // idle: the next completion is timed from its enqueue
        auto enqueue = [&](Req *r) -> bool {
            if (t_prev < 0.0) t_prev = now();
            hipStream_t s = streams[r->slot];
            fd_shot sh{r->nsrc, r->src.data(), r->d_wav, r->nrec, r->rec.data()};
            const int n1 = std::min(r->nt, r->next_step + chunk);
            int status = fdi_forward_steps(r->grid, &sh, r->nt, r->next_step, n1, r->d_rec, nullptr, 1, s);
            if (status == FD_OK && hipEventRecord(r->ev[(r->ev_head + r->ev_count) & 1], s) != hipSuccess)
                status = fdi_fail(FD_ERR_DEVICE, "event record failed");
            progressed = true;
            if (status != FD_OK) {
                active.erase(std::find(active.begin(), active.end(), r));
                // (chunks already in flight complete before finish() reads the traces)
                to_finishing(r, status);
                return false;
            }
            r->ev_steps[(r->ev_head + r->ev_count) & 1] = n1 - r->next_step;
            r->next_step = n1;
            ++r->ev_count;
            return true;
        };
        if (d.policy == FD_SERVE_SHORTEST || d.policy == FD_SERVE_RATIO) {
            if (d.policy == FD_SERVE_SHORTEST || rate <= 0.0) {
                std::stable_sort(active.begin(), active.end(), [](const Req *x, const Req *y) {
                    return x->pts * (x->nt - x->next_step) < y->pts * (y->nt - y->next_step);
                });
            } else {
                const double t = now();
                auto ratio = [&](const Req *x) {
                    const double rem = x->pts * (x->nt - x->next_step) / rate;   // seconds
                    return rem > 0.0 ? (t - x->res.t_submit + rem) / rem : 1e300;
                };
                std::stable_sort(active.begin(), active.end(),
                                 [&](const Req *x, const Req *y) { return ratio(x) > ratio(y); });
            }
            int budget = 2;
            for (const Req *r : active) budget -= r->ev_count;
            std::vector<Req *> order = active;
            for (Req *r : order) {
                while (budget > 0 && r->ev_count < 2 && r->next_step < r->nt) {
                    if (!enqueue(r)) break;
                    --budget;
                }
                if (budget <= 0) break;
            }
        } else {
            std::vector<Req *> order = active;
            for (Req *r : order)
                if (r->ev_count == 0 && r->next_step < r->nt) enqueue(r);
        }
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

extern "C" int fd_request_bytes(const fd_request *req, size_t *bytes) {
    if (!req || !bytes) return fdi_fail(FD_ERR_ARG, "null argument");
    if (!fdi_check_desc(&req->grid)) return FD_ERR_ARG;
    *bytes = footprint(req).total;
    return FD_OK;
}

extern "C" int fd_server_create(const fd_server_desc *desc, fd_server **out) {
    try {
        if (!desc || !out) return fdi_fail(FD_ERR_ARG, "null argument");
        *out = nullptr;
        if (desc->max_slots < 1 || desc->hbm_budget_bytes < 4096 || desc->steps_per_round < 0)
            return fdi_fail(FD_ERR_ARG, "max_slots >= 1, budget >= 4 KiB, steps_per_round >= 0");
        if (desc->policy != FD_SERVE_SHARE && desc->policy != FD_SERVE_SHORTEST && desc->policy != FD_SERVE_RATIO)
            return fdi_fail(FD_ERR_ARG, "policy must be FD_SERVE_SHARE, FD_SERVE_SHORTEST or FD_SERVE_RATIO");
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || desc->device < 0 || desc->device >= ndev)
            return fdi_fail(FD_ERR_ARG, "no such device %d", desc->device);
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(desc->device);
        fd_server *srv = new fd_server();
        srv->d = *desc;
        srv->t0 = std::chrono::steady_clock::now();
        if (hipMalloc((void **)&srv->arena_base, desc->hbm_budget_bytes) != hipSuccess) {
            delete srv;
            (void)hipSetDevice(prev);
            return fdi_fail(FD_ERR_NOMEM, "arena of %zu bytes", desc->hbm_budget_bytes);
        }
        srv->arena = new Arena(desc->hbm_budget_bytes);
        srv->streams.resize(desc->max_slots);
        srv->slot_busy.assign(desc->max_slots, false);
        for (int i = 0; i < desc->max_slots; ++i) {
            if (hipStreamCreateWithFlags(&srv->streams[i], hipStreamNonBlocking) != hipSuccess) {
                for (int j = 0; j < i; ++j) (void)hipStreamDestroy(srv->streams[j]);
                (void)hipFree(srv->arena_base);
                delete srv->arena;
                delete srv;
                (void)hipSetDevice(prev);
                return fdi_fail(FD_ERR_DEVICE, "stream creation failed");
            }
        }
        (void)hipSetDevice(prev);
        srv->scheduler = std::thread([srv] { srv->run_scheduler(); });
        srv->admitter = std::thread([srv] { srv->run_admitter(); });
        *out = srv;
        return FD_OK;
    } catch (const std::bad_alloc &) {
        return fdi_fail(FD_ERR_NOMEM, "host allocation failed");
    } catch (...) {
        return fdi_fail(FD_ERR_STATE, "internal error");
    }
}

extern "C" int fd_submit(fd_server *srv, const fd_request *req, uint64_t *ticket) {
    try {
        if (!srv || !req || !ticket) return fdi_fail(FD_ERR_ARG, "null argument");
        if (!fdi_check_desc(&req->grid)) return FD_ERR_ARG;
        if (req->grid.storage < FD_STORE_F32 || req->grid.storage > FD_STORE_BF16_DIFF)
            return fdi_fail(FD_ERR_ARG, "storage");
        if (req->nt < 1 || req->nsrc < 1 || req->nrec < 1 || !req->vp_host || !req->src_xyz ||
            !req->rec_xyz || !req->wavelet_host || !req->rec_out_host || !(req->dt > 0.0))
            return fdi_fail(FD_ERR_ARG, "incomplete request");
        Req *r = new Req();
        r->desc = req->grid;
        const int ndim = req->grid.ndim;
        long long phys = 1;
        for (int a = 0; a < ndim; ++a) phys *= req->grid.shape[a];
        if (req->grid.vp_padded) {
            phys = 1;
            for (int a = 0; a < ndim; ++a) phys *= req->grid.shape[a] + 2LL * req->grid.nbl;
        }
        r->vp.assign(req->vp_host, req->vp_host + phys);
        r->wav.assign(req->wavelet_host, req->wavelet_host + (size_t)req->nt * req->nsrc);
        r->src.assign(req->src_xyz, req->src_xyz + (size_t)req->nsrc * ndim);
        r->rec.assign(req->rec_xyz, req->rec_xyz + (size_t)req->nrec * ndim);
        r->nsrc = req->nsrc;
        r->nrec = req->nrec;
        r->nt = req->nt;
        r->dt = req->dt;
        r->rec_out_host = req->rec_out_host;
        r->desc.max_src = std::max(r->desc.max_src, req->nsrc);
        r->desc.max_rec = std::max(r->desc.max_rec, req->nrec);
        fd_request tmp = *req;
        tmp.grid = r->desc;
        r->fp = footprint(&tmp);
        // footprint() sized the velocity for the physical grid; a padded one is larger
        if (req->grid.vp_padded) {
            const size_t vpb = align_up(sizeof(float) * (size_t)phys, 256);
            r->fp.total += vpb - r->fp.vp;
            r->fp.vp = vpb;
        }
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stopping) {
            delete r;
            return fdi_fail(FD_ERR_STATE, "server is shutting down");
        }
        r->ticket = srv->next_ticket++;
        r->res.t_submit = srv->now();
        srv->live.insert(r->ticket);
        srv->pending.push_back(r);
        *ticket = r->ticket;
        srv->cv_admit.notify_all();
        return FD_OK;
    } catch (const std::bad_alloc &) {
        return fdi_fail(FD_ERR_NOMEM, "host allocation failed");
    } catch (...) {
        return fdi_fail(FD_ERR_STATE, "internal error");
    }
}

extern "C" int fd_wait(fd_server *srv, uint64_t ticket, double timeout_s, fd_result *result) {
    if (!srv) return fdi_fail(FD_ERR_ARG, "null server");
    std::unique_lock<std::mutex> lk(srv->mu);
    if (!srv->live.count(ticket))
        return fdi_fail(FD_ERR_ARG, "unknown or already collected ticket %llu", (unsigned long long)ticket);
    // done, or collected meanwhile by another waiter of the same ticket
    auto ready = [&] { return srv->done.count(ticket) > 0 || !srv->live.count(ticket); };
    if (timeout_s < 0) {
        srv->cv_done.wait(lk, ready);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
        return fdi_fail(FD_ERR_TIMEOUT, "ticket %llu not done", (unsigned long long)ticket);
    }
    auto it = srv->done.find(ticket);
    if (it == srv->done.end())
        return fdi_fail(FD_ERR_STATE, "ticket %llu collected by another waiter", (unsigned long long)ticket);
    Req *r = it->second;
    srv->done.erase(it);
    srv->live.erase(ticket);
    srv->cv_done.notify_all();
    if (result) *result = r->res;
    const int st = r->res.status;
    const std::string msg = r->msg;
    delete r;
    return st == FD_OK ? FD_OK
                       : fdi_fail(st, "request %llu failed: %s", (unsigned long long)ticket, msg.c_str());
}

extern "C" int fd_server_stats(fd_server *srv, size_t *peak_bytes, int *peak_slots) {
    if (!srv) return fdi_fail(FD_ERR_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (peak_bytes) *peak_bytes = srv->peak_bytes;
    if (peak_slots) *peak_slots = srv->peak_slots;
    return FD_OK;
}

extern "C" int fd_server_destroy(fd_server *srv) {
    if (!srv) return FD_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
        srv->cv_admit.notify_all();
        srv->cv_sched.notify_all();
    }
    if (srv->admitter.joinable()) srv->admitter.join();
    if (srv->scheduler.joinable()) srv->scheduler.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(srv->d.device);
    for (auto s : srv->streams) (void)hipStreamDestroy(s);
    (void)hipFree(srv->arena_base);
    (void)hipSetDevice(prev);
    for (auto &kv : srv->done) delete kv.second;
    delete srv->arena;
    delete srv;
    return FD_OK;
}
