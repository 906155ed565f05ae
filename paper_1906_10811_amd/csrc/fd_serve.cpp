// fd_serve.cpp -- continuous-batching shot server of libfd.
//
// One scheduler thread owns a device arena of hbm_budget_bytes.  Submitted
// requests wait in FIFO order; a request is admitted as soon as a slot is
// free and a first-fit block of the arena can hold its footprint (its grid
// workspace, wavelets and traces).  Every admitted request keeps its
// wavefields resident on its own stream; each scheduler round enqueues the
// next chunk of steps of every resident request, so the device interleaves
// the kernels of all resident shots, and a request arriving while others run
// starts without waiting for them to finish.  Completion is detected with
// events; the traces are copied out, the block is returned to the arena and
// the ticket is signalled.  Each request runs the same kernels with the same
// launch geometry as a lone fd_forward, so its result does not depend on the
// mix it ran in.
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
    int next_step = 0;
    hipEvent_t ev = nullptr;
    bool ev_pending = false;
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
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req *> pending;
    std::vector<Req *> active;
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
    void run();
    int admit(Req *r);
    void finish(Req *r, int status);
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
    if (hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess)
        return fdi_fail(FD_ERR_DEVICE, "event creation failed");
    r->next_step = 0;
    return FD_OK;
}

void fd_server::finish(Req *r, int status) {
    if (status != FD_OK) r->msg = fd_last_error();
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
    if (r->ev) (void)hipEventDestroy(r->ev);
    r->ev = nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if (r->slot >= 0) {
        arena->release(r->off, r->fp.total);
        slot_busy[r->slot] = false;
        r->slot = -1;
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

void fd_server::run() {
    (void)hipSetDevice(d.device);
    const int chunk = d.steps_per_round > 0 ? d.steps_per_round : 50;
    for (;;) {
        std::vector<Req *> admitted, rejected;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (active.empty() && pending.empty()) {
                if (stopping) return;
                cv_work.wait(lk, [&] { return stopping || !pending.empty(); });
                if (pending.empty() && stopping) return;
            }
            // admission: FIFO, by slot and by arena space
            while (!pending.empty()) {
                Req *r = pending.front();
                if (r->fp.total > d.hbm_budget_bytes || r->fp.total == 0) {
                    pending.pop_front();
                    rejected.push_back(r);
                    continue;
                }
                if ((int)active.size() >= d.max_slots) break;
                size_t off = 0;
                if (!arena->alloc(r->fp.total, &off)) break;
                int slot = -1;
                for (int i = 0; i < d.max_slots; ++i)
                    if (!slot_busy[i]) { slot = i; break; }
                slot_busy[slot] = true;
                r->off = off;
                r->slot = slot;
                r->res.t_start = now();
                pending.pop_front();
                active.push_back(r);
                admitted.push_back(r);
                peak_bytes = std::max(peak_bytes, arena->used());
                peak_slots = std::max(peak_slots, (int)active.size());
            }
        }
        for (Req *r : rejected) finish(r, fdi_fail(FD_ERR_NOMEM, "request needs %zu bytes > budget", r->fp.total));
        for (Req *r : admitted) {
            int rc = admit(r);
            if (rc) {
                {
                    std::lock_guard<std::mutex> lk(mu);
                    active.erase(std::find(active.begin(), active.end(), r));
                }
                finish(r, rc);
            }
        }
        // one round: next chunk of every resident request whose previous chunk is done
        bool progressed = !admitted.empty();
        std::vector<Req *> act;
        {
            std::lock_guard<std::mutex> lk(mu);
            act = active;
        }
        for (Req *r : act) {
            if (r->ev_pending) {
                const hipError_t q = hipEventQuery(r->ev);
                if (q == hipErrorNotReady) continue;
                r->ev_pending = false;
                if (q != hipSuccess) {
                    {
                        std::lock_guard<std::mutex> lk(mu);
                        active.erase(std::find(active.begin(), active.end(), r));
                    }
                    finish(r, fdi_fail(FD_ERR_DEVICE, "request %llu: %s", (unsigned long long)r->ticket,
                                       hipGetErrorString(q)));
                    progressed = true;
                    continue;
                }
            }
            if (r->next_step >= r->nt) {
                {
                    std::lock_guard<std::mutex> lk(mu);
                    active.erase(std::find(active.begin(), active.end(), r));
                }
                finish(r, FD_OK);
                progressed = true;
                continue;
            }
            hipStream_t s = streams[r->slot];
            fd_shot sh{r->nsrc, r->src.data(), r->d_wav, r->nrec, r->rec.data()};
            const int n1 = std::min(r->nt, r->next_step + chunk);
            int rc = fdi_forward_steps(r->grid, &sh, r->nt, r->next_step, n1, r->d_rec, nullptr, 1, s);
            if (rc == FD_OK && hipEventRecord(r->ev, s) != hipSuccess) rc = FD_ERR_DEVICE;
            if (rc) {
                {
                    std::lock_guard<std::mutex> lk(mu);
                    active.erase(std::find(active.begin(), active.end(), r));
                }
                finish(r, rc);
                progressed = true;
                continue;
            }
            r->next_step = n1;
            r->ev_pending = true;
            progressed = true;
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
        srv->worker = std::thread([srv] { srv->run(); });
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
        if (req->grid.storage != FD_STORE_F32 && req->grid.storage != FD_STORE_F16 &&
            req->grid.storage != FD_STORE_BF16)
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
        srv->cv_work.notify_one();
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
        srv->cv_work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
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
