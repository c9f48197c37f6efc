// Request loop for streams of independent VTS problems (vts_server_* in
// vts.h): one device pool allocated once, first-fit ranges per admitted
// request, worker threads with one non-blocking HIP stream each.  A worker
// builds the request's context inside its range, runs Algorithm 1 to the
// request's tolerances, copies rho and u to host memory and returns the
// range; admitted requests overlap on the device through their streams.
// The Newton-system MINRES solves of admitted requests with the same grid,
// levels and precision run together in one group runner per such shape:
// their smoother, transfer, operator and vector launches go out as one
// launch per kernel over the group.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "vts_internal.hpp"

using namespace vts;

namespace {

constexpr size_t kGranule = 256;

struct Request {
    int64_t id = 0;
    vts_problem pr{};
    vts_options opt{};
    std::vector<uint8_t> fixed;
    std::vector<double> f, lo, hi;
    std::string log_path;
    size_t footprint = 0;
    double t_submit = 0.0;
};

struct Finished {
    vts_request_info info{};
    std::vector<double> rho, u;
};

// first-fit ranges of the pool, coalesced on release
class RangeAllocator {
   public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool take(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

   private:
    std::map<size_t, size_t> free_;
};

}  // namespace

struct vts_server {
    int device = 0;
    char* pool = nullptr;
    size_t pool_size = 0;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> workers;

    mutable std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> pending;
    std::deque<int64_t> unpolled;
    std::map<int64_t, Finished> finished;
    RangeAllocator ranges;
    int32_t running = 0;
    int64_t next_id = 1;
    bool stop = false;
    bool batch = true;
    std::mutex rmu;
    std::map<std::string, GroupRunner*> runners;   // one per shape, created on first use

    // the group runner for problems of c's shape (nullptr: run alone)
    GroupRunner* runner_for(const Ctx& c) {
        const std::string key = std::to_string(c.prec) + ":" + std::to_string(c.nx) + "x" +
                                std::to_string(c.ny) + "x" + std::to_string(c.nz) + ":" +
                                std::to_string(c.L);
        std::lock_guard<std::mutex> lk(rmu);
        auto it = runners.find(key);
        if (it != runners.end()) return it->second;
        std::string err;
        GroupRunner* g = group_runner_create(device, err);
        runners.emplace(key, g);   // nullptr remembered too: that shape runs alone
        return g;
    }
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    // first request in arrival order whose footprint fits a free range
    bool pick(Request& r, size_t* off) {
        for (auto it = pending.begin(); it != pending.end(); ++it) {
            if (ranges.take(it->footprint, off)) {
                r = std::move(*it);
                pending.erase(it);
                return true;
            }
        }
        return false;
    }

    void work(int slot) {
        hipSetDevice(device);
        hipStream_t s = streams[slot];
        for (;;) {
            Request r;
            size_t off = 0;
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    if (stop) return;
                    if (pick(r, &off)) break;
                    cv_work.wait(lk);
                }
                ++running;
            }
            Finished fin;
            vts_request_info& in = fin.info;
            in.id = r.id;
            in.t_submit = r.t_submit;
            in.t_admit = now();
            in.footprint = r.footprint;
            vts_ctx* ctx = nullptr;
            std::string err;
            if (!r.log_path.empty()) r.opt.log_path = r.log_path.c_str();
            vts_status st = create_in(&r.pr, &r.opt, s, pool + off, r.footprint, &ctx, err);
            if (st == VTS_OK) {
                if (batch) ctx->group = runner_for(*ctx);
                vts_result res{};
                st = vts_pbm_solve(ctx, &res);
                in.outer = res.outer;
                in.newton = res.newton;
                in.minres = res.minres;
                in.compliance = res.compliance;
                in.alpha = res.alpha;
                in.sum_rho = res.sum_rho;
                in.n_dof = ctx->ndof;
                in.m = ctx->m;
                fin.rho.resize(ctx->m);
                fin.u.resize(ctx->ndof);
                hipError_t e1 = hipMemcpyAsync(fin.rho.data(), ctx->rho, ctx->m * sizeof(double),
                                               hipMemcpyDeviceToHost, s);
                hipError_t e2 = hipMemcpyAsync(fin.u.data(), ctx->u, ctx->ndof * sizeof(double),
                                               hipMemcpyDeviceToHost, s);
                hipError_t e3 = hipStreamSynchronize(s);
                if ((e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) && st == VTS_OK)
                    st = VTS_EDEVICE;
                ctx->group = nullptr;
                vts_destroy(ctx);
            }
            in.status = st;
            in.t_done = now();
            {
                std::lock_guard<std::mutex> lk(mu);
                ranges.give(off, r.footprint);
                --running;
                unpolled.push_back(r.id);
                finished.emplace(r.id, std::move(fin));
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }
};

extern "C" {

vts_status vts_server_create(int32_t slots, size_t hbm_bytes, vts_server** out) {
    if (!out || slots < 1 || hbm_bytes < kGranule) return VTS_EINVAL;
    *out = nullptr;
    vts_server* S = new (std::nothrow) vts_server();
    if (!S) return VTS_ENOMEM;
    S->pool_size = hbm_bytes / kGranule * kGranule;
    if (hipGetDevice(&S->device) != hipSuccess ||
        hipMalloc((void**)&S->pool, S->pool_size) != hipSuccess) {
        delete S;
        return VTS_ENOMEM;
    }
    S->ranges.reset(S->pool_size);
    for (int q = 0; q < slots; ++q) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t t : S->streams) hipStreamDestroy(t);
            hipFree(S->pool);
            delete S;
            return VTS_EDEVICE;
        }
        S->streams.push_back(s);
    }
    for (int q = 0; q < slots; ++q) S->workers.emplace_back(&vts_server::work, S, q);
    *out = S;
    return VTS_OK;
}

vts_status vts_server_submit(vts_server* S, const vts_problem* pr, const vts_options* opt,
                             int64_t* id) try {
    if (!S || !pr || !id) return VTS_EINVAL;
    std::string err;
    if (check_problem(pr, err) != VTS_OK) return VTS_EINVAL;
    const size_t foot = vts_footprint_bytes(pr, opt);
    if (foot == 0) return VTS_EINVAL;
    if (foot > S->pool_size) return VTS_ENOMEM;
    Request r;
    r.pr = *pr;
    if (opt) r.opt = *opt; else vts_default_options(&r.opt);
    if (r.opt.log_path) {
        r.log_path = r.opt.log_path;   // the caller's string need not outlive the call
        r.opt.log_path = nullptr;
    }
    const int64_t nn = (int64_t)(pr->nx + 1) * (pr->ny + 1) * (pr->nz + 1), m =
        (int64_t)pr->nx * pr->ny * pr->nz;
    r.fixed.assign(pr->fixed_host, pr->fixed_host + 3 * nn);
    r.f.assign(pr->f_host, pr->f_host + 3 * nn);
    r.pr.fixed_host = r.fixed.data();
    r.pr.f_host = r.f.data();
    if (pr->rho_lo_host) {
        r.lo.assign(pr->rho_lo_host, pr->rho_lo_host + m);
        r.pr.rho_lo_host = r.lo.data();
    }
    if (pr->rho_hi_host) {
        r.hi.assign(pr->rho_hi_host, pr->rho_hi_host + m);
        r.pr.rho_hi_host = r.hi.data();
    }
    r.footprint = foot;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        r.id = S->next_id++;
        r.t_submit = S->now();
        *id = r.id;
        S->pending.push_back(std::move(r));
    }
    S->cv_work.notify_all();
    return VTS_OK;
} catch (...) {
    return VTS_ENOMEM;   // host copies of the request could not be allocated
}

int32_t vts_server_poll(vts_server* S, vts_request_info* out, int32_t max, double timeout_s) {
    if (!S || !out || max < 1) return 0;
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->unpolled.empty() && timeout_s > 0)
        S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                            [&] { return !S->unpolled.empty(); });
    int32_t n = 0;
    while (n < max && !S->unpolled.empty()) {
        const int64_t id = S->unpolled.front();
        S->unpolled.pop_front();
        auto it = S->finished.find(id);
        if (it != S->finished.end()) out[n++] = it->second.info;   // else fetched already
    }
    return n;
}

vts_status vts_server_fetch(vts_server* S, int64_t id, double* rho_host, double* u_host) {
    if (!S) return VTS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->finished.find(id);
    if (it == S->finished.end()) return VTS_EINVAL;
    const Finished& f = it->second;
    if (rho_host) std::copy(f.rho.begin(), f.rho.end(), rho_host);
    if (u_host) std::copy(f.u.begin(), f.u.end(), u_host);
    S->finished.erase(it);
    // a request fetched before it was polled is not reported by a later poll
    auto up = std::find(S->unpolled.begin(), S->unpolled.end(), id);
    if (up != S->unpolled.end()) S->unpolled.erase(up);
    return VTS_OK;
}

vts_status vts_group_step(vts_ctx** ctxs, int32_t k, vts_pbmstats* stats) {
    if (!ctxs || k < 0) return VTS_EINVAL;
    for (int32_t q = 0; q < k; ++q) {
        if (!ctxs[q] || ctxs[q]->nl > 1) return VTS_EINVAL;   // one load case per context
        for (int32_t p = 0; p < q; ++p)
            if (ctxs[p] == ctxs[q]) return VTS_EINVAL;
    }
    std::vector<vts_status> st(k, VTS_OK);
    std::vector<std::thread> th;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return VTS_EDEVICE;
    // one group runner for the call: the contexts' Newton-system MINRES
    // solves advance together, one launch per kernel for contexts of one shape
    std::string err;
    GroupRunner* g = k > 1 ? group_runner_create(dev, err) : nullptr;
    for (int32_t q = 0; q < k; ++q) ctxs[q]->group = g;
    for (int32_t q = 0; q < k; ++q)
        th.emplace_back([&, q] {
            hipSetDevice(dev);
            st[q] = vts_pbm_iterate(ctxs[q], stats ? &stats[q] : nullptr);
        });
    for (std::thread& t : th) t.join();
    for (int32_t q = 0; q < k; ++q) ctxs[q]->group = nullptr;
    group_runner_destroy(g);
    for (int32_t q = 0; q < k; ++q)
        if (st[q] != VTS_OK) return st[q];
    return VTS_OK;
}

vts_status vts_server_batching(vts_server* S, int32_t on) {
    if (!S) return VTS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->next_id != 1) return VTS_ESTATE;   // only before the first submit
    S->batch = on != 0;
    return VTS_OK;
}

void vts_server_group_stats(vts_server* S, int64_t out[5]) {
    if (!S || !out) return;
    for (int q = 0; q < 5; ++q) out[q] = 0;
    std::lock_guard<std::mutex> lk(S->rmu);
    for (auto& kv : S->runners) {
        if (!kv.second) continue;
        GroupStats gs;
        group_runner_stats(kv.second, &gs);
        out[0] += gs.cycles;
        out[1] += gs.solves;
        out[2] += gs.kernel_ops;
        out[3] += gs.launches;
        out[4] = std::max(out[4], gs.max_batch);
    }
}

double vts_server_clock(const vts_server* S) { return S ? S->now() : 0.0; }

void vts_server_counts(const vts_server* S, int32_t* pending, int32_t* running,
                       int32_t* finished) {
    if (!S) return;
    std::lock_guard<std::mutex> lk(S->mu);
    if (pending) *pending = (int32_t)S->pending.size();
    if (running) *running = S->running;
    if (finished) *finished = (int32_t)S->unpolled.size();
}

void vts_server_destroy(vts_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->pending.clear();
    }
    S->cv_work.notify_all();
    for (std::thread& t : S->workers) t.join();
    for (auto& kv : S->runners) group_runner_destroy(kv.second);
    for (hipStream_t s : S->streams) hipStreamDestroy(s);
    hipFree(S->pool);
    delete S;
}

}  // extern "C"
