// Group runner: several independent MINRES solves (each the Newton system of
// eq. (3.12) of its own problem, Section 6) advanced together.  A runner
// thread owns one stream.  Each step, every solve in the group records the
// device work of its next step (the same host code as a solve on its own,
// with Ctx::rec set); solves whose recorded launch sequences are equal (the
// same kernels and grids: problems of one grid and hierarchy) are issued as
// one launch per kernel, problem = blockIdx.y, with the per-problem
// arguments in a table copied to the device once per step.  Each problem's
// arithmetic is that of its own solve (same kernels' bodies, same blocks and
// the same order), so results do not depend on the company.  One stream
// synchronization per step serves the whole group; solves join and leave
// between steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "vts_internal.hpp"

namespace vts {

namespace {

struct Job {
    Ctx* c = nullptr;
    MrState m;
    vts_linstats* out = nullptr;
    Recorder rec;
    bool started = false;
    bool finishing = false;
    bool done = false;
};

constexpr size_t kTableAlign = 256;
constexpr size_t kStageInit = size_t(4) << 20;

}  // namespace

struct GroupRunner {
    int device = 0;
    hipStream_t s = nullptr;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv_in, cv_done;
    std::deque<Job*> incoming;
    bool stop = false;
    uint8_t* host_stage = nullptr;   // pinned
    uint8_t* dev_stage = nullptr;
    size_t cap = 0;
    GroupStats stats;    // published under mu
    GroupStats step;     // this step's counts (runner thread only)

    bool grow(size_t need, std::string& err) {
        if (need <= cap) return true;
        size_t nc = cap ? cap : kStageInit;
        while (nc < need) nc *= 2;
        if (host_stage) (void)hipHostFree(host_stage);
        if (dev_stage) (void)hipFree(dev_stage);
        host_stage = nullptr;
        dev_stage = nullptr;
        cap = 0;
        if (hipHostMalloc((void**)&host_stage, nc, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void**)&dev_stage, nc) != hipSuccess) {
            err = "group runner: staging allocation failed";
            return false;
        }
        cap = nc;
        return true;
    }

    // the sequence of (kernel, grid, block, argument size) / copies: equal
    // sequences can share launches
    static std::string signature(const Recorder& r) {
        std::string sig;
        sig.reserve(r.ops.size() * 32);
        for (const RecOp& o : r.ops) {
            uintptr_t k = (uintptr_t)o.kb;
            uint32_t v[7] = {o.grid.x, o.grid.y, o.grid.z, o.block.x, o.block.y, o.block.z,
                             o.asize};
            sig.append((const char*)&k, sizeof(k));
            sig.append((const char*)v, sizeof(v));
        }
        return sig;
    }

    // issue every recorded operation of the jobs on s; false on a HIP error
    bool replay(std::vector<Job*>& jobs, std::string& err) {
        std::map<std::string, std::vector<Job*>> groups;
        for (Job* j : jobs)
            if (!j->rec.ops.empty()) groups[signature(j->rec)].push_back(j);
        // tables: for each group of two or more, for each kernel op, the
        // members' argument structs (a group of one launches the single-problem
        // kernels with the recorded arguments: no table, no copy)
        size_t total = 0;
        for (auto& kv : groups) {
            const std::vector<Job*>& g = kv.second;
            if (g.size() < 2) continue;
            for (const RecOp& o : g[0]->rec.ops)
                if (o.kb) total += (o.asize * g.size() + kTableAlign - 1) / kTableAlign * kTableAlign;
        }
        if (!grow(total, err)) return false;
        size_t off = 0;
        std::vector<size_t> offs;
        for (auto& kv : groups) {
            const std::vector<Job*>& g = kv.second;
            if (g.size() < 2) continue;
            const std::vector<RecOp>& ops = g[0]->rec.ops;
            for (size_t q = 0; q < ops.size(); ++q) {
                if (!ops[q].kb) continue;
                offs.push_back(off);
                for (size_t p = 0; p < g.size(); ++p) {
                    const RecOp& o = g[p]->rec.ops[q];
                    std::memcpy(host_stage + off + p * o.asize, g[p]->rec.bytes.data() + o.aoff,
                                o.asize);
                }
                off += (ops[q].asize * g.size() + kTableAlign - 1) / kTableAlign * kTableAlign;
            }
        }
        if (off && hipMemcpyAsync(dev_stage, host_stage, off, hipMemcpyHostToDevice, s) !=
                       hipSuccess) {
            err = "group runner: table copy failed";
            return false;
        }
        size_t t = 0;
        for (auto& kv : groups) {
            const std::vector<Job*>& g = kv.second;
            const std::vector<RecOp>& ops = g[0]->rec.ops;
            const unsigned B = (unsigned)g.size();
            for (size_t q = 0; q < ops.size(); ++q) {
                const RecOp& o = ops[q];
                if (o.kb && B == 1) {
                    void* args[] = {(void*)(g[0]->rec.bytes.data() + o.aoff)};
                    if (hipLaunchKernel(o.k, o.grid, o.block, args, 0, s) != hipSuccess) {
                        err = "group runner: launch failed";
                        return false;
                    }
                    step.kernel_ops += 1;
                    step.launches += 1;
                    if (step.max_batch < 1) step.max_batch = 1;
                } else if (o.kb) {
                    const void* tab = dev_stage + offs[t++];
                    void* args[] = {(void*)&tab};
                    if (hipLaunchKernel(o.kb, dim3(o.grid.x, B, 1), o.block, args, 0, s) !=
                        hipSuccess) {
                        err = "group runner: launch failed";
                        return false;
                    }
                    step.kernel_ops += B;
                    step.launches += 1;
                    if ((int64_t)B > step.max_batch) step.max_batch = B;
                } else {
                    for (Job* j : g) {
                        const RecOp& oc = j->rec.ops[q];
                        if (hipMemcpyAsync(oc.dst, oc.src, oc.nbytes, oc.kind, s) != hipSuccess) {
                            err = "group runner: copy failed";
                            return false;
                        }
                    }
                }
            }
        }
        return true;
    }

    void finish_all(std::vector<Job*>& jobs, vts_status st, const std::string& err) {
        std::lock_guard<std::mutex> lk(mu);
        for (Job* j : jobs) {
            if (st != VTS_OK) {
                j->m.st = st;
                j->c->err = err;
            }
            j->done = true;
        }
        jobs.clear();
        cv_done.notify_all();
    }

    void loop() {
        (void)hipSetDevice(device);
        std::vector<Job*> active;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_in.wait(lk, [&] { return stop || !incoming.empty() || !active.empty(); });
                if (stop && incoming.empty() && active.empty()) return;
                while (!incoming.empty()) {
                    active.push_back(incoming.front());
                    incoming.pop_front();
                }
            }
            // record this step of every solve
            for (Job* j : active) {
                Ctx& c = *j->c;
                c.rec = &j->rec;
                if (!j->started) {
                    mr_issue_start(c, j->m);
                    j->started = true;
                } else if (j->m.phase == MrState::kIterate) {
                    mr_issue_iter(c, j->m);
                } else if (j->m.phase == MrState::kFinish) {
                    mr_finish(c, j->m, j->out);
                    j->finishing = true;
                }
                c.rec = nullptr;
            }
            std::string err;
            if (!replay(active, err) || hipStreamSynchronize(s) != hipSuccess) {
                if (err.empty()) err = "group runner: stream synchronization failed";
                finish_all(active, VTS_EDEVICE, err);
                continue;
            }
            ++step.cycles;
            // read the step's reductions; the next step's leading work is recorded
            std::vector<Job*> left, ended;
            for (Job* j : active) {
                Ctx& c = *j->c;
                j->rec.clear();
                if (j->finishing) {
                    ++step.solves;
                    ended.push_back(j);
                    continue;
                }
                c.rec = &j->rec;
                if (j->m.phase == MrState::kStart)
                    mr_after_start(c, j->m);
                else if (j->m.phase == MrState::kIterate)
                    mr_after_iter(c, j->m);
                c.rec = nullptr;
                if (j->m.phase == MrState::kDone)
                    ended.push_back(j);     // an error: nothing more is issued
                else
                    left.push_back(j);
            }
            active.swap(left);
            {
                std::lock_guard<std::mutex> lk(mu);
                stats.cycles += step.cycles;
                stats.solves += step.solves;
                stats.kernel_ops += step.kernel_ops;
                stats.launches += step.launches;
                stats.max_batch = std::max(stats.max_batch, step.max_batch);
            }
            step = GroupStats{};
            if (!ended.empty()) finish_all(ended, VTS_OK, std::string());
        }
    }
};

GroupRunner* group_runner_create(int device, std::string& err) {
    GroupRunner* g = new GroupRunner();
    g->device = device;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != device) (void)hipSetDevice(device);
    if (hipStreamCreateWithFlags(&g->s, hipStreamNonBlocking) != hipSuccess ||
        !g->grow(kStageInit, err)) {
        if (err.empty()) err = "group runner: stream creation failed";
        if (g->s) (void)hipStreamDestroy(g->s);
        if (g->host_stage) (void)hipHostFree(g->host_stage);
        if (g->dev_stage) (void)hipFree(g->dev_stage);
        if (cur != device) (void)hipSetDevice(cur);
        delete g;
        return nullptr;
    }
    if (cur != device) (void)hipSetDevice(cur);
    g->th = std::thread([g] { g->loop(); });
    return g;
}

void group_runner_destroy(GroupRunner* g) {
    if (!g) return;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        g->stop = true;
    }
    g->cv_in.notify_all();
    if (g->th.joinable()) g->th.join();
    (void)hipStreamSynchronize(g->s);
    (void)hipStreamDestroy(g->s);
    if (g->host_stage) (void)hipHostFree(g->host_stage);
    if (g->dev_stage) (void)hipFree(g->dev_stage);
    delete g;
}

void group_runner_stats(GroupRunner* g, GroupStats* out) {
    if (!g || !out) return;
    std::lock_guard<std::mutex> lk(g->mu);
    *out = g->stats;
}

vts_status group_minres(Ctx& c, double eps, vts_linstats* out, int maxit) {
    GroupRunner* g = c.group;
    // the context's earlier work is complete before the runner's stream uses its data
    if (hipStreamSynchronize(c.s) != hipSuccess) {
        c.err = "hipStreamSynchronize failed";
        return VTS_EDEVICE;
    }
    Job job;
    job.c = &c;
    job.out = out;
    mr_init(c, job.m, eps, maxit, false);
    {
        std::lock_guard<std::mutex> lk(g->mu);
        g->incoming.push_back(&job);
    }
    g->cv_in.notify_all();
    {
        std::unique_lock<std::mutex> lk(g->mu);
        g->cv_done.wait(lk, [&] { return job.done; });
    }
    return job.m.st;
}

}  // namespace vts
