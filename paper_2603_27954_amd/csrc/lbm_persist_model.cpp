// Host model of the persistent launch's work-distribution protocol: the
// persist_walk of the device kernel (lbm_persist_protocol.h), run by host
// threads standing in for work-groups, with C++ atomics in place of the
// device's agent-scope atomics and fences.  Used by the tests to check the
// protocol on the recorded phase lists of real grids: every chunk runs
// exactly once, no chunk starts before the previous phase is complete, the
// counters are zero again after every launch, and a launch whose counters
// were not cleared, or whose work never completes, is abandoned within the
// wait's time limit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#include "../../include/lbmtree.h"
#include "lbm_grid.h"
#include "lbm_persist_protocol.h"

using namespace lbm;

namespace {

using Clock = std::chrono::steady_clock;

struct Shared {
    const int32_t *chunks;
    int n_phases;
    unsigned groups;
    unsigned abort_flag;
    double wait_s;
    int32_t stuck_phase;
    std::unique_ptr<std::atomic<int>[]> runs;  // executions per (phase, chunk)
    std::unique_ptr<std::atomic<long long>[]> finished;  // chunks of each phase run to completion
    std::vector<size_t> first;                  // index of phase p's first chunk in runs
    std::atomic<long long> order_violations{0};
    std::atomic<long long> chunks_run{0};
    std::atomic<long long> waits_given_up{0};
    unsigned *ctr;
};

// One work-group's side of the protocol.
struct HostOps {
    Shared *sh;

    int chunks(int p) const { return sh->chunks[p]; }
    unsigned groups() const { return sh->groups; }

    bool wait(unsigned *done, unsigned need)
    {
        const Clock::time_point t0 = Clock::now();
        for (;;) {
            if (__atomic_load_n(&sh->abort_flag, __ATOMIC_RELAXED) != 0u) {
                sh->waits_given_up++;
                return false;
            }
            if (__atomic_load_n(done, __ATOMIC_RELAXED) >= need)
                break;
            if (std::chrono::duration<double>(Clock::now() - t0).count() > sh->wait_s) {
                __atomic_store_n(&sh->abort_flag, 1u, __ATOMIC_RELAXED);
                sh->waits_given_up++;
                return false;
            }
            std::this_thread::yield();
        }
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
        return true;
    }

    unsigned claim(unsigned *claimed) { return __atomic_fetch_add(claimed, 1u, __ATOMIC_RELAXED); }

    void run(int p, int c)
    {
        // the previous phase must be complete: every one of its chunks run to
        // its end (the model's own count, independent of the counters)
        if (p > 0 && sh->finished[p - 1].load() < (long long)sh->chunks[p - 1])
            sh->order_violations++;
        sh->runs[sh->first[p] + (size_t)c]++;
        sh->chunks_run++;
        if (p == sh->stuck_phase) {
            // a chunk that does not finish in time (models a hung work item)
            std::this_thread::sleep_for(std::chrono::duration<double>(3.0 * sh->wait_s));
        }
    }

    void complete(unsigned *done)
    {
        sh->finished[done - (sh->ctr + sh->n_phases)]++;
        __atomic_fetch_add(done, 1u, __ATOMIC_RELEASE);
    }

    unsigned leave(unsigned *left) { return __atomic_fetch_add(left, 1u, __ATOMIC_ACQ_REL); }

    void reset(unsigned *ctr, int n)
    {
        for (int i = 0; i < n; ++i)
            __atomic_store_n(&ctr[i], 0u, __ATOMIC_RELAXED);
        __atomic_thread_fence(__ATOMIC_RELEASE);
    }
};

}  // namespace

extern "C" {

lbm_status lbm_persist_model(const int32_t *chunks, int32_t n_phases, int32_t groups, int32_t threads,
                             uint32_t *ctr, uint32_t *abort_flag, double wait_s, int32_t stuck_phase,
                             lbm_persist_model_result *out)
{
    if (!chunks || !ctr || !abort_flag || !out || n_phases <= 0 || groups <= 0 || threads <= 0 ||
        !(wait_s > 0.0))
        return grid_fail(nullptr, LBM_E_INVALID, "bad arguments");
    for (int p = 0; p < n_phases; ++p)
        if (chunks[p] < 0)
            return grid_fail(nullptr, LBM_E_INVALID, "negative chunk count");
    Shared sh;
    sh.chunks = chunks;
    sh.n_phases = n_phases;
    sh.groups = (unsigned)groups;
    sh.abort_flag = *abort_flag;
    sh.wait_s = wait_s;
    sh.stuck_phase = stuck_phase;
    sh.ctr = ctr;
    size_t total = 0;
    sh.first.resize((size_t)n_phases);
    for (int p = 0; p < n_phases; ++p) {
        sh.first[(size_t)p] = total;
        total += (size_t)chunks[p];
    }
    sh.runs.reset(new std::atomic<int>[std::max<size_t>(total, 1)]);
    for (size_t i = 0; i < total; ++i)
        sh.runs[i] = 0;
    sh.finished.reset(new std::atomic<long long>[(size_t)n_phases]);
    for (int p = 0; p < n_phases; ++p)
        sh.finished[p] = 0;
    // `threads` host threads run the work-groups in order of their index, each
    // to its end before taking the next, as a device runs a launch with more
    // work-groups than fit at once
    std::atomic<int> next{0};
    const Clock::time_point t0 = Clock::now();
    std::vector<std::thread> pool;
    for (int t = 0; t < std::min(threads, groups); ++t)
        pool.emplace_back([&]() {
            for (;;) {
                const int gidx = next.fetch_add(1);
                if (gidx >= groups)
                    return;
                HostOps o{&sh};
                persist_walk(o, n_phases, ctr);
            }
        });
    for (std::thread &th : pool)
        th.join();
    std::memset(out, 0, sizeof *out);
    out->seconds = std::chrono::duration<double>(Clock::now() - t0).count();
    out->chunks_run = sh.chunks_run;
    for (size_t i = 0; i < total; ++i) {
        const int r = sh.runs[i];
        if (r == 0)
            out->chunks_missed++;
        else if (r > 1)
            out->chunks_repeated++;
    }
    out->order_violations = sh.order_violations;
    out->waits_given_up = sh.waits_given_up;
    *abort_flag = sh.abort_flag;
    out->abandoned = sh.abort_flag != 0u ? 1 : 0;
    int zero = 1;
    for (int i = 0; i < 2 * n_phases + 1; ++i)
        zero &= ctr[i] == 0u;
    out->counters_zero = zero;
    return LBM_OK;
}

}  // extern "C"
