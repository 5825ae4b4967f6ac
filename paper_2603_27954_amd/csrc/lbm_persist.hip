// One coarse step (every level, every sub-cycled sub-step, bounce-back, force
// sums and coarse/fine transfer) as a single persistent launch.
//
// The host records the step as a list of phases (see Phase).  The work-groups
// walk the list together.  In each phase they claim chunks of the phase's work
// items from an atomic counter and count each finished chunk.  Before a phase
// starts, a work-group waits until every chunk of the previous phase is
// counted, because the next phase reads what that one wrote.  The bodies are
// the ones the per-phase kernels run.
//
// Deadlock freedom does not rest on all work-groups being resident.  A
// work-group only ever waits for chunks that running work-groups have already
// claimed, and a claimed chunk completes without waiting on anything.  A
// work-group that starts late finds the work done and leaves.  Each wave
// drains its own stores to the L2, then one agent-scope release writes the
// per-XCD L2 back before the work-group counts the chunk.  The waiter
// acquires once (which invalidates stale lines) before reading.  Every wait is still bounded: a
// wait past the bound raises the abort flag, every work-group then leaves the
// launch, and the host reports the failure.  The last work-group to leave
// resets the counters for the next launch.
#include "lbm_bodies.h"

namespace lbm {

namespace {

constexpr unsigned SPIN_LIMIT = 1u << 22;

// waits until *done reaches need (thread 0 spins, the work-group follows);
// returns false when the launch is being abandoned.  The spin polls with
// relaxed device-scope loads, which bypass the stale caches without
// invalidating them: an acquire per poll would invalidate the whole XCD L2 on
// every iteration of every waiting work-group and starve the ones still
// working.  One acquire fence follows the wait.
__device__ __forceinline__ bool wait_done(unsigned *done, unsigned need, unsigned *abort_flag, int *ok_sh)
{
    if (threadIdx.x == 0) {
        int ok = 1;
        unsigned spins = 0;
        while (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                ++spins > SPIN_LIMIT) {
                __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *ok_sh = ok;
    }
    __syncthreads();
    const bool ok = *ok_sh != 0;
    __syncthreads();
    return ok;
}

template <int B, typename S>
__device__ __forceinline__ void run_item(const Phase &p, int it, int *nb, double *sh, float (*rrec)[RESTRICT_CELLS])
{
    const int t = it * 256 + (int)threadIdx.x;
    switch (p.kind) {
    case PH_COLLIDE:
        if (p.a.dense) {
            if (!p.odd)
                collide_dense_item<S, false, false>(p.a, it);
            else if (p.rowwave)
                collide_dense_item<S, true, true>(p.a, it);
            else
                collide_dense_item<S, true, false>(p.a, it);
        } else {
            if (p.odd)
                collide_block_item<B, S, true>(p.a, it, nb);
            else
                collide_block_item<B, S, false>(p.a, it, nb);
            __syncthreads();  // nb is refilled by the next item
        }
        break;
    case PH_LINKS:
        if (p.odd)
            link_update<S, true>(p.la, t);
        else
            link_update<S, false>(p.la, t);
        break;
    case PH_BRANCH_SUM:
        link_piece_sum(p.lforce, p.pstart, it, p.piece_sum, sh);
        break;
    case PH_BRANCH_TOTAL:
        branch_totals(p.piece_sum, p.segp, p.nseg, p.sample, p.acc_branch, p.acc_total, p.ring, p.ring_pos, sh);
        break;
    case PH_AMR_MOMENTS:
        if (p.odd)
            amr_moments_item<B, S, true>(p.a, p.cells, p.n, p.om1, p.dt, p.out, t);
        else
            amr_moments_item<B, S, false>(p.a, p.cells, p.n, p.om1, p.dt, p.out, t);
        break;
    case PH_AMR_PROLONG:
        if (p.odd)
            amr_prolong_item<B, S, true>(p.a, p.cells, p.gmask, p.src, p.n, p.nsrc, p.m0, p.m1, p.om1, p.dt, t);
        else
            amr_prolong_item<B, S, false>(p.a, p.cells, p.gmask, p.src, p.n, p.nsrc, p.m0, p.m1, p.om1, p.dt, t);
        break;
    case PH_AMR_RESTRICT:
        if (p.odd && p.odd2)
            amr_restrict_item<B, S, true, true, 256, RESTRICT_CELLS>(p.a, p.b, p.cells, p.child, p.n, p.om1, p.dt, p.om2, p.dt2, it, rrec);
        else if (p.odd)
            amr_restrict_item<B, S, true, false, 256, RESTRICT_CELLS>(p.a, p.b, p.cells, p.child, p.n, p.om1, p.dt, p.om2, p.dt2, it, rrec);
        else if (p.odd2)
            amr_restrict_item<B, S, false, true, 256, RESTRICT_CELLS>(p.a, p.b, p.cells, p.child, p.n, p.om1, p.dt, p.om2, p.dt2, it, rrec);
        else
            amr_restrict_item<B, S, false, false, 256, RESTRICT_CELLS>(p.a, p.b, p.cells, p.child, p.n, p.om1, p.dt, p.om2, p.dt2, it, rrec);
        break;
    default:
        break;
    }
}

// The phase list is read-only for the whole launch; __restrict__ lets the
// compiler keep its (uniform) fields in scalar registers.  ctr holds, per
// phase, the claimed and the finished chunk counts, then the count of
// work-groups that left.
template <int B, typename S>
__global__ void __launch_bounds__(256) k_persist(const Phase *__restrict__ phases, int n_phases, unsigned *ctr,
                                                 unsigned *abort_flag)
{
    __shared__ int nb[27];
    __shared__ double sh[12];
    __shared__ float rrec[11][RESTRICT_CELLS];
    __shared__ int claim_sh, ok_sh;
    unsigned *claimed = ctr, *done = ctr + n_phases, *left = ctr + 2 * n_phases;
    for (int ph = 0; ph < n_phases; ++ph) {
        const Phase &p = phases[ph];
        if (ph > 0 && !wait_done(&done[ph - 1], (unsigned)phases[ph - 1].chunks, abort_flag, &ok_sh))
            break;
        for (;;) {
            if (threadIdx.x == 0)
                claim_sh = (int)__hip_atomic_fetch_add(&claimed[ph], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            const int c = claim_sh;
            __syncthreads();
            if (c >= p.chunks)
                break;
            const int i0 = c * p.chunk, i1 = min(i0 + p.chunk, p.items);
            for (int it = i0; it < i1; ++it)
                run_item<B, S>(p, it, nb, sh, rrec);
            // every wave's stores reach the L2, then one agent-scope release
            // writes the L2 back before the chunk is counted
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (threadIdx.x == 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_fetch_add(&done[ph], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned out = __hip_atomic_fetch_add(left, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (out == gridDim.x - 1u) {
            for (int i = 0; i < 2 * n_phases + 1; ++i)
                __hip_atomic_store(&ctr[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        }
    }
}

template <int B, typename S>
hipError_t launch_t(const Phase *phases, int n_phases, unsigned *ctr, unsigned *abort_flag, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_persist<B, S>), dim3(grid), dim3(256), 0, s, phases, n_phases, ctr, abort_flag);
    return hipGetLastError();
}

template <int B, typename S>
hipError_t max_grid_t(int *per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_persist<B, S>, 256, 0);
}

}  // namespace

hipError_t launch_persistent(int B, int storage, const Phase *phases, int n_phases, unsigned *ctr,
                             unsigned *abort_flag, int grid, hipStream_t s)
{
    if (n_phases == 0)
        return hipSuccess;
    if (B == 16) {
        if (storage == 0) return launch_t<16, float>(phases, n_phases, ctr, abort_flag, grid, s);
        if (storage == 1) return launch_t<16, __half>(phases, n_phases, ctr, abort_flag, grid, s);
        return launch_t<16, __hip_bfloat16>(phases, n_phases, ctr, abort_flag, grid, s);
    }
    if (storage == 0) return launch_t<8, float>(phases, n_phases, ctr, abort_flag, grid, s);
    if (storage == 1) return launch_t<8, __half>(phases, n_phases, ctr, abort_flag, grid, s);
    return launch_t<8, __hip_bfloat16>(phases, n_phases, ctr, abort_flag, grid, s);
}

hipError_t persistent_max_grid(int B, int storage, int device, int *grid, int *cus)
{
    int per_cu = 0, n_cu = 0;
    hipError_t e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess)
        return e;
    if (B == 16)
        e = storage == 0 ? max_grid_t<16, float>(&per_cu)
            : storage == 1 ? max_grid_t<16, __half>(&per_cu) : max_grid_t<16, __hip_bfloat16>(&per_cu);
    else
        e = storage == 0 ? max_grid_t<8, float>(&per_cu)
            : storage == 1 ? max_grid_t<8, __half>(&per_cu) : max_grid_t<8, __hip_bfloat16>(&per_cu);
    if (e != hipSuccess)
        return e;
    *grid = per_cu * n_cu;
    *cus = n_cu;
    return hipSuccess;
}

}  // namespace lbm
