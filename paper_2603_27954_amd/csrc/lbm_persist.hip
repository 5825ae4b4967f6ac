// One coarse step (every level, every sub-cycled sub-step, bounce-back, force
// sums and coarse/fine transfer) as a single persistent launch.
//
// The host records the step as a list of phases (see Phase).  The work-groups
// walk the list with the claim / count / leave protocol of persist_walk
// (lbm_persist_protocol.h): chunks of a phase's items are claimed from an
// atomic counter, each finished chunk is counted, and a phase starts once the
// previous phase's chunks are all counted.  The bodies are the ones the
// per-phase kernels run.
//
// Memory ordering across the XCDs (each has its own L2): a work-group drains
// its stores, then one agent-scope release writes its L2 back before the chunk
// is counted.  A waiting work-group polls the count with relaxed agent-scope
// loads and acquires once after the wait: an acquire per poll would invalidate
// the XCD's whole L2 on every iteration of every waiting work-group and starve
// the work-groups still computing.
//
// Every wait is bounded in time, not in polls: thread 0 reads the constant
// real-time counter and gives up once wait_ticks have passed, raising the
// abort flag.  A raised flag ends every later wait at its first poll, so the
// launch is abandoned: each work-group leaves at its next phase boundary and
// the host reports the failure.  Each wait therefore ends within wait_ticks of
// the counter's clock plus one poll, whatever a poll costs.
#include "lbm_bodies.h"
#include "lbm_persist_protocol.h"

namespace lbm {

namespace {

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

// Device side of the protocol for one work-group: thread 0 talks to the
// counters and word_sh hands its results to the whole work-group.
template <int B, typename S>
struct DevOps {
    const Phase *__restrict__ phases;
    unsigned *abort_flag;
    unsigned long long wait_ticks;
    int *nb;
    double *sh;
    float (*rrec)[RESTRICT_CELLS];
    unsigned *word_sh;

    __device__ int chunks(int p) const { return phases[p].chunks; }
    __device__ unsigned groups() const { return gridDim.x; }

    __device__ unsigned broadcast(unsigned v)
    {
        if (threadIdx.x == 0)
            *word_sh = v;
        __syncthreads();
        const unsigned r = *word_sh;
        __syncthreads();
        return r;
    }

    __device__ bool wait(unsigned *done, unsigned need)
    {
        unsigned ok = 1u;
        if (threadIdx.x == 0) {
            const unsigned long long t0 = (unsigned long long)wall_clock64();
            for (;;) {
                if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                    ok = 0u;
                    break;
                }
                if (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need)
                    break;
                if ((unsigned long long)wall_clock64() - t0 > wait_ticks) {
                    __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0u;
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        return broadcast(ok) != 0u;
    }

    __device__ unsigned claim(unsigned *claimed)
    {
        unsigned c = 0u;
        if (threadIdx.x == 0)
            c = __hip_atomic_fetch_add(claimed, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return broadcast(c);
    }

    __device__ void run(int p, int c)
    {
        const Phase &ph = phases[p];
        const int i0 = c * ph.chunk, i1 = min(i0 + ph.chunk, ph.items);
        for (int it = i0; it < i1; ++it)
            run_item<B, S>(ph, it, nb, sh, rrec);
    }

    __device__ void complete(unsigned *done)
    {
        // every wave's stores reach the L2, then one agent-scope release
        // writes the L2 back before the chunk is counted
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    __device__ unsigned leave(unsigned *left)
    {
        __syncthreads();
        unsigned v = 0u;
        if (threadIdx.x == 0)
            v = __hip_atomic_fetch_add(left, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        return broadcast(v);
    }

    __device__ void reset(unsigned *ctr, int n)
    {
        if (threadIdx.x == 0) {
            for (int i = 0; i < n; ++i)
                __hip_atomic_store(&ctr[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        }
    }
};

// The phase list is read-only for the whole launch; __restrict__ lets the
// compiler keep its (uniform) fields in scalar registers.  ctr holds, per
// phase, the claimed and the finished chunk counts, then the count of
// work-groups that left.
template <int B, typename S>
__global__ void __launch_bounds__(256) k_persist(const Phase *__restrict__ phases, int n_phases, unsigned *ctr,
                                                 unsigned *abort_flag, unsigned long long wait_ticks)
{
    __shared__ int nb[27];
    __shared__ double sh[12];
    __shared__ float rrec[11][RESTRICT_CELLS];
    __shared__ unsigned word_sh;
    DevOps<B, S> o{phases, abort_flag, wait_ticks, nb, sh, rrec, &word_sh};
    persist_walk(o, n_phases, ctr);
}

template <int B, typename S>
hipError_t launch_t(const Phase *phases, int n_phases, unsigned *ctr, unsigned *abort_flag,
                    unsigned long long wait_ticks, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_persist<B, S>), dim3(grid), dim3(256), 0, s, phases, n_phases, ctr, abort_flag,
                       wait_ticks);
    return hipGetLastError();
}

template <int B, typename S>
hipError_t max_grid_t(int *per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_persist<B, S>, 256, 0);
}

}  // namespace

hipError_t launch_persistent(int B, int storage, const Phase *phases, int n_phases, unsigned *ctr,
                             unsigned *abort_flag, unsigned long long wait_ticks, int grid, hipStream_t s)
{
    if (n_phases == 0)
        return hipSuccess;
    const unsigned long long w = wait_ticks;
    if (B == 16) {
        if (storage == 0) return launch_t<16, float>(phases, n_phases, ctr, abort_flag, w, grid, s);
        if (storage == 1) return launch_t<16, __half>(phases, n_phases, ctr, abort_flag, w, grid, s);
        return launch_t<16, __hip_bfloat16>(phases, n_phases, ctr, abort_flag, w, grid, s);
    }
    if (storage == 0) return launch_t<8, float>(phases, n_phases, ctr, abort_flag, w, grid, s);
    if (storage == 1) return launch_t<8, __half>(phases, n_phases, ctr, abort_flag, w, grid, s);
    return launch_t<8, __hip_bfloat16>(phases, n_phases, ctr, abort_flag, w, grid, s);
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
