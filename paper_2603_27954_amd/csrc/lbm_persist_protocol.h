// Work-distribution protocol of the persistent coarse-step launch, written
// once for the device kernel (lbm_persist.hip) and for the host model that
// runs it with threads standing in for work-groups (lbm_persist_model.cpp).
//
// A coarse step is a list of phases; phase p has chunks(p) chunks of work
// items, and every chunk of phase p may read what any chunk of phase p - 1
// wrote.  The counters of one launch are claimed[n], done[n] and left, in one
// array of 2n + 1 words that is zero when the launch starts.  Each work-group
// walks the phases in order:
//
//   - before phase p > 0 it waits until done[p - 1] == chunks(p - 1);
//   - it claims chunk numbers of phase p from claimed[p] until the number it
//     gets is past the last chunk; after running a claimed chunk it makes the
//     chunk's stores visible and counts the chunk in done[p];
//   - at the end it counts itself in left, and the last work-group to leave
//     sets every counter back to zero for the next launch.
//
// Progress does not rest on the work-groups being resident together: a
// work-group only waits for chunks that other work-groups have claimed, and a
// claimed chunk completes without waiting on anything.  A work-group that
// starts after the others have finished finds every chunk claimed and leaves.
// A wait ends either when the count is reached or when it gives up: the abort
// flag is up (checked first, so a raised flag ends every later wait at once)
// or the wait's time limit passed (it then raises the flag).  A work-group
// that gives up leaves the launch, so every work-group reaches the end, and
// the counters are zero again after every launch, abandoned or not.
#pragma once
#include <hip/hip_runtime.h>

namespace lbm {

// Ops supplies, for one work-group:
//   int      chunks(int p)                 chunks of phase p
//   bool     wait(unsigned *done, unsigned need)
//                                          true once *done >= need, false when
//                                          the launch is abandoned
//   unsigned claim(unsigned *claimed)      fetch-and-add 1, the old value
//   void     run(int p, int c)             the items of chunk c of phase p
//   void     complete(unsigned *done)      stores of the chunk made visible,
//                                          then *done += 1
//   unsigned leave(unsigned *left)         fetch-and-add 1, the old value
//   unsigned groups()                      work-groups of the launch
//   void     reset(unsigned *ctr, int n)   n counters set to zero, made visible
template <class Ops>
__host__ __device__ inline void persist_walk(Ops &o, int n_phases, unsigned *ctr)
{
    unsigned *claimed = ctr, *done = ctr + n_phases, *left = ctr + 2 * n_phases;
    for (int p = 0; p < n_phases; ++p) {
        if (p > 0 && !o.wait(&done[p - 1], (unsigned)o.chunks(p - 1)))
            break;
        for (;;) {
            const unsigned c = o.claim(&claimed[p]);
            if (c >= (unsigned)o.chunks(p))
                break;
            o.run(p, (int)c);
            o.complete(&done[p]);
        }
    }
    if (o.leave(left) == o.groups() - 1u)
        o.reset(ctr, 2 * n_phases + 1);
}

// Chunking of a phase of `items` work items for a launch of `groups`
// work-groups: about two claims per work-group in large phases, one item per
// claim in small ones.
__host__ __device__ inline int persist_chunk(int items, int groups)
{
    const int c = items / (2 * (groups > 0 ? groups : 1));
    return c > 1 ? c : 1;
}

}  // namespace lbm
