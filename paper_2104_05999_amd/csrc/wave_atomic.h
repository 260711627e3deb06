// Wavefront-aggregated counter updates.  Neighbouring items often add to the
// same counter (the tets around one vertex, the members of one cluster), and
// same-address atomics from one instruction serialise.  Each round takes the
// counter of the lowest pending lane; the lanes that name it are served by one
// atomic of their count, and each takes its slot by its rank among them.
// Rounds are uniform over the lanes that call; call from every lane that has
// an item (lanes without one simply do not call).
#pragma once

#include "common.h"

// counters[key] += 1 for every calling lane; returns the lane's slot (the
// counter's value before its own increment, in lane order within a round).
__device__ __forceinline__ int wave_claim(int32_t* __restrict__ counters, int key) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = (uint64_t(1) << lane) - 1;
    bool done = false;
    int slot = 0;
    while (true) {
        const uint64_t pending = __ballot(!done);
        if (pending == 0) break;
        const int leader = __ffsll(static_cast<unsigned long long>(pending)) - 1;
        const int lk = __shfl(key, leader, 64);
        const bool mine = !done && key == lk;
        const uint64_t same = __ballot(mine);
        int base = 0;
        if (lane == leader) base = atomicAdd(counters + lk, __popcll(same));
        base = __shfl(base, leader, 64);
        if (mine) {
            slot = base + __popcll(same & below);
            done = true;
        }
    }
    return slot;
}
