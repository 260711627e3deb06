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
// The rounds run on wavefront-wide masks only: the lanes of a round are those
// whose key equals the leader's (a lane served earlier holds an earlier
// leader's key, so it never matches again).  After the last round every
// leader adds its round's count in one atomic instruction (the leaders' keys
// are distinct) and each lane fetches its leader's result, so no round waits
// for an atomic.
__device__ __forceinline__ int wave_claim(int32_t* __restrict__ counters, int key) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = (uint64_t(1) << lane) - 1;
    uint64_t pending = __ballot(true), leaders = 0;
    int rank = 0, lead = 0, count = 0;
    while (pending) {
        const int leader = __builtin_ctzll(pending);
        const int lk = __builtin_amdgcn_readlane(key, leader);
        const uint64_t same = __ballot(key == lk);
        pending &= ~same;
        leaders |= uint64_t(1) << leader;
        count = lane == leader ? __popcll(same) : count;
        const bool mine = (same >> lane) & 1;
        rank = mine ? __popcll(same & below) : rank;
        lead = mine ? leader : lead;
    }
    int base = 0;
    if ((leaders >> lane) & 1) base = atomicAdd(counters + key, count);
    return __shfl(base, lead, 64) + rank;
}
