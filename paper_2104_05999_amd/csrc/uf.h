// Lock-free union-find over an int32 parent array.
#pragma once

#include "common.h"

// Connected components by lock-free union-find (used for the parts that
// cracks cut off from every Dirichlet vertex or face): the larger of two
// roots is hooked under the smaller with a compare-and-swap, so
// parent[v] <= v always holds, every find ends, and the root of a component
// is its smallest vertex (a label independent of scheduling).  A failed swap
// means another thread hooked that root; the loop then continues from the
// new root.  Finds halve the path they walk: a vertex that is not a root is
// re-pointed to its grandparent, which is an ancestor in the same tree (a
// non-root never becomes a root again, and the swaps only ever change
// roots), so the halving races with nothing.  The same code serves a parent
// array in LDS (SCOPE = workgroup) and one in global memory (the device).
template <int SCOPE = __HIP_MEMORY_SCOPE_AGENT>
__device__ __forceinline__ int32_t uf_find(int32_t* parent, int32_t v) {
    while (true) {
        const int32_t p = __hip_atomic_load(parent + v, __ATOMIC_RELAXED, SCOPE);
        if (p == v) return v;
        const int32_t gp = __hip_atomic_load(parent + p, __ATOMIC_RELAXED, SCOPE);
        if (gp == p) return p;
        __hip_atomic_store(parent + v, gp, __ATOMIC_RELAXED, SCOPE);
        v = gp;
    }
}


// Join the sets of a and b.  SCOPE is the scope of the array: the device for
// a global parent array, the workgroup for one in LDS.
template <int SCOPE = __HIP_MEMORY_SCOPE_AGENT>
__device__ __forceinline__ void uf_union(int32_t* parent, int32_t a, int32_t b) {
    int32_t ra = uf_find<SCOPE>(parent, a);
    int32_t rb = uf_find<SCOPE>(parent, b);
    while (ra != rb) {
        if (ra > rb) {
            const int32_t t = ra;
            ra = rb;
            rb = t;
        }
        int32_t old = rb;
        if (__hip_atomic_compare_exchange_strong(parent + rb, &old, ra, __ATOMIC_RELAXED, __ATOMIC_RELAXED, SCOPE))
            break;
        rb = uf_find<SCOPE>(parent, old);
        ra = uf_find<SCOPE>(parent, ra);
    }
}
