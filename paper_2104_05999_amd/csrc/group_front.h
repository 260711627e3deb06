// Front order over items that take `lanes` lanes each (a group of lanes per
// vertex or row): XCD x (blockIdx.x & 7) owns the contiguous x-th eighth of
// the items and its blocks sweep it together, so that the items in flight on
// one XCD are neighbours and the data they gather (a vertex's tets, a row's
// columns) is shared in that XCD's L2.  gridDim.x must be a multiple of 8
// (grid_xcd), and lanes must divide blockDim.x.
#pragma once

#include "common.h"

__device__ __forceinline__ FrontRange group_front(int64_t n, int lanes) {
    const int64_t xcd = blockIdx.x & 7, j = blockIdx.x >> 3, per = gridDim.x >> 3, ipb = blockDim.x / lanes;
    FrontRange r;
    r.first = n * xcd / 8 + j * ipb + threadIdx.x / lanes;
    r.step = per * ipb;
    r.end = n * (xcd + 1) / 8;
    return r;
}

#define GROUP_FRONT_LOOP(i, n, lanes)             \
    const FrontRange i##_fr = group_front((n), (lanes)); \
    for (int64_t i = i##_fr.first; i < i##_fr.end; i += i##_fr.step)
