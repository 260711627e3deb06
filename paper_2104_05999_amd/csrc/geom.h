// Small FP64 vector helpers and the textbook circumcentres, in a fixed
// operation order (kernels that decide integers from them are compiled
// without floating-point contraction).
#pragma once

#include "common.h"

struct d3 {
    double x, y, z;
};
__device__ __forceinline__ d3 sub(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ double dot(d3 a, d3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ __forceinline__ d3 cross(d3 a, d3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ d3 scale(double s, d3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ d3 load3(const double* p) { return {p[0], p[1], p[2]}; }

__device__ __forceinline__ int vget(const int4& q, int k) {
    return k == 0 ? q.x : (k == 1 ? q.y : (k == 2 ? q.z : q.w));
}

// vertex r (0..2) of local face k (the face opposite local vertex k), in the tet's order
__device__ __forceinline__ int face_local_vertex(int k, int r) { return r + (r >= k ? 1 : 0); }

// c_T = p0 + (|a|^2 (b x c) + |b|^2 (c x a) + |c|^2 (a x b)) / (2 a.(b x c))
__device__ inline d3 tet_circumcentre(d3 p0, d3 p1, d3 p2, d3 p3) {
    const d3 a = sub(p1, p0), b = sub(p2, p0), c = sub(p3, p0);
    const d3 bc = cross(b, c), ca = cross(c, a), ab = cross(a, b);
    const double sa = dot(a, a), sb = dot(b, b), sc = dot(c, c);
    const d3 num = {(sa * bc.x + sb * ca.x) + sc * ab.x, (sa * bc.y + sb * ca.y) + sc * ab.y,
                    (sa * bc.z + sb * ca.z) + sc * ab.z};
    const double den = 2.0 * dot(a, bc);
    return {p0.x + num.x / den, p0.y + num.y / den, p0.z + num.z / den};
}

// c_f = p0 + ((|a|^2 b - |b|^2 a) x (a x b)) / (2 |a x b|^2)
__device__ inline d3 tri_circumcentre(d3 p0, d3 p1, d3 p2) {
    const d3 a = sub(p1, p0), b = sub(p2, p0);
    const d3 axb = cross(a, b);
    const double sa = dot(a, a), sb = dot(b, b);
    const d3 num = cross(sub(scale(sa, b), scale(sb, a)), axb);
    const double den = 2.0 * dot(axb, axb);
    return {p0.x + num.x / den, p0.y + num.y / den, p0.z + num.z / den};
}

