// psc_device.h -- device helpers shared by the particle kernel and its adjoint:
// B-spline weights at the nodes around a particle, Esirkepov stencils, and
// interpolation from LDS tiles.
#pragma once

#include "psc_internal.h"

namespace psc {

// ---------------------------------------------------------------------------
// B-spline weights (b1 or b2 evaluated at the nodes around the particle)
// ---------------------------------------------------------------------------
// Position given as in-cell offset o in [0, 1) of cell 0.  "node" weights are
// for quantities located at integer positions, "half" weights for quantities
// located at half-integer positions (stored at their lower index).  Returns
// the first node (relative to the cell) and ORDER+1 weights.
template <int ORDER>
__device__ __forceinline__ int node_weights(float o, float w[ORDER + 1]) {
    if constexpr (ORDER == 1) {
        w[0] = 1.0f - o;
        w[1] = o;
        return 0;
    } else {
        const int up = o >= 0.5f;
        const float d = o - (float)up;  // distance from the nearest node, [-1/2, 1/2)
        const float a = 0.5f - d, b = 0.5f + d;
        w[0] = 0.5f * a * a;
        w[1] = 0.75f - d * d;
        w[2] = 0.5f * b * b;
        return up - 1;
    }
}

template <int ORDER>
__device__ __forceinline__ int half_weights(float o, float w[ORDER + 1]) {
    if constexpr (ORDER == 1) {
        const int up = o >= 0.5f;
        const float d = up ? o - 0.5f : o + 0.5f;
        w[0] = 1.0f - d;
        w[1] = d;
        return up - 1;
    } else {
        const float d = o - 0.5f;
        const float a = 0.5f - d, b = 0.5f + d;
        w[0] = 0.5f * a * a;
        w[1] = 0.75f - d * d;
        w[2] = 0.5f * b * b;
        return -1;
    }
}

// Start and end weights of one dimension on a common stencil of ORDER+2
// nodes: the particle starts at offset o0 in cell 0 and ends at offset o1 in
// cell s (|s| <= 1).  Both weight sets use node_weights so that the end
// weights equal the start weights of the next step bit for bit.
template <int ORDER>
__device__ __forceinline__ int stencil(float o0, int s, float o1, float S0[ORDER + 2], float S1[ORDER + 2]) {
    float w0[ORDER + 1], w1[ORDER + 1];
    const int b0 = node_weights<ORDER>(o0, w0);
    const int b1 = node_weights<ORDER>(o1, w1) + s;
    const int base = b0 < b1 ? b0 : b1;
    const bool k0 = b0 != base, k1 = b1 != base;
#pragma unroll
    for (int r = 0; r < ORDER + 2; ++r) {
        const float lo0 = r <= ORDER ? w0[r] : 0.0f, hi0 = r >= 1 ? w0[r - 1] : 0.0f;
        const float lo1 = r <= ORDER ? w1[r] : 0.0f, hi1 = r >= 1 ? w1[r - 1] : 0.0f;
        S0[r] = k0 ? hi0 : lo0;
        S1[r] = k1 ? hi1 : lo1;
    }
    return base;
}

// ---------------------------------------------------------------------------
// interpolation from an LDS tile
// ---------------------------------------------------------------------------
template <int ORDER>
__device__ __forceinline__ float gather2(const float *F, int pitch, int iy, int iz, const float *wy,
                                         const float *wz) {
    const float *p = F + iz * pitch + iy;
    float s = 0.0f;
#pragma unroll
    for (int b = 0; b <= ORDER; ++b) {
        float r = 0.0f;
#pragma unroll
        for (int a = 0; a <= ORDER; ++a) r = fmaf(wy[a], p[b * pitch + a], r);
        s = fmaf(wz[b], r, s);
    }
    return s;
}

// two components interleaved in one tile (same staggering, same weights)
template <int ORDER>
__device__ __forceinline__ float2 gather2_pair(const float2 *F, int pitch, int iy, int iz, const float *wy,
                                               const float *wz) {
    const float2 *p = F + iz * pitch + iy;
    float sx = 0.0f, sy = 0.0f;
#pragma unroll
    for (int b = 0; b <= ORDER; ++b) {
        float rx = 0.0f, ry = 0.0f;
#pragma unroll
        for (int a = 0; a <= ORDER; ++a) {
            const float2 f = p[b * pitch + a];
            rx = fmaf(wy[a], f.x, rx);
            ry = fmaf(wy[a], f.y, ry);
        }
        sx = fmaf(wz[b], rx, sx);
        sy = fmaf(wz[b], ry, sy);
    }
    return make_float2(sx, sy);
}

template <int ORDER>
__device__ __forceinline__ float gather3(const float *F, int px, int pxy, int ix, int iy, int iz,
                                         const float *wx, const float *wy, const float *wz) {
    const float *p = F + iz * pxy + iy * px + ix;
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c <= ORDER; ++c) {
        float t = 0.0f;
#pragma unroll
        for (int b = 0; b <= ORDER; ++b) {
            float r = 0.0f;
#pragma unroll
            for (int a = 0; a <= ORDER; ++a) r = fmaf(wx[a], p[c * pxy + b * px + a], r);
            t = fmaf(wy[b], r, t);
        }
        s = fmaf(wz[c], t, s);
    }
    return s;
}

__device__ __forceinline__ void lds_add(float *p, float v) { atomicAdd(p, v); }
__device__ __forceinline__ void lds_add(double *p, float v) { atomicAdd(p, (double)v); }

// quotient and remainder of 0 <= a < 2^22 by b >= 1 (inv_b = 1/b rounded to
// float).  (a + 1/2)/b lies at least 1/(2b) from an integer; a + 1/2 is exact
// and the two roundings (of 1/b and of the product) change the product by a
// relative 2^-23 at most, i.e. by less than 2^22/b * 2^-23 = 1/(2b), so the
// truncation is the exact quotient.
__device__ __forceinline__ int divmod_small(int a, int b, float inv_b, int &rem) {
    const int q = (int)(((float)a + 0.5f) * inv_b);
    rem = a - q * b;
    return q;
}

// 1/sqrt(x) for x >= 1 (no denormal range to guard): the hardware estimate
__device__ __forceinline__ float rsqrt_ge1(float x) { return __builtin_amdgcn_rsqf(x); }

// pointers into device memory known to be global (loads and stores become
// global_* instead of flat_*, which would also wait on LDS traffic)
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> to_global(T *p) { return (gptr<T>)p; }


}  // namespace psc
