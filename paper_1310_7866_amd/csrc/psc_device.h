// psc_device.h -- device helpers shared by the particle kernel and its adjoint:
// B-spline weights at the nodes around a particle, Esirkepov stencils, and
// interpolation from LDS tiles.
#pragma once

#include <type_traits>

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

// 2 / (1 + t^2) of the Boris rotation, t^2 >= 0, with the hardware
// reciprocal (1 ulp; the IEEE division takes ten instructions)
__device__ __forceinline__ float boris_factor(float t2) { return 2.0f * __builtin_amdgcn_rcpf(1.0f + t2); }

// s_waitcnt immediate that waits for every vector memory operation and for
// nothing else (vmcnt 0; expcnt 7 and lgkmcnt 15 do not wait)
constexpr int kWaitVmcnt0 = 0x0F70;

// Element i of a global array whose byte offsets stay below 2^32 (a species'
// arrays: at most 2^30 entries): the base stays in scalar registers and each
// lane adds a 32-bit byte offset, one address operation per lane shared by
// every array indexed with i instead of a 64-bit add per access.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *at32(__attribute__((address_space(1))) T *base,
                                                                     uint32_t i) {
    using B = typename std::conditional<std::is_const<T>::value, const uint8_t, uint8_t>::type;
    return reinterpret_cast<__attribute__((address_space(1))) T *>(
        reinterpret_cast<__attribute__((address_space(1))) B *>(base) + i * (uint32_t)sizeof(T));
}

// pointers into device memory known to be global (loads and stores become
// global_* instead of flat_*, which would also wait on LDS traffic)
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> to_global(T *p) { return (gptr<T>)p; }

// ---------------------------------------------------------------------------
// wave-level segmented sums (DPP) for frame sums of sorted particles
// ---------------------------------------------------------------------------
// Particles are sorted by cell, so the 64 lanes of a wave mostly share one or
// two cells and would hit the same LDS words with atomics.  Instead each lane
// writes what it adds (current, or the transposed interpolation of the
// adjoint) into a fixed per-cell frame and the wave forms segmented
// inclusive sums (segment = run of lanes with equal cell) over rows of SW
// lanes: DPP row shifts and row broadcasts, each multiplied by a per-lane
// 0/1 mask that is 1 only where the source lane lies in the same segment, so
// every step is one DPP multiply-add.  The last lane of each segment piece
// within a row group then adds the piece's sum to LDS.
struct RowScan {
    float m[6];    // multipliers of the six steps (1: source lane in my segment)
    bool tail;     // last lane of its segment within its group of SW lanes
};

template <int SW>
__device__ __forceinline__ RowScan row_scan_setup(int key) {
    const int lane = threadIdx.x & 63;
    const int left = __shfl_up(key, 1, 64);
    const uint64_t heads = __ballot(lane == 0 || left != key);
    const uint64_t le = lane == 63 ? ~0ull : ((2ull << lane) - 1);
    const int start = 63 - __clzll(heads & le);   // first lane of my segment
    const int row0 = lane & ~15;
    const int d = lane - (start > row0 ? start : row0);
    RowScan r;
    r.m[0] = d >= 1 ? 1.0f : 0.0f;
    r.m[1] = d >= 2 ? 1.0f : 0.0f;
    r.m[2] = d >= 4 ? 1.0f : 0.0f;
    r.m[3] = d >= 8 ? 1.0f : 0.0f;
    r.m[4] = ((lane & 16) && start < row0) ? 1.0f : 0.0f;   // from the last lane of the row below
    r.m[5] = (lane >= 32 && start < 32) ? 1.0f : 0.0f;     // from lane 31
    r.tail = lane == 63 || ((heads >> (lane + 1)) & 1ull) || (lane & (SW - 1)) == SW - 1;
    return r;
}

// Segmented inclusive sums of four independent values: every step is one
// v_fmac_f32_dpp (v += m * v[source lane]).  The four chains are interleaved
// so that a value is read through DPP three instructions after it was
// written (the hardware wants two wait states between a VALU write and a DPP
// read of the same register, five after a VALU write of EXEC; the leading
// s_nop covers whatever precedes the block).  Rows not selected by a
// broadcast's row mask keep their value.  The block is volatile: it reads
// other lanes, so it must stay where every lane of the wave executes it.
#define PSC_FMAC_DPP(CTL, M) \
    "v_fmac_f32_dpp %0, %0, " M " " CTL "\n\t" \
    "v_fmac_f32_dpp %1, %1, " M " " CTL "\n\t" \
    "v_fmac_f32_dpp %2, %2, " M " " CTL "\n\t" \
    "v_fmac_f32_dpp %3, %3, " M " " CTL "\n\t"
#define PSC_SHR(N) "row_shr:" #N " row_mask:0xf bank_mask:0xf bound_ctrl:1"

template <int SW>
__device__ __forceinline__ void row_scan4(float &a, float &b, float &c, float &d, const RowScan &r) {
    if constexpr (SW == 16) {
        asm volatile("s_nop 4\n\t" PSC_FMAC_DPP(PSC_SHR(1), "%4") PSC_FMAC_DPP(PSC_SHR(2), "%5")
                PSC_FMAC_DPP(PSC_SHR(4), "%6") PSC_FMAC_DPP(PSC_SHR(8), "%7")
            : "+v"(a), "+v"(b), "+v"(c), "+v"(d)
            : "v"(r.m[0]), "v"(r.m[1]), "v"(r.m[2]), "v"(r.m[3]));
    } else if constexpr (SW == 32) {
        asm volatile("s_nop 4\n\t" PSC_FMAC_DPP(PSC_SHR(1), "%4") PSC_FMAC_DPP(PSC_SHR(2), "%5")
                PSC_FMAC_DPP(PSC_SHR(4), "%6") PSC_FMAC_DPP(PSC_SHR(8), "%7")
                    PSC_FMAC_DPP("row_bcast:15 row_mask:0xa bank_mask:0xf", "%8")
            : "+v"(a), "+v"(b), "+v"(c), "+v"(d)
            : "v"(r.m[0]), "v"(r.m[1]), "v"(r.m[2]), "v"(r.m[3]), "v"(r.m[4]));
    } else {
        static_assert(SW == 64, "scan width 16, 32 or 64");
        asm volatile("s_nop 4\n\t" PSC_FMAC_DPP(PSC_SHR(1), "%4") PSC_FMAC_DPP(PSC_SHR(2), "%5")
                PSC_FMAC_DPP(PSC_SHR(4), "%6") PSC_FMAC_DPP(PSC_SHR(8), "%7")
                    PSC_FMAC_DPP("row_bcast:15 row_mask:0xa bank_mask:0xf", "%8")
                        PSC_FMAC_DPP("row_bcast:31 row_mask:0xc bank_mask:0xf", "%9")
            : "+v"(a), "+v"(b), "+v"(c), "+v"(d)
            : "v"(r.m[0]), "v"(r.m[1]), "v"(r.m[2]), "v"(r.m[3]), "v"(r.m[4]), "v"(r.m[5]));
    }
}
#undef PSC_SHR
#undef PSC_FMAC_DPP

// segmented sums of N values (N a multiple of 4) in place
template <int SW, int N>
__device__ __forceinline__ void row_scan(float (&v)[N], const RowScan &r) {
    static_assert(N % 4 == 0, "values come in groups of four");
#pragma unroll
    for (int k = 0; k < N; k += 4) row_scan4<SW>(v[k], v[k + 1], v[k + 2], v[k + 3], r);
}

}  // namespace psc
