// psc_push.hip -- the fused particle kernel: field interpolation, relativistic
// Boris push, position update and Esirkepov current deposit (paper: section
// "Time integration of the quasi-particle equations of motion", fig. psc_new
// particle loop; GPU design: sections "Particle Advance and Field
// Interpolation", "Current deposition" and "Fusing of GPU kernels").
//
// One workgroup takes one work item = up to `chunk` consecutive particles of
// one (run, species, patch).  It stages E and B of the patch plus ghost layers
// in LDS, zeroes an LDS current tile, pushes its particles (reading them
// through the sort permutation, writing them in sorted order into the other
// buffer set, so the physical reorder of the sort costs no extra pass), and
// adds the LDS tile into the patch's current tile in HBM.
#include <type_traits>

#include "psc_device.h"

namespace psc {

// Compile-time shape of the particle kernel (the defaults are the measured
// best on gfx950; -D overrides build the alternatives for comparison):
//   PSC_SCAN_WIDTH   lanes per group of the segmented current sums (16/32/64)
//   PSC_QUEUE_SLOTS  per-wave queue of particles whose support changes nodes
#ifndef PSC_SCAN_WIDTH
#define PSC_SCAN_WIDTH 32
#endif
#ifndef PSC_QUEUE_SLOTS
#define PSC_QUEUE_SLOTS 64
#endif
//   PSC_PACK_TAILS   segments per wave whose sums are staged and added with
//                    full-lane atomics (more fall back to per-tail atomics)
#ifndef PSC_PACK_TAILS
#define PSC_PACK_TAILS 3
#endif
//   PSC_FRAMES       0 sends every particle through the per-lane atomic
//                    deposit (the ablation of the frames and wave sums)
#ifndef PSC_FRAMES
#define PSC_FRAMES 1
#endif
//   PSC_JCOPIES      redundant copies of the LDS current tile for the
//                    per-lane atomic deposit: lane l adds into copy l mod N,
//                    the flush sums them (with PSC_FRAMES 0: the ablation of
//                    shared-memory copies against atomic conflicts)
#ifndef PSC_JCOPIES
#define PSC_JCOPIES 1
#endif
//   PSC_MIX          1: lane g of a work item takes particle
//                    (g mod 64) ceil(n / 64) + g div 64 of its n (one
//                    particle per lane), so a wave's lanes are spread over
//                    the item's cells instead of consecutive (with
//                    PSC_FRAMES 0: the ablation of mixing within super-cells)
#ifndef PSC_MIX
#define PSC_MIX 0
#endif
//   PSC_BAND         0 stages and flushes the whole patch tile for every
//                    work item instead of the band of planes its particles reach
#ifndef PSC_BAND
#define PSC_BAND 1
#endif
//   PSC_WAVES_3D1    waves per SIMD the 3-d order-1 kernel keeps room for
//                    (0: the register allocator's free choice)
#ifndef PSC_WAVES_3D1
#define PSC_WAVES_3D1 4
#endif
//   PSC_PREFETCH     1: with one particle per lane, the state of a lane's
//                    next particle (cell key, offsets, momenta) is loaded at
//                    the start of the current round and its permutation entry
//                    a round earlier, so a round waits for no memory round
//                    trip of its own (0: three dependent ones per round:
//                    permutation, key, state)
#ifndef PSC_PREFETCH
#define PSC_PREFETCH 1
#endif
//   PSC_WAVES_PER_EU occupancy the register allocator must allow for every
//                    instantiation (0: the measured per-shape choice below)
#ifndef PSC_WAVES_PER_EU
#define PSC_WAVES_PER_EU 0
#endif
// Waves per SIMD the register allocator must leave room for (0: its free
// choice).  In 2-d the LDS tiles already limit a compute unit to two
// 512-thread workgroups; the small 3-d order-1 tiles allow more, so that
// kernel keeps to 128 registers (four waves per SIMD).
template <int DIM, int ORDER, bool RUNS>
constexpr int push_waves() {
    return PSC_WAVES_PER_EU > 0 ? PSC_WAVES_PER_EU : (DIM == 3 && ORDER == 1 && !RUNS ? PSC_WAVES_3D1 : 0);
}
#define PSC_OCCUPANCY __attribute__((amdgpu_waves_per_eu(push_waves<DIM, ORDER, RUNS>())))
constexpr int kScanWidth = PSC_SCAN_WIDTH;
constexpr int kJCopies = PSC_JCOPIES;
static_assert(kJCopies >= 1 && (kJCopies == 1 || !PSC_FRAMES), "redundant tiles only for the per-lane deposit");
static_assert(!PSC_MIX || !PSC_FRAMES, "mixed lanes only for the per-lane deposit");
constexpr int kQueueSlots = PSC_QUEUE_SLOTS;
constexpr int kPackTails = PSC_PACK_TAILS;
static_assert(kQueueSlots >= 1 && kQueueSlots <= 64, "queue slots 1..64");

// words of one queued particle whose support changes nodes: packed cell and
// moves, start and end offsets, and in 2-d the out-of-plane current factor
constexpr int cross_words(int dim) { return dim == 2 ? 6 : 7; }

// LDS layout of the particle kernel (offsets in floats, each region starting
// on 16 bytes): field tile, current tile (doubles), per-wave crossing queues,
// per-wave staging of segment sums, cell table.  Returns the total.
struct PushLds {
    int cur, queue, stage, table, total;
};
__host__ __device__ constexpr int align4(int n) { return (n + 3) & ~3; }
__host__ __device__ inline PushLds push_lds_layout(int fcells, int jcells, int waves, int qwords, int swords,
                                                   int twords) {
    PushLds L{};
    L.cur = align4(6 * fcells);
    L.queue = align4(L.cur + 6 * jcells * kJCopies);   // current tile(s) in doubles
    L.stage = align4(L.queue + waves * qwords);
    L.table = align4(L.stage + waves * align4(swords));
    L.total = L.table + twords;
    return L;
}

// ---------------------------------------------------------------------------
// work items
// ---------------------------------------------------------------------------
// Work items per unit: one thread per unit writes how many chunks its
// particles need into item_start[u]; k_items_scan turns the counts into the
// exclusive prefix item_start[0..n_units].
__global__ void __launch_bounds__(256) k_unit_items(const RunDev *__restrict__ runs, const Unit *__restrict__ units,
                                                    int n_units, int cs_sel,
                                                    int32_t *__restrict__ item_start) {
    const int u = blockIdx.x * 256 + threadIdx.x;
    if (u >= n_units) return;
    const Unit U = units[u];
    const RunDev &R = runs[U.run];
    int pc[3];
    patch_coords(R, U.patch, pc);
    const int64_t kb = patch_key_base(R, pc[0], pc[1], pc[2]);
    const int64_t ke = kb + (int64_t)patch_ext(R, 0, pc[0]) * patch_ext(R, 1, pc[1]) * patch_ext(R, 2, pc[2]);
    const int32_t *cs = R.sp[U.species].cs[cs_sel];
    item_start[u] = (cs[ke] - cs[kb] + R.chunk - 1) / R.chunk;
}

// One workgroup: exclusive prefix of the per-unit item counts in place, the
// total in item_start[n_units].  The counts pass through LDS in tiles of
// kItemsTile: coalesced loads, eight consecutive counts per thread, a scan of
// the thread sums (within each wave by lane shuffles, then over the waves),
// and coalesced stores of the prefixes.  Each lane reading its own run of
// counts straight from memory would touch a separate cache line per lane and
// instruction, all on the one compute unit.  Also resets the work queues of
// the persistent launch (written before the particle kernel starts: same
// stream).
constexpr int kItemsPer = 8;
constexpr int kItemsTile = 1024 * kItemsPer;
__global__ void __launch_bounds__(1024) k_items_scan(int n_units, int32_t *__restrict__ item_start,
                                                     int32_t *__restrict__ queue) {
    __shared__ __align__(16) int32_t tile[kItemsTile];
    __shared__ int32_t wtot[16];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (queue && t < 8) queue[kQueueStride * t] = 0;
    int32_t carry = 0;
    for (int base = 0; base < n_units; base += kItemsTile) {
        const int n = imin(kItemsTile, n_units - base);
#pragma unroll
        for (int k = 0; k < kItemsPer; ++k) {
            const int i = k * 1024 + t;
            tile[i] = i < n ? item_start[base + i] : 0;
        }
        __syncthreads();
        int4 *mine = reinterpret_cast<int4 *>(tile) + 2 * t;   // counts 8t .. 8t + 7
        const int4 va = mine[0], vb = mine[1];
        const int32_t sum = va.x + va.y + va.z + va.w + vb.x + vb.y + vb.z + vb.w;
        int32_t inc = sum;   // inclusive scan over the wave's lanes
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t v = __shfl_up(inc, off, 64);
            if (lane >= off) inc += v;
        }
        if (lane == 63) wtot[wv] = inc;
        __syncthreads();
        int32_t before = carry, total = 0;   // sums of the waves below, of all waves
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            const int32_t x = wtot[w];
            before += w < wv ? x : 0;
            total += x;
        }
        int32_t run = before + inc - sum;   // exclusive prefix of count 8t
        int4 pa, pb;
        pa.x = run; run += va.x;
        pa.y = run; run += va.y;
        pa.z = run; run += va.z;
        pa.w = run; run += va.w;
        pb.x = run; run += vb.x;
        pb.y = run; run += vb.y;
        pb.z = run; run += vb.z;
        pb.w = run;
        mine[0] = pa;
        mine[1] = pb;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kItemsPer; ++k) {
            const int i = k * 1024 + t;
            if (i < n) item_start[base + i] = tile[i];
        }
        carry += total;
        __syncthreads();   // the tile and the wave totals are reused
    }
    if (t == 0) item_start[n_units] = carry;
}

hipError_t launch_items_scan(int n_units, int32_t *item_start, int32_t *queue, hipStream_t s) {
    hipLaunchKernelGGL(k_items_scan, dim3(1), dim3(1024), 0, s, n_units, item_start, queue);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Esirkepov current of one particle, added lane by lane with LDS atomics
// (general stencil: used for particles whose support changes cell)
// ---------------------------------------------------------------------------
template <int DIM, int ORDER>
__device__ __forceinline__ void deposit_lane(double *jtile, int jcells, int jx_, int jy_, int lx, int ly, int lz,
                                             const float o[3], const int s[3], const float o1[3], float jfx,
                                             float jfy, float jfz, float fxv) {
    constexpr int L = ORDER + 2;
    constexpr int JLO = ORDER;
    float S0y[L], S1y[L], S0z[L], S1z[L];
    const int by = stencil<ORDER>(o[1], s[1], o1[1], S0y, S1y);
    const int bz = stencil<ORDER>(o[2], s[2], o1[2], S0z, S1z);
    float DSy[L], DSz[L], Ay[L], Az[L], Cy[L], Cz[L];
#pragma unroll
    for (int r = 0; r < L; ++r) {
        DSy[r] = S1y[r] - S0y[r];
        DSz[r] = S1z[r] - S0z[r];
        Ay[r] = fmaf(0.5f, DSy[r], S0y[r]);
        Az[r] = fmaf(0.5f, DSz[r], S0z[r]);
        Cy[r] = r == 0 ? DSy[0] : Cy[r - 1] + DSy[r];
        Cz[r] = r == 0 ? DSz[0] : Cz[r - 1] + DSz[r];
    }
    double *Jx = jtile, *Jy = jtile + jcells, *Jz = jtile + 2 * jcells;
    if constexpr (DIM == 2) {
        const int base = (lz + bz + JLO) * jy_ + (ly + by + JLO);
#pragma unroll
        for (int b = 0; b < L; ++b)
#pragma unroll
            for (int a = 0; a < L - 1; ++a) lds_add(&Jy[base + b * jy_ + a], jfy * Cy[a] * Az[b]);
#pragma unroll
        for (int b = 0; b < L - 1; ++b)
#pragma unroll
            for (int a = 0; a < L; ++a) lds_add(&Jz[base + b * jy_ + a], jfz * Ay[a] * Cz[b]);
#pragma unroll
        for (int b = 0; b < L; ++b)
#pragma unroll
            for (int a = 0; a < L; ++a)
                lds_add(&Jx[base + b * jy_ + a], fxv * fmaf(DSy[a] * DSz[b], 1.0f / 12.0f, Ay[a] * Az[b]));
    } else {
        float S0x[L], S1x[L];
        const int bx = stencil<ORDER>(o[0], s[0], o1[0], S0x, S1x);
        float DSx[L], Ax[L], Cx[L];
#pragma unroll
        for (int r = 0; r < L; ++r) {
            DSx[r] = S1x[r] - S0x[r];
            Ax[r] = fmaf(0.5f, DSx[r], S0x[r]);
            Cx[r] = r == 0 ? DSx[0] : Cx[r - 1] + DSx[r];
        }
        const int pxy = jx_ * jy_;
        const int base = (lz + bz + JLO) * pxy + (ly + by + JLO) * jx_ + (lx + bx + JLO);
#pragma unroll
        for (int c = 0; c < L; ++c)
#pragma unroll
            for (int b = 0; b < L; ++b) {
                const float wyz = fmaf(DSy[b] * DSz[c], 1.0f / 12.0f, Ay[b] * Az[c]);
#pragma unroll
                for (int a = 0; a < L - 1; ++a) lds_add(&Jx[base + c * pxy + b * jx_ + a], jfx * Cx[a] * wyz);
            }
#pragma unroll
        for (int c = 0; c < L; ++c)
#pragma unroll
            for (int b = 0; b < L - 1; ++b)
#pragma unroll
                for (int a = 0; a < L; ++a) {
                    const float wxz = fmaf(DSx[a] * DSz[c], 1.0f / 12.0f, Ax[a] * Az[c]);
                    lds_add(&Jy[base + c * pxy + b * jx_ + a], jfy * Cy[b] * wxz);
                }
#pragma unroll
        for (int c = 0; c < L - 1; ++c)
#pragma unroll
            for (int b = 0; b < L; ++b)
#pragma unroll
                for (int a = 0; a < L; ++a) {
                    const float wxy = fmaf(DSx[a] * DSy[b], 1.0f / 12.0f, Ax[a] * Ay[b]);
                    lds_add(&Jz[base + c * pxy + b * jx_ + a], jfz * Cz[c] * wxy);
                }
    }
}

// ---------------------------------------------------------------------------
// Villasenor-Buneman current of one 1st-order particle, lane by lane: the
// straight path from offset o in its cell to s + o1 is cut where it crosses
// cell faces (at most once per dimension); each piece lies in one cell and
// adds the flux of its linear cloud through that cell's edges: along y,
// q w dy/dt times the time average of the other linear weights over the
// piece (midpoint product, plus the alternating dx dz / 12 term in 3-d).  In
// 2-d the out-of-plane current is q w v_x times the piece's share of the
// step times the linear weights at its midpoint.
// ---------------------------------------------------------------------------
template <int DIM>
__device__ __forceinline__ void deposit_lane_vb(double *jtile, int jcells, int jx_, int jy_, int lx, int ly, int lz,
                                                const float o[3], const int s[3], const float o1[3], float jfx,
                                                float jfy, float jfz, float fxv) {
    constexpr int D0 = DIM == 3 ? 0 : 1;   // first active dimension
    constexpr int JLO = 1;
    float dx[3] = {0.0f, 0.0f, 0.0f};
    float t[4];
    int nt = 0;
#pragma unroll
    for (int d = D0; d < 3; ++d) {
        dx[d] = ((float)s[d] + o1[d]) - o[d];
        if (s[d] != 0) t[nt++] = ((s[d] > 0 ? 1.0f : 0.0f) - o[d]) / dx[d];
    }
    for (int i = 1; i < nt; ++i)   // at most three cut points
        for (int k = i; k > 0 && t[k] < t[k - 1]; --k) {
            const float x = t[k];
            t[k] = t[k - 1];
            t[k - 1] = x;
        }
    t[nt] = 1.0f;
    double *Jx = jtile, *Jy = jtile + jcells, *Jz = jtile + 2 * jcells;
    const float gx = -jfx, gy = -jfy, gz = -jfz;   // q w dx_d / dt
    float ta = 0.0f;
    for (int p = 0; p <= nt; ++p) {
        const float tb = t[p];
        if (tb > ta) {
            int c[3] = {0, 0, 0};
            float m[3] = {0.0f, 0.0f, 0.0f}, dd[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int d = D0; d < 3; ++d) {
                const float pa = fmaf(ta, dx[d], o[d]), pb = fmaf(tb, dx[d], o[d]);
                const float mid = 0.5f * (pa + pb);
                c[d] = (int)floorf(mid);
                m[d] = mid - (float)c[d];
                dd[d] = pb - pa;
            }
            if constexpr (DIM == 2) {
                const int base = (lz + c[2] + JLO) * jy_ + (ly + c[1] + JLO);
                const float wy0 = 1.0f - m[1], wy1 = m[1], wz0 = 1.0f - m[2], wz1 = m[2];
                lds_add(&Jy[base], gy * dd[1] * wz0);
                lds_add(&Jy[base + jy_], gy * dd[1] * wz1);
                lds_add(&Jz[base], gz * dd[2] * wy0);
                lds_add(&Jz[base + 1], gz * dd[2] * wy1);
                const float f = fxv * (tb - ta);
                lds_add(&Jx[base], f * wy0 * wz0);
                lds_add(&Jx[base + 1], f * wy1 * wz0);
                lds_add(&Jx[base + jy_], f * wy0 * wz1);
                lds_add(&Jx[base + jy_ + 1], f * wy1 * wz1);
            } else {
                const int pxy = jx_ * jy_;
                const int base = (lz + c[2] + JLO) * pxy + (ly + c[1] + JLO) * jx_ + (lx + c[0] + JLO);
                const float w[3][2] = {{1.0f - m[0], m[0]}, {1.0f - m[1], m[1]}, {1.0f - m[2], m[2]}};
                const float xyz = dd[1] * dd[2] * (1.0f / 12.0f), xz = dd[0] * dd[2] * (1.0f / 12.0f),
                            xy = dd[0] * dd[1] * (1.0f / 12.0f);
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const float sg = b == e ? 1.0f : -1.0f;
                        lds_add(&Jx[base + e * pxy + b * jx_], gx * dd[0] * fmaf(sg, xyz, w[1][b] * w[2][e]));
                        lds_add(&Jy[base + e * pxy + b], gy * dd[1] * fmaf(sg, xz, w[0][b] * w[2][e]));
                        lds_add(&Jz[base + e * jx_ + b], gz * dd[2] * fmaf(sg, xy, w[0][b] * w[1][e]));
                    }
            }
        }
        ta = tb;
    }
}

// Node weights of one dimension on the fixed per-cell frame used by the wave
// reduction: order 1 -> nodes {0, 1}, order 2 -> nodes {-1, 0, 1, 2}.  Valid
// for a particle whose support does not change (see `stays` below).
template <int ORDER>
__device__ __forceinline__ void frame_weights(float o0, float o1, float S0[2 * ORDER], float S1[2 * ORDER]) {
    float w0[ORDER + 1], w1[ORDER + 1];
    const int b0 = node_weights<ORDER>(o0, w0);
    node_weights<ORDER>(o1, w1);
    if constexpr (ORDER == 1) {
        S0[0] = w0[0]; S0[1] = w0[1];
        S1[0] = w1[0]; S1[1] = w1[1];
    } else {
        const bool up = b0 == 0;  // support {0,1,2} instead of {-1,0,1}
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            S0[r] = up ? (r >= 1 ? w0[r - 1] : 0.0f) : (r <= 2 ? w0[r] : 0.0f);
            S1[r] = up ? (r >= 1 ? w1[r - 1] : 0.0f) : (r <= 2 ? w1[r] : 0.0f);
        }
    }
}

// does the particle's interpolation support stay on the same nodes?
template <int ORDER>
__device__ __forceinline__ bool stays(float o0, int s, float o1) {
    if constexpr (ORDER == 1) return s == 0;
    else return s + (o1 >= 0.5f ? 1 : 0) == (o0 >= 0.5f ? 1 : 0);
}

// ---------------------------------------------------------------------------
// the particle kernel
// ---------------------------------------------------------------------------
// unit u with item_start[u] <= item < item_start[u+1]
__device__ __forceinline__ int unit_of_item(const int32_t *__restrict__ item_start, int n_units, int item) {
    int lo = 0, hi = n_units;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (item_start[mid] <= item) lo = mid; else hi = mid;
    }
    return lo;
}

// Number of per-cell frame values of a particle whose support keeps its
// nodes (2-d: Jy FL(FL-1), Jz (FL-1)FL, Jx FL^2; 3-d: FL^2(FL-1) each, FL =
// 2 ORDER frame nodes per dimension), 0 where the kernel deposits per lane.
template <int DIM, int ORDER>
__host__ __device__ constexpr int frame_values() {
    return (DIM == 3 && ORDER == 2) ? 0
                                    : (DIM == 2 ? 2 * (2 * ORDER) * (2 * ORDER - 1) + (2 * ORDER) * (2 * ORDER)
                                                : 3 * (2 * ORDER) * (2 * ORDER) * (2 * ORDER - 1));
}

// LDS offset of frame value j relative to the frame's base node in the
// current tile (the order of the values is the order of the flush loops)
template <int DIM, int ORDER>
__device__ __forceinline__ int frame_offset(int j, int jx_, int jy_, int jcells) {
    constexpr int FL = 2 * ORDER;
    if constexpr (DIM == 2) {
        constexpr int NY2 = FL * (FL - 1);
        if (j < NY2) return jcells + (j / (FL - 1)) * jy_ + j % (FL - 1);
        if (j < 2 * NY2) return 2 * jcells + ((j - NY2) / FL) * jy_ + (j - NY2) % FL;
        return ((j - 2 * NY2) / FL) * jy_ + (j - 2 * NY2) % FL;
    } else {
        constexpr int NC3 = FL * FL * (FL - 1);
        const int pxy = jx_ * jy_;
        if (j < NC3) {
            const int t = j / (FL - 1);
            return (t / FL) * pxy + (t % FL) * jx_ + j % (FL - 1);
        }
        if (j < 2 * NC3) {
            const int jj = j - NC3, t = jj / FL;
            return jcells + (t / (FL - 1)) * pxy + (t % (FL - 1)) * jx_ + jj % FL;
        }
        const int jj = j - 2 * NC3, t = jj / FL;
        return 2 * jcells + (t / FL) * pxy + (t % FL) * jx_ + jj % FL;
    }
}

// One work item: stage the patch's fields, push its chunk of particles, add
// the chunk's current into the patch tile.  Ends with a barrier so the caller
// may start the next item on the same LDS.
//
// The chunk's particles are sorted by cell.  Lane g of a round pushes the K
// consecutive particles beg + g K + j (j < K, K = 1 or 2, one instantiation
// each) one after another, adding the Esirkepov current of those whose
// interpolation support keeps its nodes and whose cell is the one of the
// lane's first particle into a per-cell frame held in registers.  At the end
// of a round the wave forms segmented sums of the frames over lanes of equal
// cell (consecutive, since the particles are sorted) and the last lane of
// each segment adds them to the LDS current tile: one scan and one set of
// LDS atomics per K particles of a lane.  The other particles (support
// changes nodes, or a later cell than the lane's frame) wait in a per-wave
// queue and are deposited in batches with per-lane LDS atomics.  With K = 2
// the outputs are exchanged across the wave before the stores so that
// consecutive lanes store consecutive slots.
template <int DIM, int ORDER, int NT, bool RUNS>
__device__ __forceinline__ void push_item(const RunDev *__restrict__ runs, const Unit *__restrict__ units,
                                          const int32_t *__restrict__ item_start, int lo, int item,
                                          int front, int cs_sel, int use_perm, int K, uint32_t *__restrict__ err,
                                          float *lds) {
    constexpr int FLO = 1, FHI = ORDER;   // field ghosts
    constexpr int JLO = ORDER, JHI = ORDER + 1;
    constexpr int FL = 2 * ORDER;         // frame nodes per dimension
    constexpr int FB = ORDER == 1 ? 0 : -1;
    // the 3-d order-2 frame holds 144 values per particle: lane atomics instead
    constexpr bool kReduce = !(DIM == 3 && ORDER == 2);
    // frame values: 2-d Jy FL(FL-1), Jz (FL-1)FL, Jx FL^2; 3-d FL^2(FL-1) each
    constexpr int NY2 = FL * (FL - 1);
    constexpr int NC3 = FL * FL * (FL - 1);
    constexpr int NV = !kReduce ? 4 : (DIM == 2 ? 2 * NY2 + FL * FL : 3 * NC3);
    constexpr int SW = kScanWidth;
    constexpr int QW = cross_words(DIM);   // words of one queued crossing particle
    constexpr int QS = kQueueSlots;

    const Unit U = units[lo];
    const RunDev &R = runs[U.run];
    const SpeciesDev &S = R.sp[U.species];

    int pc[3];
    patch_coords(R, U.patch, pc);
    const int hx = DIM == 3 ? patch_ext(R, 0, pc[0]) : 1;
    const int hy = patch_ext(R, 1, pc[1]);
    const int hz = patch_ext(R, 2, pc[2]);
    const int pcells = hx * hy * hz;
    const int ox = pc[0] * R.P[0], oy = pc[1] * R.P[1], oz = pc[2] * R.P[2];
    const int64_t kb = patch_key_base(R, pc[0], pc[1], pc[2]);
    const int32_t *cs = S.cs[cs_sel];
    // cell offsets outside [0, n] (only after a counter overflow, which the
    // sort flags) must not send the item outside the particle buffers
    const int32_t np_ = (int32_t)S.n;
    const int32_t pend = imin(imax(cs[kb + pcells], 0), np_), pbeg = imin(imax(cs[kb], 0), pend);
    const int32_t beg = pbeg + (item - item_start[lo]) * R.chunk;
    const int32_t end = min(beg + R.chunk, pend);
    if (beg >= end) return;   // only with such offsets (the workgroup's item is uniform)

    // tile geometry (nominal patch size so every tile of the run has one pitch)
    const int fx = DIM == 3 ? R.P[0] + FLO + FHI : 1;
    const int fy = R.P[1] + FLO + FHI, fz = R.P[2] + FLO + FHI;
    const int fcells = fx * fy * fz;
    const int jx_ = DIM == 3 ? R.P[0] + JLO + JHI : 1;
    const int jy_ = R.P[1] + JLO + JHI, jz_ = R.P[2] + JLO + JHI;
    const int jcells = jx_ * jy_ * jz_;
    // 6 * fcells: 3-d Ex Ey Ez Bx By Bz; 2-d Ex, Bx, then (Ey, Bz) and
    // (Ez, By) interleaved in pairs: the two of a pair share their staggering,
    // so one 8-byte LDS read serves both
    // per-wave staging of the segment sums: kPackTails frames of NV values,
    // then their base offsets
    constexpr int PKW = kReduce ? kPackTails * (NV + 1) : 0;
    const PushLds LL = push_lds_layout(fcells, jcells, NT / 64, QS * QW, PKW, 0);
    float *ftile = lds;
    // 3 * jcells doubles: Jx Jy Jz.  Accumulated in double: the LDS add of
    // doubles runs at the full rate of integer atomics on this hardware,
    // the float one more than 20 times slower.
    double *jtile = reinterpret_cast<double *>(lds + LL.cur);
    // per-wave queue of particles whose support changes nodes: QW words
    // (field-major) for each of QS slots
    float *cq = lds + LL.queue + (threadIdx.x >> 6) * (QS * QW);
    float *pk = lds + LL.stage + (threadIdx.x >> 6) * align4(PKW);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    // The item's particles are sorted by cell, so they lie in the planes (2-d:
    // rows) of cells between those of its first and last particle; only the
    // tile planes their stencils reach are staged, cleared and flushed: field
    // tile lz + FLO - 1 .. lz + FLO + ORDER, current tile lz .. lz + 2 ORDER + 1.
    const int fplane = fx * fy, jplane = jx_ * jy_;
    int fr0, fr1, jr0, jr1;
    {
        int32_t sf = use_perm ? S.perm[cs_sel][beg] : beg, sl = use_perm ? S.perm[cs_sel][end - 1] : end - 1;
        if ((uint32_t)sf >= (uint32_t)S.n) sf = beg;
        if ((uint32_t)sl >= (uint32_t)S.n) sl = end - 1;
        const int32_t *ck = S.cell[front];
        const int cpl = hx * hy;   // cells per plane of the patch
        int zf = imin(imax(ck[sf] - (int32_t)kb, 0), pcells - 1) / cpl;
        int zl = imin(imax(ck[sl] - (int32_t)kb, 0), pcells - 1) / cpl;
        if (zl < zf || !PSC_BAND) {   // not in order (or banding off): the whole tile
            zf = 0;
            zl = hz - 1;
        }
        fr0 = zf + FLO - 1;
        fr1 = imin(zl + FLO + ORDER, fz - 1);
        jr0 = zf;
        jr1 = imin(zl + 2 * ORDER + 1, jz_ - 1);
    }
    const int n_fband = (fr1 - fr0 + 1) * fplane, n_jband = (jr1 - jr0 + 1) * jplane;

    // stage E, B (+ghosts), clear the current tile
    {
        const float inv_fx = 1.0f / fx, inv_fy = 1.0f / fy;
        const int64_t nc = R.ncell;
        const gptr<const float> Eg = to_global<const float>(R.E), Bg = to_global<const float>(R.B);
        for (int q = threadIdx.x; q < n_fband; q += NT) {
            const int t = fr0 * fplane + q;
            int tx = 0, ty, tz;
            if constexpr (DIM == 3) {
                const int q = divmod_small(t, fx, inv_fx, tx);
                tz = divmod_small(q, fy, inv_fy, ty);
            } else {
                tz = divmod_small(t, fy, inv_fy, ty);
            }
            const int gx = DIM == 3 ? wrap(ox + tx - FLO, R.n[0]) : 0;
            const int gy = wrap(oy + ty - FLO, R.n[1]);
            const int gz = wrap(oz + tz - FLO, R.n[2]);
            const int64_t g = gx + (int64_t)R.n[0] * (gy + (int64_t)R.n[1] * gz);
            if constexpr (DIM == 2) {
                ftile[t] = Eg[g];
                ftile[fcells + t] = Bg[g];
                reinterpret_cast<float2 *>(ftile + 2 * fcells)[t] = make_float2(Eg[nc + g], Bg[2 * nc + g]);
                reinterpret_cast<float2 *>(ftile + 4 * fcells)[t] = make_float2(Eg[2 * nc + g], Bg[nc + g]);
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    ftile[c * fcells + t] = Eg[c * nc + g];
                    ftile[(3 + c) * fcells + t] = Bg[c * nc + g];
                }
            }
        }
        for (int q = threadIdx.x; q < 3 * n_jband; q += NT) {
            const int c = q / n_jband;
#pragma unroll
            for (int cp = 0; cp < kJCopies; ++cp) jtile[(3 * cp + c) * jcells + jr0 * jplane + (q - c * n_jband)] = 0.0;
        }
    }
    __syncthreads();

    // K = 1 (its own instantiation): lane t of a round takes particle
    // beg + r0 + t, so loads and stores are coalesced.  K = 2: lane t takes
    // beg + 2 (r0 + t) and the next one; its outputs are handed across the
    // wave before the stores so that consecutive lanes store consecutive slots.
    constexpr bool single = !RUNS;
    constexpr int KS = RUNS ? 2 : 1;
    K = KS;
    const int32_t nruns = (end - beg + K - 1) / K;   // lanes' strips of K particles
    const int in = front, outb = 1 - front;
    const gptr<const int32_t> cell_in = to_global<const int32_t>(S.cell[in]);
    const gptr<const float> off_in = to_global<const float>(S.off[in]);
    const gptr<const float> u_in = to_global<const float>(S.u[in]);
    const gptr<const int32_t> id_in = to_global<const int32_t>(S.id[in]);
    const gptr<int32_t> cell_out = to_global(S.cell[outb]);
    const gptr<float> off_out = to_global(S.off[outb]);
    const gptr<float> u_out = to_global(S.u[outb]);
    const gptr<int32_t> id_out = to_global(S.id[outb]);
    const gptr<const int32_t> perm = to_global<const int32_t>(S.perm[cs_sel]);
    const gptr<uint8_t> mc = to_global(S.mc);
    // pairs of 16-bit counters.  Global (not generic) pointers here and for
    // the current flush: a pending flat atomic can complete out of order, so
    // every later wait for a load would have to drain all memory operations
    const gptr<uint32_t> cnt32 = to_global(reinterpret_cast<uint32_t *>(S.cnt));
    const int64_t cap = S.cap;
    // per-component bases of the particle arrays (uniform), indexed through
    // at32 with 32-bit slots; offsets: components (y, z) in 2-d, (x, y, z) in 3-d
    constexpr int D = DIM == 3 ? 3 : 2;
    const gptr<const float> oin[3] = {off_in, off_in + cap, D == 3 ? off_in + 2 * cap : off_in};
    const gptr<const float> uin[3] = {u_in, u_in + cap, u_in + 2 * cap};
    const gptr<float> oout[3] = {off_out, off_out + cap, D == 3 ? off_out + 2 * cap : off_out};
    const gptr<float> uout[3] = {u_out, u_out + cap, u_out + 2 * cap};
    const float h = S.qdt_2m;
    const float qw = S.qw;
    const float dt = R.dt;
    const float cfx = DIM == 3 ? dt * R.inv_dx[0] : 0.0f;
    const float cfy = dt * R.inv_dx[1], cfz = dt * R.inv_dx[2];
    const float jfx = -qw * R.dx[0] / dt, jfy = -qw * R.dx[1] / dt, jfz = -qw * R.dx[2] / dt;
    const float inv_hx = 1.0f / hx, inv_hy = 1.0f / hy;
    double *Jx = jtile, *Jy = jtile + jcells, *Jz = jtile + 2 * jcells;
    uint32_t flags = 0;
    // 1st-order runs may deposit with Villasenor-Buneman: the particles that
    // leave their cell go through the piece-wise lane deposit, and in 2-d the
    // out-of-plane frame current drops the path-average term
    const bool vb = ORDER == 1 && R.vb;
    const float x12 = vb ? 0.0f : 1.0f / 12.0f;
    double *jlane = jtile + (kJCopies > 1 ? (lane % kJCopies) * 3 * jcells : 0);   // this lane's copy
    auto deposit_one = [&](int lx_, int ly_, int lz_, const float *a0, const int *qs, const float *a1, float fx_) {
        if constexpr (ORDER == 1) {
            if (vb) {
                deposit_lane_vb<DIM>(jlane, jcells, jx_, jy_, lx_, ly_, lz_, a0, qs, a1, jfx, jfy, jfz, fx_);
                return;
            }
        }
        deposit_lane<DIM, ORDER>(jlane, jcells, jx_, jy_, lx_, ly_, lz_, a0, qs, a1, jfx, jfy, jfz, fx_);
    };

    // deposit queued particles [0, n) of this wave, one per lane
    int qn = 0;   // queued particles (the same in every lane of the wave)
    auto drain = [&](int n) {
        __builtin_amdgcn_wave_barrier();
        if (lane < n) {
            const int pk = __float_as_int(cq[lane]);
            const int qs[3] = {((pk >> 24) & 3) - 1, ((pk >> 26) & 3) - 1, ((pk >> 28) & 3) - 1};
            float a0[3] = {0.0f, 0.0f, 0.0f}, a1[3] = {0.0f, 0.0f, 0.0f};
            constexpr int D = DIM == 3 ? 3 : 2, d0 = 3 - D;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                a0[d0 + k] = cq[(1 + k) * QS + lane];
                a1[d0 + k] = cq[(1 + D + k) * QS + lane];
            }
            const float qfx = DIM == 2 ? cq[5 * QS + lane] : 0.0f;
            deposit_one(pk & 255, (pk >> 8) & 255, (pk >> 16) & 255, a0, qs, a1, qfx);
        }
        __builtin_amdgcn_wave_barrier();
    };

    // K = 1 with prefetching: the state of the lane's particle in the next
    // round (cell key, offsets, momenta, id) is loaded at the start of the
    // current round, before its stores, and its permutation entry one round
    // earlier still.  Loads and stores retire in issue order, so the next
    // round's wait for its particle leaves this round's stores in flight.
    // Lanes without a particle stand in with the chunk's first particle.
    constexpr bool prefetch = single && PSC_PREFETCH;
    int32_t p_key = 0, p_raw = beg, p_id = 0;
    float p_o[3] = {0.0f, 0.0f, 0.0f}, p_u[3] = {0.0f, 0.0f, 0.0f};
    auto lane_slot = [&](int32_t r, bool &ok) {
        int32_t g = r + (int32_t)threadIdx.x;
        if constexpr (PSC_MIX && !RUNS) g = mix_lane(g, nruns);   // ablation only
        ok = g < nruns;
        return ok ? beg + g : beg;
    };
    auto checked_src = [&](int32_t slot, int32_t raw, bool ok) {
        if ((uint32_t)raw >= (uint32_t)S.n) {   // corrupt permutation: stay in bounds
            if (ok) flags |= PSC_DEV_KEY;
            return slot;
        }
        return raw;
    };
    auto load_state = [&](int32_t src) {
        const uint32_t i = (uint32_t)src;
        p_key = *at32(cell_in, i);
        if constexpr (DIM == 3) p_o[0] = *at32(oin[0], i);
        p_o[1] = *at32(oin[D - 2], i);
        p_o[2] = *at32(oin[D - 1], i);
        p_u[0] = *at32(uin[0], i);
        p_u[1] = *at32(uin[1], i);
        p_u[2] = *at32(uin[2], i);
        p_id = id_in ? *at32(id_in, i) : 0;
    };
    if constexpr (prefetch) {
        bool ok;
        const int32_t sl = lane_slot(0, ok);
        load_state(checked_src(sl, use_perm ? *at32(perm, (uint32_t)sl) : sl, ok));
        const int32_t sl1 = lane_slot(NT, ok);
        p_raw = use_perm ? *at32(perm, (uint32_t)sl1) : sl1;
        // these loads complete here, once per item: the compiler's waits in
        // the round loop then count only the loop's own memory operations
        // (entering with the prologue's loads pending, it would wait for all
        // outstanding operations on every round)
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    }

    // every lane runs the same number of rounds and of steps per round (the
    // wave operations need all 64 lanes); lanes without a particle carry zero
    // current and write nothing
    // FULL: every lane of the round holds a particle (compile-time, so that
    // such rounds issue their loads and stores on every path)
    // K = 2: the permutation entries of a lane's two particles in the round
    // starting at r are read during the round before it (strip slots past
    // the end stand in with the chunk's first particle)
    int32_t h_raw[KS] = {};
    auto strip_slots = [&](int32_t r, int32_t slot[KS]) {
        const int32_t g_ = r + (int32_t)threadIdx.x;
        const int32_t first_ = beg + g_ * KS;
        const int32_t len_ = g_ < nruns ? imin(KS, end - first_) : 0;
#pragma unroll
        for (int j = 0; j < KS; ++j) slot[j] = j < len_ ? first_ + j : beg;
        return len_;
    };
    if constexpr (!prefetch) {
        int32_t sl[KS];
        strip_slots(0, sl);
#pragma unroll
        for (int j = 0; j < KS; ++j) h_raw[j] = use_perm ? *at32(perm, (uint32_t)sl[j]) : sl[j];
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);   // as for K = 1: the loop's waits count only its own operations
    }
    auto round = [&](int32_t r0, auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        int32_t g = r0 + (int32_t)threadIdx.x;
        if constexpr (PSC_MIX && !RUNS) g = mix_lane(g, nruns);   // ablation only
        const int32_t first = beg + g * K;                       // this lane's strip
        const int32_t len = g < nruns ? imin(K, end - first) : 0;
        int c = 0, cf = -1;   // particle's cell, cell of the lane's frame
        int lx = 0, ly = 0, lz = 0, fx_ = 0, fy_ = 0, fz_ = 0;
        auto cell_coords = [&]() {
            if constexpr (DIM == 3) {
                const int q = divmod_small(c, hx, inv_hx, lx);
                lz = divmod_small(q, hy, inv_hy, ly);
            } else {
                lz = divmod_small(c, hy, inv_hy, ly);
            }
        };
        float acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = 0.0f;
        // inputs of the frames of the lane's particles (start and end offsets,
        // out-of-plane factor, whether the particle goes into the frame)
        float fa0[3] = {0.0f, 0.0f, 0.0f}, fb0[3] = {0.0f, 0.0f, 0.0f}, fa1[3] = {0.0f, 0.0f, 0.0f},
              fb1[3] = {0.0f, 0.0f, 0.0f};
        float fx0 = 0.0f, fx1 = 0.0f;
        bool fr0 = false, fr1 = false;
        auto add_frame = [&](const float *o, const float *o1, float fxv, bool frame) {
            float S0y[FL], S1y[FL], S0z[FL], S1z[FL];
            frame_weights<ORDER>(o[1], o1[1], S0y, S1y);
            frame_weights<ORDER>(o[2], o1[2], S0z, S1z);
            float DSy[FL], DSz[FL], Ay[FL], Az[FL], Cy[FL], Cz[FL];
#pragma unroll
            for (int r = 0; r < FL; ++r) {
                DSy[r] = S1y[r] - S0y[r];
                DSz[r] = S1z[r] - S0z[r];
                Ay[r] = fmaf(0.5f, DSy[r], S0y[r]);
                Az[r] = fmaf(0.5f, DSz[r], S0z[r]);
                Cy[r] = r == 0 ? DSy[0] : Cy[r - 1] + DSy[r];
                Cz[r] = r == 0 ? DSz[0] : Cz[r - 1] + DSz[r];
            }
            const float gy = frame ? jfy : 0.0f, gz = frame ? jfz : 0.0f;
            if constexpr (DIM == 2) {
                const float gx = frame ? fxv : 0.0f;
#pragma unroll
                for (int a = 0; a < FL - 1; ++a) {
                    const float cy = gy * Cy[a], cz = gz * Cz[a];
#pragma unroll
                    for (int b = 0; b < FL; ++b) {
                        acc[b * (FL - 1) + a] = fmaf(cy, Az[b], acc[b * (FL - 1) + a]);
                        acc[NY2 + a * FL + b] = fmaf(Ay[b], cz, acc[NY2 + a * FL + b]);
                    }
                }
#pragma unroll
                for (int a = 0; a < FL; ++a) {
                    const float pa = gx * Ay[a], qa = gx * x12 * DSy[a];
#pragma unroll
                    for (int b = 0; b < FL; ++b)
                        acc[2 * NY2 + b * FL + a] = fmaf(pa, Az[b], fmaf(qa, DSz[b], acc[2 * NY2 + b * FL + a]));
                }
            } else if constexpr (ORDER == 1) {
                // in-cell move of a 1st-order particle: with displacements
                // d and path midpoints m (cell units), Jx on the edge (b, c)
                // of the cell is -jfx dx (W_b(my) W_c(mz) +- dy dz / 12),
                // W_0 = 1 - m, W_1 = m, sign + where b == c.  Summed over the
                // particles of a cell that is a combination of four moments
                // (P, P my, P mz, P (my mz + dy dz / 12)), P = -jfx dx;
                // likewise Jy with (x, z) and Jz with (x, y).  The frame holds
                // the moments, turned into edge currents after the wave sums.
                const float ex = o1[0] - o[0], ey = o1[1] - o[1], ez = o1[2] - o[2];
                const float mx = fmaf(0.5f, ex, o[0]), my = fmaf(0.5f, ey, o[1]), mz = fmaf(0.5f, ez, o[2]);
                const float px = frame ? -jfx * ex : 0.0f, py = frame ? -jfy * ey : 0.0f,
                            pz = frame ? -jfz * ez : 0.0f;
                acc[0] += px;
                acc[1] = fmaf(px, my, acc[1]);
                acc[2] = fmaf(px, mz, acc[2]);
                acc[3] = fmaf(px, fmaf(ey * ez, 1.0f / 12.0f, my * mz), acc[3]);
                acc[4] += py;
                acc[5] = fmaf(py, mx, acc[5]);
                acc[6] = fmaf(py, mz, acc[6]);
                acc[7] = fmaf(py, fmaf(ex * ez, 1.0f / 12.0f, mx * mz), acc[7]);
                acc[8] += pz;
                acc[9] = fmaf(pz, mx, acc[9]);
                acc[10] = fmaf(pz, my, acc[10]);
                acc[11] = fmaf(pz, fmaf(ex * ey, 1.0f / 12.0f, mx * my), acc[11]);
            } else {
                const float gx = frame ? jfx : 0.0f;
                float S0x[FL], S1x[FL];
                frame_weights<ORDER>(o[0], o1[0], S0x, S1x);
                float DSx[FL], Ax[FL], Cx[FL];
#pragma unroll
                for (int r = 0; r < FL; ++r) {
                    DSx[r] = S1x[r] - S0x[r];
                    Ax[r] = fmaf(0.5f, DSx[r], S0x[r]);
                    Cx[r] = r == 0 ? DSx[0] : Cx[r - 1] + DSx[r];
                }
#pragma unroll
                for (int c2 = 0; c2 < FL; ++c2)
#pragma unroll
                    for (int b = 0; b < FL; ++b) {
                        const float wyz = fmaf(DSy[b] * DSz[c2], 1.0f / 12.0f, Ay[b] * Az[c2]);
                        const float wxz = fmaf(DSx[b] * DSz[c2], 1.0f / 12.0f, Ax[b] * Az[c2]);
                        const float wxy = fmaf(DSx[b] * DSy[c2], 1.0f / 12.0f, Ax[b] * Ay[c2]);
#pragma unroll
                        for (int a = 0; a < FL - 1; ++a) {
                            // Jx(a; b, c2), Jy(b; a, c2), Jz(b, c2; a) in the index order of the flush
                            acc[(c2 * FL + b) * (FL - 1) + a] =
                                fmaf(gx * Cx[a], wyz, acc[(c2 * FL + b) * (FL - 1) + a]);
                            acc[NC3 + (c2 * (FL - 1) + a) * FL + b] =
                                fmaf(gy * Cy[a], wxz, acc[NC3 + (c2 * (FL - 1) + a) * FL + b]);
                            acc[2 * NC3 + (a * FL + c2) * FL + b] =
                                fmaf(gz * Cz[a], wxy, acc[2 * NC3 + (a * FL + c2) * FL + b]);
                        }
                    }
            }
        };
        // K = 2: the outputs of the lane's two particles, stored after both
        int32_t pk0 = 0, pk1 = 0, pi0 = 0, pi1 = 0;
        int pc0 = 0, pc1 = 0;
        float po0[3] = {0.0f, 0.0f, 0.0f}, po1[3] = {0.0f, 0.0f, 0.0f};
        float pu0[3] = {0.0f, 0.0f, 0.0f}, pu1[3] = {0.0f, 0.0f, 0.0f};

        // K = 2: both particles' keys and states, issued together at the
        // round start from the permutation entries read a round ago, then
        // the next round's entries (one memory round trip per round)
        int32_t h_key[KS] = {};
        float h_o[KS][3] = {}, h_u[KS][3] = {};
        int32_t h_id[KS] = {};
        if constexpr (!prefetch) {
            int32_t h_slot[KS];
            strip_slots(r0, h_slot);
#pragma unroll
            for (int j = 0; j < KS; ++j) {
                const int32_t src = checked_src(h_slot[j], h_raw[j], j < len);
                const uint32_t i = (uint32_t)src;
                h_key[j] = *at32(cell_in, i);
                if constexpr (DIM == 3) h_o[j][0] = *at32(oin[0], i);
                h_o[j][1] = *at32(oin[D - 2], i);
                h_o[j][2] = *at32(oin[D - 1], i);
                h_u[j][0] = *at32(uin[0], i);
                h_u[j][1] = *at32(uin[1], i);
                h_u[j][2] = *at32(uin[2], i);
                h_id[j] = id_in ? *at32(id_in, i) : 0;
            }
            int32_t n_slot[KS];
            strip_slots(r0 + NT, n_slot);
#pragma unroll
            for (int j = 0; j < KS; ++j) h_raw[j] = use_perm ? *at32(perm, (uint32_t)n_slot[j]) : n_slot[j];
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const bool valid = FULL || j < len;
            // lanes without a particle stand in with the chunk's first
            // particle (taken through the permutation, so it lies in range)
            const int32_t slot = valid ? first + j : beg;
            const int32_t key = prefetch ? p_key : h_key[j];
            c = key - (int32_t)kb;
            if (c < 0 || c >= pcells) {   // not in this patch: corrupt state
                if (valid) flags |= PSC_DEV_KEY;
                c = 0;
            }
            cell_coords();
            if (j == 0 && valid) {   // the lane's frame lies at its first particle's cell
                cf = c;
                fx_ = lx;
                fy_ = ly;
                fz_ = lz;
            }
            float o[3], ux, uy, uz;
            int32_t idv;
            if constexpr (prefetch) {
                o[0] = DIM == 3 ? p_o[0] : 0.0f;
                o[1] = p_o[1];
                o[2] = p_o[2];
                ux = p_u[0];
                uy = p_u[1];
                uz = p_u[2];
                idv = p_id;
            } else {
                o[0] = DIM == 3 ? h_o[j][0] : 0.0f;
                o[1] = h_o[j][1];
                o[2] = h_o[j][2];
                ux = h_u[j][0];
                uy = h_u[j][1];
                uz = h_u[j][2];
                idv = h_id[j];
            }
            // the next round's particle (its permutation entry was read a
            // round ago), then the permutation entry of the round after it
            // (the round loop is uniform; past the end a lane reads the
            // chunk's first particle)
            if constexpr (prefetch) {
                bool n_ok;
                const int32_t n_slot = lane_slot(r0 + NT, n_ok);
                load_state(checked_src(n_slot, p_raw, n_ok));
                const int32_t sl2 = lane_slot(r0 + 2 * NT, n_ok);
                p_raw = use_perm ? *at32(perm, (uint32_t)sl2) : sl2;
            }

            // ---- interpolation ----------------------------------------------
            float wny[ORDER + 1], why[ORDER + 1], wnz[ORDER + 1], whz[ORDER + 1];
            const int bny = node_weights<ORDER>(o[1], wny), bhy = half_weights<ORDER>(o[1], why);
            const int bnz = node_weights<ORDER>(o[2], wnz), bhz = half_weights<ORDER>(o[2], whz);
            float Ex, Ey, Ez, Bx, By, Bz;
            if constexpr (DIM == 2) {
                const int ty = ly + FLO, tz = lz + FLO;
                Ex = gather2<ORDER>(ftile, fy, ty + bny, tz + bnz, wny, wnz);
                Bx = gather2<ORDER>(ftile + fcells, fy, ty + bhy, tz + bhz, why, whz);
                const float2 EyBz = gather2_pair<ORDER>(reinterpret_cast<const float2 *>(ftile + 2 * fcells), fy,
                                                        ty + bhy, tz + bnz, why, wnz);
                const float2 EzBy = gather2_pair<ORDER>(reinterpret_cast<const float2 *>(ftile + 4 * fcells), fy,
                                                        ty + bny, tz + bhz, wny, whz);
                Ey = EyBz.x;
                Bz = EyBz.y;
                Ez = EzBy.x;
                By = EzBy.y;
            } else {
                float wnx[ORDER + 1], whx[ORDER + 1];
                const int bnx = node_weights<ORDER>(o[0], wnx), bhx = half_weights<ORDER>(o[0], whx);
                const int tx = lx + FLO, ty = ly + FLO, tz = lz + FLO;
                const int pxy = fx * fy;
                Ex = gather3<ORDER>(ftile + 0 * fcells, fx, pxy, tx + bhx, ty + bny, tz + bnz, whx, wny, wnz);
                Ey = gather3<ORDER>(ftile + 1 * fcells, fx, pxy, tx + bnx, ty + bhy, tz + bnz, wnx, why, wnz);
                Ez = gather3<ORDER>(ftile + 2 * fcells, fx, pxy, tx + bnx, ty + bny, tz + bhz, wnx, wny, whz);
                Bx = gather3<ORDER>(ftile + 3 * fcells, fx, pxy, tx + bnx, ty + bhy, tz + bhz, wnx, why, whz);
                By = gather3<ORDER>(ftile + 4 * fcells, fx, pxy, tx + bhx, ty + bny, tz + bhz, whx, wny, whz);
                Bz = gather3<ORDER>(ftile + 5 * fcells, fx, pxy, tx + bhx, ty + bhy, tz + bnz, whx, why, wnz);
            }

            // ---- relativistic Boris push: half E kick, rotation, half E kick
            {
                const float mx = fmaf(h, Ex, ux), my = fmaf(h, Ey, uy), mz = fmaf(h, Ez, uz);
                const float igm = rsqrt_ge1(1.0f + mx * mx + my * my + mz * mz);
                const float tx = h * Bx * igm, ty = h * By * igm, tz = h * Bz * igm;
                const float f = boris_factor(tx * tx + ty * ty + tz * tz);
                const float sx = f * tx, sy = f * ty, sz = f * tz;
                const float px = mx + (my * tz - mz * ty);
                const float py = my + (mz * tx - mx * tz);
                const float pz = mz + (mx * ty - my * tx);
                ux = fmaf(h, Ex, mx + (py * sz - pz * sy));
                uy = fmaf(h, Ey, my + (pz * sx - px * sz));
                uz = fmaf(h, Ez, mz + (px * sy - py * sx));
            }
            const float ig = rsqrt_ge1(1.0f + ux * ux + uy * uy + uz * uz);
            if (valid && !(ig > 0.0f)) flags |= PSC_DEV_NONFINITE;   // NaN or Inf momentum

            // ---- move: xi^{n+3/2} = xi^{n+1/2} + dt u^{n+1} / (gamma dx) ---
            int s[3] = {0, 0, 0};
            float o1[3] = {o[0], o[1], o[2]};
#pragma unroll
            for (int d = (DIM == 3 ? 0 : 1); d < 3; ++d) {
                const float cf = d == 0 ? cfx : (d == 1 ? cfy : cfz);
                const float uu = d == 0 ? ux : (d == 1 ? uy : uz);
                float disp = cf * uu * ig;
                if (!(fabsf(disp) < 0.99f)) {   // CFL broken or non-finite: keep it in bounds
                    if (valid) flags |= PSC_DEV_MOVE;
                    disp = 0.0f;
                }
                const float x1 = o[d] + disp;
                int sd = (int)floorf(x1);
                float od = x1 - (float)sd;
                if (od >= 1.0f) { od -= 1.0f; sd += 1; }
                s[d] = sd;
                o1[d] = od;
            }

            // ---- Esirkepov deposit --------------------------------------------
            const float fxv = qw * ux * ig;   // 2-d out-of-plane current factor q w v_x
            if constexpr (!kReduce) {
                if (valid)
                    deposit_one(lx, ly, lz, o, s, o1, fxv);
            } else {
                bool frame = PSC_FRAMES && valid && (single || c == cf) && stays<ORDER>(o[1], s[1], o1[1]) &&
                             stays<ORDER>(o[2], s[2], o1[2]);
                if constexpr (DIM == 3) frame = frame && stays<ORDER>(o[0], s[0], o1[0]);

                // support changes nodes: to the wave's queue; a full queue is
                // deposited with its slots' lanes busy (more crossings at once
                // than the queue holds deposit in place)
                const bool cross = valid && !frame;
                const uint64_t cm = __ballot(cross);
                if (cm) {
                    const int nq = __popcll(cm);
                    if (nq > QS) {
                        if (cross)
                            deposit_one(lx, ly, lz, o, s, o1, fxv);
                    } else {
                        if (qn + nq > QS) {
                            drain(qn);
                            qn = 0;
                        }
                        if (cross) {
                            const int slot_q = qn + (int)__builtin_amdgcn_mbcnt_hi(
                                                        (uint32_t)(cm >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)cm, 0u));
                            const int pk = lx | (ly << 8) | (lz << 16) | ((s[0] + 1) << 24) |
                                           ((s[1] + 1) << 26) | ((s[2] + 1) << 28);
                            cq[slot_q] = __int_as_float(pk);
                            constexpr int D = DIM == 3 ? 3 : 2, d0 = 3 - D;
#pragma unroll
                            for (int k = 0; k < D; ++k) {
                                cq[(1 + k) * QS + slot_q] = o[d0 + k];
                                cq[(1 + D + k) * QS + slot_q] = o1[d0 + k];
                            }
                            if constexpr (DIM == 2) cq[5 * QS + slot_q] = fxv;
                        }
                        qn += nq;
                    }
                }

                // the rest: into this lane's frame of its cell, built after
                // the lane's particles are done (keeps the frame registers
                // free while a second particle is pushed)
                if (j == 0) {
                    fa0[0] = o[0]; fa0[1] = o[1]; fa0[2] = o[2];
                    fb0[0] = o1[0]; fb0[1] = o1[1]; fb0[2] = o1[2];
                    fx0 = fxv; fr0 = frame;
                } else {
                    fa1[0] = o[0]; fa1[1] = o[1]; fa1[2] = o[2];
                    fb1[0] = o1[0]; fb1[1] = o1[1]; fb1[2] = o1[2];
                    fx1 = fxv; fr1 = frame;
                }
            }

            // ---- per (old cell, move code) counts for the sort ------------------
            // Only particles that change cell are counted (one atomic each on the
            // 32-bit word holding the 16-bit counter); the sort takes the rest of
            // a cell's particles as staying.
            {
                constexpr int CENTER = DIM == 3 ? 13 : 4;
                const int code = DIM == 3 ? (s[0] + 1) + 3 * (s[1] + 1) + 9 * (s[2] + 1) : (s[1] + 1) + 3 * (s[2] + 1);
                if (valid && code != CENTER) {
                    const int64_t w = (int64_t)code * R.ncell + kb + c;
                    atomicAdd((uint32_t *)(cnt32 + (w >> 1)), 1u << (16 * (int)(w & 1)));
                }
            }

            // ---- outputs: new cell key, move code, offsets, momenta ------------
            if (valid) {
                const int nlx = lx + s[0], nly = ly + s[1], nlz = lz + s[2];
                int32_t nkey;
                if (nlx >= 0 && nlx < hx && nly >= 0 && nly < hy && nlz >= 0 && nlz < hz) {
                    nkey = (int32_t)kb + nlx + hx * (nly + hy * nlz);
                } else {
                    const int hh[3] = {hx, hy, hz}, nl[3] = {nlx, nly, nlz};
                    nkey = (int32_t)neighbour_key(R, pc, hh, nl);
                }
                const int code = DIM == 3 ? (s[0] + 1) + 3 * (s[1] + 1) + 9 * (s[2] + 1) : (s[1] + 1) + 3 * (s[2] + 1);
                if constexpr (single) {
                    const uint32_t i = (uint32_t)slot;
                    *at32(cell_out, i) = nkey;
                    if constexpr (DIM == 3) *at32(oout[0], i) = o1[0];
                    *at32(oout[D - 2], i) = o1[1];
                    *at32(oout[D - 1], i) = o1[2];
                    *at32(mc, i) = (uint8_t)code;
                    *at32(uout[0], i) = ux;
                    *at32(uout[1], i) = uy;
                    *at32(uout[2], i) = uz;
                    if (id_out) *at32(id_out, i) = idv;
                } else if (j == 0) {
                    pk0 = nkey; po0[0] = o1[0]; po0[1] = o1[1]; po0[2] = o1[2];
                    pu0[0] = ux; pu0[1] = uy; pu0[2] = uz; pc0 = code; pi0 = idv;
                } else {
                    pk1 = nkey; po1[0] = o1[0]; po1[1] = o1[1]; po1[2] = o1[2];
                    pu1[0] = ux; pu1[1] = uy; pu1[2] = uz; pc1 = code; pi1 = idv;
                }
            }
        }
        if constexpr (!single) {
            // the wave's lanes hold the 128 consecutive slots from wbase (lane
            // l: wbase + 2l and wbase + 2l + 1); in two passes lane l stores
            // slot wbase + 64 pass + l, taken from lane 32 pass + l/2
            const int32_t wbase = beg + 2 * (r0 + (int32_t)(threadIdx.x & ~63));
            const bool odd = lane & 1;
#pragma unroll
            for (int pass = 0; pass < 2; ++pass) {
                const int src = 32 * pass + (lane >> 1);
                const int32_t slot = wbase + 64 * pass + lane;
                const bool ok = slot < end;
                auto pick = [&](auto a, auto b) {
                    const auto x = __shfl(a, src, 64), y = __shfl(b, src, 64);
                    return odd ? y : x;
                };
                const int32_t k = pick(pk0, pk1);
                const int code = pick(pc0, pc1);
                float o[3], u[3];
#pragma unroll
                for (int d = (DIM == 3 ? 0 : 1); d < 3; ++d) o[d] = pick(po0[d], po1[d]);
#pragma unroll
                for (int d = 0; d < 3; ++d) u[d] = pick(pu0[d], pu1[d]);
                if (ok) {
                    const uint32_t i = (uint32_t)slot;
                    *at32(cell_out, i) = k;
                    if constexpr (DIM == 3) *at32(oout[0], i) = o[0];
                    *at32(oout[D - 2], i) = o[1];
                    *at32(oout[D - 1], i) = o[2];
                    *at32(mc, i) = (uint8_t)code;
                    *at32(uout[0], i) = u[0];
                    *at32(uout[1], i) = u[1];
                    *at32(uout[2], i) = u[2];
                }
                if (id_out) {
                    const int32_t iv = pick(pi0, pi1);
                    if (ok) *at32(id_out, (uint32_t)slot) = iv;
                }
            }
        }

        // ---- the round's frames: segmented sums over lanes of one cell ------
        if constexpr (kReduce) {
            add_frame(fa0, fb0, fx0, fr0);
            if constexpr (!single) add_frame(fa1, fb1, fx1, fr1);
            const RowScan rs = row_scan_setup<SW>(cf);
            row_scan<SW>(acc, rs);
            if constexpr (DIM == 3 && ORDER == 1) {
                // moments (S, S_a, S_b, S_ab) of each component -> the currents
                // of its four edges (a, b) = (0,0), (1,0), (0,1), (1,1)
#pragma unroll
                for (int g3 = 0; g3 < 3; ++g3) {
                    float *m = acc + 4 * g3;
                    const float m0 = m[0], m1 = m[1], m2 = m[2], m3 = m[3];
                    m[0] = (m0 - m1) - (m2 - m3);
                    m[1] = m1 - m3;
                    m[2] = m2 - m3;
                }
            }
            const bool put = rs.tail && len > 0;
            int base;
            if constexpr (DIM == 2) base = (fz_ + FB + JLO) * jy_ + (fy_ + FB + JLO);
            else base = (fz_ + FB + JLO) * (jx_ * jy_) + (fy_ + FB + JLO) * jx_ + (fx_ + FB + JLO);
            const uint64_t tails = __ballot(put);
            const int nt = __popcll(tails);
            if (nt <= kPackTails) {
                // few segments: stage their sums, then add them with every
                // lane of the wave busy (one atomic per lane per pass)
                if (put) {
                    const int ti = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(tails >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)tails, 0u));
                    float4 *dst = reinterpret_cast<float4 *>(pk + ti * NV);
#pragma unroll
                    for (int v = 0; v < NV / 4; ++v)
                        dst[v] = make_float4(acc[4 * v], acc[4 * v + 1], acc[4 * v + 2], acc[4 * v + 3]);
                    reinterpret_cast<int32_t *>(pk + kPackTails * NV)[ti] = base;
                }
                __builtin_amdgcn_wave_barrier();
                for (int k = lane; k < nt * NV; k += 64) {
                    const int ti = k / NV, j = k - ti * NV;
                    const int b0 = reinterpret_cast<const int32_t *>(pk + kPackTails * NV)[ti];
                    lds_add(&jtile[b0 + frame_offset<DIM, ORDER>(j, jx_, jy_, jcells)], pk[k]);
                }
                __builtin_amdgcn_wave_barrier();
            } else if (put) {
                if constexpr (DIM == 2) {
#pragma unroll
                    for (int b = 0; b < FL; ++b)
#pragma unroll
                        for (int a = 0; a < FL - 1; ++a) lds_add(&Jy[base + b * jy_ + a], acc[b * (FL - 1) + a]);
#pragma unroll
                    for (int b = 0; b < FL - 1; ++b)
#pragma unroll
                        for (int a = 0; a < FL; ++a) lds_add(&Jz[base + b * jy_ + a], acc[NY2 + b * FL + a]);
#pragma unroll
                    for (int b = 0; b < FL; ++b)
#pragma unroll
                        for (int a = 0; a < FL; ++a) lds_add(&Jx[base + b * jy_ + a], acc[2 * NY2 + b * FL + a]);
                } else {
                    const int pxy = jx_ * jy_;
#pragma unroll
                    for (int c2 = 0; c2 < FL; ++c2)
#pragma unroll
                        for (int b = 0; b < FL; ++b)
#pragma unroll
                            for (int a = 0; a < FL - 1; ++a)
                                lds_add(&Jx[base + c2 * pxy + b * jx_ + a], acc[(c2 * FL + b) * (FL - 1) + a]);
#pragma unroll
                    for (int c2 = 0; c2 < FL; ++c2)
#pragma unroll
                        for (int b = 0; b < FL - 1; ++b)
#pragma unroll
                            for (int a = 0; a < FL; ++a)
                                lds_add(&Jy[base + c2 * pxy + b * jx_ + a], acc[NC3 + (c2 * (FL - 1) + b) * FL + a]);
#pragma unroll
                    for (int c2 = 0; c2 < FL - 1; ++c2)
#pragma unroll
                        for (int b = 0; b < FL; ++b)
#pragma unroll
                            for (int a = 0; a < FL; ++a)
                                lds_add(&Jz[base + c2 * pxy + b * jx_ + a], acc[2 * NC3 + (c2 * FL + b) * FL + a]);
                }
            }
        }
    };
    if constexpr (single && !PSC_MIX) {
        // the full rounds, then the item's partial last round
        int32_t r0 = 0;
        for (; r0 + NT <= nruns; r0 += NT) round(r0, std::true_type{});
        if (r0 < nruns) round(r0, std::false_type{});
    } else {
        for (int32_t r0 = 0; r0 < nruns; r0 += NT) round(r0, std::false_type{});
    }
    if constexpr (kReduce) {
        if (qn) drain(qn);
    }
    if (flags) atomicOr(err, flags);
    __syncthreads();

    if (R.jdirect) {
        // add the LDS current tile into the run's accumulator: tile entry
        // (tx, ty, tz) is cell (ox, oy, oz) + (tx, ty, tz) - JLO, periodic,
        // so the halo lands on the neighbouring patches' cells (the fold
        // done here).  Fixed point in units of jq: integer sums, so the
        // result does not depend on the order in which work items add
        const int64_t nc = R.ncell;
        const gptr<unsigned long long> acc = to_global(reinterpret_cast<unsigned long long *>(R.jacc));
        const double inv_q = R.jinvq;
        const float inv_jx = 1.0f / jx_, inv_jy = 1.0f / jy_;
        for (int q = threadIdx.x; q < n_jband; q += NT) {
            const int t = jr0 * jplane + q;
            int tx = 0, ty, tz;
            if constexpr (DIM == 3) {
                const int r = divmod_small(t, jx_, inv_jx, tx);
                tz = divmod_small(r, jy_, inv_jy, ty);
            } else {
                tz = divmod_small(t, jy_, inv_jy, ty);
            }
            const int gx = DIM == 3 ? wrap_near(ox + tx - JLO, R.n[0]) : 0;
            const int gy = wrap_near(oy + ty - JLO, R.n[1]);
            const int gz = wrap_near(oz + tz - JLO, R.n[2]);
            const int64_t g = gx + (int64_t)R.n[0] * (gy + (int64_t)R.n[1] * gz);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double v = jtile[c * jcells + t];
#pragma unroll
                for (int cp = 1; cp < kJCopies; ++cp) v += jtile[(3 * cp + c) * jcells + t];
                const long long k = (long long)__builtin_rint(v * inv_q);
                if (k != 0) atomicAdd((unsigned long long *)(acc + (c * nc + g)), (unsigned long long)k);   // two's complement
            }
        }
    } else {
        // add the LDS current tile into the patch's tile in HBM
        const gptr<float> gt = to_global(R.jtile + (int64_t)U.patch * 3 * jcells);
        for (int q = threadIdx.x; q < 3 * n_jband; q += NT) {
            const int c = q / n_jband;
            const int t = c * jcells + jr0 * jplane + (q - c * n_jband);
            double v = jtile[t];
#pragma unroll
            for (int cp = 1; cp < kJCopies; ++cp) v += jtile[3 * cp * jcells + t];
            if (v != 0.0) atomicAdd((float *)(gt + t), (float)v);
        }
    }
    __syncthreads();
}

// launch mode 0: one workgroup per item.  Workgroups are dispatched
// round-robin over the 8 XCDs; give each XCD a contiguous range of items so
// that the chunks of a patch share one L2.
template <int DIM, int ORDER, int NT, bool RUNS>
__global__ void __launch_bounds__(NT) PSC_OCCUPANCY k_push(const RunDev *__restrict__ runs, const Unit *__restrict__ units,
                                                 const int32_t *__restrict__ item_start, int n_units,
                                                 int front, int cs_sel, int use_perm, int K,
                                                 uint32_t *__restrict__ err) {
    extern __shared__ __align__(16) float lds[];   // 16-byte aligned: holds doubles and float4
    const int nb = gridDim.x;
    const int item = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
    if (item >= item_start[n_units]) return;
    push_item<DIM, ORDER, NT, RUNS>(runs, units, item_start, unit_of_item(item_start, n_units, item), item, front,
                              cs_sel, use_perm, K, err, lds);
}

// launch mode 1: persistent workgroups pull items from 8 queues, one per
// XCD (queue q owns the q-th eighth of the items, so an XCD works on
// neighbouring patches), and steal from the other queues when theirs is
// empty.  Every workgroup leaves once all queues are drained.
template <int DIM, int ORDER, int NT, bool RUNS>
__global__ void __launch_bounds__(NT) PSC_OCCUPANCY k_push_queue(const RunDev *__restrict__ runs,
                                                       const Unit *__restrict__ units,
                                                       const int32_t *__restrict__ item_start, int n_units,
                                                       int front, int cs_sel, int use_perm, int K,
                                                       uint32_t *__restrict__ err, int32_t *__restrict__ queue) {
    extern __shared__ __align__(16) float lds[];   // 16-byte aligned: holds doubles and float4
    __shared__ int s_item;
    const int total = item_start[n_units];
    const int xcd = blockIdx.x & 7;
    for (int k = 0; k < 8; ++k) {
        const int q = (xcd + k) & 7;
        const int qb = (int)((int64_t)q * total / 8), qe = (int)((int64_t)(q + 1) * total / 8);
        for (;;) {
            if (threadIdx.x == 0) {
                // a drained queue is skipped without an atomic (the counter
                // only grows; a stale read just leads to the atomic)
                int32_t *ctr = &queue[kQueueStride * q];
                s_item = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= qe - qb
                             ? qe
                             : qb + atomicAdd(ctr, 1);
            }
            __syncthreads();
            const int item = s_item;
            __syncthreads();
            if (item >= qe) break;
            push_item<DIM, ORDER, NT, RUNS>(runs, units, item_start, unit_of_item(item_start, n_units, item), item,
                                      front, cs_sel, use_perm, K, err, lds);
        }
    }
}

// launch mode 2: persistent workgroup w processes the contiguous units
// [part[w], part[w+1]) chosen by the load-balancing partition.
template <int DIM, int ORDER, int NT, bool RUNS>
__global__ void __launch_bounds__(NT) PSC_OCCUPANCY k_push_part(const RunDev *__restrict__ runs,
                                                      const Unit *__restrict__ units,
                                                      const int32_t *__restrict__ item_start, int n_units,
                                                      int front, int cs_sel, int use_perm, int K,
                                                      uint32_t *__restrict__ err, const int32_t *__restrict__ part) {
    extern __shared__ __align__(16) float lds[];   // 16-byte aligned: holds doubles and float4
    const int u0 = part[blockIdx.x], u1 = min(part[blockIdx.x + 1], n_units);
    for (int u = u0; u < u1; ++u)
        for (int item = item_start[u]; item < item_start[u + 1]; ++item)
            push_item<DIM, ORDER, NT, RUNS>(runs, units, item_start, u, item, front, cs_sel, use_perm, K, err, lds);
}

template <int DIM, int ORDER, int NT, bool RUNS>
static hipError_t launch_push_r(const Launch &L, const Unit *units, int n_units, int32_t *item_start,
                                int64_t max_items, int front, int cs_sel, int use_perm,
                                size_t lds, const PushMode &pm) {
    hipLaunchKernelGGL(k_unit_items, dim3((unsigned)imax(1, (n_units + 255) / 256)), dim3(256), 0, L.stream, L.runs_dev,
                       units, n_units, cs_sel, item_start);
    hipLaunchKernelGGL(k_items_scan, dim3(1), dim3(1024), 0, L.stream, n_units, item_start, pm.queue);
    if (pm.mode == 1) {
        hipLaunchKernelGGL((k_push_queue<DIM, ORDER, NT, RUNS>), dim3((unsigned)pm.workers), dim3(NT), lds, L.stream,
                           L.runs_dev, units, item_start, n_units, front, cs_sel, use_perm, pm.run, L.err,
                           pm.queue);
    } else if (pm.mode == 2) {
        hipLaunchKernelGGL((k_push_part<DIM, ORDER, NT, RUNS>), dim3((unsigned)pm.workers), dim3(NT), lds, L.stream,
                           L.runs_dev, units, item_start, n_units, front, cs_sel, use_perm, pm.run, L.err,
                           pm.part);
    } else {
        int64_t grid = (max_items + 7) / 8 * 8;
        if (grid < 8) grid = 8;
        hipLaunchKernelGGL((k_push<DIM, ORDER, NT, RUNS>), dim3((unsigned)grid), dim3(NT), lds, L.stream, L.runs_dev,
                           units, item_start, n_units, front, cs_sel, use_perm, pm.run, L.err);
    }
    return hipGetLastError();
}

template <int DIM, int ORDER, int NT>
static hipError_t launch_push_t(const Launch &L, const Unit *units, int n_units, int32_t *item_start,
                                int64_t max_items, int front, int cs_sel, int use_perm,
                                size_t lds, const PushMode &pm) {
    if (pm.run > 1)
        return launch_push_r<DIM, ORDER, NT, true>(L, units, n_units, item_start, max_items, front, cs_sel,
                                                   use_perm, lds, pm);
    return launch_push_r<DIM, ORDER, NT, false>(L, units, n_units, item_start, max_items, front, cs_sel,
                                                use_perm, lds, pm);
}

template <int DIM, int ORDER>
static hipError_t launch_push_nt(const Launch &L, const Unit *units, int n_units, int32_t *item_start,
                                 int64_t max_items, int front, int cs_sel, int use_perm, size_t lds,
                                 const PushMode &pm) {
    if (pm.threads == 512)
        return launch_push_t<DIM, ORDER, 512>(L, units, n_units, item_start, max_items, front, cs_sel,
                                              use_perm, lds, pm);
    if (pm.threads == 384)
        return launch_push_t<DIM, ORDER, 384>(L, units, n_units, item_start, max_items, front, cs_sel,
                                              use_perm, lds, pm);
    return launch_push_t<DIM, ORDER, 256>(L, units, n_units, item_start, max_items, front, cs_sel, use_perm,
                                          lds, pm);
}

hipError_t launch_push(const Launch &L, const Unit *units_dev, int n_units, int32_t *item_start, int64_t max_items,
                       int dim, int order, int front, int cs_sel, int use_perm, size_t lds_bytes,
                       const PushMode &pm) {
    if (dim == 2 && order == 1)
        return launch_push_nt<2, 1>(L, units_dev, n_units, item_start, max_items, front, cs_sel, use_perm,
                                    lds_bytes, pm);
    if (dim == 2 && order == 2)
        return launch_push_nt<2, 2>(L, units_dev, n_units, item_start, max_items, front, cs_sel, use_perm,
                                    lds_bytes, pm);
    if (dim == 3 && order == 1)
        return launch_push_nt<3, 1>(L, units_dev, n_units, item_start, max_items, front, cs_sel, use_perm,
                                    lds_bytes, pm);
    if (dim == 3 && order == 2)
        return launch_push_nt<3, 2>(L, units_dev, n_units, item_start, max_items, front, cs_sel, use_perm,
                                    lds_bytes, pm);
    return hipErrorInvalidValue;
}

// resident workgroups per compute unit of the persistent particle kernel of
// a launch mode (registers and LDS both counted), 0 on failure
template <int DIM, int ORDER, int NT, bool RUNS>
static int push_occupancy_r(int mode, size_t lds) {
    int n = 0;
    hipError_t e;
    if (mode == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_push_part<DIM, ORDER, NT, RUNS>, NT, lds);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_push_queue<DIM, ORDER, NT, RUNS>, NT, lds);
    return e == hipSuccess ? n : 0;
}

template <int DIM, int ORDER, int NT>
static int push_occupancy_t(int mode, int run, size_t lds) {
    return run > 1 ? push_occupancy_r<DIM, ORDER, NT, true>(mode, lds)
                   : push_occupancy_r<DIM, ORDER, NT, false>(mode, lds);
}

template <int DIM, int ORDER>
static int push_occupancy_nt(int mode, int threads, int run, size_t lds) {
    if (threads == 512) return push_occupancy_t<DIM, ORDER, 512>(mode, run, lds);
    if (threads == 384) return push_occupancy_t<DIM, ORDER, 384>(mode, run, lds);
    return push_occupancy_t<DIM, ORDER, 256>(mode, run, lds);
}

int push_occupancy(int dim, int order, int mode, int threads, int run, size_t lds) {
    if (dim == 2 && order == 1) return push_occupancy_nt<2, 1>(mode, threads, run, lds);
    if (dim == 2 && order == 2) return push_occupancy_nt<2, 2>(mode, threads, run, lds);
    if (dim == 3 && order == 1) return push_occupancy_nt<3, 1>(mode, threads, run, lds);
    if (dim == 3 && order == 2) return push_occupancy_nt<3, 2>(mode, threads, run, lds);
    return 0;
}

// particles per unit (for the load-balancing partition)
__global__ void k_unit_counts(const RunDev *__restrict__ runs, const Unit *__restrict__ units, int n_units,
                              int cs_sel, int32_t *__restrict__ out) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_units) return;
    const Unit U = units[u];
    const RunDev &R = runs[U.run];
    int pc[3];
    patch_coords(R, U.patch, pc);
    const int64_t kb = patch_key_base(R, pc[0], pc[1], pc[2]);
    const int64_t ke = kb + (int64_t)patch_ext(R, 0, pc[0]) * patch_ext(R, 1, pc[1]) * patch_ext(R, 2, pc[2]);
    const int32_t *cs = R.sp[U.species].cs[cs_sel];
    out[u] = cs[ke] - cs[kb];
}

hipError_t launch_unit_counts(const Launch &L, const Unit *units, int n_units, int cs_sel, int32_t *out) {
    hipLaunchKernelGGL(k_unit_counts, dim3((unsigned)((n_units + 255) / 256)), dim3(256), 0, L.stream, L.runs_dev,
                       units, n_units, cs_sel, out);
    return hipGetLastError();
}

// LDS bytes the particle kernel of a run needs with `threads` per workgroup
// and `run` particles per lane (the cell tables only when run > 1)
size_t push_lds_bytes(int dim, int order, const int P[3], int threads, int run) {
    const int fx = dim == 3 ? P[0] + field_lo(order) + field_hi(order) : 1;
    const int fy = P[1] + field_lo(order) + field_hi(order);
    const int fz = P[2] + field_lo(order) + field_hi(order);
    const int jx = dim == 3 ? P[0] + cur_lo(order) + cur_hi(order) : 1;
    const int jy = P[1] + cur_lo(order) + cur_hi(order);
    const int jz = P[2] + cur_lo(order) + cur_hi(order);
    const int nv = dim == 2 ? (order == 1 ? frame_values<2, 1>() : frame_values<2, 2>())
                            : (order == 1 ? frame_values<3, 1>() : frame_values<3, 2>());
    (void)run;
    const PushLds L = push_lds_layout(fx * fy * fz, jx * jy * jz, threads / 64, kQueueSlots * cross_words(dim),
                                      nv ? kPackTails * (nv + 1) : 0, 0);
    return sizeof(float) * (size_t)L.total;
}

}  // namespace psc
