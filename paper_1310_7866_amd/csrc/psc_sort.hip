// psc_sort.hip -- per-step stable counting sort of particles by cell key,
// exploiting that a particle moves at most one cell per dimension per step
// (section "Sorting and Communication": 9 move cases in 2-d, 27 in 3-d).
//
// The pushed buffer is ordered by the *old* key (the kernel wrote it in the
// previous sorted order) and each particle carries its move code m, so the new
// key is old + d(m).  The stable position of particle i with old cell o and
// move m is
//   cs_new[o + d(m)] + (arrivals into o + d(m) from source cells whose key is
//   below o's) + (earlier particles of o with the same move),
// which three integer passes compute without comparisons of particle keys:
//   count   per old cell: particles per move code          (cnt)
//   prefix  per new cell: arrivals per source, ordered     (pre, tot)
//   scan    tot -> cs_new
//   scatter per old cell: perm[position] = i
// The physical reorder is deferred into the next particle kernel, which reads
// through perm (section "Fusing of GPU kernels").
//
// Also here: the segmented exclusive scan, and the one-off general sort used
// to load particles in arbitrary order.
#include <rocprim/device/device_radix_sort.hpp>

#include "psc_device.h"
#include "psc_xcd.h"

namespace psc {

constexpr int kSortBlock = 256;

// Scatter: a workgroup owns 4 wave_cells consecutive old cells of one
// segment, each of its four waves wave_cells of them (lane q: cell cw + q),
// i.e. one contiguous range of particles (the buffer is ordered by old
// cell).  The wave walks that range 64 particles at a time with coalesced
// loads.  Each lane finds its particle's cell from the cells' first indices;
// its rank among the earlier particles of the same cell and move code is the
// population count of the code's ballot restricted to the lanes of its cell
// below it; the last such lane advances the (cell, code) counter kept in
// LDS.  Sort block b lies in scan block b / sort_per_scan of the same
// segment, whose table gives the segment.  Fewer cells per wave give more,
// shorter waves, which balances dense and sparse regions better (2-d: 32
// cells); in 3-d a wave's set-up covers 27 move codes per cell, and 64
// cells per wave measured faster.
#ifndef PSC_SORT_WAVE_CELLS_2D
#define PSC_SORT_WAVE_CELLS_2D 32
#endif
#ifndef PSC_SORT_WAVE_CELLS_3D
#define PSC_SORT_WAVE_CELLS_3D 64
#endif
constexpr int kSortThreads = 256;   // four waves
template <int DIM>
constexpr int wave_cells() { return DIM == 3 ? PSC_SORT_WAVE_CELLS_3D : PSC_SORT_WAVE_CELLS_2D; }
template <int DIM>
constexpr int sort_per_scan() { return kScanBlock / (4 * wave_cells<DIM>()); }   // workgroups per scan block
static_assert(wave_cells<2>() >= 1 && wave_cells<2>() <= 64 && kScanBlock % (4 * wave_cells<2>()) == 0 &&
                  wave_cells<3>() >= 1 && wave_cells<3>() <= 64 && kScanBlock % (4 * wave_cells<3>()) == 0,
              "sort geometry");

struct CellBlock {
    const RunDev *R;
    const SpeciesDev *S;
    int64_t cw, ce;   // this wave's cells [cw, ce)
};

template <int DIM>
__device__ __forceinline__ CellBlock cell_block(const RunDev *runs, const ScanSeg *segs, const int32_t *block_seg,
                                                const int32_t *seg_run, const int32_t *seg_sp) {
    CellBlock B;
    constexpr int WC = wave_cells<DIM>(), SPS = sort_per_scan<DIM>();
    const int64_t bid = xcd_block_sort();   // dispatch order unless PSC_XCD_SORT
    const int sg = block_seg[bid / SPS];
    B.R = &runs[seg_run[sg]];
    B.S = &B.R->sp[seg_sp[sg]];
    // the wave index as a scalar: the walk's bounds, loop counters and cell
    // masks then live in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    B.cw = (bid - SPS * segs[sg].block0) * (4 * WC) + WC * wave;
    B.ce = B.cw + WC < B.R->ncell ? B.cw + WC : B.R->ncell;
    return B;
}

// Walk the wave's particles: for each lane of a group, f(valid, i, q, m,
// rank, last) with q its cell (0..63 within the wave), m its move code, rank
// its index among the earlier particles of (q, m) in this wave, last whether
// it is the final one of (q, m) in the current group of 64; lanes past the
// end get valid = false (f is called on every lane so that a store it makes
// is issued on every group, whatever the lanes).  sb: the wave's 65 first
// indices.
//
// Lane q keeps the first index of cell q in a register.  The cell starts are
// non-decreasing, so two ballots give the cells [qa, qb] that a group of 64
// particles touches, and a lane's cell is qa plus the number of starts in
// (qa, qb] at or below its index (a short uniform loop over scalar reads;
// a binary search when the group spans many cells).  Its cell's lanes
// [lo, hi) follow from the cell's first indices.  Ranks: particles that stay
// in their cell have one ballot for the group; a lane's count of staying
// lanes below it, less that count at lane lo, is its rank, and it is the
// last one if its count plus one is the count at lane hi (both taken
// across the wave by lane shuffles).  Particles that change cell: one
// ballot per distinct (cell, move code) among them.
template <int M, typename L, typename F>
__device__ __forceinline__ void walk_cells(const int32_t *sb, int nw, int32_t pb, int32_t pe,
                                           L &&load_code, uint32_t &flags, F &&f) {
    constexpr int CENTER = M / 2;
    constexpr int kLoopCells = 8;   // longest cell range walked by the loop
    const int lane = threadIdx.x & 63;
    const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1);
    const uint64_t cells = nw >= 64 ? ~0ull : ((1ull << nw) - 1);
    const int32_t sbl = sb[lane < nw ? lane : nw];
    // Groups go in pairs, with move codes loaded two pairs ahead; every load
    // and store is issued on every group (a group past the end has no valid
    // lane), so the wait for a pair's codes (loads and stores retire in
    // issue order) leaves the stores of the last pairs in flight.  The two groups of a pair are ranked
    // in phases before either updates the counters, so that the LDS reads
    // and lane shuffles of one overlap those of the other.
    if (pb >= pe) return;
    int ma = load_code(pb + lane);
    int mb = load_code(pb + 64 + lane);
    int mc2 = load_code(pb + 128 + lane);
    int md = load_code(pb + 192 + lane);
    for (int32_t i0 = pb; i0 < pe; i0 += 128) {
        const int mh[2] = {ma, mb};
        ma = mc2;
        mb = md;
        mc2 = load_code(i0 + 256 + lane);
        md = load_code(i0 + 320 + lane);
        int32_t gi[2];
        int q[2], lend[2], lo[2], hi[2], m[2], s_me[2], s_lo[2], s_hi[2], g_me[2];
        bool valid[2], st[2];
        uint64_t stay[2], grp[2];
        // the lanes' cells
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const int32_t g0 = i0 + 64 * g;
            gi[g] = g0 + lane;
            valid[g] = gi[g] < pe;
            lend[g] = pe - g0 < 64 ? (int)(pe - g0) : 64;   // lanes [0, lend) hold particles
            const int32_t il = g0 + lend[g] - 1;
            const int qa = 63 - __clzll(__ballot(sbl <= g0) & cells);   // sb[0] = pb <= g0
            const int qb = 63 - __clzll(__ballot(sbl <= il) & cells);
            int qq = qa;
            if (qb - qa <= kLoopCells) {
                for (int k = qa + 1; k <= qb; ++k) qq += __builtin_amdgcn_readlane(sbl, k) <= gi[g] ? 1 : 0;
            } else {
                int a = qa, b = qb + 1;   // sb[a] <= i < sb[b] (or b = qb + 1)
                while (b - a > 1) {
                    const int h = (a + b) >> 1;
                    if (sb[h] <= gi[g]) a = h;
                    else b = h;
                }
                qq = a;
            }
            q[g] = qq;
        }
        // each cell's lanes [lo, hi) (q + 1 <= qb + 1 <= nw: inside sb)
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            lo[g] = imax(sb[q[g]] - (i0 + 64 * g), 0);
            hi[g] = imin(sb[q[g] + 1] - (i0 + 64 * g), lend[g]);
        }
        // codes; staying lanes below each lane
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            m[g] = -1;
            if (valid[g]) {
                m[g] = mh[g];
                if (m[g] >= M) { flags |= PSC_DEV_MOVE; m[g] = CENTER; }
            }
            st[g] = m[g] == CENTER;
            stay[g] = __ballot(st[g]);
            s_me[g] = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(stay[g] >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)stay[g], 0u));
        }
        // the counts at the cell's first lane and at its end
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            s_lo[g] = __shfl(s_me[g], lo[g], 64);
            s_hi[g] = __shfl(s_me[g], hi[g] & 63, 64);
        }
        // lanes that move: the lanes of their (cell, code)
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            uint64_t gr = 0;
            const int key = valid[g] ? q[g] * 32 + m[g] : -1;
            uint64_t mv = __ballot(valid[g] && !st[g]);
            while (mv) {
                const int k = __builtin_amdgcn_readlane(key, __ffsll((unsigned long long)mv) - 1);
                const uint64_t bk = __ballot(key == k);
                if (key == k) gr = bk;
                mv &= ~bk;
            }
            grp[g] = gr;
            g_me[g] = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(gr >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)gr, 0u));
        }
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            // grp is empty for the lanes that stay: the two ranks add
            // (written without branches)
            const int rank = g_me[g] + ((s_me[g] - s_lo[g]) & -(int)st[g]);
            // last: a staying lane whose count plus one is its cell's count
            // (all staying lanes of the group when the cell runs to lane 64);
            // a moving lane with none of its group above it (grp <= upto)
            const int s_end = hi[g] < 64 ? s_hi[g] : __popcll(stay[g]);
            const uint64_t lastm =
                (stay[g] & __ballot(s_me[g] + 1 == s_end)) | (~stay[g] & __ballot(grp[g] <= upto));
            const bool last = (lastm >> lane) & 1;
            f(valid[g], gi[g], valid[g] ? q[g] : -1, m[g], rank, last);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// decode_key in 32-bit arithmetic (keys and every product below are less
// than the run's cell count, which is below 2^31)
__device__ __forceinline__ void decode_key32(const RunDev &r, uint32_t key, int pc[3], int l[3]) {
    const uint32_t slab = (uint32_t)r.P[2] * r.n[1] * r.n[0];
    pc[2] = (int)(key / slab);
    uint32_t rem = key - (uint32_t)pc[2] * slab;
    const uint32_t hz = (uint32_t)imin(r.P[2], r.n[2] - pc[2] * r.P[2]);
    const uint32_t row = (uint32_t)r.P[1] * hz * r.n[0];
    pc[1] = (int)(rem / row);
    rem -= (uint32_t)pc[1] * row;
    const uint32_t hy = (uint32_t)imin(r.P[1], r.n[1] - pc[1] * r.P[1]);
    const uint32_t pcells = (uint32_t)r.P[0] * hy * hz;
    pc[0] = (int)(rem / pcells);
    rem -= (uint32_t)pc[0] * pcells;
    const uint32_t hx = (uint32_t)imin(r.P[0], r.n[0] - pc[0] * r.P[0]);
    const uint32_t q = rem / hx;
    l[0] = (int)(rem - q * hx);
    l[1] = (int)(q % hy);
    l[2] = (int)(q / hy);
}

// per new cell n of species S of run R: the arrivals from each source cell
// (one move against each move code), ordered by the source's key, give
// each (move, source) its arrival prefix.  The order comes in closed form
// from source_ranks; the prefix sums run through this thread's M words of
// LDS (`slot`), written in rank order.
template <int DIM>
__device__ __forceinline__ int32_t prefix_cell(const RunDev &R, const SpeciesDev &S, int64_t n, int cs_sel,
                                               uint32_t *err, int32_t *slot) {
    constexpr int M = DIM == 3 ? 27 : 9;
    constexpr int CENTER = M / 2;   // the move that stays in the cell
    const int64_t nc = R.ncell;
    int pc[3], lc[3];
    decode_key32(R, (uint32_t)n, pc, lc);
    Axis ax[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) ax[d] = axis_neighbours(R.P[d], R.n[d], R.np[d], pc[d], lc[d]);
    int rk[M];
    source_ranks<DIM>(ax, rk);
    int32_t ks[M];
    int32_t cn[M];
    // arrivals into n from each source (the particle kernel counts the
    // particles that change cell); those that stay in n are the rest of n
    // global (not generic) pointers throughout: a flat access also counts
    // against the LDS counter, so every wait for the LDS slots would wait
    // for memory as well
    const gptr<const int32_t> cs_old = to_global<const int32_t>(S.cs[cs_sel]);
    const gptr<const uint16_t> cnt = to_global<const uint16_t>(S.cnt);
    int32_t stay = cs_old[n + 1] - cs_old[n];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        int d[3];
        move_delta(DIM, m, d);
        // source cell: one step against the move (index 1 - d per axis)
        const int a0 = DIM == 3 ? 1 - d[0] : 1, a1 = 1 - d[1], a2 = 1 - d[2];
        ks[m] = (int32_t)key_of(R, ax[0].pc[a0], ax[1].pc[a1], ax[2].pc[a2], ax[0].l[a0], ax[1].l[a1], ax[2].l[a2],
                                ax[0].ext[a0], ax[1].ext[a1], ax[2].ext[a2]);
        if (m != CENTER) {
            // the code's plane of counters from a scalar base, indexed by an
            // unsigned 32-bit cell (keys and n are below 2^31): one address
            // operation per load
            const gptr<const uint16_t> cm = cnt + (int64_t)m * nc;
            cn[m] = cm[(uint32_t)ks[m]];
            stay -= cm[(uint32_t)n];   // leaving n with move m
        }
    }
    if (stay < 0) {   // counts inconsistent with the cell offsets
        atomicOr(err, PSC_DEV_OVERFULL);
        stay = 0;
    }
    cn[CENTER] = stay;
#pragma unroll
    for (int m = 0; m < M; ++m) slot[rk[m]] = cn[m];
    int32_t tot = 0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int32_t v = slot[k];
        slot[k] = tot;
        tot += v;
    }
    const gptr<uint16_t> pre = to_global(S.pre);
#pragma unroll
    for (int m = 0; m < M; ++m) (pre + (int64_t)m * nc)[(uint32_t)ks[m]] = (uint16_t)slot[rk[m]];
    if (tot > 65535) atomicOr(err, PSC_DEV_OVERFULL);
    to_global(S.tot)[n] = tot;
    return tot;
}

// Also the first pass of the scan of the totals: workgroup blk covers the
// kSortBlock cells blk % kPrefixPerScan of scan block blk / kPrefixPerScan
// (so it lies in one segment) and writes their sum to partial[blk].
constexpr int kPrefixPerScan = kScanBlock / kSortBlock;

template <int DIM>
__global__ void __launch_bounds__(kSortBlock) k_sort_prefix(const RunDev *__restrict__ runs,
                                                            const ScanSeg *__restrict__ segs,
                                                            const int32_t *__restrict__ block_seg,
                                                            const int32_t *__restrict__ seg_run,
                                                            const int32_t *__restrict__ seg_sp, int cs_sel,
                                                            int32_t *__restrict__ partial, uint32_t *err) {
    constexpr int M = DIM == 3 ? 27 : 9;
    __shared__ int32_t wsum[kSortBlock / 64];
    __shared__ int32_t slots[kSortBlock * M];   // M words per thread (odd stride: no bank conflicts in order)
    const int64_t blk = xcd_block_sort();   // dispatch order unless PSC_XCD_SORT
    const int64_t b = blk / kPrefixPerScan;
    const int sg = block_seg[b];
    const RunDev &R = runs[seg_run[sg]];
    const int64_t n = (b - segs[sg].block0) * kScanBlock + (blk - b * kPrefixPerScan) * kSortBlock + threadIdx.x;
    int32_t tot = 0;
    if (n < segs[sg].n) tot = prefix_cell<DIM>(R, R.sp[seg_sp[sg]], n, cs_sel, err, slots + threadIdx.x * M);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t s = 0;
#pragma unroll
        for (int w = 0; w < kSortBlock / 64; ++w) s += wsum[w];
        partial[blk] = s;
    }
}

// raw buffer resource of the permutation (4th word: 32-bit data format, as
// for every gfx9-family chip); offsets at or past n * 4 bytes are dropped.
// kBufferDrop lies past every buffer of at most kBufferMaxN words, also
// when the range check adds the store's 4 bytes
constexpr int kBufferWord3 = 0x00020000;
constexpr int32_t kBufferMaxN = 0x3FFFFFF0;
constexpr int kBufferDrop = (int)0xFFFFFFE0u;
static_assert(kMaxCapacity <= kBufferMaxN, "every species fits a buffer resource");

// per old cell: stable positions of its particles.  Lane q sets up the first
// position of every move code of its cell in LDS; the walk then writes
// perm[position] = index for 64 consecutive particles at a time, so the
// particles that stay (one code, consecutive positions) are stored coalesced.
template <int DIM>
__global__ void __launch_bounds__(kSortThreads) k_sort_scatter(const RunDev *__restrict__ runs,
                                                             const ScanSeg *__restrict__ segs,
                                                             const int32_t *__restrict__ block_seg,
                                                             const int32_t *__restrict__ seg_run,
                                                             const int32_t *__restrict__ seg_sp, int cs_sel,
                                                             uint32_t *err) {
    constexpr int M = DIM == 3 ? 27 : 9;
    __shared__ int32_t tab_all[4][64 * M];
    __shared__ int32_t sb_all[4][65];
    const CellBlock B = cell_block<DIM>(runs, segs, block_seg, seg_run, seg_sp);
    if (B.cw >= B.ce) return;   // whole wave
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int32_t *tab = tab_all[wave], *sb = sb_all[wave];
    const RunDev &R = *B.R;
    const SpeciesDev &S = *B.S;
    const int64_t nc = R.ncell;
    const gptr<const int32_t> cs_old = to_global<const int32_t>(S.cs[cs_sel]);
    const gptr<const int32_t> cs_new = to_global<const int32_t>(S.cs[1 - cs_sel]);
    const gptr<const uint16_t> pre = to_global<const uint16_t>(S.pre);
    const gptr<uint16_t> cnt = to_global(S.cnt);
    const int nw = (int)(B.ce - B.cw);
    sb[lane] = cs_old[B.cw + (lane < nw ? lane : nw)];
    if (lane == 0) sb[64] = cs_old[B.ce];
    if (lane < nw) {
        const int64_t o = B.cw + lane;
        int pc[3], lc[3];
        decode_key32(R, (uint32_t)o, pc, lc);
        Axis ax[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) ax[d] = axis_neighbours(R.P[d], R.n[d], R.np[d], pc[d], lc[d]);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            int d[3];
            move_delta(DIM, m, d);
            // destination cell: one step along the move (index 1 + d per axis)
            const int a0 = DIM == 3 ? 1 + d[0] : 1, a1 = 1 + d[1], a2 = 1 + d[2];
            const uint32_t dst = key_of(R, ax[0].pc[a0], ax[1].pc[a1], ax[2].pc[a2], ax[0].l[a0], ax[1].l[a1],
                                        ax[2].l[a2], ax[0].ext[a0], ax[1].ext[a1], ax[2].ext[a2]);
            tab[m * 64 + lane] = cs_new[dst] + pre[m * nc + o];
            if (m != M / 2) cnt[m * nc + o] = 0;   // consumed by the prefix pass: clear for the next push
        }
    }
    __builtin_amdgcn_wave_barrier();
    const int32_t n = (int32_t)S.n;
    uint32_t flags = 0;
    bool bad = false;
    // the wave's particle range (read from LDS: made scalar explicitly),
    // kept inside [0, n] also for offsets corrupted by a counter overflow
    const int32_t pe = imin(imax(__builtin_amdgcn_readfirstlane(sb[nw]), 0), n);
    const int32_t pb = imin(imax(__builtin_amdgcn_readfirstlane(sb[0]), 0), pe);
    auto walk = [&](auto &&load_code, auto &&store) {
        walk_cells<M>(sb, nw, pb, pe, load_code, flags,
                      [&](bool valid, int32_t i, int q, int m, int rank, bool last) {
                          const int slot = valid ? m * 64 + q : 0;
                          const int32_t p = tab[slot] + rank;
                          // out of range only after a counter overflow
                          const bool ok = valid && p >= 0 && p < n;
                          bad |= valid && !ok;
                          store(ok, p, i);   // on every lane of every group
                          if (valid && last) tab[slot] = p + 1;
                      });
    };
    // a raw buffer store: the hardware drops stores at offsets past the
    // buffer's n * 4 bytes, so lanes without a position need no other target
    const __amdgpu_buffer_rsrc_t prs =
        __builtin_amdgcn_make_buffer_rsrc(S.perm[1 - cs_sel], (short)0, (int)((uint32_t)n << 2), kBufferWord3);
    // move codes through a byte buffer of n entries: indices past the end
    // read 0 (their lanes hold no particle)
    const __amdgpu_buffer_rsrc_t mrs = __builtin_amdgcn_make_buffer_rsrc(S.mc, (short)0, n, kBufferWord3);
    walk([&](int32_t idx) { return (int)__builtin_amdgcn_raw_buffer_load_b8(mrs, idx, 0, 0); },
         [&](bool ok, int32_t p, int32_t i) {
             __builtin_amdgcn_raw_buffer_store_b32((uint32_t)i, prs, ok ? (int)((uint32_t)p << 2) : kBufferDrop, 0,
                                                   0);
         });
    if (bad) flags |= PSC_DEV_OVERFULL;
    if (flags) atomicOr(err, flags);   // also an invalid move code (PSC_DEV_MOVE)
}

// ---------------------------------------------------------------------------
// segmented exclusive scan: out[0..n] with out[n] = total, per segment
// ---------------------------------------------------------------------------
// one workgroup: segmented exclusive scan of the scan blocks' totals (each
// the sum of its kPrefixPerScan partial sums) into block_sums
__global__ void __launch_bounds__(1024) k_scan_blocks(const ScanSeg *__restrict__ segs,
                                                      const int32_t *__restrict__ block_seg, int64_t n_blocks,
                                                      const int32_t *__restrict__ partial,
                                                      int32_t *__restrict__ block_sums) {
    __shared__ int32_t val[1024];
    __shared__ int32_t flg[1024];
    const int t = threadIdx.x;
    int32_t carry = 0;
    for (int64_t cb = 0; cb < n_blocks; cb += 1024) {
        const int64_t b = cb + t;
        int32_t v = 0;
        if (b < n_blocks)
#pragma unroll
            for (int k = 0; k < kPrefixPerScan; ++k) v += partial[b * kPrefixPerScan + k];
        const int32_t f = b < n_blocks ? (b == segs[block_seg[b]].block0) : 1;
        val[t] = v;
        flg[t] = f;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int32_t av = 0, af = 0;
            if (t >= off) { av = val[t - off]; af = flg[t - off]; }
            __syncthreads();
            if (t >= off) {
                if (!flg[t]) val[t] += av;
                flg[t] |= af;
            }
            __syncthreads();
        }
        // val: inclusive segmented sum since the last head in this chunk
        const int32_t excl = val[t] - v + (flg[t] ? 0 : carry);
        const int32_t last_v = val[1023], last_f = flg[1023];
        __syncthreads();
        if (b < n_blocks) block_sums[b] = excl;
        carry = last_f ? last_v : carry + last_v;
        __syncthreads();
    }
}

// Scan block b of its segment: the block's values pass through LDS
// (coalesced loads and stores), each thread scans eight consecutive ones, and
// the thread sums are scanned within each wave by lane shuffles, then over
// the four waves.  Threads reading their eight values straight from memory
// would touch a separate cache line per lane and load.
static_assert(kScanPerThread == 8 && kScanBlock == 256 * kScanPerThread, "two int4 per thread");
__global__ void __launch_bounds__(256) k_scan_final(const ScanSeg *__restrict__ segs,
                                                    const int32_t *__restrict__ block_seg,
                                                    const int32_t *__restrict__ block_sums) {
    __shared__ __align__(16) int32_t tile[kScanBlock];
    __shared__ int32_t wtot[4];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t b = blockIdx.x;
    const ScanSeg sg = segs[block_seg[b]];
    const int32_t offset = block_sums[b];
    const int64_t base = (b - sg.block0) * kScanBlock;
    const int n = (int)(sg.n - base < kScanBlock ? sg.n - base : kScanBlock);
#pragma unroll
    for (int q = 0; q < kScanPerThread; ++q) {
        const int i = q * 256 + t;
        tile[i] = i < n ? sg.in[base + i] : 0;
    }
    __syncthreads();
    int4 *mine = reinterpret_cast<int4 *>(tile) + 2 * t;   // values 8t .. 8t + 7
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
    int32_t run = offset + inc - sum, total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const int32_t x = wtot[w];
        run += w < wv ? x : 0;
        total += x;
    }
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
    for (int q = 0; q < kScanPerThread; ++q) {
        const int i = q * 256 + t;
        if (i < n) sg.out[base + i] = tile[i];
    }
    if (t == 255 && base + kScanBlock >= sg.n) sg.out[sg.n] = offset + total;   // the segment's last block
}

// partial: kPrefixPerScan partial sums per scan block (from k_sort_prefix)
hipError_t launch_scan(const ScanSeg *segs, int, int64_t n_blocks, const int32_t *block_seg, const int32_t *partial,
                       int32_t *block_sums, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, segs, block_seg, n_blocks, partial, block_sums);
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)n_blocks), dim3(256), 0, s, segs, block_seg, block_sums);
    return hipGetLastError();
}

hipError_t launch_sort(const Launch &L, const int64_t *, const int32_t *seg_run, const int32_t *seg_sp, int n_segs,
                       int64_t, const ScanSeg *segs_dev, int64_t n_scan_blocks, int32_t *scan_tmp, int cs_sel,
                       int dim) {
    // scan_tmp: [0, n_scan_blocks) block sums; then the block -> segment
    // table; then kPrefixPerScan partial sums per scan block
    const int32_t *block_seg = scan_tmp + n_scan_blocks;
    int32_t *partial = scan_tmp + 2 * n_scan_blocks;
    const unsigned grid = (unsigned)(kPrefixPerScan * n_scan_blocks);
    const unsigned cgrid = (unsigned)((dim == 3 ? sort_per_scan<3>() : sort_per_scan<2>()) * n_scan_blocks);
    // the per (cell, move) counts come from the particle kernel
    if (dim == 3)
        hipLaunchKernelGGL(k_sort_prefix<3>, dim3(grid), dim3(kSortBlock), 0, L.stream, L.runs_dev, segs_dev,
                           block_seg, seg_run, seg_sp, cs_sel, partial, L.err);
    else
        hipLaunchKernelGGL(k_sort_prefix<2>, dim3(grid), dim3(kSortBlock), 0, L.stream, L.runs_dev, segs_dev,
                           block_seg, seg_run, seg_sp, cs_sel, partial, L.err);
    hipError_t e = launch_scan(segs_dev, n_segs, n_scan_blocks, block_seg, partial, scan_tmp, L.stream);
    if (e != hipSuccess) return e;
    if (dim == 3)
        hipLaunchKernelGGL(k_sort_scatter<3>, dim3(cgrid), dim3(kSortThreads), 0, L.stream, L.runs_dev, segs_dev,
                           block_seg, seg_run, seg_sp, cs_sel, L.err);
    else
        hipLaunchKernelGGL(k_sort_scatter<2>, dim3(cgrid), dim3(kSortThreads), 0, L.stream, L.runs_dev, segs_dev,
                           block_seg, seg_run, seg_sp, cs_sel, L.err);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// particle loading (general stable sort, once) and read-back
// ---------------------------------------------------------------------------
__global__ void k_keys(RunDev R, int64_t n, const int32_t *__restrict__ gcell, int32_t *__restrict__ keys,
                       int32_t *__restrict__ idx, uint32_t *err) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int64_t c = gcell[p];
    if (c < 0 || c >= R.ncell) {
        atomicOr(err, PSC_DEV_KEY);
        c = 0;
    }
    const int i = (int)(c % R.n[0]);
    const int j = (int)((c / R.n[0]) % R.n[1]);
    const int k = (int)(c / ((int64_t)R.n[0] * R.n[1]));
    keys[p] = (int32_t)encode_key(R, i, j, k);
    idx[p] = (int32_t)p;
}

hipError_t launch_keys(const RunDev &r, int64_t n, const int32_t *gcell, int32_t *keys, int32_t *idx,
                       uint32_t *err, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, r, n, gcell, keys, idx, err);
    return hipGetLastError();
}

__global__ void k_keys_to_cells(RunDev R, int64_t n, const int32_t *__restrict__ keys, int32_t *__restrict__ cells) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int64_t key = keys[p];
    if (key < 0 || key >= R.ncell) {
        cells[p] = -1;
        return;
    }
    int g[3];
    decode_key(R, key, g);
    cells[p] = (int32_t)(g[0] + (int64_t)R.n[0] * (g[1] + (int64_t)R.n[1] * g[2]));
}

hipError_t launch_keys_to_cells(const RunDev &r, int64_t n, const int32_t *keys, int32_t *cells, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_keys_to_cells, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, r, n, keys, cells);
    return hipGetLastError();
}

__global__ void k_load_gather(RunDev R, int sp, int64_t n, const int32_t *__restrict__ skeys,
                              const int32_t *__restrict__ sidx, const float *__restrict__ goff,
                              const float *__restrict__ gu, const int32_t *__restrict__ gid) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const SpeciesDev &S = R.sp[sp];
    const int64_t src = sidx[r];
    S.cell[0][r] = skeys[r];
    for (int d = 0; d < R.dim; ++d) S.off[0][d * S.cap + r] = goff[d * n + src];
    for (int c = 0; c < 3; ++c) S.u[0][c * S.cap + r] = gu[c * n + src];
    if (S.id[0]) S.id[0][r] = gid ? gid[src] : (int32_t)src;
}

hipError_t launch_load_gather(const RunDev &r, int species, int64_t n, const int32_t *skeys, const int32_t *sidx,
                              const float *goff, const float *gu, const int32_t *gid, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_load_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, r, species, n, skeys, sidx,
                       goff, gu, gid);
    return hipGetLastError();
}

// particles per cell of sorted keys; a cell's 65536th particle flags the
// overflow of the 16-bit per (cell, move) counters of the step sort
// Cell offsets of keys sorted ascending: cs[c] = first index whose key is at
// least c, cs[ncell] = n.  Index i writes the offsets of the cells in
// (key[i-1], key[i]] (index 0 from cell 0, index n up to ncell), so every
// entry is written once and no counting is needed.  A cell with more than
// 65535 particles (the width of the per-(cell, move) counters) sets the
// overfull flag; keys out of range or out of order set the key flag.
__global__ void k_cell_starts(int64_t n, int64_t ncell, const int32_t *__restrict__ keys, int32_t *__restrict__ cs,
                              uint32_t *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const int64_t lo = i == 0 ? -1 : keys[i - 1];
    const int64_t hi = i == n ? ncell : keys[i];
    uint32_t flags = 0;
    if (lo < -1 || hi > ncell || (i < n && hi >= ncell) || hi < lo) flags |= PSC_DEV_KEY;
    else
        for (int64_t c = lo + 1; c <= hi; ++c) cs[c] = (int32_t)i;
    if (i < n && i >= 65535 && keys[i - 65535] == keys[i]) flags |= PSC_DEV_OVERFULL;
    if (flags) atomicOr(err, flags);
}

hipError_t launch_cell_starts(int64_t n, int64_t ncell, const int32_t *keys, int32_t *cs, uint32_t *err,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_cell_starts, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, s, n, ncell, keys, cs, err);
    return hipGetLastError();
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

__global__ void k_get(RunDev R, int sp, int front, const int32_t *__restrict__ perm, int32_t *__restrict__ cell,
                      float *__restrict__ off, float *__restrict__ u, int32_t *__restrict__ id) {
    const SpeciesDev &S = R.sp[sp];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = S.n;
    if (r >= n) return;
    const int64_t src = perm ? perm[r] : r;
    if (cell) cell[r] = S.cell[front][src];
    if (off)
        for (int d = 0; d < R.dim; ++d) off[d * n + r] = S.off[front][d * S.cap + src];
    if (u)
        for (int c = 0; c < 3; ++c) u[c * n + r] = S.u[front][c * S.cap + src];
    if (id) id[r] = S.id[front] ? S.id[front][src] : -1;
}

hipError_t launch_get(const RunDev &r, int species, int front, const int32_t *perm, int32_t *cell, float *off, float *u,
                      int32_t *id, hipStream_t s) {
    const int64_t n = r.sp[species].n;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_get, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, r, species, front, perm,
                       cell, off, u, id);
    return hipGetLastError();
}

__global__ void k_iota(int32_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}

hipError_t launch_iota(int32_t *p, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t radix_sort_pairs(void *temp, size_t *temp_bytes, const int32_t *keys_in, int32_t *keys_out,
                            const int32_t *vals_in, int32_t *vals_out, int64_t n, int bits, hipStream_t s) {
    return rocprim::radix_sort_pairs(temp, *temp_bytes, keys_in, keys_out, vals_in, vals_out, (size_t)n, 0u,
                                     (unsigned)bits, s);
}

}  // namespace psc
