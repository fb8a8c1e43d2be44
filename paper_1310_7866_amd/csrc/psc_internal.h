// psc_internal.h -- device descriptors and index helpers of the HIP library.
//
// Data layout in HBM (all float32 unless noted):
//   fields   E, B, J: 3 * ncell per run, component-major, x fastest.
//   particles: per species two buffer sets (ping-pong) of SoA arrays
//            cell (int32 patch-major key), off[D] (in-cell offsets),
//            u[3] (momentum per mass), optional id (int32).
//   workspace (library-carved, caller-allocated):
//            per patch a current tile of 3 * jt[0]*jt[1]*jt[2] floats
//            (patch cells plus `order` ghost layers below and order+1
//            above, in the patch's own tile coordinates);
//            per species two cell-offset arrays cs (int32, ncell + 1),
//            the permutation (int32), per-particle move codes (uint8),
//            per-(cell, move) counts and prefixes (uint16, 3^D * ncell),
//            arrival totals (int32, ncell); per run an FP64 charge array
//            for the diagnostics; the work tables; the error word.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/psc.h"

namespace psc {

constexpr int kMaxSpecies = PSC_MAX_SPECIES;
constexpr int kBlock = 256;          // threads per workgroup of the particle kernel
constexpr int kScanPerThread = 8;    // elements per thread in the scans
constexpr int kScanBlock = 256 * kScanPerThread;
// particle slots per species buffer: indices and the sort's group offsets
// (index + 255) stay in int32
// particle slots per species buffer: the byte offsets of a species' arrays
// stay below 2^32, so the kernels address them as a base plus a 32-bit offset
constexpr int64_t kMaxCapacity = (1ll << 30) - 1024;
constexpr int kAdjBlock = 512;       // threads per workgroup of the particle adjoint
constexpr int kAdjChunk = 2048;      // particles per work item of the particle adjoint

struct SpeciesDev {
    float q, m, w;
    float qdt_2m;        // q dt / (2 m)
    float qw;            // q * w
    int32_t pad0;
    int64_t n;           // particles held
    int64_t cap;         // slots per buffer (array stride)
    int32_t *cell[2];
    float *off[2];
    float *u[2];
    int32_t *id[2];      // both null when ids are not carried
    int32_t *cs[2];      // cell start offsets, ncell + 1
    int32_t *perm[2];    // sorted slot -> index in the pushed buffer: perm[c] goes with
                         // cs[c] (the sort writes both of 1 - cs_sel, the push reads
                         // those of cs_sel; by default both name one workspace array)
    uint8_t *mc;         // move code of each pushed particle
    uint16_t *cnt;       // [m * ncell + cell]: particles of `cell` with move m != stay
                         // (counted by the particle kernel, cleared by the sort's scatter)
    uint16_t *pre;       // [m * ncell + cell]: arrivals into cell+d(m) that precede them
    int32_t *tot;        // arrivals per new cell (scan input)
    int64_t seg;         // index of this (run, species) among scan segments
};

struct RunDev {
    int dim, order;
    int vb;              // order 1: Villasenor-Buneman deposit instead of Esirkepov
    int fold_direct;     // every patch extent >= the current halo (order + 1):
                         // a tile aliases cells of its own and adjacent patches only
    int jdirect;         // the particle kernel adds its LDS tiles straight into the
                         // run's current accumulator jacc (every tile coordinate
                         // maps into [-n, 3n) per dimension)
    int n[3];            // cells
    int P[3];            // nominal patch size
    int np[3];           // patches per dimension
    int n_patches;
    int n_species;
    int chunk;           // particles per work item of the particle kernel
    int64_t ncell;
    int64_t cell_base;   // offset of the run in the flat cell space of all runs
    float dx[3];
    float inv_dx[3];
    double dxd[3];       // exact cell sizes for the float64 diagnostics
    float dt;
    int jt[3];           // current-tile extent per dimension
    int64_t jtile_cells; // jt[0]*jt[1]*jt[2]
    float *E, *B, *J;
    float *jtile;        // n_patches * 3 * jtile_cells
    long long *jacc;     // jdirect: 3 * ncell fixed-point sums of the current in units
    double jq, jinvq;    // of jq (a power of two) and its inverse
    double *rho;         // ncell, diagnostics scratch
    SpeciesDev sp[kMaxSpecies];
};

// One (run, species, patch) unit of particle work.
struct Unit {
    int32_t run, species, patch, pad;
};

// Scan segment: one (run, species) array of ncell counts.
struct ScanSeg {
    int32_t *in;         // ncell counts
    int32_t *out;        // ncell + 1 exclusive prefix
    int64_t n;
    int64_t block0;      // first scan block of the segment
};

// Adjoint step: forward state, adjoint state and scratch of one species/run.
struct AdjSpecies {
    const int32_t *key;   // forward particles at the start of the step: sorted by key,
    const float *off;     // or, with rperm, in the buffer order the step's push read
    const float *u;       // them in; off D x stride, u 3 x stride
    const int32_t *rperm; // null, or sorted slot -> buffer slot of key/off/u
    int64_t stride;       // array stride of off and u (n for sorted copies)
    const int32_t *perm;  // sort permutation of the step: next sorted slot -> slot
    int64_t n;
    float *loff, *lu;     // caller: in (next step's sorted order), out (this step's)
    float *soff, *su;     // scratch: incoming adjoints moved to this step's slots
    const int32_t *cs;    // cell offsets of the sorted keys, ncell + 1 (given, or computed
                          // into cs_scratch)
    int32_t *cs_scratch;
};

struct AdjRun {
    const float *E, *B;   // forward fields at the start of the step: E^{n+1/2}, B^n
    float *lE, *lB;       // in: adjoints of E', B2; out: adjoints of E, B
    float *B1;            // scratch: B after the first half step
    float *LJ;            // scratch: adjoint of J = -dt lE'
    float *gtile;         // scratch: per-patch transposed-interpolation tiles (6 comps)
    AdjSpecies sp[kMaxSpecies];
};

// ----------------------------------------------------------------------------
// ghost widths
// ----------------------------------------------------------------------------
// Field tile: one layer below, `order` above (interpolation supports).
// Current tile: `order` below, `order + 1` above (Esirkepov stencils of a
// particle that moves at most one cell).
__host__ __device__ inline int field_lo(int) { return 1; }
__host__ __device__ inline int field_hi(int order) { return order; }
__host__ __device__ inline int cur_lo(int order) { return order; }
__host__ __device__ inline int cur_hi(int order) { return order + 1; }

__host__ __device__ inline int imin(int a, int b) { return a < b ? a : b; }
__host__ __device__ inline int imax(int a, int b) { return a > b ? a : b; }
__host__ __device__ inline int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}
// periodic image in [0, n) of -n <= i < 3n, without a division
__host__ __device__ inline int wrap_near(int i, int n) {
    i += i < 0 ? n : 0;
    i -= i >= n ? n : 0;
    return i >= n ? i - n : i;
}
// The direct current path: a run's tile coordinate t in [0, P + lo + hi)
// along an active dimension stands for cell o + t - lo of a patch at origin
// o <= n - 1, i.e. for -lo <= i <= n + P + hi - 2; wrap_near covers that
// when lo <= n and P + hi <= 2 n + 1.
__host__ __device__ inline bool current_direct_fits(int n, int P, int order) {
    return cur_lo(order) <= n && P + cur_hi(order) <= 2 * n + 1;
}

// actual extent of patch coordinate pc along d (the last one is truncated)
__host__ __device__ inline int patch_ext(const RunDev &r, int d, int pc) {
    return imin(r.P[d], r.n[d] - pc * r.P[d]);
}

// key of the first cell of patch (pi, pj, pk)
__host__ __device__ inline int64_t patch_key_base(const RunDev &r, int pi, int pj, int pk) {
    int64_t hz = patch_ext(r, 2, pk), hy = patch_ext(r, 1, pj);
    return (int64_t)pk * r.P[2] * r.n[1] * r.n[0] + (int64_t)pj * r.P[1] * hz * r.n[0] +
           (int64_t)pi * r.P[0] * hy * hz;
}

__host__ __device__ inline void patch_coords(const RunDev &r, int p, int pc[3]) {
    pc[0] = p % r.np[0];
    pc[1] = (p / r.np[0]) % r.np[1];
    pc[2] = p / (r.np[0] * r.np[1]);
}

// patch-major key of geometric cell (i, j, k) (already wrapped)
__host__ __device__ inline int64_t encode_key(const RunDev &r, int i, int j, int k) {
    int pi = i / r.P[0], pj = j / r.P[1], pk = k / r.P[2];
    int hx = patch_ext(r, 0, pi), hy = patch_ext(r, 1, pj);
    int li = i - pi * r.P[0], lj = j - pj * r.P[1], lk = k - pk * r.P[2];
    return patch_key_base(r, pi, pj, pk) + li + (int64_t)hx * (lj + (int64_t)hy * lk);
}

// Key of the cell at local coordinates l of patch pc (extents h), where each
// l[d] lies within one cell of the patch: -1 <= l[d] <= h[d].  A coordinate
// outside the patch moves to the neighbouring patch with periodic wrap.
// Equals encode_key of the wrapped geometric cell, without divisions.
__host__ __device__ inline int64_t neighbour_key(const RunDev &r, const int pc[3], const int h[3], const int l[3]) {
    int q[3], m[3], e[3];
    for (int d = 0; d < 3; ++d) {
        q[d] = pc[d];
        m[d] = l[d];
        e[d] = h[d];
        if (l[d] < 0) {
            q[d] = pc[d] == 0 ? r.np[d] - 1 : pc[d] - 1;
            e[d] = patch_ext(r, d, q[d]);
            m[d] = e[d] - 1;
        } else if (l[d] >= h[d]) {
            q[d] = pc[d] + 1 == r.np[d] ? 0 : pc[d] + 1;
            e[d] = patch_ext(r, d, q[d]);
            m[d] = 0;
        }
    }
    return patch_key_base(r, q[0], q[1], q[2]) + m[0] + (int64_t)e[0] * (m[1] + (int64_t)e[1] * m[2]);
}

// inverse of encode_key
__host__ __device__ inline void decode_key(const RunDev &r, int64_t key, int g[3]) {
    int64_t slab = (int64_t)r.P[2] * r.n[1] * r.n[0];
    int pk = (int)(key / slab);
    int64_t rem = key - pk * slab;
    int hz = patch_ext(r, 2, pk);
    int64_t row = (int64_t)r.P[1] * hz * r.n[0];
    int pj = (int)(rem / row);
    rem -= pj * row;
    int hy = patch_ext(r, 1, pj);
    int64_t pcells = (int64_t)r.P[0] * hy * hz;
    int pi = (int)(rem / pcells);
    rem -= pi * pcells;
    int hx = patch_ext(r, 0, pi);
    int li = (int)(rem % hx);
    rem /= hx;
    int lj = (int)(rem % hy);
    int lk = (int)(rem / hy);
    g[0] = pi * r.P[0] + li;
    g[1] = pj * r.P[1] + lj;
    g[2] = pk * r.P[2] + lk;
}

// Lane map of the mixed-lane ablation of the particle kernel: lane g of a
// work item with `nruns` lane strips takes strip (g mod 64) M + g div 64,
// M = ceil(nruns / 64), so the 64 lanes of a wave are spread over the item
// instead of lying on consecutive strips.  A bijection of [0, 64 M) onto
// itself; g >= 64 M gives nruns (no strip).  The kernel's rounds visit every
// g < 64 M since a workgroup is a whole number of waves.
__host__ __device__ inline int32_t mix_lane(int32_t g, int32_t nruns) {
    const int32_t M = (nruns + 63) >> 6;
    return g < 64 * M ? (g & 63) * M + (g >> 6) : nruns;
}

// number of move codes and the code of "stays in its cell"
__host__ __device__ inline int n_moves(int dim) { return dim == 3 ? 27 : 9; }

// displacement (-1, 0, 1 per dimension) of move code m
__host__ __device__ inline void move_delta(int dim, int m, int d[3]) {
    if (dim == 3) {
        d[0] = m % 3 - 1;
        d[1] = (m / 3) % 3 - 1;
        d[2] = m / 9 - 1;
    } else {
        d[0] = 0;
        d[1] = m % 3 - 1;
        d[2] = m / 3 - 1;
    }
}

// Patch coordinate, local coordinate and patch extent of each cell along
// one dimension, and of its neighbours one cell down (index 0) and up (2):
// a move of at most one cell leaves the patch only at its faces, so the
// neighbour's patch is the same or the adjacent one (periodic) and needs
// no division.
struct Axis {
    int pc[3], l[3], ext[3];
};

__host__ __device__ inline Axis axis_neighbours(int P, int n, int np, int pc, int l) {
    Axis a;
    const int ext = imin(P, n - pc * P);
    const int pdn = pc == 0 ? np - 1 : pc - 1, pup = pc == np - 1 ? 0 : pc + 1;
    const int edn = imin(P, n - pdn * P);
    a.pc[1] = pc;
    a.l[1] = l;
    a.ext[1] = ext;
    const bool out_dn = l == 0;
    a.pc[0] = out_dn ? pdn : pc;
    a.l[0] = out_dn ? edn - 1 : l - 1;
    a.ext[0] = out_dn ? edn : ext;
    const bool out_up = l == ext - 1;
    a.pc[2] = out_up ? pup : pc;
    a.l[2] = out_up ? 0 : l + 1;
    a.ext[2] = out_up ? imin(P, n - pup * P) : ext;
    return a;
}

// key of the cell at (patch, local) coordinates, extents given
__host__ __device__ inline uint32_t key_of(const RunDev &r, int p0, int p1, int p2, int l0, int l1, int l2, int e0,
                                           int e1, int e2) {
    return (uint32_t)p2 * r.P[2] * r.n[1] * r.n[0] + (uint32_t)p1 * r.P[1] * e2 * r.n[0] +
           (uint32_t)p0 * r.P[0] * e1 * e2 + (uint32_t)(l0 + e0 * (l1 + e1 * l2));
}

// Rank, in key order, of the source cell of each move code m of a new
// cell (the cell one move against m; ax: the new cell's per-axis
// candidates below / own / above from axis_neighbours).  Keys order cells
// by patch coordinate (z, y, x), then by local coordinate (z, y, x), so per
// axis it is enough to know, for each candidate a, how many of the three
// lie in a lower patch (lo), in the same patch (eq, a included) and in the
// same patch at a lower local coordinate (in):
//   rank = lo_z 3 K + eq_z (lo_y K + eq_y lo_x) + in_z eq_y eq_x + in_y eq_x + in_x
// with K the candidates per x (3 in 3-d; 2-d: x inactive, lo = in = 0,
// eq = 1).  Distinct source cells (every active axis has >= 3 cells) get
// the ranks 0 .. M - 1.
template <int DIM>
__host__ __device__ inline void source_ranks(const Axis ax[3], int rank[]) {
    constexpr int M = DIM == 3 ? 27 : 9;
    constexpr int K = DIM == 3 ? 3 : 1;
    int lo[3][3], eq[3][3], in[3][3];
    for (int d = 0; d < 3; ++d)
        for (int a = 0; a < 3; ++a) {
            lo[d][a] = 0;
            eq[d][a] = 1;
            in[d][a] = 0;
            if (DIM == 2 && d == 0) continue;
            for (int b = 0; b < 3; ++b) {
                if (b == a) continue;
                lo[d][a] += ax[d].pc[b] < ax[d].pc[a] ? 1 : 0;
                eq[d][a] += ax[d].pc[b] == ax[d].pc[a] ? 1 : 0;
                in[d][a] += ax[d].pc[b] == ax[d].pc[a] && ax[d].l[b] < ax[d].l[a] ? 1 : 0;
            }
        }
    for (int m = 0; m < M; ++m) {
        int dm[3];
        move_delta(DIM, m, dm);
        const int x = DIM == 3 ? 1 - dm[0] : 1, y = 1 - dm[1], z = 1 - dm[2];
        const int r = lo[2][z] * 3 * K + eq[2][z] * (lo[1][y] * K + eq[1][y] * lo[0][x]) +
                      in[2][z] * eq[1][y] * eq[0][x] + in[1][y] * eq[0][x] + in[0][x];
        rank[m] = r < M - 1 ? r : M - 1;
    }
}

// ----------------------------------------------------------------------------
// launchers (defined in the .hip files)
// ----------------------------------------------------------------------------
struct Launch {
    const RunDev *runs_dev;   // device copy of the run table
    const RunDev *runs_host;  // host copy
    int n_runs;
    hipStream_t stream;
    uint32_t *err;            // device error word
};

// the persistent particle kernel's 8 queue counters, one per 128-byte line
constexpr int kQueueStride = 32;

// how the particle kernel is launched: 0 one workgroup per work item,
// 1 persistent workgroups with per-XCD queues, 2 persistent workgroups over a
// load-balanced partition of the units
struct PushMode {
    int mode = 0;
    int threads = 256;         // workgroup size: 256, 384 or 512
    int run = 1;               // consecutive particles per lane and round (1 or 2)
    int workers = 0;           // persistent workgroups (modes 1, 2)
    int32_t *queue = nullptr;  // 8 counters (mode 1; reset every launch)
    const int32_t *part = nullptr;  // workers + 1 unit boundaries (mode 2)
};

hipError_t launch_push(const Launch &L, const Unit *units_dev, int n_units, int32_t *item_start, int64_t max_items,
                       int dim, int order, int front, int cs_sel, int use_perm, size_t lds_bytes,
                       const PushMode &pm);
hipError_t launch_unit_counts(const Launch &L, const Unit *units, int n_units, int cs_sel, int32_t *out);
hipError_t launch_fields(const Launch &L, int op, int64_t total_cells, const int64_t *run_cell_base_dev);
// fold: runs with fold_direct by patch (one workgroup row per patch; bit
// 1 << dim of direct_dims set when such a run has that dimension), the
// others by cell with the alias search
hipError_t launch_fold(const Launch &L, int64_t total_cells, const int64_t *run_cell_base_dev, int64_t total_patches,
                       const int64_t *run_patch_base_dev, int max_patch_cells, int direct_dims, bool any_search);
// J = jacc * jq and jacc = 0 in the runs with jdirect
hipError_t launch_finish_current(const Launch &L, int64_t total_cells, const int64_t *run_cell_base_dev);
hipError_t launch_sort(const Launch &L, const int64_t *seg_cell_base_dev, const int32_t *seg_run_dev,
                       const int32_t *seg_species_dev, int n_segs, int64_t total_seg_cells,
                       const ScanSeg *segs_dev, int64_t n_scan_blocks, int32_t *scan_tmp, int cs_sel,
                       int max_dim);
hipError_t launch_scan(const ScanSeg *segs_dev, int n_segs, int64_t n_blocks, const int32_t *block_seg_dev,
                       const int32_t *partial, int32_t *block_sums, hipStream_t s);
hipError_t launch_keys(const RunDev &r, int64_t n, const int32_t *gcell, int32_t *keys, int32_t *idx,
                       uint32_t *err, hipStream_t s);
hipError_t launch_keys_to_cells(const RunDev &r, int64_t n, const int32_t *keys, int32_t *cells,
                                hipStream_t s);
hipError_t launch_load_gather(const RunDev &r, int species, int64_t n, const int32_t *sorted_keys,
                              const int32_t *sorted_idx, const float *goff, const float *gu,
                              const int32_t *gid, hipStream_t s);
hipError_t launch_cell_starts(int64_t n, int64_t ncell, const int32_t *sorted_keys, int32_t *cs, uint32_t *err,
                              hipStream_t s);
hipError_t launch_get(const RunDev &r, int species, int front, const int32_t *perm, int32_t *cell,
                      float *off, float *u, int32_t *id, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_items_scan(int n_units, int32_t *item_start, int32_t *queue, hipStream_t s);
hipError_t launch_adj_seed(const float *E, const float *B, float *lE, float *lB, int64_t n, float dV,
                           hipStream_t s);
hipError_t launch_iota(int32_t *p, int64_t n, hipStream_t s);
hipError_t launch_diag(const Launch &L, double *out, double *gauss, int64_t total_cells,
                       const int64_t *run_cell_base_dev, int front);
hipError_t launch_marder(const Launch &L, const double *ref, double d, int iters, int64_t total_cells,
                         const int64_t *run_cell_base_dev, int front);
size_t adjoint_lds_bytes(int dim, int order, const int P[3]);
hipError_t launch_adjoint(const Launch &L, const AdjRun *adj_dev, const AdjRun *adj_host, const Unit *units,
                          int n_units, int32_t *item_start, int64_t max_items, int chunk, int dim, int order,
                          int64_t total_cells, const int64_t *run_base, size_t lds, hipStream_t s);
hipError_t radix_sort_pairs(void *temp, size_t *temp_bytes, const int32_t *keys_in, int32_t *keys_out,
                            const int32_t *vals_in, int32_t *vals_out, int64_t n, int bits,
                            hipStream_t s);

}  // namespace psc
