// psc_adjoint.hip -- hand-written reverse of one time step (2-d and 3-d runs).
//
// The paper has no adjoint; this is the exact transpose of the discrete step
// of fig. psc_new as implemented by the forward kernels:
//   B1 = B  - dt/2 curl^+ E                    (B half step)
//   particles: gather E, B1 -> Boris -> move -> Esirkepov J
//   B2 = B1 - dt/2 curl^+ E                    (B half step)
//   E' = E  + dt (curl^- B2 - J)               (E full step)
// Given the adjoints (lE', lB2, lx', lu') of the step's output it returns
// (lE, lB, lx, lu) of its input.  On a periodic Yee grid curl^+ and curl^- are
// transposes of each other.  The particle part recomputes the forward of every
// particle and back-propagates through the deposit, the move, the Boris
// rotation and the interpolation; the transpose of the interpolation scatters
// into LDS tiles that are added into the grid adjoints like the current fold.
#include "psc_device.h"

namespace psc {

// derivatives of node_weights / half_weights with respect to the offset
template <int ORDER>
__device__ __forceinline__ void node_dweights(float o, float dw[ORDER + 1]) {
    if constexpr (ORDER == 1) {
        dw[0] = -1.0f;
        dw[1] = 1.0f;
    } else {
        const float d = o - (o >= 0.5f ? 1.0f : 0.0f);
        dw[0] = -(0.5f - d);
        dw[1] = -2.0f * d;
        dw[2] = 0.5f + d;
    }
}

template <int ORDER>
__device__ __forceinline__ void half_dweights(float o, float dw[ORDER + 1]) {
    if constexpr (ORDER == 1) {
        dw[0] = -1.0f;
        dw[1] = 1.0f;
    } else {
        const float d = o - 0.5f;
        dw[0] = -(0.5f - d);
        dw[1] = -2.0f * d;
        dw[2] = 0.5f + d;
    }
}

// stencil() with the derivatives of the placed weights
template <int ORDER>
__device__ __forceinline__ int stencil_d(float o0, int s, float o1, float S0[ORDER + 2], float S1[ORDER + 2],
                                        float D0[ORDER + 2], float D1[ORDER + 2]) {
    float w0[ORDER + 1], w1[ORDER + 1], d0[ORDER + 1], d1[ORDER + 1];
    const int b0 = node_weights<ORDER>(o0, w0);
    const int b1 = node_weights<ORDER>(o1, w1) + s;
    node_dweights<ORDER>(o0, d0);
    node_dweights<ORDER>(o1, d1);
    const int base = b0 < b1 ? b0 : b1;
    const bool k0 = b0 != base, k1 = b1 != base;
#pragma unroll
    for (int r = 0; r < ORDER + 2; ++r) {
        S0[r] = k0 ? (r >= 1 ? w0[r - 1] : 0.0f) : (r <= ORDER ? w0[r] : 0.0f);
        S1[r] = k1 ? (r >= 1 ? w1[r - 1] : 0.0f) : (r <= ORDER ? w1[r] : 0.0f);
        D0[r] = k0 ? (r >= 1 ? d0[r - 1] : 0.0f) : (r <= ORDER ? d0[r] : 0.0f);
        D1[r] = k1 ? (r >= 1 ? d1[r - 1] : 0.0f) : (r <= ORDER ? d1[r] : 0.0f);
    }
    return base;
}

// interpolation of one component with its offset derivatives
template <int ORDER>
__device__ __forceinline__ float gather2_d(const float *F, int pitch, int iy, int iz, const float *wy,
                                           const float *dwy, const float *wz, const float *dwz, float &gy,
                                           float &gz) {
    const float *p = F + iz * pitch + iy;
    float s = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
    for (int b = 0; b <= ORDER; ++b) {
        float r = 0.0f, rd = 0.0f;
#pragma unroll
        for (int a = 0; a <= ORDER; ++a) {
            const float f = p[b * pitch + a];
            r = fmaf(wy[a], f, r);
            rd = fmaf(dwy[a], f, rd);
        }
        s = fmaf(wz[b], r, s);
        sy = fmaf(wz[b], rd, sy);
        sz = fmaf(dwz[b], r, sz);
    }
    gy = sy;
    gz = sz;
    return s;
}

// Transposed interpolation through per-cell frames.  Along one dimension a
// particle of a cell touches a fixed window of nodes: order 1 node-centred
// 0..1, order 2 node-centred -1..2 (the first node moves with the offset),
// half-centred -1..1 at both orders.  Each lane writes lam * wy * wz over the
// window of its cell; lanes of one cell are summed with the segmented wave
// scan and only the last lane of each cell adds the frame to LDS.
template <int ORDER, bool HALF>
struct AdjFrame {
    static constexpr int len = HALF ? 3 : (ORDER == 1 ? 2 : 4);
    static constexpr int origin = HALF ? -1 : (ORDER == 1 ? 0 : -1);
};

// the ORDER+1 weights with first node b (relative to the cell) on the window
template <int ORDER, bool HALF>
__device__ __forceinline__ void frame_place(int b, const float *w, float *f) {
    constexpr int n = AdjFrame<ORDER, HALF>::len;
    if constexpr (n == ORDER + 1) {
#pragma unroll
        for (int k = 0; k < n; ++k) f[k] = w[k];
    } else {
        const bool up = b != AdjFrame<ORDER, HALF>::origin;
#pragma unroll
        for (int k = 0; k < n; ++k) f[k] = up ? (k >= 1 ? w[k - 1] : 0.0f) : (k <= ORDER ? w[k] : 0.0f);
    }
}

template <int ORDER, bool HY, bool HZ>
constexpr int frame_size() {
    return AdjFrame<ORDER, HY>::len * AdjFrame<ORDER, HZ>::len;
}

template <int ORDER, bool HY, bool HZ>
__device__ __forceinline__ void frame_put(float *v, float lam, const float *fy, const float *fz) {
    constexpr int ny = AdjFrame<ORDER, HY>::len, nz = AdjFrame<ORDER, HZ>::len;
#pragma unroll
    for (int b = 0; b < nz; ++b) {
        const float lb = lam * fz[b];
#pragma unroll
        for (int a = 0; a < ny; ++a) v[a + ny * b] = lb * fy[a];
    }
}

template <int ORDER, bool HY, bool HZ>
__device__ __forceinline__ void frame_add(double *G, int pitch, int ty, int tz, const float *v) {
    constexpr int ny = AdjFrame<ORDER, HY>::len, nz = AdjFrame<ORDER, HZ>::len;
    double *p = G + (tz + AdjFrame<ORDER, HZ>::origin) * pitch + ty + AdjFrame<ORDER, HY>::origin;
#pragma unroll
    for (int b = 0; b < nz; ++b)
#pragma unroll
        for (int a = 0; a < ny; ++a) lds_add(p + b * pitch + a, v[a + ny * b]);
}

__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 add3(float3 a, float3 b) { return make_float3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 scale3(float3 a, float s) { return make_float3(a.x * s, a.y * s, a.z * s); }

// ---------------------------------------------------------------------------
// field parts of the reverse step
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_run_a(const int64_t *base, int n_runs, int64_t c) {
    int lo = 0, hi = n_runs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= c) lo = mid; else hi = mid;
    }
    return lo;
}

// Call f(R, A, idx) for cell c of the flat cell space; R and A are uniform
// over the workgroup (scalar loads) when all its cells lie in one run.
template <typename F>
__device__ __forceinline__ void with_run_adj(const RunDev *runs, const AdjRun *adj, const int64_t *base, int n_runs,
                                             int64_t total, F &&f) {
    const int64_t c0 = (int64_t)blockIdx.x * blockDim.x, c = c0 + threadIdx.x;
    const int64_t c1 = (c0 + blockDim.x < total ? c0 + blockDim.x : total) - 1;
    const int rb = find_run_a(base, n_runs, c0);
    const bool one = base[rb + 1] > c1;
    if (c >= total) return;
    if (one) {
        f(runs[rb], adj[rb], c - base[rb]);
    } else {
        const int r = find_run_a(base, n_runs, c);
        f(runs[r], adj[r], c - base[r]);
    }
}

// grid coordinates of cell idx of a run (32-bit: fewer than 2^31 cells)
__device__ __forceinline__ void adj_grid_coords(const RunDev &R, int64_t idx, int g[3]) {
    const uint32_t id = (uint32_t)idx, nx = (uint32_t)R.n[0], ny = (uint32_t)R.n[1];
    const uint32_t q = R.dim == 3 ? id / nx : id;
    g[0] = (int)(id - q * nx);
    const uint32_t k = q / ny;
    g[1] = (int)(q - k * ny);
    g[2] = (int)k;
}

// op 0: LJ = -dt lE ; lB += dt curl^+ lE
// op 1: lE -= dt/2 curl^- lB ; B1 = B - dt/2 curl^+ E
// op 2: lE -= dt/2 curl^- lB
// Every load of a cell before its stores; in 2-d the x neighbours are the
// cell itself and ix is zero, so their terms are zero.
__device__ __forceinline__ void adj_field_cell(const RunDev &R, const AdjRun &A, int64_t idx, int op) {
    const int nx = R.n[0], ny = R.n[1], nz = R.n[2];
    int g[3];
    adj_grid_coords(R, idx, g);
    const int i = g[0], j = g[1], k = g[2];
    const int64_t nc = R.ncell;
    const float ix = R.dim == 3 ? R.inv_dx[0] : 0.0f, iy = R.inv_dx[1], iz = R.inv_dx[2];
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const int64_t ip = i + 1 < nx ? idx + 1 : idx - (nx - 1);
    const int64_t jp = j + 1 < ny ? idx + sy : idx - (int64_t)(ny - 1) * sy;
    const int64_t kp = k + 1 < nz ? idx + sz : idx - (int64_t)(nz - 1) * sz;
    const int64_t im = i > 0 ? idx - 1 : idx + (nx - 1);
    const int64_t jm = j > 0 ? idx - sy : idx + (int64_t)(ny - 1) * sy;
    const int64_t km = k > 0 ? idx - sz : idx + (int64_t)(nz - 1) * sz;
    auto curl_plus = [&](const gptr<const float> F, float &cx, float &cy, float &cz) {
        const float fx = F[idx], fy = F[nc + idx], fz = F[2 * nc + idx];
        const float fz_j = F[2 * nc + jp], fy_k = F[nc + kp], fx_k = F[kp], fz_i = F[2 * nc + ip], fy_i = F[nc + ip],
                    fx_j = F[jp];
        cx = (fz_j - fz) * iy - (fy_k - fy) * iz;
        cy = (fx_k - fx) * iz - (fz_i - fz) * ix;
        cz = (fy_i - fy) * ix - (fx_j - fx) * iy;
    };
    auto curl_minus = [&](const gptr<const float> F, float &cx, float &cy, float &cz) {
        const float fx = F[idx], fy = F[nc + idx], fz = F[2 * nc + idx];
        const float fz_j = F[2 * nc + jm], fy_k = F[nc + km], fx_k = F[km], fz_i = F[2 * nc + im], fy_i = F[nc + im],
                    fx_j = F[jm];
        cx = (fz - fz_j) * iy - (fy - fy_k) * iz;
        cy = (fx - fx_k) * iz - (fz - fz_i) * ix;
        cz = (fy - fy_i) * ix - (fx - fx_j) * iy;
    };
    const float dt = R.dt;
    float cx, cy, cz;
    if (op == 0) {
        curl_plus(to_global<const float>(A.lE), cx, cy, cz);
        const float e0 = to_global(A.lE)[idx], e1 = to_global(A.lE)[nc + idx], e2 = to_global(A.lE)[2 * nc + idx];
        const float b0 = to_global(A.lB)[idx], b1 = to_global(A.lB)[nc + idx], b2 = to_global(A.lB)[2 * nc + idx];
        to_global(A.LJ)[idx] = -dt * e0;
        to_global(A.LJ)[nc + idx] = -dt * e1;
        to_global(A.LJ)[2 * nc + idx] = -dt * e2;
        to_global(A.lB)[idx] = b0 + dt * cx;
        to_global(A.lB)[nc + idx] = b1 + dt * cy;
        to_global(A.lB)[2 * nc + idx] = b2 + dt * cz;
    } else {
        curl_minus(to_global<const float>(A.lB), cx, cy, cz);
        float ex = 0.0f, ey = 0.0f, ez = 0.0f, bx = 0.0f, by = 0.0f, bz = 0.0f;
        const float e0 = to_global(A.lE)[idx], e1 = to_global(A.lE)[nc + idx], e2 = to_global(A.lE)[2 * nc + idx];
        if (op == 1) {
            curl_plus(to_global(A.E), ex, ey, ez);
            bx = to_global(A.B)[idx];
            by = to_global(A.B)[nc + idx];
            bz = to_global(A.B)[2 * nc + idx];
        }
        to_global(A.lE)[idx] = e0 - 0.5f * dt * cx;
        to_global(A.lE)[nc + idx] = e1 - 0.5f * dt * cy;
        to_global(A.lE)[2 * nc + idx] = e2 - 0.5f * dt * cz;
        if (op == 1) {
            to_global(A.B1)[idx] = bx - 0.5f * dt * ex;
            to_global(A.B1)[nc + idx] = by - 0.5f * dt * ey;
            to_global(A.B1)[2 * nc + idx] = bz - 0.5f * dt * ez;
        }
    }
}

__global__ void __launch_bounds__(256) k_adj_fields(const RunDev *__restrict__ runs, const AdjRun *__restrict__ adj,
                                                    int n_runs, const int64_t *__restrict__ run_base, int64_t total,
                                                    int op) {
    with_run_adj(runs, adj, run_base, n_runs, total,
                 [&](const RunDev &R, const AdjRun &A, int64_t idx) { adj_field_cell(R, A, idx, op); });
}

// move the incoming particle adjoints (next step's sorted order) to this
// step's slots: slot perm[j] holds the particle that the sort put at j
__global__ void k_adj_unpermute(const AdjRun *__restrict__ adj, int r, int s, int dim) {
    const AdjSpecies &S = adj[r].sp[s];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= S.n) return;
    const int64_t p = to_global(S.perm)[j];
    if (p < 0 || p >= S.n) return;
    const gptr<float> soff = to_global(S.soff), su = to_global(S.su);
    const gptr<const float> loff = to_global<const float>(S.loff), lu = to_global<const float>(S.lu);
    for (int d = 0; d < dim; ++d) soff[d * S.n + p] = loff[d * S.n + j];
    for (int c = 0; c < 3; ++c) su[c * S.n + p] = lu[c * S.n + j];
}

// work items of the particle adjoint per unit (one thread per unit); the
// prefix over units follows with launch_items_scan
__global__ void __launch_bounds__(256) k_adj_unit_items(const RunDev *__restrict__ runs,
                                                        const AdjRun *__restrict__ adj,
                                                        const Unit *__restrict__ units, int n_units, int chunk,
                                                        int32_t *__restrict__ item_start) {
    const int u = blockIdx.x * 256 + threadIdx.x;
    if (u >= n_units) return;
    const Unit U = units[u];
    const RunDev &R = runs[U.run];
    int pc[3];
    patch_coords(R, U.patch, pc);
    const int64_t kb = patch_key_base(R, pc[0], pc[1], pc[2]);
    const int64_t ke = kb + (int64_t)patch_ext(R, 0, pc[0]) * patch_ext(R, 1, pc[1]) * patch_ext(R, 2, pc[2]);
    const int32_t *cs = adj[U.run].sp[U.species].cs;
    item_start[u] = (cs[ke] - cs[kb] + chunk - 1) / chunk;
}

// ---------------------------------------------------------------------------
// the particle adjoint kernel (2-d)
// ---------------------------------------------------------------------------
// LDS layout (offsets in floats, regions on 16 bytes): the field tile of E and
// B1 (6 components, field-tile geometry), the tile of the current adjoint LJ
// (3 components, current-tile geometry), the transposed-interpolation tile
// (6 components in double, field-tile geometry).
struct AdjLds {
    int lj, gt, total;
};
__host__ __device__ inline AdjLds adj_lds_layout(int fcells, int jcells) {
    AdjLds L{};
    L.lj = (6 * fcells + 3) & ~3;
    L.gt = (L.lj + 3 * jcells + 3) & ~3;
    L.total = L.gt + 12 * fcells;
    return L;
}

template <int ORDER>
__global__ void __launch_bounds__(kAdjBlock) k_adj_particles(const RunDev *__restrict__ runs,
                                                             const AdjRun *__restrict__ adj,
                                                             const Unit *__restrict__ units,
                                                             const int32_t *__restrict__ item_start, int n_units,
                                                             int chunk) {
    extern __shared__ __align__(16) float lds[];   // 16-byte aligned: holds doubles
    constexpr int L = ORDER + 2;
    constexpr int FLO = 1, FHI = ORDER;
    constexpr int JLO = ORDER, JHI = ORDER + 1;
    constexpr int NT = kAdjBlock;

    const int nb = gridDim.x;
    const int item = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
    const int total = item_start[n_units];
    if (item >= total) return;
    int lo = 0, hi = n_units;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (item_start[mid] <= item) lo = mid; else hi = mid;
    }
    const Unit U = units[lo];
    const RunDev &R = runs[U.run];
    const AdjRun &A = adj[U.run];
    const SpeciesDev &S = R.sp[U.species];
    const AdjSpecies &AS = A.sp[U.species];

    int pc[3];
    patch_coords(R, U.patch, pc);
    const int hy = patch_ext(R, 1, pc[1]), hz = patch_ext(R, 2, pc[2]);
    const int oy = pc[1] * R.P[1], oz = pc[2] * R.P[2];
    const int64_t kb = patch_key_base(R, 0, pc[1], pc[2]);
    const int32_t pbeg = to_global(AS.cs)[kb], pend = to_global(AS.cs)[kb + (int64_t)hy * hz];
    const int32_t beg = pbeg + (item - item_start[lo]) * chunk;
    const int32_t end = min(beg + chunk, pend);

    const int fy = R.P[1] + FLO + FHI, fz = R.P[2] + FLO + FHI;
    const int fcells = fy * fz;
    const int jy = R.P[1] + JLO + JHI, jz = R.P[2] + JLO + JHI;
    const int jcells = jy * jz;
    const AdjLds LL = adj_lds_layout(fcells, jcells);
    float *ftile = lds;               // E, B1
    float *ljt = lds + LL.lj;         // LJ
    // transposed interpolation of E, B1, accumulated in double (the LDS add
    // of doubles runs at the rate of integer atomics, the float one far slower)
    double *gt = reinterpret_cast<double *>(lds + LL.gt);
    const int64_t nc = R.ncell;
    // The chunk's particles are sorted by cell, so they lie in the cell rows
    // between those of its first and last particle; only the tile rows their
    // stencils reach are staged, cleared and flushed.  Field-tile rows:
    // lz + FLO - 1 .. lz + FLO + ORDER; current-tile rows: lz .. lz + 2 ORDER + 1.
    const int pc_cells = hy * hz;
    // buffer slot of the forward particle at sorted slot i
    auto slot_of = [&](int32_t i) -> int64_t {
        if (!AS.rperm) return i;
        const int32_t q = to_global(AS.rperm)[i];
        return (uint32_t)q < (uint32_t)AS.stride ? q : 0;   // a corrupt permutation stays in bounds
    };
    const int lf = imin(imax(to_global(AS.key)[slot_of(beg)] - (int32_t)kb, 0), pc_cells - 1);
    const int ll = imin(imax(to_global(AS.key)[slot_of(end - 1)] - (int32_t)kb, 0), pc_cells - 1);
    const int zf = lf / hy, zl = ll / hy;
    const int fr0 = zf + FLO - 1, fr1 = imin(zl + FLO + ORDER, fz - 1);   // field-tile rows [fr0, fr1]
    const int jr0 = zf, jr1 = imin(zl + 2 * ORDER + 1, jz - 1);           // current-tile rows [jr0, jr1]
    {
        const float inv_fy = 1.0f / fy;
        const int n_f = (fr1 - fr0 + 1) * fy;
        for (int q = threadIdx.x; q < n_f; q += NT) {
            int ty;
            const int tz = fr0 + divmod_small(q, fy, inv_fy, ty);
            const int t = tz * fy + ty;
            const int64_t g = wrap(oy + ty - FLO, R.n[1]) + (int64_t)R.n[1] * wrap(oz + tz - FLO, R.n[2]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                ftile[c * fcells + t] = to_global(A.E)[c * nc + g];
                ftile[(3 + c) * fcells + t] = to_global(A.B1)[c * nc + g];
                gt[c * fcells + t] = 0.0;
                gt[(3 + c) * fcells + t] = 0.0;
            }
        }
        const float inv_jy = 1.0f / jy;
        const int n_j = (jr1 - jr0 + 1) * jy;
        for (int q = threadIdx.x; q < n_j; q += NT) {
            int ty;
            const int tz = jr0 + divmod_small(q, jy, inv_jy, ty);
            const int t = tz * jy + ty;
            const int64_t g = wrap(oy + ty - JLO, R.n[1]) + (int64_t)R.n[1] * wrap(oz + tz - JLO, R.n[2]);
#pragma unroll
            for (int c = 0; c < 3; ++c) ljt[c * jcells + t] = to_global(A.LJ)[c * nc + g];
        }
    }
    __syncthreads();

    const int64_t n = AS.n;
    const float h = S.qdt_2m, qw = S.qw, dt = R.dt;
    const float cfy = dt * R.inv_dx[1], cfz = dt * R.inv_dx[2];
    const float jfy = -qw * R.dx[1] / dt, jfz = -qw * R.dx[2] / dt;
    const float inv_hy = 1.0f / hy;

    // every round gives each thread one particle; the rounds are uniform over
    // the workgroup so that the wave scans see all lanes.  A round's buffer
    // slot is read through the permutation a round ahead, and the round's
    // loads (state and incoming adjoints) are issued together at its start
    auto round_slot = [&](int32_t b0) {
        const int32_t ii = b0 + (int32_t)threadIdx.x;
        return slot_of(ii < end ? ii : beg);
    };
    int64_t p_q = round_slot(beg);
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);   // the loop's waits then count only its own operations
    for (int32_t base = beg; base < end; base += NT) {
        const bool valid = base + (int32_t)threadIdx.x < end;
        const int32_t i = valid ? base + (int32_t)threadIdx.x : beg;
        const int64_t q = p_q;
        const int64_t st = AS.stride;
        const int32_t key = to_global(AS.key)[q];
        int local = key - (int32_t)kb;
        if (local < 0 || local >= hy * hz) local = 0;
        int ly;
        const int lz = divmod_small(local, hy, inv_hy, ly);
        const float oyv = to_global(AS.off)[q], ozv = to_global(AS.off)[st + q];
        const float3 u0 = make_float3(to_global(AS.u)[q], to_global(AS.u)[st + q], to_global(AS.u)[2 * st + q]);
        const float lx1_0 = to_global(AS.soff)[i], lx1_1 = to_global(AS.soff)[n + i];   // adjoint of the moved offsets
        const float3 lun0 = make_float3(to_global(AS.su)[i], to_global(AS.su)[n + i], to_global(AS.su)[2 * n + i]);
        p_q = round_slot(base + NT);

        // ---- forward recompute: interpolation (with offset derivatives) ----
        float wny[ORDER + 1], why[ORDER + 1], wnz[ORDER + 1], whz[ORDER + 1];
        float dny[ORDER + 1], dhy[ORDER + 1], dnz[ORDER + 1], dhz[ORDER + 1];
        const int bny = node_weights<ORDER>(oyv, wny), bhy = half_weights<ORDER>(oyv, why);
        const int bnz = node_weights<ORDER>(ozv, wnz), bhz = half_weights<ORDER>(ozv, whz);
        node_dweights<ORDER>(oyv, dny);
        half_dweights<ORDER>(oyv, dhy);
        node_dweights<ORDER>(ozv, dnz);
        half_dweights<ORDER>(ozv, dhz);
        const int ty = ly + FLO, tz = lz + FLO;
        // component c: (y index, z index, y weights, z weights)
        const int cy_[6] = {ty + bny, ty + bhy, ty + bny, ty + bhy, ty + bny, ty + bhy};
        const int cz_[6] = {tz + bnz, tz + bnz, tz + bhz, tz + bhz, tz + bhz, tz + bnz};
        float F[6], Gy[6], Gz[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const bool hyc = c == 1 || c == 3 || c == 5;
            const bool hzc = c == 2 || c == 3 || c == 4;
            F[c] = gather2_d<ORDER>(ftile + c * fcells, fy, cy_[c], cz_[c], hyc ? why : wny, hyc ? dhy : dny,
                                    hzc ? whz : wnz, hzc ? dhz : dnz, Gy[c], Gz[c]);
        }
        const float3 Ep = make_float3(F[0], F[1], F[2]);
        const float3 Bp = make_float3(F[3], F[4], F[5]);

        // ---- Boris with intermediates ---------------------------------------
        const float3 um = add3(u0, scale3(Ep, h));
        const float igm = rsqrt_ge1(1.0f + dot3(um, um));
        const float3 t = scale3(Bp, h * igm);
        const float t2 = dot3(t, t);
        const float f = boris_factor(t2);
        const float3 s = scale3(t, f);
        const float3 up = add3(um, cross3(um, t));
        const float3 uq = add3(um, cross3(up, s));
        const float3 un = add3(uq, scale3(Ep, h));
        const float ig = rsqrt_ge1(1.0f + dot3(un, un));

        // ---- move -------------------------------------------------------------
        int sh[2];
        float o1[2];
        const float o0[2] = {oyv, ozv};
        const float cf[2] = {cfy, cfz};
        const float uu[2] = {un.y, un.z};
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            float disp = cf[d] * uu[d] * ig;
            if (!(fabsf(disp) < 0.99f)) disp = 0.0f;
            const float x1 = o0[d] + disp;
            int sd = (int)floorf(x1);
            float od = x1 - (float)sd;
            if (od >= 1.0f) { od -= 1.0f; sd += 1; }
            sh[d] = sd;
            o1[d] = od;
        }

        // ---- reverse ----------------------------------------------------------
        float lx1[2] = {lx1_0, lx1_1};
        float3 lun = lun0;
        float lo0[2] = {0.0f, 0.0f};
        float lig = 0.0f;

        // deposit: J values on the stencil, adjoint read from the LJ tile
        {
            float S0y[L], S1y[L], S0z[L], S1z[L], D0y[L], D1y[L], D0z[L], D1z[L];
            const int by = stencil_d<ORDER>(oyv, sh[0], o1[0], S0y, S1y, D0y, D1y);
            const int bz = stencil_d<ORDER>(ozv, sh[1], o1[1], S0z, S1z, D0z, D1z);
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
            const float vx = un.x * ig;
            const float fxv = qw * vx;
            float gCy[L], gCz[L], gAy[L], gAz[L], gDy[L], gDz[L];
#pragma unroll
            for (int r = 0; r < L; ++r) gCy[r] = gCz[r] = gAy[r] = gAz[r] = gDy[r] = gDz[r] = 0.0f;
            float gfxv = 0.0f;
            const float *lj = ljt + (lz + bz + JLO) * jy + (ly + by + JLO);
#pragma unroll
            for (int b = 0; b < L; ++b) {
#pragma unroll
                for (int a = 0; a < L; ++a) {
                    const int q = b * jy + a;
                    const float ljx = lj[q], ljy = lj[jcells + q], ljz = lj[2 * jcells + q];
                    if (a < L - 1) {   // J_y(a, b) = jfy Cy[a] Az[b]
                        gCy[a] += jfy * ljy * Az[b];
                        gAz[b] += jfy * ljy * Cy[a];
                    }
                    if (b < L - 1) {   // J_z(a, b) = jfz Ay[a] Cz[b]
                        gAy[a] += jfz * ljz * Cz[b];
                        gCz[b] += jfz * ljz * Ay[a];
                    }
                    // J_x(a, b) = fxv (Ay Az + DSy DSz / 12)
                    gAy[a] += fxv * ljx * Az[b];
                    gAz[b] += fxv * ljx * Ay[a];
                    gDy[a] += fxv * ljx * DSz[b] * (1.0f / 12.0f);
                    gDz[b] += fxv * ljx * DSy[a] * (1.0f / 12.0f);
                    gfxv += ljx * fmaf(DSy[a] * DSz[b], 1.0f / 12.0f, Ay[a] * Az[b]);
                }
            }
            // cumulative sums: C[r] = sum_{r' <= r} DS[r'], used for r < L-1
            float accy = 0.0f, accz = 0.0f;
#pragma unroll
            for (int r = L - 1; r >= 0; --r) {
                accy += r < L - 1 ? gCy[r] : 0.0f;
                accz += r < L - 1 ? gCz[r] : 0.0f;
                gDy[r] += accy;
                gDz[r] += accz;
            }
            // A = S0 + DS/2, DS = S1 - S0
            float l1y = 0.0f, l1z = 0.0f;
#pragma unroll
            for (int r = 0; r < L; ++r) {
                const float dsy = gDy[r] + 0.5f * gAy[r], dsz = gDz[r] + 0.5f * gAz[r];
                lo0[0] += (gAy[r] - dsy) * D0y[r];
                lo0[1] += (gAz[r] - dsz) * D0z[r];
                l1y += dsy * D1y[r];
                l1z += dsz * D1z[r];
            }
            lx1[0] += l1y;
            lx1[1] += l1z;
            // fxv = qw un.x ig
            lun.x += qw * ig * gfxv;
            lig += qw * un.x * gfxv;
        }
        // move: x1 = o0 + cf un ig
        lo0[0] += lx1[0];
        lo0[1] += lx1[1];
        lun.y += cfy * ig * lx1[0];
        lun.z += cfz * ig * lx1[1];
        lig += cfy * un.y * lx1[0] + cfz * un.z * lx1[1];
        lun = add3(lun, scale3(un, -ig * ig * ig * lig));

        // Boris reverse
        float3 lE = scale3(lun, h);
        const float3 luq = lun;
        float3 lum = luq;
        const float3 lup = cross3(s, luq);
        const float3 ls = cross3(luq, up);
        lum = add3(lum, add3(lup, cross3(t, lup)));
        float3 lt = cross3(lup, um);
        // s = f t with f = 2 / (1 + |t|^2), df/dt = -f^2 t
        lt = add3(lt, add3(scale3(ls, f), scale3(t, -f * f * dot3(ls, t))));
        const float3 lB = scale3(lt, h * igm);
        const float ligm = h * dot3(Bp, lt);
        lum = add3(lum, scale3(um, -igm * igm * igm * ligm));
        lE = add3(lE, scale3(lum, h));
        const float3 lu0 = lum;

        // interpolation reverse: offsets, then the transposed interpolation
        // through per-cell frames (lanes past the end add zeros in a segment
        // of their own)
        const float lF[6] = {lE.x, lE.y, lE.z, lB.x, lB.y, lB.z};
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            lo0[0] += lF[c] * Gy[c];
            lo0[1] += lF[c] * Gz[c];
        }
        if (valid) {
            to_global(AS.loff)[i] = lo0[0];
            to_global(AS.loff)[n + i] = lo0[1];
            to_global(AS.lu)[i] = lu0.x;
            to_global(AS.lu)[n + i] = lu0.y;
            to_global(AS.lu)[2 * n + i] = lu0.z;
        }
        float fny[AdjFrame<ORDER, false>::len], fhy[AdjFrame<ORDER, true>::len];
        float fnz[AdjFrame<ORDER, false>::len], fhz[AdjFrame<ORDER, true>::len];
        frame_place<ORDER, false>(bny, wny, fny);
        frame_place<ORDER, true>(bhy, why, fhy);
        frame_place<ORDER, false>(bnz, wnz, fnz);
        frame_place<ORDER, true>(bhz, whz, fhz);
        const float vm = valid ? 1.0f : 0.0f;
        const RowScan rs = row_scan_setup<64>(valid ? local : -1);
        const bool add = rs.tail && valid;
        {   // E: (node, node), (half, node), (node, half)
            constexpr int n0 = frame_size<ORDER, false, false>(), n1 = frame_size<ORDER, true, false>();
            constexpr int n2 = frame_size<ORDER, false, true>();
            constexpr int NV = (n0 + n1 + n2 + 3) & ~3;
            float v[NV];
#pragma unroll
            for (int k = n0 + n1 + n2; k < NV; ++k) v[k] = 0.0f;
            frame_put<ORDER, false, false>(v, vm * lF[0], fny, fnz);
            frame_put<ORDER, true, false>(v + n0, vm * lF[1], fhy, fnz);
            frame_put<ORDER, false, true>(v + n0 + n1, vm * lF[2], fny, fhz);
            row_scan<64>(v, rs);
            if (add) {
                frame_add<ORDER, false, false>(gt, fy, ty, tz, v);
                frame_add<ORDER, true, false>(gt + fcells, fy, ty, tz, v + n0);
                frame_add<ORDER, false, true>(gt + 2 * fcells, fy, ty, tz, v + n0 + n1);
            }
        }
        {   // B: (half, half), (node, half), (half, node)
            constexpr int n0 = frame_size<ORDER, true, true>(), n1 = frame_size<ORDER, false, true>();
            constexpr int n2 = frame_size<ORDER, true, false>();
            constexpr int NV = (n0 + n1 + n2 + 3) & ~3;
            float v[NV];
#pragma unroll
            for (int k = n0 + n1 + n2; k < NV; ++k) v[k] = 0.0f;
            frame_put<ORDER, true, true>(v, vm * lF[3], fhy, fhz);
            frame_put<ORDER, false, true>(v + n0, vm * lF[4], fny, fhz);
            frame_put<ORDER, true, false>(v + n0 + n1, vm * lF[5], fhy, fnz);
            row_scan<64>(v, rs);
            if (add) {
                frame_add<ORDER, true, true>(gt + 3 * fcells, fy, ty, tz, v);
                frame_add<ORDER, false, true>(gt + 4 * fcells, fy, ty, tz, v + n0);
                frame_add<ORDER, true, false>(gt + 5 * fcells, fy, ty, tz, v + n0 + n1);
            }
        }
    }
    __syncthreads();
    const gptr<float> gp = to_global(A.gtile + (int64_t)U.patch * 6 * fcells);
    const int n_f = (fr1 - fr0 + 1) * fy;
    for (int q = threadIdx.x; q < 6 * n_f; q += NT) {
        const int c = q / n_f, r = q - c * n_f;
        const int t2 = c * fcells + fr0 * fy + r;
        const double v = gt[t2];
        if (v != 0.0) atomicAdd((float *)(gp + t2), (float)v);
    }
}

// interpolation of one component in 3-d with its offset derivatives (g: d/dx, d/dy, d/dz)
template <int ORDER>
__device__ __forceinline__ float gather3_d(const float *F, int px, int pxy, int ix, int iy, int iz, const float *wx,
                                           const float *dwx, const float *wy, const float *dwy, const float *wz,
                                           const float *dwz, float g[3]) {
    const float *p = F + iz * pxy + iy * px + ix;
    float s = 0.0f, sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
    for (int c = 0; c <= ORDER; ++c) {
        float t = 0.0f, tx = 0.0f, ty = 0.0f;
#pragma unroll
        for (int b = 0; b <= ORDER; ++b) {
            float r = 0.0f, rx = 0.0f;
#pragma unroll
            for (int a = 0; a <= ORDER; ++a) {
                const float f = p[c * pxy + b * px + a];
                r = fmaf(wx[a], f, r);
                rx = fmaf(dwx[a], f, rx);
            }
            t = fmaf(wy[b], r, t);
            tx = fmaf(wy[b], rx, tx);
            ty = fmaf(dwy[b], r, ty);
        }
        s = fmaf(wz[c], t, s);
        sx = fmaf(wz[c], tx, sx);
        sy = fmaf(wz[c], ty, sy);
        sz = fmaf(dwz[c], t, sz);
    }
    g[0] = sx;
    g[1] = sy;
    g[2] = sz;
    return s;
}

// Transposed interpolation of one component in 3-d through a per-cell frame:
// each lane forms lam * wx * wy * wz over the window of its cell (the
// AdjFrame windows per dimension), the lanes of one cell are summed with the
// segmented wave scan, and the last lane of each cell adds the frame to the
// double LDS tile.  Every lane of the wave must call it.
template <int ORDER, bool HX, bool HY, bool HZ>
__device__ __forceinline__ void frame3_scan_add(double *G, int px, int pxy, int tx, int ty, int tz, float lam,
                                                const float *wx, const float *wy, const float *wz,
                                                const RowScan &rs, bool add) {
    constexpr int nx = AdjFrame<ORDER, HX>::len, ny = AdjFrame<ORDER, HY>::len, nz = AdjFrame<ORDER, HZ>::len;
    constexpr int N = nx * ny * nz, NV = (N + 3) & ~3;
    float v[NV];
#pragma unroll
    for (int k = 0; k < nz; ++k)
#pragma unroll
        for (int b = 0; b < ny; ++b) {
            const float lyz = lam * wy[b] * wz[k];
#pragma unroll
            for (int a = 0; a < nx; ++a) v[(k * ny + b) * nx + a] = lyz * wx[a];
        }
#pragma unroll
    for (int k = N; k < NV; ++k) v[k] = 0.0f;
    row_scan<64>(v, rs);
    if (add) {
        double *p = G + (tz + AdjFrame<ORDER, HZ>::origin) * pxy + (ty + AdjFrame<ORDER, HY>::origin) * px + tx +
                    AdjFrame<ORDER, HX>::origin;
#pragma unroll
        for (int k = 0; k < nz; ++k)
#pragma unroll
            for (int b = 0; b < ny; ++b)
#pragma unroll
                for (int a = 0; a < nx; ++a) lds_add(p + k * pxy + b * px + a, v[(k * ny + b) * nx + a]);
    }
}

// ---------------------------------------------------------------------------
// the particle adjoint kernel (3-d)
// ---------------------------------------------------------------------------
// The same reverse as the 2-d kernel with the third dimension: the forward of
// every particle is recomputed (gather with weight derivatives, Boris, move),
// then reversed through the 3-d Esirkepov deposit (J_x(a; b, c) = jfx C_x(a)
// (A_y(b) A_z(c) + DS_y(b) DS_z(c) / 12) and its two rotations, A = S0 + DS/2,
// C the running sum of DS = S1 - S0), the move, the Boris rotation and the
// interpolation.  The transposed interpolation goes through per-cell frames
// and the segmented wave scan (as in 2-d; at order 2, whose frames would not
// fit the registers, by per-lane atomics) into a double LDS tile per work
// item, added at the end straight into lE and lB with the tile's halo
// wrapped onto the neighbouring cells (float atomics: the summation order of
// a cell's contributions varies between runs).
template <int ORDER>
__global__ void __launch_bounds__(kAdjBlock) k_adj_particles3(const RunDev *__restrict__ runs,
                                                              const AdjRun *__restrict__ adj,
                                                              const Unit *__restrict__ units,
                                                              const int32_t *__restrict__ item_start, int n_units,
                                                              int chunk) {
    extern __shared__ __align__(16) float lds[];   // 16-byte aligned: holds doubles
    constexpr int L = ORDER + 2;
    constexpr int FLO = 1, FHI = ORDER;
    constexpr int JLO = ORDER, JHI = ORDER + 1;
    constexpr int NT = kAdjBlock;
    // half-grid flags (x, y, z) of Ex, Ey, Ez, Bx, By, Bz
    constexpr bool HS[6][3] = {{true, false, false}, {false, true, false}, {false, false, true},
                               {false, true, true},  {true, false, true},  {true, true, false}};

    const int nb = gridDim.x;
    const int item = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
    const int total = item_start[n_units];
    if (item >= total) return;
    int lo = 0, hi = n_units;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (item_start[mid] <= item) lo = mid; else hi = mid;
    }
    const Unit U = units[lo];
    const RunDev &R = runs[U.run];
    const AdjRun &A = adj[U.run];
    const SpeciesDev &S = R.sp[U.species];
    const AdjSpecies &AS = A.sp[U.species];

    int pc[3];
    patch_coords(R, U.patch, pc);
    const int hx = patch_ext(R, 0, pc[0]), hy = patch_ext(R, 1, pc[1]), hz = patch_ext(R, 2, pc[2]);
    const int ox = pc[0] * R.P[0], oy = pc[1] * R.P[1], oz = pc[2] * R.P[2];
    const int64_t kb = patch_key_base(R, pc[0], pc[1], pc[2]);
    const int pcells = hx * hy * hz;
    // offsets outside [0, n] (a corrupt input) must not send the item outside the buffers
    const int32_t n32 = (int32_t)AS.n;
    const int32_t pend = min(max(to_global(AS.cs)[kb + pcells], 0), n32), pbeg = min(max(to_global(AS.cs)[kb], 0), pend);
    const int32_t beg = pbeg + (item - item_start[lo]) * chunk;
    const int32_t end = min(beg + chunk, pend);

    const int fx = R.P[0] + FLO + FHI, fy = R.P[1] + FLO + FHI, fz = R.P[2] + FLO + FHI;
    const int fxy = fx * fy, fcells = fxy * fz;
    const int jx = R.P[0] + JLO + JHI, jy = R.P[1] + JLO + JHI, jz = R.P[2] + JLO + JHI;
    const int jxy = jx * jy, jcells = jxy * jz;
    const AdjLds LL = adj_lds_layout(fcells, jcells);
    float *ftile = lds;               // E, B1
    float *ljt = lds + LL.lj;         // LJ
    double *gt = reinterpret_cast<double *>(lds + LL.gt);
    const int64_t nc = R.ncell;
    auto tile_cell = [&](int q, int px, int pxy, int lo_, int64_t &g) {
        const int tz = q / pxy, r = q - tz * pxy, ty = r / px, tx = r - ty * px;
        g = wrap(ox + tx - lo_, R.n[0]) +
            (int64_t)R.n[0] * (wrap(oy + ty - lo_, R.n[1]) + (int64_t)R.n[1] * wrap(oz + tz - lo_, R.n[2]));
    };
    for (int q = threadIdx.x; q < fcells; q += NT) {
        int64_t g;
        tile_cell(q, fx, fxy, FLO, g);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ftile[c * fcells + q] = to_global(A.E)[c * nc + g];
            ftile[(3 + c) * fcells + q] = to_global(A.B1)[c * nc + g];
            gt[c * fcells + q] = 0.0;
            gt[(3 + c) * fcells + q] = 0.0;
        }
    }
    for (int q = threadIdx.x; q < jcells; q += NT) {
        int64_t g;
        tile_cell(q, jx, jxy, JLO, g);
#pragma unroll
        for (int c = 0; c < 3; ++c) ljt[c * jcells + q] = to_global(A.LJ)[c * nc + g];
    }
    __syncthreads();

    const int64_t n = AS.n, st = AS.stride;
    const float h = S.qdt_2m, qw = S.qw, dt = R.dt;
    const float cf[3] = {dt * R.inv_dx[0], dt * R.inv_dx[1], dt * R.inv_dx[2]};
    const float jf[3] = {-qw * R.dx[0] / dt, -qw * R.dx[1] / dt, -qw * R.dx[2] / dt};
    auto slot_of = [&](int32_t i) -> int64_t {
        if (!AS.rperm) return i;
        const int32_t q = to_global(AS.rperm)[i];
        return (uint32_t)q < (uint32_t)AS.stride ? q : 0;   // a corrupt permutation stays in bounds
    };

    // every round gives each thread one particle; at order 1 the rounds are
    // uniform over the workgroup so that the wave scans see all lanes (lanes
    // past the end recompute the item's first particle and add zeros in a
    // segment of their own)
    // (a round's buffer slot is read through the permutation a round ahead,
    // and its loads are issued together at its start)
    auto round_slot = [&](int32_t b0) {
        const int32_t ii = b0 + (int32_t)threadIdx.x;
        return slot_of(ii < end ? ii : beg);
    };
    int64_t p_q = round_slot(beg);
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);   // the loop's waits then count only its own operations
    for (int32_t base = beg; base < end; base += NT) {
        const bool valid = base + (int32_t)threadIdx.x < end;
        const int64_t q = p_q;
        p_q = round_slot(base + NT);
        if constexpr (ORDER != 1) {
            if (!valid) continue;   // no wave scans at order 2
        }
        const int32_t i = valid ? base + (int32_t)threadIdx.x : beg;
        int local = to_global(AS.key)[q] - (int32_t)kb;
        if (local < 0 || local >= pcells) local = 0;
        const int lz = local / (hx * hy), rr = local - lz * hx * hy, ly = rr / hx, lx = rr - ly * hx;
        const float o0[3] = {to_global(AS.off)[q], to_global(AS.off)[st + q], to_global(AS.off)[2 * st + q]};
        const float3 u0 = make_float3(to_global(AS.u)[q], to_global(AS.u)[st + q], to_global(AS.u)[2 * st + q]);
        const float lx1_0[3] = {to_global(AS.soff)[i], to_global(AS.soff)[n + i], to_global(AS.soff)[2 * n + i]};
        const float lun_0[3] = {to_global(AS.su)[i], to_global(AS.su)[n + i], to_global(AS.su)[2 * n + i]};

        // ---- forward recompute: interpolation (with offset derivatives) ----
        float wn[3][ORDER + 1], wh[3][ORDER + 1], dn[3][ORDER + 1], dh[3][ORDER + 1];
        int bn[3], bh[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            bn[d] = node_weights<ORDER>(o0[d], wn[d]);
            bh[d] = half_weights<ORDER>(o0[d], wh[d]);
            node_dweights<ORDER>(o0[d], dn[d]);
            half_dweights<ORDER>(o0[d], dh[d]);
        }
        float F[6], G[6][3];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const int ix = lx + FLO + (HS[c][0] ? bh[0] : bn[0]);
            const int iy = ly + FLO + (HS[c][1] ? bh[1] : bn[1]);
            const int iz = lz + FLO + (HS[c][2] ? bh[2] : bn[2]);
            F[c] = gather3_d<ORDER>(ftile + c * fcells, fx, fxy, ix, iy, iz, HS[c][0] ? wh[0] : wn[0],
                                    HS[c][0] ? dh[0] : dn[0], HS[c][1] ? wh[1] : wn[1], HS[c][1] ? dh[1] : dn[1],
                                    HS[c][2] ? wh[2] : wn[2], HS[c][2] ? dh[2] : dn[2], G[c]);
        }
        const float3 Ep = make_float3(F[0], F[1], F[2]);
        const float3 Bp = make_float3(F[3], F[4], F[5]);

        // ---- Boris with intermediates ---------------------------------------
        const float3 um = add3(u0, scale3(Ep, h));
        const float igm = rsqrt_ge1(1.0f + dot3(um, um));
        const float3 t = scale3(Bp, h * igm);
        const float t2 = dot3(t, t);
        const float f = boris_factor(t2);
        const float3 sv = scale3(t, f);
        const float3 up = add3(um, cross3(um, t));
        const float3 uq = add3(um, cross3(up, sv));
        const float3 un = add3(uq, scale3(Ep, h));
        const float ig = rsqrt_ge1(1.0f + dot3(un, un));
        const float unv[3] = {un.x, un.y, un.z};

        // ---- move -------------------------------------------------------------
        int sh[3];
        float o1[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            float disp = cf[d] * unv[d] * ig;
            if (!(fabsf(disp) < 0.99f)) disp = 0.0f;
            const float x1 = o0[d] + disp;
            int sd = (int)floorf(x1);
            float od = x1 - (float)sd;
            if (od >= 1.0f) { od -= 1.0f; sd += 1; }
            sh[d] = sd;
            o1[d] = od;
        }

        // ---- reverse ----------------------------------------------------------
        float lx1[3] = {lx1_0[0], lx1_0[1], lx1_0[2]};   // adjoint of the moved offsets
        float lun[3] = {lun_0[0], lun_0[1], lun_0[2]};
        float lo0[3] = {0.0f, 0.0f, 0.0f};
        float lig = 0.0f;

        // deposit: J values on the stencil, adjoint read from the LJ tile
        {
            float S0[3][L], S1[3][L], D0[3][L], D1[3][L];
            int bs[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) bs[d] = stencil_d<ORDER>(o0[d], sh[d], o1[d], S0[d], S1[d], D0[d], D1[d]);
            float DS[3][L], Aw[3][L], C[3][L], gC[3][L], gA[3][L], gD[3][L];
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int r = 0; r < L; ++r) {
                    DS[d][r] = S1[d][r] - S0[d][r];
                    Aw[d][r] = fmaf(0.5f, DS[d][r], S0[d][r]);
                    C[d][r] = r == 0 ? DS[d][0] : C[d][r - 1] + DS[d][r];
                    gC[d][r] = gA[d][r] = gD[d][r] = 0.0f;
                }
            const float *lj = ljt + ((lz + bs[2] + JLO) * jy + (ly + bs[1] + JLO)) * jx + (lx + bs[0] + JLO);
            constexpr float k12 = 1.0f / 12.0f;
#pragma unroll
            for (int c = 0; c < L; ++c)
#pragma unroll
                for (int b = 0; b < L; ++b)
#pragma unroll
                    for (int a = 0; a < L; ++a) {
                        const int idx = (c * jy + b) * jx + a;
                        if (a < L - 1) {   // J_x(a; b, c) = jfx C_x(a) (A_y(b) A_z(c) + DS_y(b) DS_z(c) / 12)
                            const float lam = jf[0] * lj[idx];
                            gC[0][a] += lam * fmaf(DS[1][b] * DS[2][c], k12, Aw[1][b] * Aw[2][c]);
                            const float tt = lam * C[0][a];
                            gA[1][b] += tt * Aw[2][c];
                            gA[2][c] += tt * Aw[1][b];
                            gD[1][b] += tt * DS[2][c] * k12;
                            gD[2][c] += tt * DS[1][b] * k12;
                        }
                        if (b < L - 1) {   // J_y(a; b, c) = jfy C_y(b) (A_x(a) A_z(c) + DS_x(a) DS_z(c) / 12)
                            const float lam = jf[1] * lj[jcells + idx];
                            gC[1][b] += lam * fmaf(DS[0][a] * DS[2][c], k12, Aw[0][a] * Aw[2][c]);
                            const float tt = lam * C[1][b];
                            gA[0][a] += tt * Aw[2][c];
                            gA[2][c] += tt * Aw[0][a];
                            gD[0][a] += tt * DS[2][c] * k12;
                            gD[2][c] += tt * DS[0][a] * k12;
                        }
                        if (c < L - 1) {   // J_z(a, b; c) = jfz C_z(c) (A_x(a) A_y(b) + DS_x(a) DS_y(b) / 12)
                            const float lam = jf[2] * lj[2 * jcells + idx];
                            gC[2][c] += lam * fmaf(DS[0][a] * DS[1][b], k12, Aw[0][a] * Aw[1][b]);
                            const float tt = lam * C[2][c];
                            gA[0][a] += tt * Aw[1][b];
                            gA[1][b] += tt * Aw[0][a];
                            gD[0][a] += tt * DS[1][b] * k12;
                            gD[1][b] += tt * DS[0][a] * k12;
                        }
                    }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                // C(r) = sum_{r' <= r} DS(r'), used for r < L - 1
                float acc = 0.0f;
#pragma unroll
                for (int r = L - 1; r >= 0; --r) {
                    acc += r < L - 1 ? gC[d][r] : 0.0f;
                    gD[d][r] += acc;
                }
                // A = S0 + DS/2, DS = S1 - S0
                float l1 = 0.0f;
#pragma unroll
                for (int r = 0; r < L; ++r) {
                    const float ds = gD[d][r] + 0.5f * gA[d][r];
                    lo0[d] += (gA[d][r] - ds) * D0[d][r];
                    l1 += ds * D1[d][r];
                }
                lx1[d] += l1;
            }
        }
        // move: x1 = o0 + cf un ig
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lo0[d] += lx1[d];
            lun[d] += cf[d] * ig * lx1[d];
            lig += cf[d] * unv[d] * lx1[d];
        }
        float3 lu3 = add3(make_float3(lun[0], lun[1], lun[2]), scale3(un, -ig * ig * ig * lig));

        // Boris reverse
        float3 lE = scale3(lu3, h);
        const float3 luq = lu3;
        float3 lum = luq;
        const float3 lup = cross3(sv, luq);
        const float3 ls = cross3(luq, up);
        lum = add3(lum, add3(lup, cross3(t, lup)));
        float3 lt = cross3(lup, um);
        // s = f t with f = 2 / (1 + |t|^2), df/dt = -f^2 t
        lt = add3(lt, add3(scale3(ls, f), scale3(t, -f * f * dot3(ls, t))));
        const float3 lB = scale3(lt, h * igm);
        const float ligm = h * dot3(Bp, lt);
        lum = add3(lum, scale3(um, -igm * igm * igm * ligm));
        lE = add3(lE, scale3(lum, h));
        const float3 lu0 = lum;

        // interpolation reverse: offsets, then the transposed interpolation
        const float lF[6] = {lE.x, lE.y, lE.z, lB.x, lB.y, lB.z};
#pragma unroll
        for (int c = 0; c < 6; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) lo0[d] += lF[c] * G[c][d];
        if (valid) {
            to_global(AS.loff)[i] = lo0[0];
            to_global(AS.loff)[n + i] = lo0[1];
            to_global(AS.loff)[2 * n + i] = lo0[2];
            to_global(AS.lu)[i] = lu0.x;
            to_global(AS.lu)[n + i] = lu0.y;
            to_global(AS.lu)[2 * n + i] = lu0.z;
        }
        if constexpr (ORDER == 1) {
            float fn[3][AdjFrame<ORDER, false>::len], fh[3][AdjFrame<ORDER, true>::len];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                frame_place<ORDER, false>(bn[d], wn[d], fn[d]);
                frame_place<ORDER, true>(bh[d], wh[d], fh[d]);
            }
            const float vm = valid ? 1.0f : 0.0f;
            const RowScan rs = row_scan_setup<64>(valid ? local : -1);
            const bool add = rs.tail && valid;
            const int tx = lx + FLO, ty = ly + FLO, tz = lz + FLO;
            frame3_scan_add<ORDER, true, false, false>(gt, fx, fxy, tx, ty, tz, vm * lF[0], fh[0], fn[1], fn[2], rs, add);
            frame3_scan_add<ORDER, false, true, false>(gt + fcells, fx, fxy, tx, ty, tz, vm * lF[1], fn[0], fh[1], fn[2],
                                                       rs, add);
            frame3_scan_add<ORDER, false, false, true>(gt + 2 * fcells, fx, fxy, tx, ty, tz, vm * lF[2], fn[0], fn[1],
                                                       fh[2], rs, add);
            frame3_scan_add<ORDER, false, true, true>(gt + 3 * fcells, fx, fxy, tx, ty, tz, vm * lF[3], fn[0], fh[1],
                                                      fh[2], rs, add);
            frame3_scan_add<ORDER, true, false, true>(gt + 4 * fcells, fx, fxy, tx, ty, tz, vm * lF[4], fh[0], fn[1],
                                                      fh[2], rs, add);
            frame3_scan_add<ORDER, true, true, false>(gt + 5 * fcells, fx, fxy, tx, ty, tz, vm * lF[5], fh[0], fh[1],
                                                      fn[2], rs, add);
        } else {
            // order 2: the frames would not fit the registers; per-lane atomics
            if (valid) {
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const float *wxx = HS[c][0] ? wh[0] : wn[0], *wyy = HS[c][1] ? wh[1] : wn[1],
                                *wzz = HS[c][2] ? wh[2] : wn[2];
                    const int ix = lx + FLO + (HS[c][0] ? bh[0] : bn[0]);
                    const int iy = ly + FLO + (HS[c][1] ? bh[1] : bn[1]);
                    const int iz = lz + FLO + (HS[c][2] ? bh[2] : bn[2]);
                    double *g0 = gt + c * fcells + (iz * fy + iy) * fx + ix;
#pragma unroll
                    for (int cz = 0; cz <= ORDER; ++cz)
#pragma unroll
                        for (int by = 0; by <= ORDER; ++by) {
                            const float lyz = lF[c] * wyy[by] * wzz[cz];
#pragma unroll
                            for (int ax = 0; ax <= ORDER; ++ax) lds_add(g0 + (cz * fy + by) * fx + ax, lyz * wxx[ax]);
                        }
                }
            }
        }
    }
    __syncthreads();
    // the tile into lE, lB: entry (tx, ty, tz) is cell (ox, oy, oz) + (tx, ty, tz) - FLO, periodic
    for (int q = threadIdx.x; q < fcells; q += NT) {
        int64_t g;
        tile_cell(q, fx, fxy, FLO, g);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double ve = gt[c * fcells + q], vb = gt[(3 + c) * fcells + q];
            if (ve != 0.0) atomicAdd((float *)(to_global(A.lE) + (c * nc + g)), (float)ve);
            if (vb != 0.0) atomicAdd((float *)(to_global(A.lB) + (c * nc + g)), (float)vb);
        }
    }
}

// fold the transposed-interpolation tiles (field-tile geometry) into lE, lB
// Runs whose patches are all at least as wide as the current halo (so also
// as the field tile's): per dimension the patch below (when l < hi), the
// own patch and the patch above (when l >= ext - lo), every load issued
// before the sums and the clearing stores, as in the forward fold.
__device__ __forceinline__ void adj_fold_direct(const RunDev &R, const AdjRun &A, int64_t idx) {
    int g3[3];
    adj_grid_coords(R, idx, g3);
    const int l0[2] = {g3[1], g3[2]};   // 2-d: (y, z)
    const int lo = 1, hi = R.order;
    const int fy = R.P[1] + lo + hi, fz = R.P[2] + lo + hi;
    const int64_t fcells = (int64_t)fy * fz;
    int pcs[2][3], ls[2][3];
    bool on[2][3];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        const int P = R.P[d + 1], n = R.n[d + 1], np = R.np[d + 1];
        const int pc = l0[d] / P, l = l0[d] - pc * P;
        const int ext = imin(P, n - pc * P);
        const int pdn = pc == 0 ? np - 1 : pc - 1;
        on[d][0] = l < hi;
        pcs[d][0] = pdn;
        ls[d][0] = l + imin(P, n - pdn * P);
        on[d][1] = true;
        pcs[d][1] = pc;
        ls[d][1] = l;
        on[d][2] = l >= ext - lo;
        pcs[d][2] = pc == np - 1 ? 0 : pc + 1;
        ls[d][2] = l - ext;
    }
    const int64_t own = (int64_t)(R.np[0] * (pcs[0][1] + R.np[1] * pcs[1][1])) * 6 * fcells + (ls[0][1] + lo) +
                        (int64_t)fy * (ls[1][1] + lo);
    float v[9][6];
    int64_t at[9];
#pragma unroll
    for (int z = 0; z < 3; ++z)
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            const int k = z * 3 + y;
            const bool use = on[1][z] && on[0][y];
            const int p = R.np[0] * (pcs[0][y] + R.np[1] * pcs[1][z]);
            at[k] = use ? (int64_t)p * 6 * fcells + (ls[0][y] + lo) + (int64_t)fy * (ls[1][z] + lo) : own;
            float w[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) w[q] = to_global(A.gtile)[q * fcells + at[k]];
#pragma unroll
            for (int q = 0; q < 6; ++q) v[k][q] = use ? w[q] : 0.0f;
        }
    const int64_t nc = R.ncell;
    float cur[6];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        cur[q] = to_global(A.lE)[q * nc + idx];
        cur[3 + q] = to_global(A.lB)[q * nc + idx];
    }
    float acc[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int q = 0; q < 6; ++q) acc[q] += v[k][q];
#pragma unroll
    for (int z = 0; z < 3; ++z)
#pragma unroll
        for (int y = 0; y < 3; ++y)
            if (on[1][z] && on[0][y])
#pragma unroll
                for (int q = 0; q < 6; ++q) to_global(A.gtile)[q * fcells + at[z * 3 + y]] = 0.0f;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        to_global(A.lE)[q * nc + idx] = cur[q] + acc[q];
        to_global(A.lB)[q * nc + idx] = cur[3 + q] + acc[3 + q];
    }
}

__global__ void __launch_bounds__(256) k_adj_fold(const RunDev *__restrict__ runs, const AdjRun *__restrict__ adj,
                                                  int n_runs, const int64_t *__restrict__ run_base, int64_t total) {
    {
        // the usual case: the workgroup in one run whose patches allow the direct fold
        const int64_t c0 = (int64_t)blockIdx.x * blockDim.x;
        const int64_t c1 = (c0 + blockDim.x < total ? c0 + blockDim.x : total) - 1;
        const int rb = find_run_a(run_base, n_runs, c0);
        if (run_base[rb + 1] > c1 && runs[rb].fold_direct) {
            const int64_t c = c0 + threadIdx.x;
            if (c < total) adj_fold_direct(runs[rb], adj[rb], c - run_base[rb]);
            return;
        }
    }
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= total) return;
    const int r = find_run_a(run_base, n_runs, c);
    const RunDev &R = runs[r];
    const AdjRun &A = adj[r];
    const int64_t idx = c - R.cell_base;
    const int g[2] = {(int)(idx % R.n[1]), (int)(idx / R.n[1])};   // 2-d: (y, z)
    const int lo = 1, hi = R.order;
    const int fy = R.P[1] + lo + hi, fz = R.P[2] + lo + hi;
    const int64_t fcells = (int64_t)fy * fz;
    int cand[2][3], ncand[2];
    for (int d = 0; d < 2; ++d) {
        const int own = g[d] / R.P[d + 1];
        ncand[d] = 0;
        for (int t = -1; t <= 1; ++t) {
            const int pcd = wrap(own + t, R.np[d + 1]);
            bool dup = false;
            for (int q = 0; q < ncand[d]; ++q) dup |= cand[d][q] == pcd;
            if (!dup) cand[d][ncand[d]++] = pcd;
        }
    }
    float acc[6] = {0, 0, 0, 0, 0, 0};
    for (int a1 = 0; a1 < ncand[1]; ++a1)
        for (int a0 = 0; a0 < ncand[0]; ++a0) {
            const int pcy = cand[0][a0], pcz = cand[1][a1];
            const int p = R.np[0] * (pcy + R.np[1] * pcz);
            const gptr<float> tile = to_global(A.gtile + (int64_t)p * 6 * fcells);
            int ls[2][3], nl[2];
            const int pcs[2] = {pcy, pcz};
            for (int d = 0; d < 2; ++d) {
                nl[d] = 0;
                const int ext = patch_ext(R, d + 1, pcs[d]);
                const int base = g[d] - pcs[d] * R.P[d + 1];
                for (int m = -1; m <= 1; ++m) {
                    const int l = base + m * R.n[d + 1];
                    if (l >= -lo && l < ext + hi) ls[d][nl[d]++] = l;
                }
            }
            for (int z = 0; z < nl[1]; ++z)
                for (int y = 0; y < nl[0]; ++y) {
                    const int64_t t = (ls[0][y] + lo) + (int64_t)fy * (ls[1][z] + lo);
                    for (int q = 0; q < 6; ++q) {
                        acc[q] += tile[q * fcells + t];
                        tile[q * fcells + t] = 0.0f;
                    }
                }
        }
    const int64_t nc = R.ncell;
    for (int q = 0; q < 3; ++q) {
        to_global(A.lE)[q * nc + idx] += acc[q];
        to_global(A.lB)[q * nc + idx] += acc[3 + q];
    }
}

// Adjoint seed of W = 1/2 sum(E^2 + B^2) dV at the final state: dW/dE = E dV,
// dW/dB = B dV (n = 3 ncell values of one run).
__global__ void k_adj_seed(const float *__restrict__ E, const float *__restrict__ B, float *__restrict__ lE,
                           float *__restrict__ lB, int64_t n, float dV) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    lE[i] = E[i] * dV;
    lB[i] = B[i] * dV;
}

hipError_t launch_adj_seed(const float *E, const float *B, float *lE, float *lB, int64_t n, float dV,
                           hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_seed, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, E, B, lE, lB, n, dV);
    return hipGetLastError();
}

size_t adjoint_lds_bytes(int dim, int order, const int P[3]) {
    const int fx = dim == 3 ? P[0] + 1 + order : 1, jx = dim == 3 ? P[0] + 2 * order + 1 : 1;
    const int fcells = fx * (P[1] + 1 + order) * (P[2] + 1 + order);
    const int jcells = jx * (P[1] + 2 * order + 1) * (P[2] + 2 * order + 1);
    return sizeof(float) * (size_t)adj_lds_layout(fcells, jcells).total;
}

hipError_t launch_adjoint(const Launch &L, const AdjRun *adj_dev, const AdjRun *adj_host, const Unit *units,
                          int n_units, int32_t *item_start, int64_t max_items, int chunk, int dim, int order,
                          int64_t total_cells, const int64_t *run_base, size_t lds, hipStream_t s) {
    const unsigned gc = (unsigned)((total_cells + 255) / 256);
    // (1) LJ = -dt lE', lB2 = lB' + dt curl^+ lE'
    hipLaunchKernelGGL(k_adj_fields, dim3(gc), dim3(256), 0, s, L.runs_dev, adj_dev, L.n_runs, run_base, total_cells, 0);
    // (2) lE -= dt/2 curl^- lB2, B1 = B - dt/2 curl^+ E
    hipLaunchKernelGGL(k_adj_fields, dim3(gc), dim3(256), 0, s, L.runs_dev, adj_dev, L.n_runs, run_base, total_cells, 1);
    // (3) particle adjoints to this step's slots; cell offsets of the forward keys
    for (int r = 0; r < L.n_runs; ++r) {
        const RunDev &R = L.runs_host[r];
        for (int sp = 0; sp < R.n_species; ++sp) {
            const AdjSpecies &S = adj_host[r].sp[sp];
            if (S.n > 0)
                hipLaunchKernelGGL(k_adj_unpermute, dim3((unsigned)((S.n + 255) / 256)), dim3(256), 0, s, adj_dev, r,
                                   sp, R.dim);
            if (S.cs == S.cs_scratch) {   // offsets not given: from the sorted keys
                hipError_t e = launch_cell_starts(S.n, R.ncell, S.key, S.cs_scratch, L.err, s);
                if (e != hipSuccess) return e;
            }
        }
    }
    // (4) particles
    hipLaunchKernelGGL(k_adj_unit_items, dim3((unsigned)imax(1, (n_units + 255) / 256)), dim3(256), 0, s, L.runs_dev,
                       adj_dev, units, n_units, chunk, item_start);
    {
        hipError_t e = launch_items_scan(n_units, item_start, nullptr, s);
        if (e != hipSuccess) return e;
    }
    int64_t grid = (max_items + 7) / 8 * 8;
    if (grid < 8) grid = 8;
    if (dim == 3) {
        // the 3-d kernel adds its transposed interpolation into lE, lB1 itself
        if (order == 1)
            hipLaunchKernelGGL(k_adj_particles3<1>, dim3((unsigned)grid), dim3(kAdjBlock), lds, s, L.runs_dev, adj_dev,
                               units, item_start, n_units, chunk);
        else
            hipLaunchKernelGGL(k_adj_particles3<2>, dim3((unsigned)grid), dim3(kAdjBlock), lds, s, L.runs_dev, adj_dev,
                               units, item_start, n_units, chunk);
    } else {
        if (order == 1)
            hipLaunchKernelGGL(k_adj_particles<1>, dim3((unsigned)grid), dim3(kAdjBlock), lds, s, L.runs_dev, adj_dev,
                               units, item_start, n_units, chunk);
        else
            hipLaunchKernelGGL(k_adj_particles<2>, dim3((unsigned)grid), dim3(kAdjBlock), lds, s, L.runs_dev, adj_dev,
                               units, item_start, n_units, chunk);
        // (5) transposed interpolation into lE, lB1
        hipLaunchKernelGGL(k_adj_fold, dim3(gc), dim3(256), 0, s, L.runs_dev, adj_dev, L.n_runs, run_base,
                           total_cells);
    }
    // (6) lE -= dt/2 curl^- lB1   (lB = lB1 is the adjoint of B^n)
    hipLaunchKernelGGL(k_adj_fields, dim3(gc), dim3(256), 0, s, L.runs_dev, adj_dev, L.n_runs, run_base, total_cells, 2);
    return hipGetLastError();
}

}  // namespace psc
