// psc_fields.hip -- Yee FDTD field update, fold of the per-patch current tiles
// into J, and the double-precision diagnostics.
//
// FDTD (section "FDTD method for solving Maxwell's equations"): forward curl
// curl^+ E on faces, backward curl curl^- B on edges, leap-frog split as in
// fig. psc_new (two B half steps around the particle loop, one E full step).
// All kernels index a flat cell space spanning every run; the run of a cell is
// found by binary search over the runs' cell offsets.
#include "psc_device.h"
#include "psc_xcd.h"

namespace psc {

__device__ __forceinline__ int find_run(const int64_t *base, int n_runs, int64_t c) {
    int lo = 0, hi = n_runs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= c) lo = mid; else hi = mid;
    }
    return lo;
}

// The run of every cell of this workgroup when they lie in one run (the
// usual case: then the run's fields are read once, through scalar loads),
// else -1.
__device__ __forceinline__ int block_run(const int64_t *base, int n_runs, int64_t total) {
    const int64_t c0 = (int64_t)xcd_block() * blockDim.x;
    const int64_t c1 = (c0 + blockDim.x < total ? c0 + blockDim.x : total) - 1;
    const int r = find_run(base, n_runs, c0);
    return base[r + 1] > c1 ? r : -1;
}

// Call f(R, idx) for the cell c of the flat cell space (idx: its index in
// run R), with R uniform over the workgroup when block_run finds one run.
template <typename F>
__device__ __forceinline__ void with_run(const RunDev *runs, const int64_t *base, int n_runs, int64_t total, F &&f) {
    const int64_t c = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
    const int rb = block_run(base, n_runs, total);
    if (c >= total) return;
    if (rb >= 0) {
        f(runs[rb], c - base[rb]);
    } else {
        const int r = find_run(base, n_runs, c);
        f(runs[r], c - base[r]);
    }
}

// grid coordinates of cell idx of a run (32-bit: a run has fewer than 2^31
// cells; a 2-d run has n[0] == 1)
__device__ __forceinline__ void grid_coords(const RunDev &R, int64_t idx, int g[3]) {
    const uint32_t id = (uint32_t)idx;
    const uint32_t nx = (uint32_t)R.n[0], ny = (uint32_t)R.n[1];
    const uint32_t q = R.dim == 3 ? id / nx : id;
    g[0] = (int)(id - q * nx);
    const uint32_t k = q / ny;
    g[1] = (int)(q - k * ny);
    g[2] = (int)k;
}

__device__ __forceinline__ void field_step(const RunDev &R, int64_t idx, int op) {
    const int nx = R.n[0], ny = R.n[1], nz = R.n[2];
    int g[3];
    grid_coords(R, idx, g);
    const int i = g[0], j = g[1], k = g[2];
    const int64_t nc = R.ncell;
    const bool three = R.dim == 3;
    const float ix = three ? R.inv_dx[0] : 0.0f, iy = R.inv_dx[1], iz = R.inv_dx[2];
    const int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
    const gptr<float> E = to_global(R.E), B = to_global(R.B), J = to_global(R.J);
    // every load before the arithmetic and the stores (in 2-d the x
    // neighbour is the cell itself and ix is zero, so its term is zero)
    if (op == PSC_B_HALF) {
        const float h = 0.5f * R.dt;
        const int64_t ip = i + 1 < nx ? idx + sx : idx - (int64_t)(nx - 1) * sx;
        const int64_t jp = j + 1 < ny ? idx + sy : idx - (int64_t)(ny - 1) * sy;
        const int64_t kp = k + 1 < nz ? idx + sz : idx - (int64_t)(nz - 1) * sz;
        const gptr<float> Ex = E, Ey = E + nc, Ez = E + 2 * nc;
        const float ex = Ex[idx], ey = Ey[idx], ez = Ez[idx];
        const float ez_j = Ez[jp], ey_k = Ey[kp], ex_k = Ex[kp], ez_i = Ez[ip], ey_i = Ey[ip], ex_j = Ex[jp];
        const float bx = B[idx], by = B[nc + idx], bz = B[2 * nc + idx];
        const float cx = (ez_j - ez) * iy - (ey_k - ey) * iz;
        const float cy = (ex_k - ex) * iz - (ez_i - ez) * ix;
        const float cz = (ey_i - ey) * ix - (ex_j - ex) * iy;
        B[idx] = bx - h * cx;
        B[nc + idx] = by - h * cy;
        B[2 * nc + idx] = bz - h * cz;
    } else {
        const float h = R.dt;
        const int64_t im = i > 0 ? idx - sx : idx + (int64_t)(nx - 1) * sx;
        const int64_t jm = j > 0 ? idx - sy : idx + (int64_t)(ny - 1) * sy;
        const int64_t km = k > 0 ? idx - sz : idx + (int64_t)(nz - 1) * sz;
        const gptr<float> Bx = B, By = B + nc, Bz = B + 2 * nc;
        const float bx = Bx[idx], by = By[idx], bz = Bz[idx];
        const float bz_j = Bz[jm], by_k = By[km], bx_k = Bx[km], bz_i = Bz[im], by_i = By[im], bx_j = Bx[jm];
        const float ex = E[idx], ey = E[nc + idx], ez = E[2 * nc + idx];
        const float jx = J[idx], jy = J[nc + idx], jz = J[2 * nc + idx];
        const float cx = (bz - bz_j) * iy - (by - by_k) * iz;
        const float cy = (bx - bx_k) * iz - (bz - bz_i) * ix;
        const float cz = (by - by_i) * ix - (bx - bx_j) * iy;
        E[idx] = ex + h * (cx - jx);
        E[nc + idx] = ey + h * (cy - jy);
        E[2 * nc + idx] = ez + h * (cz - jz);
    }
}

// B <- B - (dt/2) curl^+ E (op 0) or E <- E + dt (curl^- B - J) (op 1)
__global__ void __launch_bounds__(256) k_fields(const RunDev *__restrict__ runs, int n_runs,
                                                const int64_t *__restrict__ run_base, int64_t total, int op) {
    with_run(runs, run_base, n_runs, total, [&](const RunDev &R, int64_t idx) { field_step(R, idx, op); });
}

hipError_t launch_fields(const Launch &L, int op, int64_t total, const int64_t *run_base) {
    const unsigned grid = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(k_fields, dim3(grid), dim3(256), 0, L.stream, L.runs_dev, L.n_runs, run_base, total, op);
    return hipGetLastError();
}

// J from the fixed-point sums of the runs whose particle kernel adds its
// current tiles into jacc (integer sums: the same whatever order the work
// items added in), and jacc cleared for the next push
__global__ void __launch_bounds__(256) k_finish_current(const RunDev *__restrict__ runs, int n_runs,
                                                        const int64_t *__restrict__ run_base, int64_t total) {
    with_run(runs, run_base, n_runs, total, [&](const RunDev &R, int64_t idx) {
        if (!R.jdirect) return;
        const int64_t nc = R.ncell;
        const gptr<long long> acc = to_global(R.jacc);
        const gptr<float> J = to_global(R.J);
        long long a[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) a[c] = acc[c * nc + idx];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            J[c * nc + idx] = (float)((double)a[c] * R.jq);
            acc[c * nc + idx] = 0;
        }
    });
}

hipError_t launch_finish_current(const Launch &L, int64_t total, const int64_t *run_base) {
    const unsigned grid = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(k_finish_current, dim3(grid), dim3(256), 0, L.stream, L.runs_dev, L.n_runs, run_base, total);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// J fold: J(cell) = sum of every patch tile entry that maps onto the cell
// (own patch and the halos of its neighbours, periodic), in a fixed order;
// each tile entry maps onto exactly one cell, so it is cleared here too.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_fold(const RunDev *__restrict__ runs, int n_runs,
                                              const int64_t *__restrict__ run_base, int64_t total) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= total) return;
    const int r = find_run(run_base, n_runs, c);
    const RunDev &R = runs[r];
    const int64_t idx = c - R.cell_base;
    int g[3];
    grid_coords(R, idx, g);
    const int lo = cur_lo(R.order), hi = cur_hi(R.order);
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    const int64_t jc = R.jtile_cells;
    const int64_t nc = R.ncell;
    if (R.fold_direct || R.jdirect) return;   // folded by patch (k_fold_patch), or J is complete
    // candidate patch coordinates per dimension (deduplicated), and for each
    // the tile-local coordinates that alias this cell
    int cand[3][3], ncand[3];
    for (int d = 0; d < 3; ++d) {
        const int own = g[d] / R.P[d];
        ncand[d] = 0;
        for (int t = -1; t <= 1; ++t) {
            const int pcd = wrap(own + t, R.np[d]);
            bool dup = false;
            for (int q = 0; q < ncand[d]; ++q) dup |= cand[d][q] == pcd;
            if (!dup) cand[d][ncand[d]++] = pcd;
        }
    }
    for (int a2 = 0; a2 < ncand[2]; ++a2)
        for (int a1 = 0; a1 < ncand[1]; ++a1)
            for (int a0 = 0; a0 < ncand[0]; ++a0) {
                const int pc[3] = {cand[0][a0], cand[1][a1], cand[2][a2]};
                const int p = pc[0] + R.np[0] * (pc[1] + R.np[1] * pc[2]);
                float *tile = R.jtile + (int64_t)p * 3 * jc;
                // aliases along each dimension: l = g - origin + m*n, l in [-lo, ext+hi)
                int ls[3][3], nl[3];
                for (int d = 0; d < 3; ++d) {
                    nl[d] = 0;
                    if (R.dim == 2 && d == 0) { ls[0][0] = 0; nl[0] = 1; continue; }
                    const int ext = patch_ext(R, d, pc[d]);
                    const int base = g[d] - pc[d] * R.P[d];
                    for (int m = -1; m <= 1; ++m) {
                        const int l = base + m * R.n[d];
                        if (l >= -lo && l < ext + hi) ls[d][nl[d]++] = l;
                    }
                }
                for (int z = 0; z < nl[2]; ++z)
                    for (int y = 0; y < nl[1]; ++y)
                        for (int x = 0; x < nl[0]; ++x) {
                            const int tx = R.dim == 3 ? ls[0][x] + lo : 0;
                            const int64_t t = tx + (int64_t)R.jt[0] * ((ls[1][y] + lo) + (int64_t)R.jt[1] * (ls[2][z] + lo));
                            sx += tile[t];
                            sy += tile[jc + t];
                            sz += tile[2 * jc + t];
                            tile[t] = 0.0f;
                            tile[jc + t] = 0.0f;
                            tile[2 * jc + t] = 0.0f;
                        }
            }
    R.J[idx] = sx;
    R.J[nc + idx] = sy;
    R.J[2 * nc + idx] = sz;
}

// Runs whose patches are all at least as wide as the current halo: a tile
// aliases cells of its own patch and, across each face, of the adjacent
// patch only.  Workgroup row (patch, part) folds part of the patch's cells:
// per dimension the patch below (whose upper halo reaches the cell when
// l < hi), the own patch and the patch above (lower halo, when
// l >= ext - lo), in that order.  With 1 or 2 patches along a dimension
// these are different aliases within the same tile.  A patch's tile is read
// by its own workgroups and, at the faces, its neighbours', so the reads
// stay within a few contiguous tiles at a time.
constexpr int kFoldBlock = 256;

template <int DIM>
__global__ void __launch_bounds__(kFoldBlock) k_fold_patch(const RunDev *__restrict__ runs, int n_runs,
                                                           const int64_t *__restrict__ patch_base) {
    constexpr int X0 = DIM == 3 ? 0 : 1, X1 = DIM == 3 ? 2 : 1;   // x candidates (2-d: the own one)
    const int64_t gp = blockIdx.x;
    const int r = find_run(patch_base, n_runs, gp);
    const RunDev &R = runs[r];
    if (!R.fold_direct || R.jdirect || R.dim != DIM) return;
    const int p = (int)(gp - patch_base[r]);
    int pc[3], ext[3];
    pc[0] = p % R.np[0];
    pc[1] = (p / R.np[0]) % R.np[1];
    pc[2] = p / (R.np[0] * R.np[1]);
#pragma unroll
    for (int d = 0; d < 3; ++d) ext[d] = imin(R.P[d], R.n[d] - pc[d] * R.P[d]);
    const uint32_t ncells = (uint32_t)(ext[0] * ext[1] * ext[2]);
    const int lo = cur_lo(R.order), hi = cur_hi(R.order);
    const int64_t jc = R.jtile_cells;
    const int64_t nc = R.ncell;
    const gptr<float> jtile = to_global(R.jtile), J = to_global(R.J);
    for (uint32_t t = blockIdx.y * kFoldBlock + threadIdx.x; t < ncells; t += gridDim.y * kFoldBlock) {
        int l[3];
        const uint32_t q = t / (uint32_t)ext[0];
        l[0] = (int)(t - q * (uint32_t)ext[0]);
        l[2] = (int)(q / (uint32_t)ext[1]);
        l[1] = (int)(q - (uint32_t)l[2] * (uint32_t)ext[1]);
        // candidates per dimension: 0 below, 1 own, 2 above
        int pcs[3][3], ls[3][3];
        bool on[3][3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (DIM == 2 && d == 0) {
                on[0][1] = true;
                pcs[0][1] = 0;
                ls[0][1] = -lo;   // tile x index 0
                continue;
            }
            const int pdn = pc[d] == 0 ? R.np[d] - 1 : pc[d] - 1;
            on[d][0] = l[d] < hi;
            pcs[d][0] = pdn;
            ls[d][0] = l[d] + imin(R.P[d], R.n[d] - pdn * R.P[d]);
            on[d][1] = true;
            pcs[d][1] = pc[d];
            ls[d][1] = l[d];
            on[d][2] = l[d] >= ext[d] - lo;
            pcs[d][2] = pc[d] == R.np[d] - 1 ? 0 : pc[d] + 1;
            ls[d][2] = l[d] - ext[d];
        }
        // every load before the sums and the clearing stores, and every
        // load issued (an unused candidate reads the own entry, counted as
        // zero), so that a cell's reads are in flight together
        float v[27][3];
        const int64_t own = (int64_t)p * 3 * jc + (ls[0][1] + lo) +
                            (int64_t)R.jt[0] * ((l[1] + lo) + (int64_t)R.jt[1] * (l[2] + lo));
#pragma unroll
        for (int z = 0; z < 3; ++z)
#pragma unroll
            for (int y = 0; y < 3; ++y)
#pragma unroll
                for (int x = X0; x <= X1; ++x) {
                    const int k = (z * 3 + y) * 3 + x;
                    const int pq = pcs[0][x] + R.np[0] * (pcs[1][y] + R.np[1] * pcs[2][z]);
                    const bool use = on[2][z] && on[1][y] && on[0][x];
                    const int64_t at = use ? (int64_t)pq * 3 * jc + (ls[0][x] + lo) +
                                                 (int64_t)R.jt[0] * ((ls[1][y] + lo) + (int64_t)R.jt[1] * (ls[2][z] + lo))
                                           : own;
                    const float a = jtile[at], b = jtile[jc + at], c = jtile[2 * jc + at];
                    v[k][0] = use ? a : 0.0f;
                    v[k][1] = use ? b : 0.0f;
                    v[k][2] = use ? c : 0.0f;
                }
        float sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
        for (int z = 0; z < 3; ++z)
#pragma unroll
            for (int y = 0; y < 3; ++y)
#pragma unroll
                for (int x = X0; x <= X1; ++x) {
                    const int k = (z * 3 + y) * 3 + x;
                    sx += v[k][0];
                    sy += v[k][1];
                    sz += v[k][2];
                }
#pragma unroll
        for (int z = 0; z < 3; ++z)
#pragma unroll
            for (int y = 0; y < 3; ++y)
#pragma unroll
                for (int x = X0; x <= X1; ++x) {
                    if (on[2][z] && on[1][y] && on[0][x]) {   // the address again: fewer live registers
                        const int pq = pcs[0][x] + R.np[0] * (pcs[1][y] + R.np[1] * pcs[2][z]);
                        const int64_t at = (int64_t)pq * 3 * jc + (ls[0][x] + lo) +
                                           (int64_t)R.jt[0] * ((ls[1][y] + lo) + (int64_t)R.jt[1] * (ls[2][z] + lo));
                        jtile[at] = 0.0f;
                        jtile[jc + at] = 0.0f;
                        jtile[2 * jc + at] = 0.0f;
                    }
                }
        const int64_t idx = (pc[0] * R.P[0] + l[0]) +
                            (int64_t)R.n[0] * ((pc[1] * R.P[1] + l[1]) + (int64_t)R.n[1] * (pc[2] * R.P[2] + l[2]));
        J[idx] = sx;
        J[nc + idx] = sy;
        J[2 * nc + idx] = sz;
    }
}

hipError_t launch_fold(const Launch &L, int64_t total, const int64_t *run_base, int64_t total_patches,
                       const int64_t *patch_base, int max_patch_cells, int direct_dims, bool any_search) {
    const unsigned parts = (unsigned)imin((max_patch_cells + kFoldBlock - 1) / kFoldBlock, 1024);
    if ((direct_dims & 4) && total_patches > 0)
        hipLaunchKernelGGL(k_fold_patch<2>, dim3((unsigned)total_patches, parts), dim3(kFoldBlock), 0, L.stream,
                           L.runs_dev, L.n_runs, patch_base);
    if ((direct_dims & 8) && total_patches > 0)
        hipLaunchKernelGGL(k_fold_patch<3>, dim3((unsigned)total_patches, parts), dim3(kFoldBlock), 0, L.stream,
                           L.runs_dev, L.n_runs, patch_base);
    if (any_search) {
        const unsigned grid = (unsigned)((total + 255) / 256);
        hipLaunchKernelGGL(k_fold, dim3(grid), dim3(256), 0, L.stream, L.runs_dev, L.n_runs, run_base, total);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// diagnostics in float64
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}
// atomic max of a non-negative double through its bit pattern
__device__ __forceinline__ void atomic_max_nonneg(double *p, double v) {
    atomicMax(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ double bs(int order, double s) {
    const double a = fabs(s);
    if (order == 1) return a < 1.0 ? 1.0 - a : 0.0;
    if (a <= 0.5) return 0.75 - a * a;
    if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
    return 0.0;
}

// charge density at nodes from one species, float64 atomics
__global__ void __launch_bounds__(256) k_rho(const RunDev *__restrict__ runs, int r, int sp, int front,
                                             double *__restrict__ out) {
    const RunDev &R = runs[r];
    const SpeciesDev &S = R.sp[sp];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= S.n) return;
    int g[3];
    decode_key(R, S.cell[front][p], g);
    double x[3] = {0, 0, 0};
    const int D = R.dim;
    for (int d = 0; d < D; ++d) x[3 - D + d] = (double)S.off[front][d * S.cap + p];
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 3 - D; d < 3; ++d) {
        lo[d] = -2;
        hi[d] = 2;
    }
    const double qw = (double)S.q * (double)S.w;
    for (int c = lo[2]; c <= hi[2]; ++c) {
        const double wz = bs(R.order, x[2] - c);
        if (wz == 0.0) continue;
        for (int b = lo[1]; b <= hi[1]; ++b) {
            const double wy = bs(R.order, x[1] - b);
            if (wy == 0.0) continue;
            for (int a = lo[0]; a <= hi[0]; ++a) {
                const double wx = D == 3 ? bs(R.order, x[0] - a) : 1.0;
                if (wx == 0.0) continue;
                const int gx = D == 3 ? wrap(g[0] + a, R.n[0]) : 0;
                const int64_t cell = gx + (int64_t)R.n[0] * (wrap(g[1] + b, R.n[1]) + (int64_t)R.n[1] * wrap(g[2] + c, R.n[2]));
                atomicAdd(&out[cell], qw * wx * wy * wz);
            }
        }
    }
}

// kinetic energy per species
__global__ void __launch_bounds__(256) k_kinetic(const RunDev *__restrict__ runs, int r, int sp, int front,
                                                 double *__restrict__ out) {
    const RunDev &R = runs[r];
    const SpeciesDev &S = R.sp[sp];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (p < S.n) {
        const double ux = S.u[front][p], uy = S.u[front][S.cap + p], uz = S.u[front][2 * S.cap + p];
        const double u2 = ux * ux + uy * uy + uz * uz;
        v = u2 / (sqrt(1.0 + u2) + 1.0);   // gamma - 1 without cancellation
    }
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0 && v != 0.0) {
        const double dV = R.dxd[1] * R.dxd[2] * (R.dim == 3 ? R.dxd[0] : 1.0);
        atomicAdd(&out[2 + sp], (double)S.m * S.w * dV * v);
    }
}

// field energies, Gauss residual, div B, total charge
__global__ void __launch_bounds__(256) k_field_diag(const RunDev *__restrict__ runs, int n_runs,
                                                    const int64_t *__restrict__ run_base, int64_t total,
                                                    double *__restrict__ out, double *__restrict__ gauss) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int r = 0;
    double we = 0, wb = 0, gmax = 0, bmax = 0, rsum = 0;
    if (c < total) {
        r = find_run(run_base, n_runs, c);
        const RunDev &R = runs[r];
        const int64_t idx = c - R.cell_base;
        const int nx = R.n[0], ny = R.n[1], nz = R.n[2];
        int g[3];
        grid_coords(R, idx, g);
        const int i = g[0], j = g[1], k = g[2];
        const int64_t nc = R.ncell;
        const bool three = R.dim == 3;
        const double dV = R.dxd[1] * R.dxd[2] * (three ? R.dxd[0] : 1.0);
        const double ix = three ? 1.0 / R.dxd[0] : 0.0, iy = 1.0 / R.dxd[1], iz = 1.0 / R.dxd[2];
        for (int q = 0; q < 3; ++q) {
            const double e = R.E[q * nc + idx], b = R.B[q * nc + idx];
            we += e * e;
            wb += b * b;
        }
        we *= 0.5 * dV;
        wb *= 0.5 * dV;
        const int64_t im = i > 0 ? idx - 1 : idx + (nx - 1);
        const int64_t jm = j > 0 ? idx - nx : idx + (int64_t)(ny - 1) * nx;
        const int64_t km = k > 0 ? idx - (int64_t)nx * ny : idx + (int64_t)(nz - 1) * nx * ny;
        const int64_t ip = i + 1 < nx ? idx + 1 : idx - (nx - 1);
        const int64_t jp = j + 1 < ny ? idx + nx : idx - (int64_t)(ny - 1) * nx;
        const int64_t kp = k + 1 < nz ? idx + (int64_t)nx * ny : idx - (int64_t)(nz - 1) * nx * ny;
        const double dive = ((double)R.E[idx] - R.E[im]) * ix + ((double)R.E[nc + idx] - R.E[nc + jm]) * iy +
                            ((double)R.E[2 * nc + idx] - R.E[2 * nc + km]) * iz;
        const double divb = ((double)R.B[ip] - R.B[idx]) * ix + ((double)R.B[nc + jp] - R.B[nc + idx]) * iy +
                            ((double)R.B[2 * nc + kp] - R.B[2 * nc + idx]) * iz;
        const double rho = R.rho[idx];
        const double G = dive - rho;
        if (gauss) gauss[c] = G;
        gmax = fabs(G);
        bmax = fabs(divb);
        rsum = rho * dV;
    }
    // runs can change inside a wave; reduce per lane group with the same run
    const int r0 = __shfl(r, 0, 64);
    const bool uniform = __all(r == r0);
    if (uniform) {
        we = wave_sum(we);
        wb = wave_sum(wb);
        rsum = wave_sum(rsum);
        gmax = wave_max(gmax);
        bmax = wave_max(bmax);
        if ((threadIdx.x & 63) == 0 && c - (threadIdx.x & 63) < total) {
            double *o = out + (int64_t)r0 * PSC_DIAG_STRIDE;
            atomicAdd(&o[0], we);
            atomicAdd(&o[1], wb);
            atomicAdd(&o[8], rsum);
            atomic_max_nonneg(&o[6], gmax);
            atomic_max_nonneg(&o[7], bmax);
        }
    } else if (c < total) {
        double *o = out + (int64_t)r * PSC_DIAG_STRIDE;
        atomicAdd(&o[0], we);
        atomicAdd(&o[1], wb);
        atomicAdd(&o[8], rsum);
        atomic_max_nonneg(&o[6], gmax);
        atomic_max_nonneg(&o[7], bmax);
    }
}

__global__ void k_zero_f64(double *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void k_count(const RunDev *__restrict__ runs, int n_runs, double *out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_runs) return;
    double n = 0;
    for (int s = 0; s < runs[r].n_species; ++s) n += (double)runs[r].sp[s].n;
    out[(int64_t)r * PSC_DIAG_STRIDE + 9] = n;
}

// Marder cleaning, residual: F = (div^- E - rho) - ref at every node, written
// over rho (which holds the charge density of the current particles)
__global__ void __launch_bounds__(256) k_marder_residual(const RunDev *__restrict__ runs, int n_runs,
                                                         const int64_t *__restrict__ run_base, int64_t total,
                                                         const double *__restrict__ ref) {
    with_run(runs, run_base, n_runs, total, [&](const RunDev &R, int64_t idx) {
        const int64_t c = R.cell_base + idx;
        const int nx = R.n[0], ny = R.n[1], nz = R.n[2];
        int g[3];
        grid_coords(R, idx, g);
        const int i = g[0], j = g[1], k = g[2];
        const int64_t nc = R.ncell;
        const double ix = R.dim == 3 ? 1.0 / R.dxd[0] : 0.0, iy = 1.0 / R.dxd[1], iz = 1.0 / R.dxd[2];
        const int64_t im = i > 0 ? idx - 1 : idx + (nx - 1);
        const int64_t jm = j > 0 ? idx - nx : idx + (int64_t)(ny - 1) * nx;
        const int64_t km = k > 0 ? idx - (int64_t)nx * ny : idx + (int64_t)(nz - 1) * nx * ny;
        const double dive = ((double)R.E[idx] - R.E[im]) * ix + ((double)R.E[nc + idx] - R.E[nc + jm]) * iy +
                            ((double)R.E[2 * nc + idx] - R.E[2 * nc + km]) * iz;
        R.rho[idx] = dive - R.rho[idx] - (ref ? ref[c] : 0.0);
    });
}

// Marder cleaning, update: E += d dt grad^+ F (the forward difference of the
// node field F lies where each E component is staggered)
__global__ void __launch_bounds__(256) k_marder_update(const RunDev *__restrict__ runs, int n_runs,
                                                       const int64_t *__restrict__ run_base, int64_t total, double d) {
    with_run(runs, run_base, n_runs, total, [&](const RunDev &R, int64_t idx) {
        const int nx = R.n[0], ny = R.n[1], nz = R.n[2];
        int g[3];
        grid_coords(R, idx, g);
        const int i = g[0], j = g[1], k = g[2];
        const int64_t nc = R.ncell;
        const double h = d * (double)R.dt;
        const double ix = R.dim == 3 ? h / R.dxd[0] : 0.0, iy = h / R.dxd[1], iz = h / R.dxd[2];
        const int64_t ip = i + 1 < nx ? idx + 1 : idx - (nx - 1);
        const int64_t jp = j + 1 < ny ? idx + nx : idx - (int64_t)(ny - 1) * nx;
        const int64_t kp = k + 1 < nz ? idx + (int64_t)nx * ny : idx - (int64_t)(nz - 1) * nx * ny;
        const double *F = R.rho;
        const double f = F[idx], fi = F[ip], fj = F[jp], fk = F[kp];
        const float ex = R.E[idx], ey = R.E[nc + idx], ez = R.E[2 * nc + idx];
        R.E[idx] = (float)(ex + (fi - f) * ix);
        R.E[nc + idx] = (float)(ey + (fj - f) * iy);
        R.E[2 * nc + idx] = (float)(ez + (fk - f) * iz);
    });
}

// charge density of the current particles into every run's rho
static void launch_rho(const Launch &L, int front) {
    for (int r = 0; r < L.n_runs; ++r) {
        const RunDev &R = L.runs_host[r];
        hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((R.ncell + 255) / 256)), dim3(256), 0, L.stream, R.rho,
                           R.ncell);
        for (int s = 0; s < R.n_species; ++s) {
            const int64_t n = R.sp[s].n;
            if (n == 0) continue;
            hipLaunchKernelGGL(k_rho, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, L.stream, L.runs_dev, r, s,
                               front, R.rho);
        }
    }
}

hipError_t launch_marder(const Launch &L, const double *ref, double d, int iters, int64_t total,
                         const int64_t *run_base, int front) {
    const unsigned g = (unsigned)((total + 255) / 256);
    for (int it = 0; it < iters; ++it) {
        launch_rho(L, front);
        hipLaunchKernelGGL(k_marder_residual, dim3(g), dim3(256), 0, L.stream, L.runs_dev, L.n_runs, run_base, total,
                           ref);
        hipLaunchKernelGGL(k_marder_update, dim3(g), dim3(256), 0, L.stream, L.runs_dev, L.n_runs, run_base, total, d);
    }
    return hipGetLastError();
}

hipError_t launch_diag(const Launch &L, double *out, double *gauss, int64_t total, const int64_t *run_base,
                       int front) {
    const int64_t nout = (int64_t)L.n_runs * PSC_DIAG_STRIDE;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, L.stream, out, nout);
    for (int r = 0; r < L.n_runs; ++r) {
        const RunDev &R = L.runs_host[r];
        hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((R.ncell + 255) / 256)), dim3(256), 0, L.stream, R.rho,
                           R.ncell);
        for (int s = 0; s < R.n_species; ++s) {
            const int64_t n = R.sp[s].n;
            if (n == 0) continue;
            const unsigned g = (unsigned)((n + 255) / 256);
            hipLaunchKernelGGL(k_rho, dim3(g), dim3(256), 0, L.stream, L.runs_dev, r, s, front, R.rho);
            hipLaunchKernelGGL(k_kinetic, dim3(g), dim3(256), 0, L.stream, L.runs_dev, r, s, front,
                               out + (int64_t)r * PSC_DIAG_STRIDE);
        }
    }
    hipLaunchKernelGGL(k_field_diag, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, L.stream, L.runs_dev,
                       L.n_runs, run_base, total, out, gauss);
    hipLaunchKernelGGL(k_count, dim3((unsigned)((L.n_runs + 63) / 64)), dim3(64), 0, L.stream, L.runs_dev, L.n_runs,
                       out);
    return hipGetLastError();
}

}  // namespace psc
