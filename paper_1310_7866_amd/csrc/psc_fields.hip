// psc_fields.hip -- Yee FDTD field update, fold of the per-patch current tiles
// into J, and the double-precision diagnostics.
//
// FDTD (section "FDTD method for solving Maxwell's equations"): forward curl
// curl^+ E on faces, backward curl curl^- B on edges, leap-frog split as in
// fig. psc_new (two B half steps around the particle loop, one E full step).
// All kernels index a flat cell space spanning every run; the run of a cell is
// found by binary search over the runs' cell offsets.
#include "psc_internal.h"

namespace psc {

__device__ __forceinline__ int find_run(const int64_t *base, int n_runs, int64_t c) {
    int lo = 0, hi = n_runs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= c) lo = mid; else hi = mid;
    }
    return lo;
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

// B <- B - (dt/2) curl^+ E (op 0) or E <- E + dt (curl^- B - J) (op 1)
__global__ void __launch_bounds__(256) k_fields(const RunDev *__restrict__ runs, int n_runs,
                                                const int64_t *__restrict__ run_base, int64_t total, int op) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= total) return;
    const int r = find_run(run_base, n_runs, c);
    const RunDev &R = runs[r];
    const int64_t idx = c - R.cell_base;
    const int nx = R.n[0], ny = R.n[1], nz = R.n[2];
    int g[3];
    grid_coords(R, idx, g);
    const int i = g[0], j = g[1], k = g[2];
    const int64_t nc = R.ncell;
    const bool three = R.dim == 3;
    const float ix = three ? R.inv_dx[0] : 0.0f, iy = R.inv_dx[1], iz = R.inv_dx[2];
    const int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
    if (op == PSC_B_HALF) {
        const float h = 0.5f * R.dt;
        const int64_t ip = i + 1 < nx ? idx + sx : idx - (int64_t)(nx - 1) * sx;
        const int64_t jp = j + 1 < ny ? idx + sy : idx - (int64_t)(ny - 1) * sy;
        const int64_t kp = k + 1 < nz ? idx + sz : idx - (int64_t)(nz - 1) * sz;
        const float *Ex = R.E, *Ey = R.E + nc, *Ez = R.E + 2 * nc;
        const float ex = Ex[idx], ey = Ey[idx], ez = Ez[idx];
        const float cx = (Ez[jp] - ez) * iy - (Ey[kp] - ey) * iz;
        const float cy = (Ex[kp] - ex) * iz - (three ? (Ez[ip] - ez) * ix : 0.0f);
        const float cz = (three ? (Ey[ip] - ey) * ix : 0.0f) - (Ex[jp] - ex) * iy;
        R.B[idx] -= h * cx;
        R.B[nc + idx] -= h * cy;
        R.B[2 * nc + idx] -= h * cz;
    } else {
        const float h = R.dt;
        const int64_t im = i > 0 ? idx - sx : idx + (int64_t)(nx - 1) * sx;
        const int64_t jm = j > 0 ? idx - sy : idx + (int64_t)(ny - 1) * sy;
        const int64_t km = k > 0 ? idx - sz : idx + (int64_t)(nz - 1) * sz;
        const float *Bx = R.B, *By = R.B + nc, *Bz = R.B + 2 * nc;
        const float bx = Bx[idx], by = By[idx], bz = Bz[idx];
        const float cx = (bz - Bz[jm]) * iy - (by - By[km]) * iz;
        const float cy = (bx - Bx[km]) * iz - (three ? (bz - Bz[im]) * ix : 0.0f);
        const float cz = (three ? (by - By[im]) * ix : 0.0f) - (bx - Bx[jm]) * iy;
        R.E[idx] += h * (cx - R.J[idx]);
        R.E[nc + idx] += h * (cy - R.J[nc + idx]);
        R.E[2 * nc + idx] += h * (cz - R.J[2 * nc + idx]);
    }
}

hipError_t launch_fields(const Launch &L, int op, int64_t total, const int64_t *run_base) {
    const unsigned grid = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(k_fields, dim3(grid), dim3(256), 0, L.stream, L.runs_dev, L.n_runs, run_base, total, op);
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
    if (R.fold_direct) {
        // Per dimension: the patch below (whose upper halo reaches this cell
        // when l < hi), the own patch, the patch above (lower halo, when
        // l >= ext - lo), in that order, with the tile-local coordinate of
        // the cell in each.  With 1 or 2 patches along a dimension these are
        // different aliases within the same tile.
        int pcs[3][3], ls[3][3], nd[3];
        for (int d = 0; d < 3; ++d) {
            if (R.dim == 2 && d == 0) {
                pcs[0][0] = 0;
                ls[0][0] = -lo;   // tile x index 0
                nd[0] = 1;
                continue;
            }
            const int pc = g[d] / R.P[d];
            const int l = g[d] - pc * R.P[d];
            const int ext = imin(R.P[d], R.n[d] - pc * R.P[d]);
            int k = 0;
            if (l < hi) {
                const int pdn = pc == 0 ? R.np[d] - 1 : pc - 1;
                pcs[d][k] = pdn;
                ls[d][k++] = l + imin(R.P[d], R.n[d] - pdn * R.P[d]);
            }
            pcs[d][k] = pc;
            ls[d][k++] = l;
            if (l >= ext - lo) {
                pcs[d][k] = pc == R.np[d] - 1 ? 0 : pc + 1;
                ls[d][k++] = l - ext;
            }
            nd[d] = k;
        }
        for (int z = 0; z < nd[2]; ++z)
            for (int y = 0; y < nd[1]; ++y)
                for (int x = 0; x < nd[0]; ++x) {
                    const int p = pcs[0][x] + R.np[0] * (pcs[1][y] + R.np[1] * pcs[2][z]);
                    float *tile = R.jtile + (int64_t)p * 3 * jc;
                    const int64_t t = (ls[0][x] + lo) + (int64_t)R.jt[0] * ((ls[1][y] + lo) + (int64_t)R.jt[1] * (ls[2][z] + lo));
                    sx += tile[t];
                    sy += tile[jc + t];
                    sz += tile[2 * jc + t];
                    tile[t] = 0.0f;
                    tile[jc + t] = 0.0f;
                    tile[2 * jc + t] = 0.0f;
                }
        R.J[idx] = sx;
        R.J[nc + idx] = sy;
        R.J[2 * nc + idx] = sz;
        return;
    }
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

hipError_t launch_fold(const Launch &L, int64_t total, const int64_t *run_base) {
    const unsigned grid = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(k_fold, dim3(grid), dim3(256), 0, L.stream, L.runs_dev, L.n_runs, run_base, total);
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
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= total) return;
    const RunDev &R = runs[find_run(run_base, n_runs, c)];
    const int64_t idx = c - R.cell_base;
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
}

// Marder cleaning, update: E += d dt grad^+ F (the forward difference of the
// node field F lies where each E component is staggered)
__global__ void __launch_bounds__(256) k_marder_update(const RunDev *__restrict__ runs, int n_runs,
                                                       const int64_t *__restrict__ run_base, int64_t total, double d) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= total) return;
    const RunDev &R = runs[find_run(run_base, n_runs, c)];
    const int64_t idx = c - R.cell_base;
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
    const double f = F[idx];
    R.E[idx] = (float)(R.E[idx] + (F[ip] - f) * ix);
    R.E[nc + idx] = (float)(R.E[nc + idx] + (F[jp] - f) * iy);
    R.E[2 * nc + idx] = (float)(R.E[2 * nc + idx] + (F[kp] - f) * iz);
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
