// psc_capi.hip -- the C ABI: validation, workspace carving, device descriptor
// tables, call sequencing and HIP graph capture of whole time steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "psc_internal.h"

namespace psc {
size_t push_lds_bytes(int dim, int order, const int P[3], int threads, int run);
int push_occupancy(int dim, int order, int mode, int threads, int run, size_t lds);
void hilbert_patch_order(int dim, const int np[3], std::vector<int32_t> &order);
}

using namespace psc;

// LDS one workgroup may allocate on gfx950 (160 KiB per compute unit)
static constexpr size_t kMaxLds = 160 * 1024;
// adjoint tables in flight: each call fills a pinned host slot and a device
// slot of its own, so calls queue on the stream without a host wait (a slot
// is reused only after the call that last used it has finished)
static constexpr int kAdjRing = 4;
// run-table entries in flight from psc_set_particle_buffers (pinned slots,
// reused once the upload that last used them has finished)
static constexpr int kRunRing = 8;

// Library-held workspace of psc_bind_static, one per device (each device
// that loads the library holds its own copy until the process ends).  Host
// code never passes the array's name to a kernel or copy: it is a host-side
// stand-in, and the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[PSC_STATIC_WORKSPACE_BYTES];

struct psc_ctx {
    std::vector<psc_run_desc> desc;
    std::vector<RunDev> runs;   // host mirror of the device table
    int n_runs = 0, dim = 2, order = 1, chunk = 8192;
    // particle-kernel LDS bytes for a workgroup size and particles per lane
    size_t push_lds(int threads, int run) const {
        size_t m = 0;
        for (const psc_run_desc &d : desc) {
            const size_t b = push_lds_bytes(d.dim, d.order, d.patch, threads, run);
            if (b > m) m = b;
        }
        return m;
    }

    // workspace layout (offsets in bytes)
    size_t ws_bytes = 0;
    char *ws = nullptr;
    std::vector<Unit> units;
    int unit_order = PSC_ORDER_ROWMAJOR;  // patch order of the units within a run
    int64_t max_items = 0;
    int64_t total_cells = 0;
    std::vector<int64_t> run_base;       // n_runs + 1
    std::vector<int64_t> patch_base;     // n_runs + 1: first patch of each run in the flat patch space
    int max_patch_cells = 0;             // cells of the largest patch of any run
    int fold_direct_dims = 0;            // bit 1 << dim: a run of that dimension folds by patch
    bool any_jdirect = false;            // a run whose particle kernel adds into fixed-point current sums
    bool any_fold_search = false;
    int n_segs = 0;
    std::vector<int64_t> seg_base;       // n_segs + 1
    std::vector<int32_t> seg_run, seg_sp;
    int64_t total_seg_cells = 0;
    int64_t n_scan_blocks = 0;
    std::vector<int32_t> block_seg;
    std::vector<ScanSeg> segs_host[2];   // scan segments per cs_sel, filled at bind (sized at init)
    int64_t max_cap = 0, max_ncell = 0;
    size_t rsort_bytes = 0;

    struct Off {
        size_t runs, units, item_start, run_base, patch_base, seg_base, seg_run, seg_sp, segs0, segs1, scan_tmp, err;
        size_t load_keys, load_idx, load_keys_s, load_idx_s, rsort;
        size_t adj_runs;
        size_t queue, part, unit_counts;
    } off{};
    PushMode pm;                             // particle-kernel launch shape
    int max_workers = 0;
    std::vector<size_t> off_jtile, off_jacc, off_rho;
    std::vector<std::vector<size_t>> off_cs0, off_cs1, off_perm, off_mc, off_cnt, off_pre, off_tot;
    // adjoint scratch (PSC_RUN_ADJOINT)
    bool adjoint = false;
    size_t adj_lds = 0;
    int64_t adj_items = 0;                  // work items of the particle adjoint (kAdjChunk particles)
    std::vector<AdjRun> adj;                 // host mirror of the adjoint table
    RunDev *run_pinned = nullptr;            // kRunRing staged copies of the run and segment tables (pinned)
    hipEvent_t run_done[kRunRing] = {};
    uint64_t run_calls = 0;
    bool runs_dirty = false;                 // host run table changed since its last upload
    bool segs_dirty = false;                 // ... and with it the scan segments' output offsets
    AdjRun *adj_pinned = nullptr;            // kAdjRing * n_runs tables in pinned host memory
    hipEvent_t adj_done[kAdjRing] = {};      // completion of the call that last used each slot
    uint64_t adj_calls = 0;
    std::vector<size_t> off_b1, off_lj, off_gt;
    std::vector<std::vector<size_t>> off_soff, off_su, off_acs;

    int static_dev = -1;                 // device whose library-held workspace this context is bound to

    // state
    bool bound = false;
    bool stepped = false;
    std::vector<std::vector<bool>> loaded;
    int front = 0, cs_sel = 0, perm_pending = 0, mc_valid = 0;
    std::map<std::tuple<int, int, int>, hipGraphExec_t> graphs;
    hipStream_t cap_stream = nullptr;   // private stream used only to record graphs
    std::string last_error;

    template <class T>
    T *at(size_t o) const { return reinterpret_cast<T *>(ws + o); }
    uint32_t *err() const { return at<uint32_t>(off.err); }

    ~psc_ctx() {
        for (hipEvent_t &e : adj_done)
            if (e) hipEventDestroy(e);
        if (adj_pinned) hipHostFree(adj_pinned);
        for (hipEvent_t &e : run_done)
            if (e) hipEventDestroy(e);
        if (run_pinned) hipHostFree(run_pinned);
    }
};

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

psc_status fail(psc_ctx *c, psc_status s, const std::string &msg) {
    if (c) c->last_error = msg;
    return s;
}

psc_status hipfail(psc_ctx *c, hipError_t e, const char *where) {
    if (e == hipSuccess) return PSC_OK;
    if (c) c->last_error = std::string(where) + ": " + hipGetErrorString(e);
    return PSC_ERR_HIP;
}

#define HIPCHECK(call, where)                                         \
    do {                                                              \
        hipError_t e_ = (call);                                       \
        if (e_ != hipSuccess) return hipfail(ctx, e_, where);         \
    } while (0)

Launch make_launch(psc_ctx *ctx, hipStream_t s) {
    Launch L;
    L.runs_dev = ctx->at<RunDev>(ctx->off.runs);
    L.runs_host = ctx->runs.data();
    L.n_runs = ctx->n_runs;
    L.stream = s;
    L.err = ctx->err();
    return L;
}

// Upload the host run table if psc_set_particle_buffers / psc_set_sort_outputs
// changed it: one copy through a pinned staging slot, ordered on the stream,
// without a host wait (a slot is reused once its copy has completed).
// Called by every entry point that launches kernels reading the table.
static psc_status sync_runs(psc_ctx *ctx, hipStream_t s) {
    if (!ctx->runs_dirty) return PSC_OK;
    // one staging block per slot: the run table, then both segment tables
    const size_t run_bytes = sizeof(RunDev) * ctx->n_runs, seg_bytes = 2 * sizeof(ScanSeg) * ctx->n_segs;
    if (!ctx->run_pinned) {
        HIPCHECK(hipHostMalloc((void **)&ctx->run_pinned, (run_bytes + seg_bytes) * kRunRing, hipHostMallocDefault),
                 "run table staging");
        for (hipEvent_t &e : ctx->run_done) HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
    }
    const int slot = (int)(ctx->run_calls++ % kRunRing);
    HIPCHECK(hipEventSynchronize(ctx->run_done[slot]), "run table slot");
    char *staged = reinterpret_cast<char *>(ctx->run_pinned) + (run_bytes + seg_bytes) * slot;
    std::memcpy(staged, ctx->runs.data(), run_bytes);
    size_t bytes = run_bytes;
    if (ctx->segs_dirty) {
        // the scan writes the new cell offsets through the segment tables
        // (table c for cs_sel == c: into cs[1 - c])
        ScanSeg *sg = reinterpret_cast<ScanSeg *>(staged + run_bytes);
        for (int c = 0; c < 2; ++c)
            for (int g = 0; g < ctx->n_segs; ++g) {
                ScanSeg &t = ctx->segs_host[c][g];
                t.out = ctx->runs[ctx->seg_run[g]].sp[ctx->seg_sp[g]].cs[1 - c];
                sg[(size_t)c * ctx->n_segs + g] = t;
            }
        bytes += seg_bytes;
        ctx->segs_dirty = false;
    }
    HIPCHECK(hipMemcpyAsync(ctx->at<void>(ctx->off.runs), staged, bytes, hipMemcpyHostToDevice, s), "upload runs");
    HIPCHECK(hipEventRecord(ctx->run_done[slot], s), "run table event");
    ctx->runs_dirty = false;
    return PSC_OK;
}

// the (run, species, patch) units: runs one after another, each run's
// patches in row-major order or along its Hilbert curve, the species of a
// patch together
void build_units(psc_ctx *ctx) {
    ctx->units.clear();
    std::vector<int32_t> order;
    for (int r = 0; r < ctx->n_runs; ++r) {
        const RunDev &R = ctx->runs[r];
        if (ctx->unit_order == PSC_ORDER_HILBERT) {
            hilbert_patch_order(R.dim, R.np, order);
        } else {
            order.resize(R.n_patches);
            for (int p = 0; p < R.n_patches; ++p) order[p] = p;
        }
        for (int p : order)
            for (int s = 0; s < R.n_species; ++s) ctx->units.push_back(Unit{r, s, p, 0});
    }
}

// device addresses of `scratch` (taken once per device with that device
// current) and the context each device's copy is bound to
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
psc_ctx *g_scratch_owner[kMaxDevices] = {};

// work items of the particle kernel at most: every unit may start one that
// is not full, plus the chunks of every species' capacity at its run's chunk
int64_t count_items(const psc_ctx *ctx) {
    int64_t items = (int64_t)ctx->units.size();
    for (const RunDev &R : ctx->runs)
        for (int s = 0; s < R.n_species; ++s) items += (R.sp[s].cap + R.chunk - 1) / R.chunk;
    return items;
}

}  // namespace

extern "C" {

const char *psc_status_string(psc_status s) {
    switch (s) {
        case PSC_OK: return "ok";
        case PSC_ERR_INVALID: return "invalid argument";
        case PSC_ERR_CFL: return "time step violates the CFL limit";
        case PSC_ERR_LDS: return "patch tile does not fit in LDS";
        case PSC_ERR_HIP: return "HIP runtime error";
        case PSC_ERR_NONFINITE: return "non-finite particle momentum";
        case PSC_ERR_PARTICLE: return "particle moved more than one cell or has an invalid cell";
        case PSC_ERR_UNSUPPORTED: return "unsupported combination";
        case PSC_ERR_STATE: return "call out of order";
    }
    return "unknown status";
}

psc_status psc_last_error(const psc_ctx *ctx, char *buf, size_t n) {
    if (!ctx || !buf || n == 0) return PSC_ERR_INVALID;
    std::snprintf(buf, n, "%s", ctx->last_error.c_str());
    return PSC_OK;
}

psc_status psc_init_patches(const psc_run_desc *runs, int n_runs, int chunk, psc_ctx **out) {
    if (!out) return PSC_ERR_INVALID;
    *out = nullptr;
    if (!runs || n_runs < 1 || n_runs > PSC_MAX_RUNS || chunk < 0) return PSC_ERR_INVALID;
    psc_ctx *ctx = new psc_ctx();
    ctx->n_runs = n_runs;
    ctx->desc.assign(runs, runs + n_runs);
    ctx->dim = runs[0].dim;
    ctx->order = runs[0].order;
    ctx->chunk = chunk ? chunk : 8192;
    for (int r = 0; r < n_runs; ++r) {
        const psc_run_desc &d = runs[r];
        char msg[256];
        if (d.dim != ctx->dim || d.order != ctx->order) {
            std::snprintf(msg, sizeof msg, "run %d: every run of a context needs the same dim and order", r);
            psc_status s = fail(ctx, PSC_ERR_UNSUPPORTED, msg);
            delete ctx;
            return s;
        }
        bool ok = (d.dim == 2 || d.dim == 3) && (d.order == 1 || d.order == 2) && d.n_species >= 1 &&
                  d.n_species <= PSC_MAX_SPECIES && d.dt > 0.0;
        if (ok && d.dim == 2) ok = d.gdims[0] == 1 && d.patch[0] == 1;
        for (int k = 0; ok && k < 3; ++k) {
            const bool active = d.dim == 3 || k > 0;
            ok = d.patch[k] >= 1 && d.patch[k] <= d.gdims[k] && (!active || (d.gdims[k] >= 3 && d.dx[k] > 0.0));
        }
        double ncell = ok ? (double)d.gdims[0] * d.gdims[1] * d.gdims[2] : 0.0;
        if (ok && ncell >= 2147483647.0) ok = false;
        for (int s = 0; ok && s < d.n_species; ++s)
            ok = d.m[s] > 0.0 && d.capacity[s] >= 0 && d.capacity[s] <= kMaxCapacity;
        if (!ok) {
            std::snprintf(msg, sizeof msg, "run %d: invalid descriptor", r);
            psc_status s = fail(ctx, PSC_ERR_INVALID, msg);
            delete ctx;
            return s;
        }
        // the current fold gathers a cell's current from the tiles of its own
        // patch and its two neighbours, so with more than three patches along
        // a dimension every patch (the truncated last one too) must be at
        // least as wide as the tile's halo of order + 1 cells
        for (int k = (d.dim == 3 ? 0 : 1); k < 3; ++k) {
            const int np = (d.gdims[k] + d.patch[k] - 1) / d.patch[k];
            const int last = d.gdims[k] - (np - 1) * d.patch[k];
            if (np > 3 && (d.patch[k] < d.order + 1 || last < d.order + 1)) {
                std::snprintf(msg, sizeof msg, "run %d: patches along dimension %d are narrower than the current halo "
                              "(%d cells; patch %d, last patch %d)", r, k, d.order + 1, d.patch[k], last);
                psc_status s = fail(ctx, PSC_ERR_INVALID, msg);
                delete ctx;
                return s;
            }
        }
        if ((d.flags & PSC_RUN_VB) && (d.order != 1 || (d.flags & PSC_RUN_ADJOINT))) {
            std::snprintf(msg, sizeof msg, "run %d: the Villasenor-Buneman deposit is for 1st order, without adjoint", r);
            psc_status s = fail(ctx, PSC_ERR_UNSUPPORTED, msg);
            delete ctx;
            return s;
        }
        double inv2 = 0.0;
        for (int k = (d.dim == 3 ? 0 : 1); k < 3; ++k) inv2 += 1.0 / (d.dx[k] * d.dx[k]);
        if (d.dt >= 1.0 / std::sqrt(inv2)) {
            std::snprintf(msg, sizeof msg, "run %d: dt %.6g >= CFL limit %.6g", r, d.dt, 1.0 / std::sqrt(inv2));
            psc_status s = fail(ctx, PSC_ERR_CFL, msg);
            delete ctx;
            return s;
        }
        const size_t lds = push_lds_bytes(d.dim, d.order, d.patch, 256, 1);
        if (d.patch[0] > 255 || d.patch[1] > 255 || d.patch[2] > 255 || lds > kMaxLds) {
            std::snprintf(msg, sizeof msg, "run %d: patch tile needs %zu bytes of LDS (max %zu)", r, lds, kMaxLds);
            psc_status s = fail(ctx, PSC_ERR_LDS, msg);
            delete ctx;
            return s;
        }
    }

    // host mirrors and layout
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + (bytes ? bytes : 1));
        return at;
    };
    ctx->runs.resize(n_runs);
    ctx->run_base.assign(n_runs + 1, 0);
    ctx->patch_base.assign(n_runs + 1, 0);
    ctx->loaded.assign(n_runs, std::vector<bool>(PSC_MAX_SPECIES, false));
    for (int r = 0; r < n_runs; ++r) {
        const psc_run_desc &d = runs[r];
        RunDev &R = ctx->runs[r];
        std::memset(&R, 0, sizeof R);
        R.dim = d.dim;
        R.order = d.order;
        R.vb = (d.flags & PSC_RUN_VB) != 0;
        for (int k = 0; k < 3; ++k) {
            R.n[k] = d.gdims[k];
            R.P[k] = d.patch[k];
            R.np[k] = (d.gdims[k] + d.patch[k] - 1) / d.patch[k];
            const bool active = d.dim == 3 || k > 0;
            R.dx[k] = active ? (float)d.dx[k] : 1.0f;
            R.inv_dx[k] = active ? (float)(1.0 / d.dx[k]) : 0.0f;
            R.dxd[k] = active ? d.dx[k] : 1.0;
            R.jt[k] = active ? d.patch[k] + cur_lo(d.order) + cur_hi(d.order) : 1;
        }
        R.n_patches = R.np[0] * R.np[1] * R.np[2];
        R.fold_direct = 1;
        R.jdirect = (d.flags & PSC_RUN_TILE_FOLD) == 0;
        for (int k = (d.dim == 3 ? 0 : 1); k < 3; ++k) {
            const int last = d.gdims[k] - (R.np[k] - 1) * d.patch[k];
            const int halo = imax(cur_lo(d.order), cur_hi(d.order));
            if (d.patch[k] < halo || last < halo) R.fold_direct = 0;
            if (!current_direct_fits(d.gdims[k], d.patch[k], d.order)) R.jdirect = 0;
        }
        ctx->patch_base[r + 1] = ctx->patch_base[r] + R.n_patches;
        ctx->max_patch_cells = imax(ctx->max_patch_cells, d.patch[0] * d.patch[1] * d.patch[2]);
        if (R.jdirect) ctx->any_jdirect = true;
        else if (R.fold_direct) ctx->fold_direct_dims |= 1 << d.dim;
        else ctx->any_fold_search = true;
        R.n_species = d.n_species;
        R.ncell = (int64_t)d.gdims[0] * d.gdims[1] * d.gdims[2];
        R.cell_base = ctx->total_cells;
        ctx->total_cells += R.ncell;
        ctx->run_base[r + 1] = ctx->total_cells;
        R.dt = (float)d.dt;
        R.jtile_cells = (int64_t)R.jt[0] * R.jt[1] * R.jt[2];
        if (R.ncell > ctx->max_ncell) ctx->max_ncell = R.ncell;
        for (int s = 0; s < d.n_species; ++s) {
            SpeciesDev &S = R.sp[s];
            S.q = (float)d.q[s];
            S.m = (float)d.m[s];
            S.w = (float)d.w[s];
            S.qdt_2m = (float)(d.q[s] * d.dt / (2.0 * d.m[s]));
            S.qw = (float)(d.q[s] * d.w[s]);
            S.cap = d.capacity[s];
            S.n = 0;
            if (S.cap > ctx->max_cap) ctx->max_cap = S.cap;
        }
        if (R.jdirect) {
            // Fixed-point unit of the current sums: a particle adds at most
            // bound = 4 max|q w| max(dx / dt, 1) to one current component of a
            // cell in a push (an Esirkepov or Villasenor-Buneman flux of at most
            // one cell's worth, or the 2-d q w v_x term), and a cell's sum over
            // the run's particle slots stays below 2^62 units:
            // jq = bound * 2^(ceil(log2 slots) - 62), a power of two.
            double qw = 0.0, slots = 1.0, dxdt = 1.0;
            for (int s = 0; s < d.n_species; ++s) {
                qw = std::max(qw, std::fabs(d.q[s] * d.w[s]));
                slots += (double)d.capacity[s];
            }
            for (int k = (d.dim == 3 ? 0 : 1); k < 3; ++k) dxdt = std::max(dxdt, d.dx[k] / d.dt);
            const double bound = 4.0 * (qw > 0.0 ? qw : 1.0) * dxdt;   // no charge: any unit
            const int e = std::min(std::max((int)std::ceil(std::log2(bound)) + (int)std::ceil(std::log2(slots)) - 62,
                                            -1000), 1000);
            R.jq = std::ldexp(1.0, e);
            R.jinvq = std::ldexp(1.0, -e);
        }
    }
    build_units(ctx);
    for (RunDev &R : ctx->runs) R.chunk = ctx->chunk;
    ctx->max_items = count_items(ctx);

    // scan segments: one per (run, species)
    ctx->seg_base.push_back(0);
    for (int r = 0; r < n_runs; ++r)
        for (int s = 0; s < runs[r].n_species; ++s) {
            ctx->seg_run.push_back(r);
            ctx->seg_sp.push_back(s);
            ctx->runs[r].sp[s].seg = ctx->n_segs++;
            const int64_t nb = (ctx->runs[r].ncell + kScanBlock - 1) / kScanBlock;
            for (int64_t b = 0; b < nb; ++b) ctx->block_seg.push_back(ctx->n_segs - 1);
            ctx->n_scan_blocks += nb;
            ctx->total_seg_cells += ctx->runs[r].ncell;
            ctx->seg_base.push_back(ctx->total_seg_cells);
        }

    const int M = n_moves(ctx->dim);
    // the run table and the two scan-segment tables in one block (one upload)
    static_assert(sizeof(RunDev) % alignof(ScanSeg) == 0, "segment tables follow the run table");
    ctx->off.runs = take(sizeof(RunDev) * n_runs + 2 * sizeof(ScanSeg) * ctx->n_segs);
    ctx->off.segs0 = ctx->off.runs + sizeof(RunDev) * n_runs;
    ctx->off.segs1 = ctx->off.segs0 + sizeof(ScanSeg) * ctx->n_segs;
    ctx->off.units = take(sizeof(Unit) * ctx->units.size());
    ctx->off.item_start = take(sizeof(int32_t) * (ctx->units.size() + 1));
    ctx->off.run_base = take(sizeof(int64_t) * (n_runs + 1));
    ctx->off.patch_base = take(sizeof(int64_t) * (n_runs + 1));
    ctx->off.seg_base = take(sizeof(int64_t) * (ctx->n_segs + 1));
    ctx->off.seg_run = take(sizeof(int32_t) * ctx->n_segs);
    ctx->off.seg_sp = take(sizeof(int32_t) * ctx->n_segs);
    ctx->segs_host[0].resize(ctx->n_segs);
    ctx->segs_host[1].resize(ctx->n_segs);
    // block sums, block -> segment table, partial sums (kScanBlock / 256 per block)
    ctx->off.scan_tmp = take(sizeof(int32_t) * (2 + kScanBlock / 256) * ctx->n_scan_blocks);
    ctx->off.err = take(sizeof(uint32_t) * 64);
    ctx->max_workers = 256 * 16;
    ctx->off.queue = take(sizeof(int32_t) * 8 * kQueueStride);
    ctx->off.part = take(sizeof(int32_t) * (ctx->max_workers + 1));
    ctx->off.unit_counts = take(sizeof(int32_t) * ctx->units.size());
    ctx->off.load_keys = take(sizeof(int32_t) * ctx->max_cap);
    ctx->off.load_idx = take(sizeof(int32_t) * ctx->max_cap);
    ctx->off.load_keys_s = take(sizeof(int32_t) * ctx->max_cap);
    ctx->off.load_idx_s = take(sizeof(int32_t) * ctx->max_cap);
    ctx->off_jtile.resize(n_runs);
    ctx->off_jacc.resize(n_runs);
    ctx->off_rho.resize(n_runs);
    ctx->off_cs0.assign(n_runs, std::vector<size_t>(PSC_MAX_SPECIES, 0));
    ctx->off_cs1 = ctx->off_perm = ctx->off_mc = ctx->off_cnt = ctx->off_pre = ctx->off_tot = ctx->off_cs0;
    for (int r = 0; r < n_runs; ++r) {
        const RunDev &R = ctx->runs[r];
        ctx->off_jtile[r] = take(R.jdirect ? 0 : sizeof(float) * (size_t)R.n_patches * 3 * R.jtile_cells);
        ctx->off_jacc[r] = take(R.jdirect ? sizeof(long long) * 3 * (size_t)R.ncell : 0);
        ctx->off_rho[r] = take(sizeof(double) * R.ncell);
        for (int s = 0; s < R.n_species; ++s) {
            ctx->off_cs0[r][s] = take(sizeof(int32_t) * (R.ncell + 1));
            ctx->off_cs1[r][s] = take(sizeof(int32_t) * (R.ncell + 1));
            ctx->off_perm[r][s] = take(sizeof(int32_t) * R.sp[s].cap);
            ctx->off_mc[r][s] = take(R.sp[s].cap);
            ctx->off_cnt[r][s] = take(sizeof(uint16_t) * (M * R.ncell + 2));   // whole 32-bit words
            ctx->off_pre[r][s] = take(sizeof(uint16_t) * M * R.ncell);
            ctx->off_tot[r][s] = take(sizeof(int32_t) * R.ncell);
        }
    }
    // adjoint scratch
    for (int r = 0; r < n_runs; ++r) ctx->adjoint |= (runs[r].flags & PSC_RUN_ADJOINT) != 0;
    if (ctx->adjoint) {
        ctx->off.adj_runs = take(sizeof(AdjRun) * n_runs * kAdjRing);
        ctx->adj.assign(n_runs, AdjRun{});
        ctx->off_b1.resize(n_runs);
        ctx->off_lj.resize(n_runs);
        ctx->off_gt.resize(n_runs);
        ctx->off_soff = ctx->off_su = ctx->off_acs = ctx->off_cs0;
        for (int r = 0; r < n_runs; ++r) {
            const RunDev &R = ctx->runs[r];
            const size_t lds = adjoint_lds_bytes(R.dim, R.order, R.P);
            if (lds > ctx->adj_lds) ctx->adj_lds = lds;
            const int fy = R.P[1] + 1 + R.order, fz = R.P[2] + 1 + R.order;
            ctx->off_b1[r] = take(sizeof(float) * 3 * R.ncell);
            ctx->off_lj[r] = take(sizeof(float) * 3 * R.ncell);
            // 2-d: per-patch transposed-interpolation tiles, folded by k_adj_fold
            // (the 3-d kernel adds its tiles into the grid adjoints itself)
            ctx->off_gt[r] = take(R.dim == 2 ? sizeof(float) * (size_t)R.n_patches * 6 * fy * fz : 0);
            for (int s = 0; s < R.n_species; ++s) {
                ctx->off_soff[r][s] = take(sizeof(float) * R.dim * R.sp[s].cap);
                ctx->off_su[r][s] = take(sizeof(float) * 3 * R.sp[s].cap);
                ctx->off_acs[r][s] = take(sizeof(int32_t) * (R.ncell + 1));
                ctx->adj_items += (R.sp[s].cap + kAdjChunk - 1) / kAdjChunk;
            }
        }
        ctx->adj_items += (int64_t)ctx->units.size();
        if (ctx->adj_lds > kMaxLds) {
            psc_status st = fail(ctx, PSC_ERR_LDS, "adjoint patch tiles do not fit in 160 KiB of LDS");
            delete ctx;
            return st;
        }
    }
    if (ctx->adjoint) {
        hipError_t e = hipHostMalloc((void **)&ctx->adj_pinned, sizeof(AdjRun) * n_runs * kAdjRing, hipHostMallocDefault);
        for (int k = 0; k < kAdjRing && e == hipSuccess; ++k)
            e = hipEventCreateWithFlags(&ctx->adj_done[k], hipEventDisableTiming);
        if (e != hipSuccess) {
            psc_status st = hipfail(ctx, e, "adjoint table staging");
            delete ctx;
            return st;
        }
    }
    ctx->off.rsort = o;     // radix-sort temp storage goes last, sized in psc_workspace_size
    ctx->ws_bytes = o;
    *out = ctx;
    return PSC_OK;
}

psc_status psc_workspace_size(const psc_ctx *cctx, size_t *bytes) {
    psc_ctx *ctx = const_cast<psc_ctx *>(cctx);
    if (!ctx || !bytes) return PSC_ERR_INVALID;
    if (ctx->rsort_bytes == 0) {
        size_t tb = 0;
        int bits = 1;
        while ((int64_t(1) << bits) < ctx->max_ncell) ++bits;
        hipError_t e = radix_sort_pairs(nullptr, &tb, nullptr, nullptr, nullptr, nullptr,
                                        ctx->max_cap > 0 ? ctx->max_cap : 1, bits, 0);
        if (e != hipSuccess) return hipfail(ctx, e, "radix sort size query");
        ctx->rsort_bytes = align256(tb + 256);
    }
    *bytes = ctx->off.rsort + ctx->rsort_bytes;
    return PSC_OK;
}

psc_status psc_bind(psc_ctx *ctx, const psc_run_bufs *bufs, int n_runs, void *workspace, void *stream) {
    if (!ctx || !bufs || n_runs != ctx->n_runs || !workspace) return PSC_ERR_INVALID;
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(ctx, PSC_ERR_INVALID, "workspace not 256-byte aligned");
    if (ctx->rsort_bytes == 0) {
        size_t b;
        psc_status st = psc_workspace_size(ctx, &b);
        if (st != PSC_OK) return st;
    }
    if (ctx->static_dev >= 0) {   // leaves the library-held workspace for the caller's
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (g_scratch_owner[ctx->static_dev] == ctx) g_scratch_owner[ctx->static_dev] = nullptr;
        ctx->static_dev = -1;
    }
    hipStream_t s = (hipStream_t)stream;
    ctx->bound = false;
    ctx->ws = (char *)workspace;
    for (int r = 0; r < ctx->n_runs; ++r) {
        RunDev &R = ctx->runs[r];
        const psc_run_bufs &b = bufs[r];
        if (!b.E || !b.B || !b.J) return fail(ctx, PSC_ERR_INVALID, "null field buffer");
        R.E = b.E;
        R.B = b.B;
        R.J = b.J;
        R.jtile = ctx->at<float>(ctx->off_jtile[r]);
        R.jacc = ctx->at<long long>(ctx->off_jacc[r]);
        R.rho = ctx->at<double>(ctx->off_rho[r]);
        for (int sp = 0; sp < R.n_species; ++sp) {
            SpeciesDev &S = R.sp[sp];
            const bool any_id = b.id[sp][0] || b.id[sp][1];
            for (int k = 0; k < 2; ++k) {
                if (S.cap > 0 && (!b.cell[sp][k] || !b.off[sp][k] || !b.u[sp][k]))
                    return fail(ctx, PSC_ERR_INVALID, "null particle buffer");
                if (any_id && !b.id[sp][k]) return fail(ctx, PSC_ERR_INVALID, "ids must be given for both buffers");
                S.cell[k] = b.cell[sp][k];
                S.off[k] = b.off[sp][k];
                S.u[k] = b.u[sp][k];
                S.id[k] = b.id[sp][k];
            }
            S.cs[0] = ctx->at<int32_t>(ctx->off_cs0[r][sp]);
            S.cs[1] = ctx->at<int32_t>(ctx->off_cs1[r][sp]);
            S.perm[0] = S.perm[1] = ctx->at<int32_t>(ctx->off_perm[r][sp]);
            S.mc = ctx->at<uint8_t>(ctx->off_mc[r][sp]);
            S.cnt = ctx->at<uint16_t>(ctx->off_cnt[r][sp]);
            S.pre = ctx->at<uint16_t>(ctx->off_pre[r][sp]);
            S.tot = ctx->at<int32_t>(ctx->off_tot[r][sp]);
        }
    }
    std::vector<ScanSeg> &segs0 = ctx->segs_host[0], &segs1 = ctx->segs_host[1];
    {
        int64_t b0 = 0;
        for (int g = 0; g < ctx->n_segs; ++g) {
            const RunDev &R = ctx->runs[ctx->seg_run[g]];
            const SpeciesDev &S = R.sp[ctx->seg_sp[g]];
            segs0[g] = ScanSeg{S.tot, S.cs[1], R.ncell, b0};   // cs_sel 0: new offsets go to cs[1]
            segs1[g] = ScanSeg{S.tot, S.cs[0], R.ncell, b0};
            b0 += (R.ncell + kScanBlock - 1) / kScanBlock;
        }
    }
    HIPCHECK(hipMemcpyAsync(ctx->at<void>(ctx->off.runs), ctx->runs.data(), sizeof(RunDev) * ctx->n_runs,
                            hipMemcpyHostToDevice, s), "upload runs");
    HIPCHECK(hipMemcpyAsync(ctx->at<void>(ctx->off.units), ctx->units.data(), sizeof(Unit) * ctx->units.size(),
                            hipMemcpyHostToDevice, s), "upload units");
    HIPCHECK(hipMemcpyAsync(ctx->at<void>(ctx->off.run_base), ctx->run_base.data(), sizeof(int64_t) * (ctx->n_runs + 1),
                            hipMemcpyHostToDevice, s), "upload run base");
    HIPCHECK(hipMemcpyAsync(ctx->at<void>(ctx->off.patch_base), ctx->patch_base.data(),
                            sizeof(int64_t) * (ctx->n_runs + 1), hipMemcpyHostToDevice, s),
             "upload patch base");
    HIPCHECK(hipMemcpyAsync(ctx->at<void>(ctx->off.seg_base), ctx->seg_base.data(), sizeof(int64_t) * (ctx->n_segs + 1),
                            hipMemcpyHostToDevice, s), "upload seg base");
    HIPCHECK(hipMemcpyAsync(ctx->at<void>(ctx->off.seg_run), ctx->seg_run.data(), sizeof(int32_t) * ctx->n_segs,
                            hipMemcpyHostToDevice, s), "upload seg run");
    HIPCHECK(hipMemcpyAsync(ctx->at<void>(ctx->off.seg_sp), ctx->seg_sp.data(), sizeof(int32_t) * ctx->n_segs,
                            hipMemcpyHostToDevice, s), "upload seg species");
    HIPCHECK(hipMemcpyAsync(ctx->at<void>(ctx->off.segs0), segs0.data(), sizeof(ScanSeg) * ctx->n_segs,
                            hipMemcpyHostToDevice, s), "upload segs0");
    HIPCHECK(hipMemcpyAsync(ctx->at<void>(ctx->off.segs1), segs1.data(), sizeof(ScanSeg) * ctx->n_segs,
                            hipMemcpyHostToDevice, s), "upload segs1");
    ctx->runs_dirty = ctx->segs_dirty = false;   // the bound table is the one uploaded here
    HIPCHECK(hipMemcpyAsync(ctx->at<int32_t>(ctx->off.scan_tmp) + ctx->n_scan_blocks, ctx->block_seg.data(),
                            sizeof(int32_t) * ctx->n_scan_blocks, hipMemcpyHostToDevice, s), "upload block table");
    HIPCHECK(hipMemsetAsync(ctx->err(), 0, sizeof(uint32_t), s), "clear error word");
    // clear the current tiles and every cell-offset array once
    for (int r = 0; r < ctx->n_runs; ++r) {
        const RunDev &R = ctx->runs[r];
        if (R.jdirect)
            HIPCHECK(hipMemsetAsync(R.jacc, 0, sizeof(long long) * 3 * (size_t)R.ncell, s), "clear accumulators");
        else
            HIPCHECK(hipMemsetAsync(R.jtile, 0, sizeof(float) * (size_t)R.n_patches * 3 * R.jtile_cells, s),
                     "clear tiles");
        for (int sp = 0; sp < R.n_species; ++sp) {
            HIPCHECK(hipMemsetAsync(R.sp[sp].cs[0], 0, sizeof(int32_t) * (R.ncell + 1), s), "clear cs");
            HIPCHECK(hipMemsetAsync(R.sp[sp].cs[1], 0, sizeof(int32_t) * (R.ncell + 1), s), "clear cs");
            HIPCHECK(hipMemsetAsync(R.sp[sp].cnt, 0, sizeof(uint16_t) * (n_moves(R.dim) * R.ncell + 2), s),
                     "clear move counts");
        }
    }
    if (ctx->adjoint) {
        for (int r = 0; r < ctx->n_runs; ++r) {
            const RunDev &R = ctx->runs[r];
            AdjRun &A = ctx->adj[r];
            A.B1 = ctx->at<float>(ctx->off_b1[r]);
            A.LJ = ctx->at<float>(ctx->off_lj[r]);
            A.gtile = ctx->at<float>(ctx->off_gt[r]);
            const int fy = R.P[1] + 1 + R.order, fz = R.P[2] + 1 + R.order;
            if (R.dim == 2)   // the only runs with per-patch adjoint tiles
                HIPCHECK(hipMemsetAsync(A.gtile, 0, sizeof(float) * (size_t)R.n_patches * 6 * fy * fz, s),
                         "clear adj tiles");
            for (int sp = 0; sp < R.n_species; ++sp) {
                AdjSpecies &S = A.sp[sp];
                S.soff = ctx->at<float>(ctx->off_soff[r][sp]);
                S.su = ctx->at<float>(ctx->off_su[r][sp]);
                S.cs = S.cs_scratch = ctx->at<int32_t>(ctx->off_acs[r][sp]);
            }
        }
    }
    HIPCHECK(hipStreamSynchronize(s), "bind sync");
    ctx->bound = true;
    ctx->stepped = false;
    ctx->front = ctx->cs_sel = ctx->perm_pending = ctx->mc_valid = 0;
    // default launch: persistent queues with the largest workgroup that fits;
    // two particles per lane for 2-d order-2 runs, one otherwise (the
    // autotuner's choices on gfx950)
    const int run = ctx->dim == 2 && ctx->order == 2 ? 2 : 1;
    for (int threads : {512, 384, 256}) {
        if (ctx->push_lds(threads, run) > kMaxLds) continue;
        psc_status st = psc_set_launch(ctx, PSC_LAUNCH_QUEUE, 0, 0, threads, run, stream);
        if (st != PSC_ERR_LDS) return st;
    }
    return PSC_OK;
}

psc_status psc_bind_static(psc_ctx *ctx, const psc_run_bufs *bufs, int n_runs, void *stream) {
    if (!ctx || !bufs || n_runs != ctx->n_runs) return PSC_ERR_INVALID;
    size_t need = 0;
    psc_status st = psc_workspace_size(ctx, &need);
    if (st != PSC_OK) return st;
    if (need > (size_t)PSC_STATIC_WORKSPACE_BYTES)
        return fail(ctx, PSC_ERR_INVALID,
                    "the runs need " + std::to_string(need) + " bytes of workspace; the library-held workspace " +
                        "holds " + std::to_string((size_t)PSC_STATIC_WORKSPACE_BYTES) + " (use psc_bind)");
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev), "get device");
    if (dev < 0 || dev >= kMaxDevices) return fail(ctx, PSC_ERR_INVALID, "device index beyond the static table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "address of the static workspace");
        if (!p || reinterpret_cast<uintptr_t>(p) % 256) return fail(ctx, PSC_ERR_HIP, "static workspace address");
        g_scratch_ptr[dev] = p;
    }
    // the previous holder of this device's copy loses it (its workspace is
    // about to be overwritten): it must be bound again before further use
    psc_ctx *prev = g_scratch_owner[dev];
    if (prev && prev != ctx) {
        prev->bound = false;
        prev->static_dev = -1;
        prev->last_error = "the library-held workspace was bound to another context";
    }
    g_scratch_owner[dev] = nullptr;
    if (ctx->static_dev >= 0 && ctx->static_dev != dev) g_scratch_owner[ctx->static_dev] = nullptr;
    ctx->static_dev = -1;
    st = psc_bind(ctx, bufs, n_runs, g_scratch_ptr[dev], stream);
    if (st != PSC_OK) return st;
    ctx->static_dev = dev;
    g_scratch_owner[dev] = ctx;
    return PSC_OK;
}

// zero the per (cell, move) counts the particle kernel accumulates (needed
// only when a push was not followed by the sort, which clears them)
static psc_status clear_move_counts(psc_ctx *ctx, hipStream_t s) {
    for (int r = 0; r < ctx->n_runs; ++r) {
        const RunDev &R = ctx->runs[r];
        for (int sp = 0; sp < R.n_species; ++sp)
            HIPCHECK(launch_fill_i32(reinterpret_cast<int32_t *>(R.sp[sp].cnt),
                                     (n_moves(R.dim) * R.ncell + 2) / 2, 0, s),
                     "clear move counts");
    }
    return PSC_OK;
}

psc_status psc_load_particles(psc_ctx *ctx, int run, int species, int64_t n, const int32_t *gcell, const float *goff,
                              const float *gu, const int32_t *gid, void *stream) {
    if (!ctx || !ctx->bound) return PSC_ERR_STATE;
    if (run < 0 || run >= ctx->n_runs || species < 0 || species >= ctx->runs[run].n_species)
        return PSC_ERR_INVALID;
    if (ctx->stepped || ctx->front || ctx->cs_sel || ctx->perm_pending) {
        // restart: the particle state of every species lives in buffer set 0
        // again, so every species has to be loaded before the next step
        if (ctx->mc_valid) {
            psc_status st = clear_move_counts(ctx, (hipStream_t)stream);
            if (st != PSC_OK) return st;
        }
        ctx->stepped = false;
        ctx->front = ctx->cs_sel = ctx->perm_pending = ctx->mc_valid = 0;
        for (auto &v : ctx->loaded) std::fill(v.begin(), v.end(), false);
    }
    RunDev &R = ctx->runs[run];
    SpeciesDev &S = R.sp[species];
    if (n < 0 || n > S.cap) return fail(ctx, PSC_ERR_INVALID, "particle count exceeds capacity");
    if (n > 0 && (!gcell || !goff || !gu)) return PSC_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    int32_t *keys = ctx->at<int32_t>(ctx->off.load_keys), *idx = ctx->at<int32_t>(ctx->off.load_idx);
    int32_t *keys_s = ctx->at<int32_t>(ctx->off.load_keys_s), *idx_s = ctx->at<int32_t>(ctx->off.load_idx_s);
    HIPCHECK(launch_keys(R, n, gcell, keys, idx, ctx->err(), s), "load keys");
    if (n > 0) {
        int bits = 1;
        while ((int64_t(1) << bits) < R.ncell) ++bits;
        size_t tb = ctx->rsort_bytes;
        HIPCHECK(radix_sort_pairs(ctx->at<void>(ctx->off.rsort), &tb, keys, keys_s, idx, idx_s, n, bits, s), "load sort");
    }
    HIPCHECK(launch_load_gather(R, species, n, keys_s, idx_s, goff, gu, gid, s), "load gather");
    HIPCHECK(launch_cell_starts(n, R.ncell, keys_s, S.cs[0], ctx->err(), s), "load cell offsets");
    S.n = n;
    HIPCHECK(hipMemcpyAsync(ctx->at<RunDev>(ctx->off.runs) + run, &R, sizeof(RunDev), hipMemcpyHostToDevice, s),
             "upload run");
    HIPCHECK(hipStreamSynchronize(s), "load sync");
    ctx->loaded[run][species] = true;
    return PSC_OK;
}

psc_status psc_load_sorted(psc_ctx *ctx, int run, int species, int64_t n, const int32_t *key, const float *off,
                           const float *u, const int32_t *id, void *stream) {
    if (!ctx || !ctx->bound) return PSC_ERR_STATE;
    if (run < 0 || run >= ctx->n_runs || species < 0 || species >= ctx->runs[run].n_species)
        return PSC_ERR_INVALID;
    if (ctx->stepped || ctx->front || ctx->cs_sel || ctx->perm_pending) {
        // restart, as psc_load_particles
        if (ctx->mc_valid) {
            psc_status st = clear_move_counts(ctx, (hipStream_t)stream);
            if (st != PSC_OK) return st;
        }
        ctx->stepped = false;
        ctx->front = ctx->cs_sel = ctx->perm_pending = ctx->mc_valid = 0;
        for (auto &v : ctx->loaded) std::fill(v.begin(), v.end(), false);
    }
    RunDev &R = ctx->runs[run];
    SpeciesDev &S = R.sp[species];
    if (n < 0 || n > S.cap) return fail(ctx, PSC_ERR_INVALID, "particle count exceeds capacity");
    if (n > 0 && (!key || !off || !u)) return PSC_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    if (n > 0) {
        const size_t row = sizeof(float) * (size_t)n, pitch = sizeof(float) * (size_t)S.cap;
        HIPCHECK(hipMemcpyAsync(S.cell[0], key, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s), "load keys");
        HIPCHECK(hipMemcpy2DAsync(S.off[0], pitch, off, row, row, R.dim, hipMemcpyDeviceToDevice, s), "load offsets");
        HIPCHECK(hipMemcpy2DAsync(S.u[0], pitch, u, row, row, 3, hipMemcpyDeviceToDevice, s), "load momenta");
        if (S.id[0]) {
            if (id) HIPCHECK(hipMemcpyAsync(S.id[0], id, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s), "load ids");
            else HIPCHECK(launch_iota(S.id[0], n, s), "load ids");
        }
    }
    HIPCHECK(launch_cell_starts(n, R.ncell, S.cell[0], S.cs[0], ctx->err(), s), "load cell offsets");
    S.n = n;
    HIPCHECK(hipMemcpyAsync(ctx->at<RunDev>(ctx->off.runs) + run, &R, sizeof(RunDev), hipMemcpyHostToDevice, s),
             "upload run");
    HIPCHECK(hipStreamSynchronize(s), "load sync");
    ctx->loaded[run][species] = true;
    return PSC_OK;
}

static psc_status require_loaded(psc_ctx *ctx) {
    if (!ctx || !ctx->bound) return PSC_ERR_STATE;
    for (int r = 0; r < ctx->n_runs; ++r)
        for (int s = 0; s < ctx->runs[r].n_species; ++s)
            if (!ctx->loaded[r][s]) return fail(ctx, PSC_ERR_STATE, "species not loaded");
    return PSC_OK;
}

psc_status psc_push_fields(psc_ctx *ctx, int op, void *stream) {
    if (!ctx || !ctx->bound) return PSC_ERR_STATE;
    if (op != PSC_B_HALF && op != PSC_E_FULL) return PSC_ERR_INVALID;
    if (psc_status rs = sync_runs(ctx, (hipStream_t)stream); rs != PSC_OK) return rs;
    Launch L = make_launch(ctx, (hipStream_t)stream);
    HIPCHECK(launch_fields(L, op, ctx->total_cells, ctx->at<int64_t>(ctx->off.run_base)), "push fields");
    return PSC_OK;
}

psc_status psc_push_particles(psc_ctx *ctx, void *stream) {
    psc_status st = require_loaded(ctx);
    if (st != PSC_OK) return st;
    if (ctx->mc_valid && (st = clear_move_counts(ctx, (hipStream_t)stream)) != PSC_OK) return st;
    if (psc_status rs = sync_runs(ctx, (hipStream_t)stream); rs != PSC_OK) return rs;
    Launch L = make_launch(ctx, (hipStream_t)stream);
    PushMode pm = ctx->pm;
    pm.queue = ctx->at<int32_t>(ctx->off.queue);
    pm.part = ctx->at<int32_t>(ctx->off.part);
    HIPCHECK(launch_push(L, ctx->at<Unit>(ctx->off.units), (int)ctx->units.size(),
                         ctx->at<int32_t>(ctx->off.item_start), ctx->max_items, ctx->dim, ctx->order,
                         ctx->front, ctx->cs_sel, ctx->perm_pending, ctx->push_lds(pm.threads, pm.run), pm),
             "push particles");
    ctx->front = 1 - ctx->front;
    ctx->perm_pending = 0;
    ctx->mc_valid = 1;
    ctx->stepped = true;
    return PSC_OK;
}

psc_status psc_deposit_current(psc_ctx *ctx, void *stream) {
    if (!ctx || !ctx->bound) return PSC_ERR_STATE;
    if (psc_status rs = sync_runs(ctx, (hipStream_t)stream); rs != PSC_OK) return rs;
    Launch L = make_launch(ctx, (hipStream_t)stream);
    if (ctx->any_jdirect)
        HIPCHECK(launch_finish_current(L, ctx->total_cells, ctx->at<int64_t>(ctx->off.run_base)), "finish current");
    if (ctx->fold_direct_dims == 0 && !ctx->any_fold_search) return PSC_OK;   // no run keeps tiles
    HIPCHECK(launch_fold(L, ctx->total_cells, ctx->at<int64_t>(ctx->off.run_base), ctx->patch_base[ctx->n_runs],
                         ctx->at<int64_t>(ctx->off.patch_base), ctx->max_patch_cells, ctx->fold_direct_dims,
                         ctx->any_fold_search),
             "deposit current");
    return PSC_OK;
}

psc_status psc_sort(psc_ctx *ctx, void *stream) {
    psc_status st = require_loaded(ctx);
    if (st != PSC_OK) return st;
    if (!ctx->mc_valid) return fail(ctx, PSC_ERR_STATE, "psc_sort needs a preceding psc_push_particles");
    if (psc_status rs = sync_runs(ctx, (hipStream_t)stream); rs != PSC_OK) return rs;
    Launch L = make_launch(ctx, (hipStream_t)stream);
    HIPCHECK(launch_sort(L, ctx->at<int64_t>(ctx->off.seg_base), ctx->at<int32_t>(ctx->off.seg_run),
                         ctx->at<int32_t>(ctx->off.seg_sp), ctx->n_segs, ctx->total_seg_cells,
                         ctx->at<ScanSeg>(ctx->cs_sel == 0 ? ctx->off.segs0 : ctx->off.segs1), ctx->n_scan_blocks,
                         ctx->at<int32_t>(ctx->off.scan_tmp), ctx->cs_sel, ctx->dim),
             "sort");
    ctx->cs_sel = 1 - ctx->cs_sel;
    ctx->perm_pending = 1;
    ctx->mc_valid = 0;
    return PSC_OK;
}

psc_status psc_sort_radix(psc_ctx *ctx, void *stream) {
    psc_status st = require_loaded(ctx);
    if (st != PSC_OK) return st;
    if (!ctx->mc_valid) return fail(ctx, PSC_ERR_STATE, "psc_sort_radix needs a preceding psc_push_particles");
    hipStream_t s = (hipStream_t)stream;
    int32_t *idx = ctx->at<int32_t>(ctx->off.load_idx), *keys_s = ctx->at<int32_t>(ctx->off.load_keys_s);
    for (int r = 0; r < ctx->n_runs; ++r) {
        const RunDev &R = ctx->runs[r];
        int bits = 1;
        while ((int64_t(1) << bits) < R.ncell) ++bits;
        for (int sp = 0; sp < R.n_species; ++sp) {
            const SpeciesDev &S = R.sp[sp];
            if (S.n > 0) {
                HIPCHECK(launch_iota(idx, S.n, s), "radix sort indices");
                size_t tb = ctx->rsort_bytes;
                HIPCHECK(radix_sort_pairs(ctx->at<void>(ctx->off.rsort), &tb, S.cell[ctx->front], keys_s, idx, S.perm[1 - ctx->cs_sel],
                                          S.n, bits, s),
                         "radix sort");
            }
            HIPCHECK(launch_cell_starts(S.n, R.ncell, keys_s, S.cs[1 - ctx->cs_sel], ctx->err(), s),
                     "radix sort offsets");
        }
    }
    // the per (cell, move) counts of the push are consumed by psc_sort only
    if ((st = clear_move_counts(ctx, s)) != PSC_OK) return st;
    ctx->cs_sel = 1 - ctx->cs_sel;
    ctx->perm_pending = 1;
    ctx->mc_valid = 0;
    return PSC_OK;
}

static psc_status one_step(psc_ctx *ctx, void *stream) {
    psc_status st;
    if ((st = psc_push_fields(ctx, PSC_B_HALF, stream)) != PSC_OK) return st;
    if ((st = psc_push_particles(ctx, stream)) != PSC_OK) return st;
    if ((st = psc_push_fields(ctx, PSC_B_HALF, stream)) != PSC_OK) return st;
    if ((st = psc_deposit_current(ctx, stream)) != PSC_OK) return st;
    if ((st = psc_push_fields(ctx, PSC_E_FULL, stream)) != PSC_OK) return st;
    return psc_sort(ctx, stream);
}

psc_status psc_step(psc_ctx *ctx, int nsteps, int use_graph, void *stream) {
    psc_status st = require_loaded(ctx);
    if (st != PSC_OK) return st;
    if (nsteps < 0) return PSC_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    if ((st = sync_runs(ctx, s)) != PSC_OK) return st;   // before any capture
    for (int k = 0; k < nsteps; ++k) {
        if (!use_graph) {
            if ((st = one_step(ctx, stream)) != PSC_OK) return st;
            continue;
        }
        const auto key = std::make_tuple(ctx->front, ctx->cs_sel, ctx->perm_pending);
        auto it = ctx->graphs.find(key);
        if (it == ctx->graphs.end()) {
            const int f = ctx->front, c = ctx->cs_sel, p = ctx->perm_pending, m = ctx->mc_valid;
            const bool was_stepped = ctx->stepped;
            // record on a private stream (the caller's may be the legacy null
            // stream, which cannot be captured); recording runs nothing
            if (!ctx->cap_stream) HIPCHECK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking), "capture stream");
            HIPCHECK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
            st = one_step(ctx, (void *)ctx->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
            if (st != PSC_OK) return st;
            if (e != hipSuccess) return hipfail(ctx, e, "end capture");
            hipGraphExec_t ex = nullptr;
            e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            if (e != hipSuccess) return hipfail(ctx, e, "graph instantiate");
            it = ctx->graphs.emplace(key, ex).first;
            // capture recorded the work without running it: restore the state
            ctx->front = f;
            ctx->cs_sel = c;
            ctx->perm_pending = p;
            ctx->mc_valid = m;
            ctx->stepped = was_stepped;
        }
        HIPCHECK(hipGraphLaunch(it->second, s), "graph launch");
        ctx->front = 1 - ctx->front;
        ctx->cs_sel = 1 - ctx->cs_sel;
        ctx->perm_pending = 1;
        ctx->mc_valid = 0;
        ctx->stepped = true;
    }
    return PSC_OK;
}

psc_status psc_get_particles(psc_ctx *ctx, int run, int species, int32_t *cell, float *off, float *u, int32_t *id,
                             void *stream) {
    if (!ctx || !ctx->bound) return PSC_ERR_STATE;
    if (run < 0 || run >= ctx->n_runs || species < 0 || species >= ctx->runs[run].n_species) return PSC_ERR_INVALID;
    const SpeciesDev &Sg = ctx->runs[run].sp[species];
    HIPCHECK(launch_get(ctx->runs[run], species, ctx->front, ctx->perm_pending ? Sg.perm[ctx->cs_sel] : nullptr, cell, off,
                        u, id, (hipStream_t)stream),
             "get particles");
    return PSC_OK;
}

psc_status psc_keys_to_cells(psc_ctx *ctx, int run, int64_t n, const int32_t *keys, int32_t *cells, void *stream) {
    if (!ctx || run < 0 || run >= ctx->n_runs || n < 0 || (n > 0 && (!keys || !cells))) return PSC_ERR_INVALID;
    HIPCHECK(launch_keys_to_cells(ctx->runs[run], n, keys, cells, (hipStream_t)stream), "keys to cells");
    return PSC_OK;
}

psc_status psc_particle_count(const psc_ctx *ctx, int run, int species, int64_t *n) {
    if (!ctx || !n || run < 0 || run >= ctx->n_runs || species < 0 || species >= ctx->runs[run].n_species)
        return PSC_ERR_INVALID;
    *n = ctx->runs[run].sp[species].n;
    return PSC_OK;
}

psc_status psc_front(const psc_ctx *ctx, int *front, int *perm_pending) {
    if (!ctx) return PSC_ERR_INVALID;
    if (front) *front = ctx->front;
    if (perm_pending) *perm_pending = ctx->perm_pending;
    return PSC_OK;
}

psc_status psc_sort_view(const psc_ctx *ctx, int run, int species, const int32_t **perm, const int32_t **cell_start) {
    if (!ctx || !ctx->bound || run < 0 || run >= ctx->n_runs || species < 0 || species >= ctx->runs[run].n_species)
        return PSC_ERR_INVALID;
    if (perm) *perm = ctx->runs[run].sp[species].perm[ctx->cs_sel];
    if (cell_start) *cell_start = ctx->runs[run].sp[species].cs[ctx->cs_sel];
    return PSC_OK;
}

psc_status psc_diagnostics(psc_ctx *ctx, double *out_dev, double *gauss_dev, void *stream) {
    if (!ctx || !ctx->bound || !out_dev) return PSC_ERR_INVALID;
    if (psc_status rs = sync_runs(ctx, (hipStream_t)stream); rs != PSC_OK) return rs;
    Launch L = make_launch(ctx, (hipStream_t)stream);
    HIPCHECK(launch_diag(L, out_dev, gauss_dev, ctx->total_cells, ctx->at<int64_t>(ctx->off.run_base), ctx->front),
             "diagnostics");
    return PSC_OK;
}

psc_status psc_marder(psc_ctx *ctx, const double *ref, double d, int iters, void *stream) {
    psc_status st = require_loaded(ctx);
    if (st != PSC_OK) return st;
    if (iters < 0 || !(d > 0.0)) return PSC_ERR_INVALID;
    if (ctx->mc_valid) return fail(ctx, PSC_ERR_STATE, "psc_marder runs between steps, not after a bare push");
    for (const psc_run_desc &r : ctx->desc) {
        double lap = 0.0;
        for (int k = (r.dim == 3 ? 0 : 1); k < 3; ++k) lap += 4.0 / (r.dx[k] * r.dx[k]);
        if (d * r.dt * lap > 2.0) return fail(ctx, PSC_ERR_INVALID, "Marder coefficient above the stability bound");
    }
    if (psc_status rs = sync_runs(ctx, (hipStream_t)stream); rs != PSC_OK) return rs;
    Launch L = make_launch(ctx, (hipStream_t)stream);
    HIPCHECK(launch_marder(L, ref, d, iters, ctx->total_cells, ctx->at<int64_t>(ctx->off.run_base), ctx->front),
             "marder");
    return PSC_OK;
}

psc_status psc_partition(const double *L, int n_patches, const double *C, int n_ranks, int32_t *N) {
    if (!L || !C || !N || n_patches < 0 || n_ranks < 1) return PSC_ERR_INVALID;
    // App. A: walk the patches along the curve, tentatively adding each to
    // rank r.  The appendix never resets the running load when it moves to
    // the next rank, so the running load is cumulative and is compared with
    // the cumulative target T_hat * (C_0 + ... + C_r) of ranks 0..r (a
    // per-rank target against a cumulative load could not work; a per-rank
    // target with a per-rank load would pass every boundary's rounding on
    // to the last rank).  At the patch that crosses the target it stays on r
    // or opens r + 1, whichever leaves the boundary closer to the target (a
    // rank keeps at least one patch); once only as many patches as ranks
    // remain, each remaining rank gets one.  The last rank takes the rest.
    double ltot = 0.0, ctot = 0.0;
    for (int p = 0; p < n_patches; ++p) ltot += L[p];
    for (int r = 0; r < n_ranks; ++r) {
        if (!(C[r] > 0.0)) return PSC_ERR_INVALID;
        ctot += C[r];
        N[r] = 0;
    }
    const double that = ltot / ctot;
    int r = 0, ncur = 0;
    double lcur = 0.0, tdone = 0.0;   // cumulative load so far, cumulative target of ranks < r
    for (int p = 0; p < n_patches; ++p) {
        lcur += L[p];
        ncur += 1;
        if (r < n_ranks - 1) {
            const double tcur = tdone + that * C[r];
            if (lcur > tcur || n_ranks - r >= n_patches - p) {
                const double above = lcur - tcur;
                const double below = tcur - (lcur - L[p]);
                if (above > below && ncur > 1) {
                    N[r] = ncur - 1;   // patch p opens the next rank
                    ncur = 1;
                } else {
                    N[r] = ncur;       // patch p closes this rank
                    ncur = 0;
                }
                tdone = tcur;
                ++r;
            }
        }
        if (p == n_patches - 1) N[n_ranks - 1] += ncur;
    }
    return PSC_OK;
}

psc_status psc_balance(psc_ctx *ctx, double cell_cost, void *stream) {
    psc_status st = require_loaded(ctx);
    if (st != PSC_OK) return st;
    const int workers = ctx->pm.workers;
    if (workers < 1) return fail(ctx, PSC_ERR_STATE, "psc_balance needs a persistent launch shape");
    hipStream_t s = (hipStream_t)stream;
    if (psc_status rs = sync_runs(ctx, s); rs != PSC_OK) return rs;
    Launch L = make_launch(ctx, s);
    const int nu = (int)ctx->units.size();
    HIPCHECK(launch_unit_counts(L, ctx->at<Unit>(ctx->off.units), nu, ctx->cs_sel, ctx->at<int32_t>(ctx->off.unit_counts)),
             "unit counts");
    std::vector<int32_t> cnt(nu);
    HIPCHECK(hipMemcpyAsync(cnt.data(), ctx->at<int32_t>(ctx->off.unit_counts), sizeof(int32_t) * nu,
                            hipMemcpyDeviceToHost, s), "read unit counts");
    HIPCHECK(hipStreamSynchronize(s), "balance sync");
    std::vector<double> load(nu), cap(workers, 1.0);
    for (int u = 0; u < nu; ++u) {
        const Unit &U = ctx->units[u];
        const RunDev &R = ctx->runs[U.run];
        int pc[3];
        patch_coords(R, U.patch, pc);
        const double cells = (double)patch_ext(R, 0, pc[0]) * patch_ext(R, 1, pc[1]) * patch_ext(R, 2, pc[2]);
        load[u] = cnt[u] + cell_cost * cells;
    }
    std::vector<int32_t> N(workers);
    st = psc_partition(load.data(), nu, cap.data(), workers, N.data());
    if (st != PSC_OK) return st;
    std::vector<int32_t> part(workers + 1, 0);
    for (int w = 0; w < workers; ++w) part[w + 1] = part[w] + N[w];
    HIPCHECK(hipMemcpyAsync(ctx->at<int32_t>(ctx->off.part), part.data(), sizeof(int32_t) * (workers + 1),
                            hipMemcpyHostToDevice, s), "upload partition");
    HIPCHECK(hipStreamSynchronize(s), "balance sync");
    return PSC_OK;
}

psc_status psc_set_launch(psc_ctx *ctx, int mode, int chunk, int workers, int threads, int run, void *stream) {
    if (!ctx || !ctx->bound || mode < 0 || mode > 2 || chunk < 0 || workers < 0 || workers > ctx->max_workers ||
        (threads != 0 && threads != 256 && threads != 384 && threads != 512) || run < 0 || run > 2)
        return PSC_ERR_INVALID;
    if (ctx->push_lds(threads ? threads : ctx->pm.threads, run ? run : ctx->pm.run) > kMaxLds) return PSC_ERR_LDS;
    if (threads) ctx->pm.threads = threads;
    if (run) ctx->pm.run = run;
    if (chunk > 0) {   // every run's chunk
        bool change = false;
        for (RunDev &R : ctx->runs) {
            change = change || R.chunk != chunk;
            R.chunk = chunk;
        }
        ctx->chunk = chunk;
        ctx->max_items = count_items(ctx);
        if (change) {
            hipStream_t s = (hipStream_t)stream;
            HIPCHECK(hipMemcpyAsync(ctx->at<void>(ctx->off.runs), ctx->runs.data(), sizeof(RunDev) * ctx->n_runs,
                                    hipMemcpyHostToDevice, s), "upload runs");
            HIPCHECK(hipStreamSynchronize(s), "launch sync");
        }
    }
    if (mode != 0 && workers == 0) {
        int dev = 0, cus = 0;
        HIPCHECK(hipGetDevice(&dev), "get device");
        HIPCHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
        int per = push_occupancy(ctx->dim, ctx->order, mode, ctx->pm.threads, ctx->pm.run,
                                 ctx->push_lds(ctx->pm.threads, ctx->pm.run));
        if (per < 1) per = 1;
        workers = cus * per;
        if (workers > ctx->max_workers) workers = ctx->max_workers;
    }
    ctx->pm.mode = mode;
    ctx->pm.workers = mode == 0 ? 0 : workers;
    for (auto &kv : ctx->graphs) hipGraphExecDestroy(kv.second);
    ctx->graphs.clear();
    if (mode == 2) {
        psc_status st = psc_balance(ctx, 1.0, stream);
        if (st != PSC_OK) return st;
    }
    return PSC_OK;
}

psc_status psc_set_run_chunk(psc_ctx *ctx, int run, int chunk, void *stream) {
    if (!ctx || !ctx->bound || run < 0 || run >= ctx->n_runs || chunk < 1) return PSC_ERR_INVALID;
    if (ctx->runs[run].chunk == chunk) return PSC_OK;
    hipStream_t s = (hipStream_t)stream;
    ctx->runs[run].chunk = chunk;
    ctx->max_items = count_items(ctx);
    HIPCHECK(hipMemcpyAsync(ctx->at<RunDev>(ctx->off.runs) + run, &ctx->runs[run], sizeof(RunDev),
                            hipMemcpyHostToDevice, s), "upload run");
    HIPCHECK(hipStreamSynchronize(s), "run chunk sync");
    for (auto &kv : ctx->graphs) hipGraphExecDestroy(kv.second);
    ctx->graphs.clear();
    if (ctx->pm.mode == 2) return psc_balance(ctx, 1.0, stream);
    return PSC_OK;
}

psc_status psc_set_unit_order(psc_ctx *ctx, int order, void *stream) {
    if (!ctx || !ctx->bound || (order != PSC_ORDER_ROWMAJOR && order != PSC_ORDER_HILBERT)) return PSC_ERR_INVALID;
    if (order == ctx->unit_order) return PSC_OK;
    hipStream_t s = (hipStream_t)stream;
    ctx->unit_order = order;
    build_units(ctx);
    HIPCHECK(hipMemcpyAsync(ctx->at<void>(ctx->off.units), ctx->units.data(), sizeof(Unit) * ctx->units.size(),
                            hipMemcpyHostToDevice, s), "upload units");
    HIPCHECK(hipStreamSynchronize(s), "unit order sync");
    for (auto &kv : ctx->graphs) hipGraphExecDestroy(kv.second);
    ctx->graphs.clear();
    if (ctx->pm.mode == 2) return psc_balance(ctx, 1.0, stream);
    return PSC_OK;
}

psc_status psc_get_cell_offsets(psc_ctx *ctx, int run, int species, int32_t *out, void *stream) {
    if (!ctx || !ctx->bound || run < 0 || run >= ctx->n_runs || species < 0 || species >= ctx->runs[run].n_species ||
        !out)
        return PSC_ERR_INVALID;
    const RunDev &R = ctx->runs[run];
    HIPCHECK(hipMemcpyAsync(out, R.sp[species].cs[ctx->cs_sel], sizeof(int32_t) * (R.ncell + 1),
                            hipMemcpyDeviceToDevice, (hipStream_t)stream),
             "copy cell offsets");
    return PSC_OK;
}

psc_status psc_set_particle_buffers(psc_ctx *ctx, int run, int species, int set, int32_t *cell, float *off, float *u,
                                    int32_t *id, void *stream) {
    if (!ctx || !ctx->bound || run < 0 || run >= ctx->n_runs || species < 0 || species >= ctx->runs[run].n_species ||
        set < 0 || set > 1)
        return PSC_ERR_INVALID;
    RunDev &R = ctx->runs[run];
    SpeciesDev &S = R.sp[species];
    if (S.cap > 0 && (!cell || !off || !u)) return fail(ctx, PSC_ERR_INVALID, "null particle buffer");
    if ((id != nullptr) != (S.id[set] != nullptr))
        return fail(ctx, PSC_ERR_INVALID, "ids must be given exactly when the context carries them");
    (void)stream;
    S.cell[set] = cell;
    S.off[set] = off;
    S.u[set] = u;
    S.id[set] = id;
    ctx->runs_dirty = true;   // uploaded before the next launch
    for (auto &kv : ctx->graphs) hipGraphExecDestroy(kv.second);
    ctx->graphs.clear();
    return PSC_OK;
}

psc_status psc_set_sort_outputs(psc_ctx *ctx, int run, int species, int32_t *perm, int32_t *cs, void *stream) {
    if (!ctx || !ctx->bound || run < 0 || run >= ctx->n_runs || species < 0 || species >= ctx->runs[run].n_species ||
        (perm == nullptr) != (cs == nullptr))
        return PSC_ERR_INVALID;
    RunDev &R = ctx->runs[run];
    SpeciesDev &S = R.sp[species];
    hipStream_t s = (hipStream_t)stream;
    if (perm) {
        S.perm[1 - ctx->cs_sel] = perm;
        S.cs[1 - ctx->cs_sel] = cs;
    } else {
        // back to the workspace's arrays, keeping the current offsets and
        // the pending permutation
        int32_t *ws_perm = ctx->at<int32_t>(ctx->off_perm[run][species]);
        int32_t *ws_cs[2] = {ctx->at<int32_t>(ctx->off_cs0[run][species]), ctx->at<int32_t>(ctx->off_cs1[run][species])};
        const int c = ctx->cs_sel;
        if (S.cs[c] != ws_cs[c])
            HIPCHECK(hipMemcpyAsync(ws_cs[c], S.cs[c], sizeof(int32_t) * (R.ncell + 1), hipMemcpyDeviceToDevice, s),
                     "keep cell offsets");
        if (ctx->perm_pending && S.perm[c] != ws_perm && S.n > 0)
            HIPCHECK(hipMemcpyAsync(ws_perm, S.perm[c], sizeof(int32_t) * S.n, hipMemcpyDeviceToDevice, s),
                     "keep permutation");
        S.perm[0] = S.perm[1] = ws_perm;
        S.cs[0] = ws_cs[0];
        S.cs[1] = ws_cs[1];
    }
    ctx->runs_dirty = ctx->segs_dirty = true;   // uploaded before the next launch
    for (auto &kv : ctx->graphs) hipGraphExecDestroy(kv.second);
    ctx->graphs.clear();
    return PSC_OK;
}

psc_status psc_get_perm(psc_ctx *ctx, int run, int species, int32_t *perm, void *stream) {
    if (!ctx || !ctx->bound || run < 0 || run >= ctx->n_runs || species < 0 || species >= ctx->runs[run].n_species ||
        !perm)
        return PSC_ERR_INVALID;
    if (!ctx->perm_pending) return fail(ctx, PSC_ERR_STATE, "no permutation: psc_sort has not run since the last push");
    const SpeciesDev &S = ctx->runs[run].sp[species];
    HIPCHECK(hipMemcpyAsync(perm, S.perm[ctx->cs_sel], sizeof(int32_t) * S.n, hipMemcpyDeviceToDevice, (hipStream_t)stream),
             "copy permutation");
    return PSC_OK;
}

psc_status psc_adjoint_step(psc_ctx *ctx, const psc_adj_fwd *fwd, const psc_adj_state *adj, void *stream) {
    if (!ctx || !ctx->bound || !fwd || !adj) return PSC_ERR_INVALID;
    if (!ctx->adjoint) return fail(ctx, PSC_ERR_STATE, "context was created without PSC_RUN_ADJOINT");
    for (int r = 0; r < ctx->n_runs; ++r)
        if (ctx->runs[r].vb)
            return fail(ctx, PSC_ERR_UNSUPPORTED, "the adjoint step differentiates the Esirkepov deposit");
    hipStream_t s = (hipStream_t)stream;
    for (int r = 0; r < ctx->n_runs; ++r) {
        const RunDev &R = ctx->runs[r];
        AdjRun &A = ctx->adj[r];
        if (!fwd[r].E || !fwd[r].B || !adj[r].lE || !adj[r].lB) return PSC_ERR_INVALID;
        A.E = fwd[r].E;
        A.B = fwd[r].B;
        A.lE = adj[r].lE;
        A.lB = adj[r].lB;
        for (int sp = 0; sp < R.n_species; ++sp) {
            AdjSpecies &S = A.sp[sp];
            S.n = R.sp[sp].n;
            if (S.n > 0 && (!fwd[r].cell[sp] || !fwd[r].off[sp] || !fwd[r].u[sp] || !fwd[r].perm[sp] ||
                            !adj[r].loff[sp] || !adj[r].lu[sp]))
                return PSC_ERR_INVALID;
            S.key = fwd[r].cell[sp];
            S.off = fwd[r].off[sp];
            S.u = fwd[r].u[sp];
            S.perm = fwd[r].perm[sp];
            S.rperm = fwd[r].read_perm[sp];
            S.stride = fwd[r].stride[sp] > 0 ? fwd[r].stride[sp] : S.n;
            if (S.rperm && S.stride < S.n) return fail(ctx, PSC_ERR_INVALID, "forward buffer stride below n");
            S.cs = fwd[r].cell_start[sp] ? fwd[r].cell_start[sp] : S.cs_scratch;
            S.loff = adj[r].loff[sp];
            S.lu = adj[r].lu[sp];
        }
    }
    const int slot = (int)(ctx->adj_calls++ % kAdjRing);
    HIPCHECK(hipEventSynchronize(ctx->adj_done[slot]), "adjoint table slot");   // done long ago
    AdjRun *host = ctx->adj_pinned + (size_t)slot * ctx->n_runs;
    AdjRun *dev = ctx->at<AdjRun>(ctx->off.adj_runs) + (size_t)slot * ctx->n_runs;
    std::copy(ctx->adj.begin(), ctx->adj.end(), host);
    HIPCHECK(hipMemcpyAsync(dev, host, sizeof(AdjRun) * ctx->n_runs, hipMemcpyHostToDevice, s),
             "upload adjoint table");
    if (psc_status rs = sync_runs(ctx, s); rs != PSC_OK) return rs;
    Launch L = make_launch(ctx, s);
    HIPCHECK(launch_adjoint(L, dev, ctx->adj.data(), ctx->at<Unit>(ctx->off.units),
                            (int)ctx->units.size(), ctx->at<int32_t>(ctx->off.item_start), ctx->adj_items, kAdjChunk,
                            ctx->dim, ctx->order, ctx->total_cells, ctx->at<int64_t>(ctx->off.run_base), ctx->adj_lds, s),
             "adjoint step");
    HIPCHECK(hipEventRecord(ctx->adj_done[slot], s), "adjoint step event");
    return PSC_OK;
}

psc_status psc_adjoint_seed(psc_ctx *ctx, const psc_adj_state *adj, void *stream) {
    if (!ctx || !ctx->bound || !adj) return PSC_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    for (int r = 0; r < ctx->n_runs; ++r) {
        const RunDev &R = ctx->runs[r];
        const psc_run_desc &d = ctx->desc[r];
        if (!adj[r].lE || !adj[r].lB) return PSC_ERR_INVALID;
        const double dV = d.dx[1] * d.dx[2] * (R.dim == 3 ? d.dx[0] : 1.0);
        HIPCHECK(launch_adj_seed(R.E, R.B, adj[r].lE, adj[r].lB, 3 * R.ncell, (float)dV, s), "adjoint seed");
        for (int sp = 0; sp < R.n_species; ++sp) {
            const int64_t n = R.sp[sp].n;
            if (n == 0) continue;
            if (!adj[r].loff[sp] || !adj[r].lu[sp]) return PSC_ERR_INVALID;
            HIPCHECK(launch_fill_i32(reinterpret_cast<int32_t *>(adj[r].loff[sp]), R.dim * n, 0, s), "adjoint seed");
            HIPCHECK(launch_fill_i32(reinterpret_cast<int32_t *>(adj[r].lu[sp]), 3 * n, 0, s), "adjoint seed");
        }
    }
    return PSC_OK;
}

psc_status psc_check(psc_ctx *ctx, void *stream, uint32_t *word, int clear) {
    if (!ctx || !ctx->bound) return PSC_ERR_STATE;
    hipStream_t s = (hipStream_t)stream;
    HIPCHECK(hipStreamSynchronize(s), "check sync");
    uint32_t w = 0;
    HIPCHECK(hipMemcpy(&w, ctx->err(), sizeof w, hipMemcpyDeviceToHost), "read error word");
    if (clear) HIPCHECK(hipMemset(ctx->err(), 0, sizeof(uint32_t)), "clear error word");
    if (word) *word = w;
    if (w & PSC_DEV_NONFINITE) return fail(ctx, PSC_ERR_NONFINITE, "non-finite momentum");
    if (w & (PSC_DEV_MOVE | PSC_DEV_KEY | PSC_DEV_OVERFULL))
        return fail(ctx, PSC_ERR_PARTICLE, "particle moved too far, had a bad key, or a cell overflowed");
    return PSC_OK;
}

psc_status psc_destroy(psc_ctx *ctx) {
    if (!ctx) return PSC_ERR_INVALID;
    if (ctx->static_dev >= 0) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (g_scratch_owner[ctx->static_dev] == ctx) g_scratch_owner[ctx->static_dev] = nullptr;
    }
    for (auto &kv : ctx->graphs) hipGraphExecDestroy(kv.second);
    if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return PSC_OK;
}

}  // extern "C"
