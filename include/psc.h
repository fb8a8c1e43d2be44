/*
 * psc.h -- C ABI of the MI355X particle-in-cell hot path.
 *
 * One explicit electromagnetic PIC time step in the staggered order of the
 * paper's optimized time step (Germaschewski et al., "The Plasma Simulation
 * Code", fig. psc_new): B half step, particle loop (field interpolation,
 * relativistic Boris push, position update, charge-conserving current
 * deposit), B half step, fold of the per-patch current halos, E full step,
 * and the per-step sort of particles by patch and cell (section "Sorting and
 * Communication").  Everything runs in hand-written HIP kernels for gfx950 on
 * the stream the caller passes; the library allocates no particle or field
 * state.
 *
 * Units: c = eps0 = 1.  Maxwell: dE/dt = curl B - J, dB/dt = -curl E,
 * div E = rho.  Motion: du/dt = (q/m)(E + u x B / gamma), u = gamma v.
 * A particle of species s carries charge density q_s * w_s.
 *
 * Grid (section "FDTD method", fig. grid): cells (nx, ny, nz), x fastest;
 * a 2-d run is the (y, z) plane with nx == 1 and no x derivatives.  Field
 * arrays are float32, component-major, 3 * ncell elements, cell index
 * i + nx*(j + ny*k).  Yee staggering, each value stored at its lower index:
 * E_x (i+1/2, j, k), E_y (i, j+1/2, k), E_z (i, j, k+1/2);
 * B_x (i, j+1/2, k+1/2), B_y (i+1/2, j, k+1/2), B_z (i+1/2, j+1/2, k);
 * J located like E.  Periodic in every direction.
 *
 * Particles (structure of arrays, float32 precision with an integer cell):
 *   cell  int32    patch-major cell key (see below) of the particle's cell
 *   off   float32  D arrays of in-cell offsets in [0, 1) (D = 2: y, z;
 *                  D = 3: x, y, z), array d at off + d * capacity
 *   u     float32  3 arrays of momentum per mass u = gamma v / c, array c
 *                  at u + c * capacity
 *   id    int32    optional user tag carried through pushes and sorts
 * Cell key: patches of patch[d] cells tile the grid in row-major patch order
 * (x fastest), the last patch along a dimension truncated at the grid edge;
 * cells inside a patch are numbered row-major; the key is the cell's rank in
 * this enumeration.  Sorting by key groups particles by patch, then by cell.
 *
 * Ownership: the caller allocates every device buffer (fields, two particle
 * buffer sets per species used as ping-pong, and one workspace block whose
 * size psc_workspace_size reports) and keeps them alive until psc_destroy.
 * The context object itself is host memory owned by the library.  A context
 * is used by one host thread at a time; all device work is ordered on the
 * stream argument.
 *
 * Errors: every call returns a psc_status.  Argument problems are reported
 * synchronously.  Device-side problems (non-finite momenta, a particle that
 * would move more than one cell, a cell key out of range, an overfull cell)
 * set a sticky device error word that psc_check returns.  HIP runtime
 * failures return PSC_ERR_HIP; psc_last_error gives the text.
 */
#ifndef PSC_H
#define PSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PSC_OK = 0,
    PSC_ERR_INVALID = 1,      /* bad argument or descriptor                  */
    PSC_ERR_CFL = 2,          /* dt violates the CFL limit                    */
    PSC_ERR_LDS = 3,          /* patch tile does not fit in LDS               */
    PSC_ERR_HIP = 4,          /* HIP runtime error                            */
    PSC_ERR_NONFINITE = 5,    /* a momentum became NaN/Inf (device word)      */
    PSC_ERR_PARTICLE = 6,     /* move > 1 cell or key out of range (device)   */
    PSC_ERR_UNSUPPORTED = 7,  /* valid but not implemented combination        */
    PSC_ERR_STATE = 8         /* call out of order (e.g. no particles loaded) */
} psc_status;

#define PSC_MAX_SPECIES 4
#define PSC_MAX_RUNS 4096

/* Field operations of psc_push_fields (fig. psc_new: push_field_B_half,
 * push_field_E). */
#define PSC_B_HALF 0   /* B <- B - (dt/2) curl^+ E                            */
#define PSC_E_FULL 1   /* E <- E + dt (curl^- B - J)                          */

/* Error word bits (psc_check / psc_error_word). */
#define PSC_DEV_NONFINITE 1u
#define PSC_DEV_MOVE 2u
#define PSC_DEV_KEY 4u
#define PSC_DEV_OVERFULL 8u

typedef struct {
    int dim;                        /* 2 or 3                                        */
    int gdims[3];                   /* cells along x, y, z (gdims[0] == 1 in 2-d);   */
                                    /* active dimensions need >= 3 cells             */
    int patch[3];                   /* patch size in cells (patch[0] == 1 in 2-d)    */
    double dx[3];                   /* cell sizes (dx[0] ignored in 2-d)             */
    double dt;                      /* time step, below the Yee CFL limit            */
    int order;                      /* 1: b1 interpolation weights, 2: b2            */
    int n_species;                  /* 1 .. PSC_MAX_SPECIES                          */
    double q[PSC_MAX_SPECIES];      /* charge                                        */
    double m[PSC_MAX_SPECIES];      /* mass                                          */
    double w[PSC_MAX_SPECIES];      /* density weight per particle                   */
    int64_t capacity[PSC_MAX_SPECIES]; /* particle slots per buffer, <= 2^30 - 1024  */
    int flags;                      /* PSC_RUN_* bits                                 */
} psc_run_desc;

/* psc_run_desc.flags: reserve workspace for psc_adjoint_step */
#define PSC_RUN_ADJOINT 1
/* psc_run_desc.flags: deposit the current of this 1st-order run with the
 * Villasenor-Buneman scheme (the paper's choice at 1st order: the path is
 * cut at cell faces and each piece adds the flux of its linear cloud; in
 * 2-d the out-of-plane current takes the linear weights at each piece's
 * midpoint) instead of Esirkepov's.  Order 2: PSC_ERR_UNSUPPORTED.  Not
 * with PSC_RUN_ADJOINT (the reverse step differentiates Esirkepov). */
#define PSC_RUN_VB 2
/* psc_run_desc.flags: accumulate this run's current in per-patch float
 * tiles with halos in the workspace (float atomics), folded into J by
 * psc_deposit_current (fig. psc_new: add_and_fill_ghosts_j as a pass of its
 * own).  Without it the particle kernel adds each work item's LDS tile
 * straight into a per-cell accumulator of the run, its halo wrapped onto the
 * neighbouring patches' cells (the fold fused into the deposit, section
 * "Fusing of GPU kernels"), in 64-bit fixed point: integer sums, so J does
 * not depend on the order in which work items add and a step is bitwise
 * reproducible; psc_deposit_current then converts the sums to J (one
 * elementwise pass) and clears them.  The unit is a power of two chosen
 * from the run's largest |q w|, dx/dt and particle capacity so that no sum
 * can overflow; each tile value added is rounded to it, by at most 2^-29 of
 * the bound on one particle's contribution.  Runs too small for the direct path (an active dimension
 * with fewer cells than order, or with 2 * cells + 1 < patch + order + 1)
 * always take the tiles. */
#define PSC_RUN_TILE_FOLD 4

typedef struct {
    float *E, *B, *J;                          /* 3 * ncell float32 each               */
    int32_t *cell[PSC_MAX_SPECIES][2];         /* ping-pong particle buffer sets       */
    float *off[PSC_MAX_SPECIES][2];            /* D * capacity                          */
    float *u[PSC_MAX_SPECIES][2];              /* 3 * capacity                          */
    int32_t *id[PSC_MAX_SPECIES][2];           /* optional: all NULL or all set         */
} psc_run_bufs;

typedef struct psc_ctx psc_ctx;

/* Validate run descriptors and create a context (host only, no device work).
 * runs: n_runs descriptors (1 <= n_runs <= PSC_MAX_RUNS), copied.
 * chunk: particles per work item of the particle kernel (0 = default 8192).
 * Synchronous errors: PSC_ERR_INVALID (also: more than three patches along a
 * dimension with a patch, or the truncated last one, narrower than order + 1
 * cells, the current tile's halo), PSC_ERR_CFL (dt >= CFL limit),
 * PSC_ERR_LDS (a patch's field and current tiles plus the per-wave queues of
 * a 256-thread workgroup exceed the 160 KiB of LDS of a workgroup, or a patch
 * side exceeds 255 cells). */
psc_status psc_init_patches(const psc_run_desc *runs, int n_runs, int chunk, psc_ctx **out);

/* Bytes of device workspace the context needs (per-patch current tiles,
 * cell offsets, sort counters, permutation, work tables, error word). */
psc_status psc_workspace_size(const psc_ctx *ctx, size_t *bytes);

/* Attach caller buffers: bufs[r] for each run, and a device workspace of at
 * least psc_workspace_size bytes (256-byte aligned).  Uploads the device
 * descriptor tables on `stream` (a hipStream_t, NULL = default stream). */
psc_status psc_bind(psc_ctx *ctx, const psc_run_bufs *bufs, int n_runs, void *workspace, void *stream);

/* Size of the library-held workspace of psc_bind_static, per device. */
#define PSC_STATIC_WORKSPACE_BYTES (64u * 1024u * 1024u)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): psc_bind
 * with the workspace taken from a device array the library holds, of
 * PSC_STATIC_WORKSPACE_BYTES on each device, instead of a caller block.  The
 * caller still allocates and passes the fields and particle buffers (bufs).
 * The array of the current device (hipGetDevice) is used; its address is
 * looked up once per device.  Clears what must start at zero (error word,
 * current tiles, cell offsets, move counters) as psc_bind does: the array
 * otherwise keeps whatever the last call left in it.  Calls no hipMalloc,
 * hipFree or allocating library routine (the context's host tables were
 * sized by psc_init_patches); synchronizes `stream` like psc_bind.
 * Sharing: one context at a time holds a device's array.  Binding another
 * context with this call hands the array to it; the previous holder is left
 * unbound (its calls return PSC_ERR_STATE, and psc_last_error says why) until
 * it is bound again, and its device state is lost.  Calls of two contexts
 * that overlap on one device race on the array.  psc_bind or psc_destroy of
 * the holder releases it.
 * Errors: PSC_ERR_INVALID if psc_workspace_size exceeds
 * PSC_STATIC_WORKSPACE_BYTES (psc_last_error states both sizes), otherwise
 * as psc_bind. */
psc_status psc_bind_static(psc_ctx *ctx, const psc_run_bufs *bufs, int n_runs, void *stream);

/* Load the particles of one (run, species) from caller device arrays in
 * geometric form: gcell int32 (n) geometric cell index i + nx*(j + ny*k),
 * goff float32 (D, n) row-major (array d at goff + d*n), gu float32 (3, n),
 * gid int32 (n) or NULL.  Converts cells to patch-major keys and stably sorts
 * by key into buffer set 0 (input order kept among equal keys).  n must not
 * exceed the species capacity.  Call for every species before stepping.
 * Loading after steps have run restarts the context: every species must be
 * loaded again before the next step (used to restore checkpoints). */
psc_status psc_load_particles(psc_ctx *ctx, int run, int species, int64_t n, const int32_t *gcell,
                              const float *goff, const float *gu, const int32_t *gid, void *stream);

/* Load the particles of one (run, species) that are already in sorted key
 * order, in the layout psc_get_particles writes (stride n): key int32 (n)
 * patch-major cell keys, off float32 (D, n), u float32 (3, n), id int32 (n)
 * or NULL (ids are then 0 .. n-1 if the context carries them).  No
 * conversion and no sort: the arrays are copied into buffer set 0 and the
 * cell offsets taken from the key boundaries; a key outside the run's cells
 * or a decreasing pair sets PSC_DEV_KEY in the error word (psc_check).
 * Otherwise as psc_load_particles (restores a checkpoint taken with
 * psc_get_particles without sorting it again). */
psc_status psc_load_sorted(psc_ctx *ctx, int run, int species, int64_t n, const int32_t *key, const float *off,
                           const float *u, const int32_t *id, void *stream);

/* Field update of every run (section "FDTD method"; fig. psc_new).
 * op: PSC_B_HALF or PSC_E_FULL. */
psc_status psc_push_fields(psc_ctx *ctx, int op, void *stream);

/* Particle loop of every run and species (fig. psc_new: push_particle_p,
 * push_particle_x, deposit_j), fused in one kernel: per patch, E and B are
 * staged in LDS with ghost layers; each particle is interpolated (b1/b2
 * weights of its Yee component), pushed with the relativistic Boris scheme,
 * moved, and its Esirkepov current is accumulated in an LDS tile that is
 * added into the run's fixed-point current sums (or, under
 * PSC_RUN_TILE_FOLD, the patch's float tile); psc_deposit_current turns
 * them into J.  Reads the particles
 * through the permutation left by psc_sort (if any), writes them in that
 * sorted order into the other buffer set, and records each particle's move
 * code for the next psc_sort. */
psc_status psc_push_particles(psc_ctx *ctx, void *stream);

/* J of the last psc_push_particles, then the accumulators cleared: the
 * runs' fixed-point sums (whose halos the particle kernel already wrapped)
 * converted to float; for the runs that keep tiles (PSC_RUN_TILE_FOLD or too
 * small for the direct path) the per-patch tiles with their halos folded
 * into J with periodic wrap, in a fixed order (fig. psc_new:
 * add_and_fill_ghosts_j). */
psc_status psc_deposit_current(psc_ctx *ctx, void *stream);

/* Stable counting sort of every species by cell key (section "Sorting and
 * Communication"): uses the move codes of the last psc_push_particles (each
 * particle moved by at most one cell per dimension), computes the new cell
 * offsets and the permutation into key order, equal keys in their current
 * order.  The physical reorder is deferred into the next
 * psc_push_particles. */
psc_status psc_sort(psc_ctx *ctx, void *stream);

/* The same stable order as psc_sort by a general least-significant-digit
 * radix sort of the new keys (rocPRIM, several passes over all particles),
 * the multi-pass baseline that the paper's single-pass sort replaces
 * (section "Sorting and Communication"): for timing the two against each
 * other.  Same outputs and state change as psc_sort (permutation, cell
 * offsets, reorder deferred into the next push); the push's move counts are
 * cleared unused.  Uses the load path's scratch.  May not be recorded into
 * a graph. */
psc_status psc_sort_radix(psc_ctx *ctx, void *stream);

/* nsteps full steps in the order of fig. psc_new: B half, particles, B half,
 * fold J, E full, sort.  use_graph != 0 records the step into a HIP graph
 * once per buffer parity and replays it. */
psc_status psc_step(psc_ctx *ctx, int nsteps, int use_graph, void *stream);

/* Launch shape of the particle kernel (batching and autotuning).  psc_bind
 * sets PSC_LAUNCH_QUEUE with 512 threads (or the largest workgroup whose LDS
 * fits), two particles per lane for 2-d order-2 runs and one otherwise (the
 * shapes the autotuner chose on gfx950).
 * mode: PSC_LAUNCH_GRID      one workgroup per work item;
 *       PSC_LAUNCH_QUEUE     persistent workgroups pulling work items from
 *                            eight queues (one per XCD, with stealing);
 *       PSC_LAUNCH_PARTITION persistent workgroups, each over a contiguous
 *                            segment of (run, patch, species) units chosen
 *                            by psc_balance (called here once).
 * chunk: particles per work item of every run (0 keeps the current values).
 * workers: persistent workgroups (0 = compute units x workgroups that fit
 * in one unit's LDS).  threads: workgroup size, 256, 384 or 512 (0 keeps;
 * the LDS tiles of a work item are shared by all its waves; PSC_ERR_LDS if
 * the tiles and per-wave queues exceed 160 KiB).  run: consecutive
 * particles a lane pushes in sequence, 1 or 2 (0 keeps; default 1: one
 * particle per lane, consecutive particles on consecutive lanes; 2: a lane
 * accumulates the current of both when they share a cell, halving the
 * wave-level sums, and the outputs are exchanged across the wave so that
 * the stores stay coalesced).  Drops recorded step graphs.  May
 * synchronize. */
#define PSC_LAUNCH_GRID 0
#define PSC_LAUNCH_QUEUE 1
#define PSC_LAUNCH_PARTITION 2
psc_status psc_set_launch(psc_ctx *ctx, int mode, int chunk, int workers, int threads, int run,
                          void *stream);

/* Particles per work item of one run's (species, patch) units (batching
 * with runs of different occupancy: the launch shape is one per context,
 * the chunk can differ per run; psc_set_launch with chunk > 0 sets every
 * run's).  chunk >= 1.  Uploads the run's table entry and synchronizes
 * `stream`, drops recorded step graphs, and recomputes the partition under
 * PSC_LAUNCH_PARTITION.  PSC_ERR_INVALID for a bad run or chunk or an
 * unbound context. */
psc_status psc_set_run_chunk(psc_ctx *ctx, int run, int chunk, void *stream);

/* Recompute the PSC_LAUNCH_PARTITION split from the current particle
 * counts (App. A, "Load balancing algorithm", with every workgroup of equal
 * capability): unit loads L = N_particles + cell_cost * N_cells (the load
 * estimate of the load-balancing section), in unit order.  Synchronizes
 * `stream`. */
psc_status psc_balance(psc_ctx *ctx, double cell_cost, void *stream);

/* The greedy partition of App. A on host arrays: loads L[n_patches] in
 * space-filling-curve order and capabilities C[n_ranks] give N[n_ranks],
 * the number of consecutive patches of each rank.  Pure host function. */
psc_status psc_partition(const double *L, int n_patches, const double *C, int n_ranks, int32_t *N);

/* Order in which the (run, species, patch) units of the particle work are
 * handed out (section "Dynamic load balancing using space filling curves":
 * patches enumerated along a Hilbert-Peano curve, so that a contiguous
 * segment of the enumeration is a compact block of the domain).  The units
 * of a run follow its patches in this order, the species of a patch
 * together, runs one after another.  It decides which patches the eighth of
 * the work items owned by one XCD's queue (PSC_LAUNCH_QUEUE), a contiguous
 * item range (PSC_LAUNCH_GRID) or one workgroup's partition segment
 * (PSC_LAUNCH_PARTITION) covers; it does not change the particle layout,
 * the cell keys or any result beyond the summation order of the current.
 * PSC_ORDER_ROWMAJOR is the default: it hands each XCD a contiguous range of
 * the patch-major particle arrays, and on one GPU it is the faster of the
 * two (the Hilbert order spreads an XCD's items over the arrays). */
#define PSC_ORDER_ROWMAJOR 0   /* patch index order, x fastest               */
#define PSC_ORDER_HILBERT 1    /* psc_hilbert_order                           */

/* Set the unit order of a bound context: uploads the unit table on `stream`
 * and synchronizes it, drops recorded step graphs, and recomputes the
 * partition (psc_balance) under PSC_LAUNCH_PARTITION.  PSC_ERR_INVALID for an
 * unknown order or an unbound context. */
psc_status psc_set_unit_order(psc_ctx *ctx, int order, void *stream);

/* The Hilbert order of the patches of a grid of np[0] x np[1] x np[2]
 * patches (x fastest; np[0] == 1 when dim == 2): order[t] is the row-major
 * patch index p = px + np[0]*(py + np[1]*pz) of the t-th patch along the
 * curve, for t < np[0]*np[1]*np[2] (at most 2^24 patches).  The curve is
 * the n-dimensional Hilbert curve (Skilling's construction) of the smallest
 * power-of-two cube holding the grid, restricted to it, with the grid axes
 * mapped onto the curve's coordinates by the permutation that leaves the
 * fewest consecutive pairs that are not face neighbours (none for a cube of
 * side 2^k, or a 2:1 box in 2-d, 2:1:1 or 2:2:1 in 3-d).  `order` is caller
 * host memory.  Pure host function; PSC_ERR_INVALID for bad sizes. */
psc_status psc_hilbert_order(int dim, const int32_t np[3], int32_t *order);

/* Write the particles of (run, species) in sorted key order into caller
 * device arrays (same layout as the buffers, stride n): cell keys, offsets,
 * momenta, ids (any pointer may be NULL to skip it). */
psc_status psc_get_particles(psc_ctx *ctx, int run, int species, int32_t *cell, float *off, float *u,
                             int32_t *id, void *stream);

/* Convert patch-major keys to geometric cell indices for (run): n keys in,
 * n geometric indices out (device arrays). */
psc_status psc_keys_to_cells(psc_ctx *ctx, int run, int64_t n, const int32_t *keys, int32_t *cells,
                             void *stream);

/* Per-step state queries (host side, no device work). */
psc_status psc_particle_count(const psc_ctx *ctx, int run, int species, int64_t *n);
psc_status psc_front(const psc_ctx *ctx, int *front, int *perm_pending);

/* Device views for tests: the permutation (int32, capacity) and the current
 * cell offsets (int32, ncell + 1) of (run, species). */
psc_status psc_sort_view(const psc_ctx *ctx, int run, int species, const int32_t **perm,
                         const int32_t **cell_start);

/* Double-precision diagnostics of every run (the only FP64 on the GPU), on
 * the stored time levels E^{n+1/2}, B^n, u^n.  out_dev: device float64,
 * n_runs * PSC_DIAG_STRIDE values per run:
 *   [0] 1/2 sum E^2 dV   [1] 1/2 sum B^2 dV   [2..5] sum m w dV (gamma-1) per species
 *   [6] max |div^- E - rho|   [7] max |div^+ B|   [8] sum rho dV   [9] particle count
 * gauss_dev: optional float64 (sum of ncell over runs) receiving div^- E - rho
 * per node, runs concatenated. */
#define PSC_DIAG_STRIDE 10
psc_status psc_diagnostics(psc_ctx *ctx, double *out_dev, double *gauss_dev, void *stream);

/* Marder's divergence cleaning, the iterative method the paper names for
 * dissipating the violations of Gauss's law that single-precision runs
 * accumulate over many steps (section "Time integration of the
 * quasi-particle equations of motion").  iters times: F = div^- E - rho - ref
 * at every node (rho of the current particles, FP64), then
 * E += d dt grad^+ F, which changes only the longitudinal part of E.
 * ref: optional device float64 array laid out like psc_diagnostics' gauss
 * output (e.g. the residual at the start of the run, so that only its drift
 * is removed); NULL means zero.  d: diffusion coefficient (length^2/time),
 * 0 < d dt sum_d 4/dx_d^2 <= 2 in every run, else PSC_ERR_INVALID (the step
 * would amplify the residual).  Call between steps (PSC_ERR_STATE right after
 * a bare psc_push_particles).  Overwrites the diagnostics' charge scratch.
 * Asynchronous on `stream`. */
psc_status psc_marder(psc_ctx *ctx, const double *ref, double d, int iters, void *stream);

/* Copy the permutation of the last psc_sort of (run, species) to a caller
 * device array (int32, n): entry j is the slot, in the order the last
 * psc_push_particles wrote, of the particle that sorts to position j. */
psc_status psc_get_perm(psc_ctx *ctx, int run, int species, int32_t *perm, void *stream);

/* Copy the current cell offsets of (run, species) (int32, ncell + 1: the
 * sorted particles of cell key c are slots [out[c], out[c+1]) of the order
 * psc_get_particles writes) to a caller device array. */
psc_status psc_get_cell_offsets(psc_ctx *ctx, int run, int species, int32_t *out, void *stream);

/* Replace the device arrays of particle buffer set `set` (0 or 1) of (run,
 * species) with caller arrays of the same capacity and layout (cell, off,
 * u, and id exactly when the context carries ids).  The set psc_front does
 * not name is the one the next psc_push_particles writes, so swapping it
 * before each step keeps every step's particles in arrays of their own (the
 * adjoint's recomputed segments); swapping the front set is allowed only
 * with arrays that hold the same particles.  The run table is uploaded on
 * the stream of the next call that launches kernels (one copy through a
 * pinned staging slot for all changes since the last upload, no host
 * wait); drops recorded step graphs.  `stream` is unused. */
psc_status psc_set_particle_buffers(psc_ctx *ctx, int run, int species, int set, int32_t *cell, float *off, float *u,
                                    int32_t *id, void *stream);

/* Direct the outputs of the next psc_sort (or psc_sort_radix) of (run,
 * species) to caller device arrays: its permutation into `perm` (int32,
 * the species' capacity) and its new cell offsets into `cs` (int32, ncell
 * + 1).  The following psc_push_particles reads them there, and
 * psc_get_perm / psc_get_cell_offsets copy from there, so a caller that
 * redirects every step keeps each step's permutation and offsets in arrays
 * of their own without copies (the adjoint's recomputed segments).  perm ==
 * cs == NULL returns to the workspace's own arrays, copying the current
 * offsets (and a pending permutation) back into them on `stream`.  Both or
 * neither must be NULL (PSC_ERR_INVALID otherwise).  The run table is
 * uploaded before the next launch, as with psc_set_particle_buffers; drops
 * recorded step graphs. */
psc_status psc_set_sort_outputs(psc_ctx *ctx, int run, int species, int32_t *perm, int32_t *cs, void *stream);

/* Forward state of one step, per run, as the adjoint needs it: fields at the
 * start of the step (E^{n+1/2}, B^n), the particles at the start of the step,
 * and the permutation of the step's sort (psc_get_perm after the step).
 * The particles come either in sorted key order (as psc_get_particles
 * writes them, stride n; read_perm NULL) or as the buffer set the step's
 * push read them from, with read_perm the permutation of the previous sort
 * (sorted slot -> buffer slot, as psc_get_perm returned it before the step)
 * and stride the buffers' capacity.  cell_start: optional cell offsets of
 * the sorted keys (ncell + 1, as psc_get_cell_offsets returned them before
 * the step); NULL computes them from sorted keys (read_perm NULL only). */
typedef struct {
    const float *E, *B;
    const int32_t *cell[PSC_MAX_SPECIES];
    const float *off[PSC_MAX_SPECIES];
    const float *u[PSC_MAX_SPECIES];
    const int32_t *perm[PSC_MAX_SPECIES];
    const int32_t *read_perm[PSC_MAX_SPECIES];   /* NULL: particles in sorted order   */
    const int32_t *cell_start[PSC_MAX_SPECIES];  /* NULL: from the sorted keys         */
    int64_t stride[PSC_MAX_SPECIES];             /* 0: n                               */
} psc_adj_fwd;

/* Adjoint state, per run: on entry the adjoints of the step's outputs
 * (E^{n+3/2}, B^{n+1}, particle offsets and momenta in the sorted order of the
 * next step); on return those of its inputs (E^{n+1/2}, B^n, particles in the
 * sorted order of this step).  Float32, same layouts as the state; updated in
 * place. */
typedef struct {
    float *lE, *lB;
    float *loff[PSC_MAX_SPECIES];   /* D x n */
    float *lu[PSC_MAX_SPECIES];     /* 3 x n */
} psc_adj_state;

/* Reverse of one full time step (transpose of the discrete step of
 * fig. psc_new: E full step, second B half step, particle loop with the
 * Esirkepov deposit, move, Boris rotation and interpolation, first B half
 * step).  The paper defines no adjoint; this is the exact derivative of the
 * forward kernels' arithmetic.  Needs PSC_RUN_ADJOINT in every run's flags;
 * 2-d and 3-d runs (in 3-d the particle part adds its transposed
 * interpolation into lE, lB with float atomics, so its summation order varies
 * between calls; the 2-d fold is in a fixed order); PSC_ERR_UNSUPPORTED with
 * PSC_RUN_VB.  fwd and adj hold n_runs entries.  Asynchronous on `stream` (the pointer tables are copied before
 * the call returns): the buffers must stay valid until the stream reaches
 * the call's end.  Successive calls on different streams must be ordered by
 * the caller, since they share the adjoint scratch. */
psc_status psc_adjoint_step(psc_ctx *ctx, const psc_adj_fwd *fwd, const psc_adj_state *adj, void *stream);

/* Seed of the reverse pass for W = final field energy, 1/2 sum(E^2 + B^2) dV
 * (psc_diagnostics [0] + [1]), from the context's current fields: per run
 * lE = dW/dE = E dV, lB = dW/dB = B dV, and the particle adjoints loff, lu
 * (D x n and 3 x n, n the current particle count) zero.  adj holds n_runs
 * entries of caller device arrays.  Asynchronous on `stream`. */
psc_status psc_adjoint_seed(psc_ctx *ctx, const psc_adj_state *adj, void *stream);

/* Synchronize `stream` and return the device error word as a status:
 * PSC_OK, PSC_ERR_NONFINITE, PSC_ERR_PARTICLE. *word (optional) receives the
 * raw bits (PSC_DEV_*). clear != 0 resets the word. */
psc_status psc_check(psc_ctx *ctx, void *stream, uint32_t *word, int clear);

const char *psc_status_string(psc_status s);
psc_status psc_last_error(const psc_ctx *ctx, char *buf, size_t n);
psc_status psc_destroy(psc_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* PSC_H */
