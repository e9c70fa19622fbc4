/*
 * pic.h -- C ABI of libpic, an MI355X (gfx950) library for particle-in-cell current
 * deposition with cell-sorted particles (MatrixPIC, arXiv 2601.08277).
 *
 * What the library computes
 *   pic_deposit           Eq. 1 (Sec. 3.1): J_c(node) = sum_p q W_p v_{p,c} S(node - x_p),
 *                         with the separable shape S = s_x s_y s_z of Sec. 4.2.1, B-splines
 *                         of order 1..3, on a Yee-staggered Jx/Jy/Jz grid, accumulated per
 *                         cell / per tile ("rhocell", Sec. 3.4, Eq. 4-5) instead of global
 *                         atomics.
 *   pic_rebin             keeps particles sorted by cell: the start-up counting sort
 *                         (GlobalSortParticlesByCell, Alg. 1), the per-step incremental
 *                         update of movers with gapped bins (Sec. 4.3), local rebuilds and
 *                         the global re-sort policy (Sec. 4.4).
 *   pic_deposit_backward  adjoint of pic_deposit: gathers dL/dJ back to the particles and
 *                         returns dL/dx, dL/du, dL/dw (gather = field interpolation, Sec. 3.1).
 *   pic_plan_* / pic_deposit_batched
 *                         many independent patches of uneven size in one persistent launch.
 *
 * Conventions (every entry point)
 *   - Pointers named in pic_particles, J*, G*, d* are DEVICE pointers owned by the caller
 *     (allocated with hipMalloc or by a framework such as PyTorch). Descriptor structs
 *     (pic_grid, pic_sort_policy, pic_rebin_stats) are HOST memory, read (or written)
 *     during the call only.
 *   - Work is enqueued asynchronously on `stream` (0 = the null stream). Calls neither
 *     allocate nor synchronise, except pic_bins_create/destroy, pic_plan_create/destroy,
 *     pic_rebin_stats_read and pic_check, which say so.
 *   - Argument errors return a negative pic_status at once and enqueue nothing; the
 *     message is available from pic_last_error() (thread-local). Device-side errors
 *     (particle out of the domain, non-finite position, capacity) set flags inside the
 *     bins object; pic_check() / pic_rebin_stats_read() synchronise and report them.
 *   - Grid arrays (J, G) are float32, x fastest:
 *        J[((k + gz) * Ny + (j + gy)) * Nx + (i + gx)],  N_d = n_d + 2 g_d,
 *     g_d = ng on a guard dimension and 0 on a periodic one. In 2D there is no k term.
 *     Component c sits half a cell along its own axis (Jx at i + 1/2, ...).
 */
#ifndef PIC_H
#define PIC_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PIC_OK = 0,
  PIC_ERR_INVALID_ARG = -1,       /* bad descriptor, size, pointer or mode            */
  PIC_ERR_UNSUPPORTED = -2,       /* valid request the library does not implement     */
  PIC_ERR_OUT_OF_DOMAIN = -3,     /* a particle (or its stencil) left the domain       */
  PIC_ERR_CAPACITY = -4,          /* particle arrays too small for bins with slack     */
  PIC_ERR_INVALID_PARTICLE = -5,  /* non-finite position                              */
  PIC_ERR_HIP = -6                /* a HIP runtime call failed                        */
} pic_status;

enum { PIC_BC_PERIODIC = 0, PIC_BC_GUARD = 1 };

/* Deposition paths. All accumulate in float32; the split-MFMA paths feed the matrix
 * cores hi/lo pairs of bf16 or fp16 operands (three products per pair). */
enum {
  PIC_PATH_AUTO = 0,         /* pick per order and density: pic_tuning_load's cache, else */
                             /* the per-cell VALU path                                    */
  PIC_PATH_ATOMIC = 1,       /* one particle per lane, LDS-atomic tile accumulation        */
  PIC_PATH_CELL_VALU = 2,    /* per-cell register accumulation (rhocell on VALU)           */
  PIC_PATH_MFMA_BF16 = 3,    /* per-row outer-product contraction on MFMA, split bf16     */
  PIC_PATH_MFMA_FP16 = 4,    /* same with scaled split fp16                                */
  PIC_PATH_UNSORTED = 5      /* no bins: one particle per lane, global atomics             */
};

enum { PIC_REBIN_FULL = 0, PIC_REBIN_INCREMENTAL = 1, PIC_REBIN_AUTO = 2 };

enum {
  PIC_F_ACCUMULATE = 1u,     /* add into J instead of overwriting it                       */
                             /* (bit 2u is not used: rejected as an unknown flag)          */
  PIC_F_EMIT_MOVERS = 4u,    /* pic_deposit records particles whose cell no longer matches */
                             /* their bin, for the next PIC_REBIN_INCREMENTAL              */
  PIC_F_DRIFT = 8u,          /* pic_deposit then moves every particle x += v dt (grid dt)  */
                             /* and records movers against the moved positions            */
  PIC_F_MIDPOINT = 16u       /* time-centred current: deposit at the midpoint of the move  */
                             /* x -> x + v dt (grid dt): at x + v dt / 2 with PIC_F_DRIFT, */
                             /* else at x - v dt / 2 (x already advanced by a push)        */
};

#define PIC_INVALID_ID (-1)  /* id of an empty (gap) slot; gap slots also carry w = 0 */

typedef struct {
  int dim;          /* 2 (x, y) or 3                                              */
  int n[3];         /* cells per dimension; n[2] = 1 in 2D                        */
  double x0[3];     /* position of node 0                                         */
  double dx[3];     /* cell size                                                  */
  double inv_dx[3]; /* 1 / dx, used as given (the cell index is (x - x0) * inv_dx) */
  int bc[3];        /* PIC_BC_PERIODIC or PIC_BC_GUARD per dimension               */
  int ng;           /* guard nodes per side on guard dimensions (>= 1, 2, 2 for   */
                    /* orders 1, 2, 3)                                            */
  int order;        /* shape order 1, 2 or 3                                      */
  float q;          /* charge of the species                                      */
  double dt;        /* time step of PIC_F_DRIFT, PIC_F_MIDPOINT and pic_drift       */
} pic_grid;

typedef struct {
  int64_t nslots;   /* length of every array below (slots, valid or gap)          */
  double *x, *y, *z;/* positions (z unused in 2D but must be a valid pointer)     */
  float *ux, *uy, *uz; /* proper velocity u = gamma v (c = 1)                     */
  float *w;         /* macro-particle weight                                      */
  int32_t *id;      /* particle id, PIC_INVALID_ID in gap slots                    */
} pic_particles;

typedef struct pic_bins pic_bins;   /* opaque, library-owned device memory */
typedef struct pic_plan pic_plan;   /* opaque batched-launch plan          */

/* Global re-sort policy, Sec. 4.4; defaults from the parameter table (Appendix A). */
typedef struct {
  int min_interval;     /* 10   */
  int interval;         /* 50   */
  int rebuild_count;    /* 100  */
  double empty_ratio;   /* 0.15 */
  double full_ratio;    /* 0.85 */
  int perf_enable;      /* 1    */
  double perf_degrad;   /* 0.80 */
} pic_sort_policy;

typedef struct {
  int64_t n_valid;            /* particles held by the bins                          */
  int64_t n_moved;            /* movers found by the last rebin                       */
  int64_t n_overflow;         /* movers that found their destination bin full         */
  int64_t n_mover_drop;       /* movers beyond the mover-list capacity (retried)      */
  int32_t n_local_rebuilds;   /* tiles rebuilt by the last rebin                       */
  int32_t n_global_sorts;     /* full sorts since the bins were created               */
  double empty_slot_ratio;    /* empty slots / slots inside bins                       */
  int32_t global_sort_recommended; /* policy decision after the last rebin (0/1)      */
  int32_t last_mode;          /* PIC_REBIN_FULL or PIC_REBIN_INCREMENTAL as executed  */
  uint32_t error_flags;       /* bit 0 out of domain, 1 non-finite, 2 capacity, 3 stencil */
                              /* outside the stored nodes, 4 move of a cell or more     */
} pic_rebin_stats;

/* Default policy values. */
void pic_sort_policy_default(pic_sort_policy* out);

/* Host-side policy decision of Sec. 4.4 (prioritised triggers 1..5); returns 1 to run a
 * global sort. `trigger` (nullable) receives the deciding rule number, 0 if none. A
 * negative empty_slot_ratio means "not known yet" and skips trigger 4. */
int pic_policy_decide(const pic_sort_policy* p, int steps_since_sort, int rebuilds_since_sort,
                      double empty_slot_ratio, double perf, double perf_baseline, int* trigger);

/* Create bins (the cell-sorted index structure that Alg. 1 keeps per tile, with gapped
 * per-cell slots as in Sec. 4.3.1) for particles stored in arrays of `nslots` slots. tile[3] is the particle
 * tile (cells per tile per dimension, tile[2] = 1 in 2D). `slack` is the fraction of
 * extra slots a full sort gives every cell (at least one per cell). `max_movers`
 * bounds the mover list (0 = nslots / 8 + 4096). Allocates device memory (synchronous).
 * Bins hold nothing until the first pic_rebin(PIC_REBIN_FULL). */
pic_status pic_bins_create(const pic_grid* grid, const int tile[3], double slack,
                           int64_t nslots, int64_t max_movers, pic_bins** out);
pic_status pic_bins_destroy(pic_bins* bins);

/* Device views of the bin tables, for inspection and tests. Bins are ordered tile by
 * tile (tiles x fastest), cells x fastest inside a tile. Bin b owns slots
 * [off[b], off[b+1]); its first len[b] slots hold its particles, the rest are gaps. */
typedef struct {
  int64_t nbins, ntiles;
  int32_t ntile[3];
  const int32_t* off;       /* nbins + 1 */
  const int32_t* len;       /* nbins     */
  const int32_t* bin_cell;  /* nbins: flat x-fastest cell of every bin */
} pic_bins_view;
pic_status pic_bins_get_view(const pic_bins* bins, pic_bins_view* out);
/* Synchronises `stream` and copies the bin tables to host arrays (each nullable):
 * off_host nbins + 1 entries, len_host and cell_host nbins entries. */
pic_status pic_bins_copy_tables(const pic_bins* bins, int32_t* off_host, int32_t* len_host,
                                int32_t* cell_host, hipStream_t stream);

/* Sort particles into cells. FULL: counting sort of every valid slot into bins with
 * fresh slack (Alg. 1, GlobalSortParticlesByCell). INCREMENTAL: move only the particles
 * whose cell changed since the last rebin (Sec. 4.3): insert into the destination bin's
 * gap slots, compact the source bin, rebuild any tile whose bins overflowed with fresh
 * uniform gaps. Uses the mover list of the last pic_deposit(PIC_F_EMIT_MOVERS) when it
 * is fresh, otherwise scans all particles first. A mover that finds no slot stays in its
 * old bin (deposition still handles it correctly) and is retried next time. AUTO:
 * INCREMENTAL unless the policy asks for FULL; the policy reads the statistics of the
 * calls up to PIC_POLICY_LAG calls back (waiting for the copy of call s - 2 if it has not
 * landed; the stream is not synchronised). Particle payload moves between slots; ids
 * travel with it. `policy` may be NULL (defaults). Not capturable into a graph: refused
 * (UNSUPPORTED) while `stream` is capturing. */
pic_status pic_rebin(const pic_grid* grid, pic_particles* p, pic_bins* bins, int mode,
                     const pic_sort_policy* policy, hipStream_t stream);

/* Synchronises `stream` and returns the statistics of the last pic_rebin. */
pic_status pic_rebin_stats_read(pic_bins* bins, hipStream_t stream, pic_rebin_stats* out);

/* One rebin call as the bins recorded it: what the policy (Alg. 1, "Global Sort
 * Decision"; Sec. 4.4) saw and decided, then the call's own statistics. Calls are numbered
 * from 0 (the first FULL) per bins object. The decision of call s sees the statistics of
 * calls up to s - 2 only (PIC_POLICY_LAG): pic_rebin waits for those if they have not come
 * back yet, so the host runs at most two rebins ahead of the device and the decisions do
 * not depend on timing. */
#define PIC_POLICY_LAG 2
typedef struct {
  int64_t seq;                  /* call number                                          */
  int32_t mode;                 /* executed: PIC_REBIN_FULL or PIC_REBIN_INCREMENTAL     */
  int32_t trigger;              /* AUTO: deciding rule 0..5 (0: none fired); -1 explicit */
  int32_t steps_since_sort;     /* policy inputs at the decision                         */
  int32_t rebuilds_since_sort;  /*   local rebuilds of calls after the last FULL, <= s-2 */
  double known_empty_ratio;     /*   empty-slot ratio of call s-2 (-1: before the FULL)  */
  int64_t n_valid;              /* statistics of this call (valid once `complete`)       */
  int64_t n_moved, n_overflow, n_mover_drop;
  int32_t n_local_rebuilds;
  uint32_t error_flags;
  double empty_slot_ratio;
  int32_t complete;             /* 1 once the statistics have come back                  */
  int32_t pad;
} pic_rebin_record;

/* Synchronises `stream` and copies the records of calls first .. first + max - 1 (those
 * still kept: the newest 65,536 calls) to `out` (host array of `max`); *count receives the
 * number copied. Errors: INVALID_ARG (NULL pointers, negative first or max). */
pic_status pic_rebin_history(pic_bins* bins, hipStream_t stream, int64_t first, int32_t max,
                             pic_rebin_record* out, int32_t* count);

/* Optional performance sample for policy trigger 5 (higher is better, e.g. particles/s). */
pic_status pic_bins_report_perf(pic_bins* bins, double perf);

/* Current deposition (Eq. 1). Overwrites Jx, Jy, Jz unless PIC_F_ACCUMULATE. `bins` must
 * come from pic_rebin on these particles (any path except PIC_PATH_UNSORTED, which
 * ignores bins and may take NULL). Particles whose cell differs from their bin's cell are
 * still deposited exactly. With PIC_F_DRIFT the positions are advanced by v dt after
 * their current is deposited (periodic dimensions wrap). PIC_F_MIDPOINT deposits each
 * particle at x +- (dt/2) u / gamma, the offset formed in float32 and added to x in
 * float64, wrapped on periodic dimensions (positions are not changed by it); it is taken by
 * PIC_PATH_AUTO, PIC_PATH_CELL_VALU and PIC_PATH_UNSORTED (UNSUPPORTED on the other
 * paths). Repeatability: the per-cell and matrix paths sum in a fixed order, so equal
 * inputs and bins give bitwise equal J, except for stencil nodes outside the tile's
 * window, which go to J with float atomics; only a particle whose cell lies outside its
 * bin's tile has such nodes (a mover no bin had room for, or a particle moved across a
 * tile boundary without a rebin). The LDS-atomic and unsorted paths use float atomics
 * throughout.
 * The bins themselves are always left in a deterministic order by pic_rebin. */
pic_status pic_deposit(const pic_grid* grid, pic_particles* p, pic_bins* bins,
                       float* Jx, float* Jy, float* Jz, int path, unsigned flags,
                       hipStream_t stream);

/* pic_deposit for callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): same arguments, checks, paths,
 * flags and results as pic_deposit, but the per-tile stencil windows between the
 * deposition kernel and the window sum live in one fixed 32 MiB device array of the
 * library (one per GPU, held until the process ends) instead of the bins' allocation.
 * Allocates nothing. Bins whose windows need more than 32 MiB (ntiles x 3 x wmax x 4 B,
 * wmax = prod_d (tile_d + 4): 14 MB for 64^3 cells in 8x8x4 tiles, 113 MB for 128^3) are
 * refused with PIC_ERR_INVALID_ARG before anything is enqueued. Every call on one GPU shares the array: calls that overlap on one
 * GPU (other streams, other host threads) race. */
pic_status pic_deposit_noalloc(const pic_grid* grid, pic_particles* p, pic_bins* bins,
                               float* Jx, float* Jy, float* Jz, int path, unsigned flags,
                               hipStream_t stream);

/* Adjoint of pic_deposit for L = sum_c <G_c, J_c>. Writes per slot (gap slots get 0):
 * dL/dx, dL/dy, dL/dz (dz ignored in 2D; may be NULL there), dL/dux, dL/duy, dL/duz and,
 * if dw is not NULL, dL/dw. Shape weights are recomputed, not stored. `bins` may be NULL
 * (particle-parallel gather, no tiles). flags must be 0. */
pic_status pic_deposit_backward(const pic_grid* grid, const pic_particles* p,
                                const pic_bins* bins, const float* Gx, const float* Gy,
                                const float* Gz, float* dx, float* dy, float* dz,
                                float* dux, float* duy, float* duz, float* dw,
                                unsigned flags, hipStream_t stream);

/* Charge density rho(m) = sum_p q W_p prod_d B_o(m_d - xi_{p,d}): the scalar, nodal
 * counterpart of pic_deposit (no velocity, no staggering in any dimension), i.e. the
 * charge/mass assignment of the paper's Appendix B on the same sorted tiles. `rho` is one
 * float32 grid in the layout of a J component (device, caller-owned); it is overwritten
 * unless PIC_F_ACCUMULATE (the only flag accepted). Needs bins filled by pic_rebin.
 * Errors: INVALID_ARG (bad arguments, other flags, no bins), UNSUPPORTED (tile window over
 * the LDS limit); out-of-domain and non-finite positions are reported by pic_check. */
pic_status pic_deposit_rho(const pic_grid* grid, const pic_particles* p, pic_bins* bins,
                           float* rho, unsigned flags, hipStream_t stream);

/* Field gather: E and B interpolated to every particle with the deposition's shape
 * factors (field interpolation, Sec. 3.1). E_c is staggered half a cell along its own axis
 * (the J_c location), B_c half a cell along the two other axes (Yee faces); in 2D, Ez is
 * nodal and Bz is staggered in x and y. Fields: six float32 grids in the J layout (device,
 * read only). Outputs: six float32 arrays of nslots (device, caller-owned), 0 on gap
 * slots. With bins (filled by pic_rebin) each tile's window of the fields is read once into
 * LDS; without bins the gather reads global memory per particle. Errors: INVALID_ARG (bad
 * arguments, bins for another grid); stencil nodes outside the stored grid and
 * out-of-domain positions are reported by pic_check. */
pic_status pic_gather_fields(const pic_grid* grid, const pic_particles* p, pic_bins* bins,
                             const float* Ex, const float* Ey, const float* Ez,
                             const float* Bx, const float* By, const float* Bz, float* ex,
                             float* ey, float* ez, float* bx, float* by, float* bz,
                             hipStream_t stream);

/* Particle push: the field gather above, then the relativistic Boris rotation and the move
 * (the push half of the PIC cycle, Sec. 3.1, which the paper's Alg. 1 leaves to the host
 * code). With c = 1 and h = qm dt / 2: u- = u + h E, t = h B / gamma(u-),
 * s = 2 t / (1 + |t|^2), u+ = u- + (u- + u- x t) x s, u <- u+ + h E (float32, like the
 * stored momenta), then x <- x + dt u / gamma(u) (float64, like the positions) with the
 * operation order and periodic wrap of pic_drift. qm: charge-to-mass ratio of the species; E, B: as for
 * pic_gather_fields (device, read only). Updates x, y, z, ux, uy, uz of every valid
 * particle in place; gap slots and out-of-domain particles are left alone. With bins the
 * tile windows of the fields are read once into LDS (particles that left their tile are
 * pushed from global memory), and the bins' mover list is marked stale, so the next
 * pic_rebin detects movers itself. flags must be 0. Errors: INVALID_ARG (bad arguments,
 * non-finite qm or dt, bins for another grid); out-of-domain positions and stencil nodes
 * outside the stored grid are reported by pic_check. */
pic_status pic_push(const pic_grid* grid, pic_particles* p, pic_bins* bins, const float* Ex,
                    const float* Ey, const float* Ez, const float* Bx, const float* By,
                    const float* Bz, double qm, double dt, unsigned flags, hipStream_t stream);

/* Charge-conserving current (Esirkepov's density decomposition, the scheme the paper lists
 * as unsupported in Sec. 7): for each valid particle moving from (x_old, y_old, z_old) to
 * its current position in p during grid->dt, J_d on the faces i+1/2 is
 * -q W dx_d/dt times the running sum along d of W_d, with W_d built from the 1D nodal
 * weights at the two positions (order grid->order, o+2 nodes per dimension), so that
 * (rho_new - rho_old)/dt + div J = 0 holds for the charge density of pic_deposit_rho. In
 * 2D, Jz = q W v_z times the time-averaged weights (v from u). x_old, y_old, z_old: device
 * float64 arrays of nslots in p's slot order (z_old unused in 2D). Periodic moves take the
 * nearest image; a move of a cell or more along a dimension is skipped and reported by
 * pic_check (INVALID_PARTICLE), as are non-finite and out-of-domain positions. Overwrites
 * J unless PIC_F_ACCUMULATE (the only flag). With bins (filled by pic_rebin, for either
 * position) each tile accumulates in LDS and adds its window to J with float atomics;
 * without bins every particle adds its box with float atomics. The order of the atomic
 * additions varies, so results agree between calls to float32 rounding, not bitwise.
 * Errors: INVALID_ARG (bad arguments, dt zero or non-finite, bins for another grid). */
pic_status pic_deposit_esirkepov(const pic_grid* grid, const pic_particles* p, pic_bins* bins,
                                 const double* x_old, const double* y_old, const double* z_old,
                                 float* Jx, float* Jy, float* Jz, unsigned flags,
                                 hipStream_t stream);

/* Constant-velocity move of every valid particle, x += v dt (float64), with periodic
 * wrap: the stand-in for the particle push of the PIC cycle (Sec. 3.1; Alg. 1 moves the
 * particles between depositions). */
pic_status pic_drift(const pic_grid* grid, pic_particles* p, double dt, hipStream_t stream);

/* ---- batched patches ---------------------------------------------------------------
 * Many independent 3D patches (uneven sizes, densities and shape orders) deposited by one
 * persistent kernel that pulls (patch, tile) work items from a device counter, longest
 * items first (the tile decomposition of Sec. 4.1, batched). `bins[k]` must have been made
 * for `grids[k]` (its tile shape is the autotuner's choice, applied at pic_bins_create) and
 * filled by pic_rebin(PIC_REBIN_FULL) before the first call. `tune_cache_json` is a host
 * path to the autotuner's JSON cache or NULL; the plan reads its "blocks_per_cu" entry
 * (persistent workgroups per compute unit, capped by occupancy; default: occupancy).
 * pic_plan_create allocates device and pinned memory and synchronises; pic_plan_destroy
 * synchronises the device and frees them. Errors: INVALID_ARG (bad grid, bins for another
 * grid, unreadable cache), UNSUPPORTED (2D patch, tile window over the LDS limit). */
pic_status pic_plan_create(const pic_grid* grids, int npatch, pic_bins* const* bins,
                           const char* tune_cache_json, pic_plan** out);
pic_status pic_plan_destroy(pic_plan* plan);
/* Deposits every patch: particles[k] (host array of npatch descriptors; device SoA
 * pointers) into J3[3k], J3[3k+1], J3[3k+2] (host array of 3 npatch device pointers), with
 * the flags of pic_deposit (overwrite unless PIC_F_ACCUMULATE; PIC_F_DRIFT uses grids[k].dt;
 * PIC_F_EMIT_MOVERS fills each patch's mover list for pic_rebin). path: PIC_PATH_AUTO or
 * PIC_PATH_CELL_VALU (else UNSUPPORTED); under AUTO, patches the plan put on a matrix path
 * (pic_plan_patch_path) run as their own launches after the persistent one, except with
 * PIC_F_MIDPOINT, which only the per-cell path has. Enqueues three kernels on `stream`
 * (plus two per matrix-path patch) and nothing else once the pointer set has been uploaded: the first call with new pointers copies the
 * patch descriptors from pinned memory (and waits for the previous copy of that buffer),
 * which is refused (INVALID_ARG) while `stream` is capturing. Calls with unchanged pointers
 * allocate nothing, do not synchronise and contain no memset: safe to capture into a HIP
 * graph. Calls that overlap on one plan race. */
pic_status pic_deposit_batched(pic_plan* plan, const pic_particles* particles,
                               float* const* J3, int path, unsigned flags, hipStream_t stream);
/* Work items, persistent workgroups, workgroups per CU and LDS bytes per workgroup of a
 * plan (any pointer may be NULL). */
pic_status pic_plan_info(const pic_plan* plan, int* nitems, int* blocks, int* blocks_per_cu,
                         int64_t* lds_bytes);

/* Path choice of PIC_PATH_AUTO by density (the paper runs its matrix kernel in dense
 * regions and vector kernels in sparse ones: Sec. 6.1, Sec. 7). pic_tuning_load reads the
 * autotuner's JSON cache (host path; NULL clears it): each entry {"order": o, "ppc": p,
 * "path": "cell_valu" | "mfma_fp16" | "mfma_bf16" | "atomic", ...} names the fastest path
 * measured for shape order o at p particles per cell. AUTO then takes, for the grid's
 * order, the entry whose ppc is nearest (log scale) to the bins' particles per cell (the
 * count of the newest rebin statistics the host has read, else nslots / ((1 + slack)
 * nbins)); with no entry for the order, or no cache, the per-cell VALU path. The table is
 * process-wide. Errors: INVALID_ARG (unreadable file, malformed entry, unknown path). */
pic_status pic_tuning_load(const char* json_path);
/* The path PIC_PATH_AUTO would take now for these bins (PIC_PATH_CELL_VALU on bad input). */
int pic_auto_path(const pic_grid* grid, const pic_bins* bins);
/* The path a batched plan runs patch `patch` on under PIC_PATH_AUTO, fixed by the tuning
 * table when the plan was created (PIC_PATH_CELL_VALU or a matrix path; matrix-path patches
 * are launched on their own after the persistent kernel). */
pic_status pic_plan_patch_path(const pic_plan* plan, int patch, int* path);

/* Synchronises `stream` and reports the first device-side error recorded in `bins`
 * (PIC_OK if none); clears the flags. With bins NULL it reports the errors of calls made
 * without bins. (Device-side errors are the paper's silent cases made explicit: a particle
 * outside the domain, a non-finite position, bins without room.) */
pic_status pic_check(pic_bins* bins, hipStream_t stream);

const char* pic_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PIC_H */
