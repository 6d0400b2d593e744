/*
 * dpd.h -- C-ABI of the MI355X (gfx950) DPD solvent library.
 *
 * The library advances a periodic box of dissipative-particle-dynamics
 * solvent particles on one GPU.  One time step is the hot path of the
 * Mirheo paper (arXiv 1911.04712):
 *
 *   1. cell binning: particles are sorted into unit cells (edge r_c = 1) by a
 *      stable counting sort (Sec. 3.2; time-stepping step 1 of Sec. 3.1);
 *   2. pair forces: F_i = sum_j (F^C_ij + F^D_ij + F^R_ij) over r_ij < r_c
 *      (Sec. 2.1, Eqs. 2-5, with w_R = w = 1 - r, w_D = w^2,
 *      sigma^2 = 2 gamma kT), the random term being sigma w xi_ij / sqrt(dt);
 *      plus the optional periodic-Poiseuille body force (Sec. 4.2, Eq. 11);
 *   3. fused velocity-Verlet (Sec. 3.1, time-stepping step 5):
 *      v^{n+1/2} = v^{n-1/2} + dt f^n / m,  x^{n+1} = x^n + dt v^{n+1/2},
 *      followed by the periodic wrap; FP64 reductions of momentum, kinetic
 *      energy and the flow profile are fused into this step.
 *
 * xi_ij is Box-Muller applied to the first two words of Philox4x32-10
 * (Salmon et al., SC'11) with counter (min id, max id, step mod 2^32, 0)
 * and key (seed mod 2^32, seed >> 32); u1 = ((w0 >> 8) + 1) 2^-24,
 * u2 = (w1 >> 8) 2^-24, xi = sqrt(-2 ln u1) cos(2 pi u2).  `step` counts
 * force evaluations since dpd_set_state.
 *
 * Conventions shared by every call:
 *   - Every call returns an int status (DPD_OK or a negative DPD_E* code)
 *     and never throws.  dpd_last_error() gives a thread-local message for
 *     the last failing call of the calling thread.
 *   - Device memory is the caller's: the box lives inside a workspace the
 *     caller allocates (size from dpd_workspace_bytes) and frees after
 *     dpd_destroy.  The library never frees caller memory.  It allocates no
 *     device memory for particle state.
 *   - Pointers flagged `where` are host pointers for DPD_HOST and device
 *     pointers for DPD_DEVICE.
 *   - Work is enqueued on the HIP stream given at creation.  dpd_step is
 *     asynchronous; reads and stats synchronise that stream.
 *   - Particle arrays exchanged with the caller are row i = particle id i,
 *     three floats per row (x, y, z).  Internally particles are kept in cell
 *     order; dpd_read_raw exposes that order.
 *   - Units: r_c = 1, so a box of cells (L_x, L_y, L_z) has edges L_x, L_y,
 *     L_z; every edge is an integer >= 3.
 *   - Positions live on a fixed grid: every stored coordinate is a multiple
 *     of q = spacing of FP32 numbers at max(L_x, L_y, L_z)
 *     (2^(floor(log2 L_max) - 23)).  Positions passed to dpd_set_state are
 *     rounded to that grid; dpd_position_grid returns q.
 */
#ifndef DPD_H
#define DPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
enum {
    DPD_OK = 0,
    DPD_EINVAL = -1,     /* invalid argument (null pointer, size, range)        */
    DPD_ENOMEM = -2,     /* workspace or pool too small; host allocation failed */
    DPD_EDEVICE = -3,    /* a HIP call failed; message in dpd_last_error()     */
    DPD_ESTATE = -4,     /* call out of order (e.g. step before set_state)     */
    DPD_ENONFINITE = -5, /* a non-finite force, velocity or position, or a    */
                         /* pair force of magnitude >= 2^19, was seen          */
    DPD_EAGAIN = -6,     /* result not ready yet                                */
    DPD_EBUSY = -7,      /* no free slot or memory right now                    */
    DPD_ENOTFOUND = -8   /* unknown ticket                                      */
};

enum { DPD_HOST = 0, DPD_DEVICE = 1 };

/* most species of one box (dpd_set_species) */
enum { DPD_MAX_TYPES = 8 };

/* quantities for dpd_read */
enum {
    DPD_POS = 0,          /* x^n (after the last step), wrapped into [0, L)           */
    DPD_VEL = 1,          /* stored half-step velocity v^{n-1/2}                      */
    DPD_VEL_CENTRED = 2,  /* v^{n-1/2} - dt f^{n-1} / (2m): time level of the last force */
    DPD_FORCE = 3         /* f^{n-1}: total force of the last step (pairs + body)     */
};

/* flags of dpd_params.flags */
enum {
    DPD_FLAG_VIRIAL = 1,          /* also accumulate the conservative virial each step   */
    DPD_FLAG_REFERENCE_FORCE = 2, /* use the one-thread-per-particle gather kernel for
                                     the pair forces instead of the LDS tile kernel (same
                                     bits; a reference for validation)                    */
    DPD_FLAG_BODY_UNIFORM = 4     /* body force +body_f along flow_axis everywhere (flow
                                     between walls) instead of Eq. 11's two halves        */
};

/* walls of dpd_params.wall_kind (Sec. 2.3): the wall surface is the zero of a
 * signed distance function, negative in the fluid */
enum {
    DPD_WALL_NONE = 0,
    DPD_WALL_PLATES = 1,  /* two plates normal to grad_axis: sdf = |y - L_y/2| - wall_h   */
    DPD_WALL_PIPE = 2,    /* a pipe along flow_axis through the box centre:
                             sdf = (distance to the axis) - wall_h                      */
    DPD_WALL_CYLINDERS = 3 /* two coaxial cylinders along flow_axis through the box
                             centre (Taylor-Couette, Sec. 4.3): sdf = max(wall_r_in - q,
                             q - wall_h), q the distance to the axis; the inner one
                             turns at omega_in, the outer at omega_out             */
};

typedef struct dpd_box_s* dpd_box;

/* Box geometry: edges in unit cells (each >= 3) and particle count. */
typedef struct {
    int32_t cells[3];
    int32_t reserved;     /* must be 0 */
    int64_t n;            /* 0 <= n <= 715 827 882 ((2^31 - 1) / 3: row offsets
                             3 i of the n x 3 arrays stay 32-bit)            */
} dpd_geom;

/* Model parameters (Sec. 2.1, Eqs. 3-5; Sec. 4.2, Eq. 11).
 * sigma = sqrt(2 gamma kT) is derived.  Required: dt > 0, mass > 0,
 * gamma >= 0, kT >= 0, all finite; flow_axis != grad_axis in {0,1,2};
 * profile_bins in [0, 4096]; 0 <= kexp <= 1. */
typedef struct {
    double a;             /* conservative amplitude                                */
    double gamma;         /* dissipative coefficient                               */
    double kT;            /* temperature                                           */
    double dt;            /* time step                                             */
    double mass;          /* particle mass                                         */
    double body_f;        /* periodic-Poiseuille amplitude f (0 = no body force):
                             -f along flow_axis where the grad_axis coordinate is
                             <= L/2, +f above                                      */
    int32_t flow_axis;
    int32_t grad_axis;
    int32_t profile_bins; /* slabs along grad_axis for the flow profile (0 = off)  */
    int32_t flags;        /* DPD_FLAG_*                                            */
    double kexp;          /* exponent k of the random-term kernel w_R = (1 - r)^k;
                             the dissipative kernel is w_D = w_R^2 and the
                             conservative weight stays 1 - r (Sec. 2.1).
                             0 < k <= 1; 0 selects k = 1                           */
    int32_t wall_kind;    /* DPD_WALL_*: a fluid particle whose drift ends inside the
                             wall (sdf > 0) is put back at the collision point, the
                             sdf's zero along the drift, with its velocity reversed
                             (bounce-back, Sec. 3.3)                               */
    int32_t reserved2;    /* must be 0                                             */
    double wall_h;        /* plate half-gap, pipe radius or outer cylinder radius; the
                             wall and its frozen layer (thickness r_c = 1) must fit
                             inside the box: wall_h + 1 < L/2 on every axis the sdf
                             depends on                                            */
    double wall_r_in;     /* DPD_WALL_CYLINDERS: inner radius, 0 < wall_r_in < wall_h */
    double omega_in;      /* DPD_WALL_CYLINDERS: angular velocities of the inner and   */
    double omega_out;     /* outer cylinder, right-handed about +flow_axis.  A wall's
                             velocity is omega x r; a bounce reverses the velocity in
                             the frame of the wall (v -> 2 u_wall - v), and a turning
                             cylinder's frozen particles turn rigidly with it by
                             omega dt per step, carrying its velocity               */
} dpd_params;

/* Diagnostics, all reduced in FP64 on the GPU in a fixed order.
 * "last" values describe the most recent step n -> n+1. */
typedef struct {
    double momentum[3];       /* last: sum m v^{n+1/2}                                 */
    double ke_half;           /* last: sum m |v^{n+1/2}|^2 / 2                        */
    double ke_centred;        /* last: sum m |v^{n-1/2} + dt f^n/(2m)|^2 / 2           */
    double kT_centred;        /* last: 2 ke_centred / (3 (N - 1)), N = free particles  */
    double virial;            /* last: sum_{i<j} r_ij . F^C_ij (DPD_FLAG_VIRIAL)      */
    double pressure;          /* last: rho kT_centred + virial / (3 V)                */
    double sum_kT_centred;    /* sums over the steps since the last reset ...         */
    double sum_pressure;
    double sum_momentum[3];
    uint64_t nsamples;        /* ... and their number                                  */
    uint64_t step;            /* force evaluations since dpd_set_state                 */
    int32_t nonfinite;        /* 1 if a non-finite value was seen since set_state      */
    int32_t escaped;          /* 1 if a particle moved >= 1 per axis in one step       */
} dpd_stats;

/* ---- single box -------------------------------------------------------- */

/* Spacing q of the position grid of a geometry (see conventions). */
int dpd_position_grid(const dpd_geom* geom, double* q);

/* Bytes of device memory the box needs (also its admission footprint). */
int dpd_workspace_bytes(const dpd_geom* geom, size_t* bytes);

/* Create a box inside `dev_ws` (device memory of at least
 * dpd_workspace_bytes, 256-byte aligned), working on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  The workspace must outlive the
 * box.  DPD_ENOMEM if ws_bytes is too small. */
int dpd_create(const dpd_geom* geom, void* dev_ws, size_t ws_bytes, void* hip_stream, dpd_box* out);

/* Set model parameters; validated as documented at dpd_params. */
int dpd_set_params(dpd_box box, const dpd_params* params);

/* Species: several fluids in one box, each pair of species with its own
 * conservative amplitude, dissipative coefficient and cutoff (fluids of
 * different viscosity side by side, Sec. 2.3, Sec. 5.2 and Sec. 5.3 of the
 * paper; a cross entry gamma = 0 couples two fluids through the
 * conservative force alone; several cutoffs, Sec. 3.1).  a_tab, gamma_tab
 * and rc_tab are host arrays of ntypes x ntypes doubles, row-major,
 * symmetric, finite, gamma >= 0, 1/16 <= rc <= 1 (the cell edge; rc_tab
 * NULL: every cutoff 1); the pair (s, t) then takes a = a_tab[s][t],
 * gamma = gamma_tab[s][t], sigma = sqrt(2 gamma kT) and the cutoff
 * r_c = rc_tab[s][t] with w = 1 - r / r_c, and dpd_params.a / .gamma are
 * ignored.  kT, dt, the mass and the kernel exponent stay shared.  ntypes in
 * 1..DPD_MAX_TYPES; ntypes = 0 returns to one species described by
 * dpd_params.  DPD_EINVAL if a particle already has a species >= ntypes.
 * The tables are copied; may be called at any time (also between steps) and
 * take effect from the next step. */
int dpd_set_species(dpd_box box, int32_t ntypes, const double* a_tab, const double* gamma_tab,
                    const double* rc_tab);

/* Number of species set by dpd_set_species (0: one species from params). */
int dpd_get_species(dpd_box box, int32_t* ntypes);

/* Species of each particle: type_host[i] (host array of n int32) is the
 * species of particle id i, each in 0..ntypes-1 (DPD_EINVAL otherwise,
 * DPD_ESTATE before dpd_set_species or without a state).  dpd_set_state and
 * dpd_init_random make every particle species 0.  Synchronises. */
int dpd_set_types(dpd_box box, const int32_t* type_host);

/* Read the species back, row i = particle id i (host array of n int32).
 * Synchronises. */
int dpd_get_types(dpd_box box, int32_t* type_host);

/* Frozen wall particles (Sec. 2.3): frozen_host[i] != 0 marks particle id i
 * (host array of n bytes) as part of a wall's frozen layer.  Frozen
 * particles take part in every pair force but move only with their wall
 * (their velocity is set to the wall's: 0 for plates and pipes, omega x r
 * for a turning cylinder, which turns them), and are left out of the momentum,
 * kinetic energy, kT (3 (N_fluid - 1) degrees of freedom) and flow profile.
 * dpd_set_state and dpd_init_random clear the marks.  DPD_ESTATE without a
 * state; DPD_EINVAL if fewer than 2 particles stay free.  Synchronises. */
int dpd_set_frozen(dpd_box box, const uint8_t* frozen_host);

/* The frozen marks, row i = particle id i (host array of n bytes, 0 or 1). */
int dpd_get_frozen(dpd_box box, uint8_t* frozen_host);

/* Signed wall distance of every particle's current position, row i =
 * particle id i (host array of n floats; negative in the fluid), for the
 * box's wall_kind and wall_h (DPD_ESTATE when the params name no wall).
 * Frozen layers are cut from an equilibrated fluid with it.  Synchronises. */
int dpd_wall_sdf(dpd_box box, float* sdf_host);

/* Cell-tile shape of the LDS pair-force kernel: tile[3] edges in cells
 * (each 1..16), or {0, 0, 0} for the default: from a short list per
 * density class (rho <= 4.5 or above), the first shape that gives at least
 * 512 tiles and fits a CU's LDS, each with its own workgroup size.
 * Positions, velocities and forces do not depend on the tile shape
 * (bitwise); the FP64 diagnostics are folded per tile, in a fixed order, so
 * their last bits follow the tile. */
int dpd_set_tile(dpd_box box, const int32_t tile[3]);

/* The tile shape in use (after clamping to the box). */
int dpd_get_tile(dpd_box box, int32_t tile[3]);

/* Workgroup size of the LDS pair-force kernel: 256, 512 or 1024 threads
 * (4, 8 or 16 waves sharing one tile), or 0 for the default (the default
 * tile's own size, 512 with a tile set by dpd_set_tile).  Results do not
 * depend on it (bitwise).  DPD_EINVAL for other values, or if the current
 * tile would then need more LDS than a CU has. */
int dpd_set_force_threads(dpd_box box, int32_t threads);

/* The workgroup size in use. */
int dpd_get_force_threads(dpd_box box, int32_t* threads);

/* Autotuner: time the LDS pair-force kernel on the box's current positions
 * for a fixed list of tile shapes, each with 256, 512 and 1024 threads per
 * workgroup (those whose LDS fits a CU), `reps` launches each with HIP
 * events on the box stream, keep the fastest pair and report the tile in
 * tile_out (the workgroup size through dpd_get_force_threads) and *ms_out
 * (mean ms per launch; may be NULL).  The box is timed with the kernel its
 * steps run, forces with the kick-drift fused (with the walls' conditions
 * when it has walls); the state, the
 * diagnostics and the flow profile are put back afterwards.  The
 * state does not advance (the box is left holding its cell list, as after
 * dpd_build_cells) and, since the trajectory does not depend on the tile,
 * no position, velocity or force changes.  Synchronises. */
int dpd_tune_tile(dpd_box box, int32_t reps, int32_t tile_out[3], double* ms_out);

/* Autotuner cache: a JSON file (path NULL or "" turns the cache off) that
 * dpd_tune_tile and dpd_batch_tune consult before timing anything.  Entries
 * are keyed by the GPU architecture, the revision of the force kernel's
 * sources the library was built from, and the box (cells, particles per
 * occupied cell, species table on or off, kernel exponent k = 1 or not) or,
 * for a batch, the list of its boxes with their own tile requests.  A hit
 * applies the stored tile and workgroup size (if they still fit a CU's LDS)
 * without timing and reports the stored ms; a miss times as usual and adds
 * the winner to the file (rewritten whole; an unwritable place keeps the
 * entries in memory only).  Process-wide; thread-safe.  Trajectories never
 * depend on the tile, so the cache changes speed (and the last bits of the
 * FP64 diagnostics) only. */
int dpd_set_tune_cache(const char* path);

/* Set the 64-bit seed of the random term. */
int dpd_set_seed(dpd_box box, uint64_t seed);

/* Load the state: pos and vel are n x 3 floats, row i = particle id i.
 * pos must lie in [0, L) per axis (DPD_EINVAL otherwise; checked on the
 * host for DPD_HOST, on the device for DPD_DEVICE), and is rounded to the
 * position grid.  vel is taken as v^{-1/2}.  Resets the step counter and
 * the accumulators.  Synchronises the stream. */
int dpd_set_state(dpd_box box, const float* pos_n3, const float* vel_n3, int where);

/* Set the step counter: the index of the next force evaluation, which
 * selects the random term's noise.  With dpd_set_state of a run's DPD_POS and
 * DPD_VEL (and dpd_set_types / dpd_set_frozen), this resumes the run: the
 * trajectory continues bit for bit, whatever the internal order (forces are
 * order-independent sums).  DPD_ESTATE without a state.  Synchronises. */
int dpd_set_step(dpd_box box, uint64_t step);

/* Load a random state generated on the device: positions uniform on [0, L)
 * (on the position grid), velocities Maxwellian N(0, kT/m) per component
 * with the centre-of-mass velocity removed, particle i = id i.  Drawn from
 * Philox4x32-10 keyed by `seed` on counters disjoint from the pair noise.
 * Needs params (for m).  Resets the step counter and accumulators.
 * Synchronises. */
int dpd_init_random(dpd_box box, double kT, uint64_t seed);

/* Bin the current state into cells without stepping (so dpd_read_raw
 * reports the cell list of the current positions). */
int dpd_build_cells(dpd_box box);

/* Enqueue nsteps >= 0 full steps (bin, forces, integrate).  Requires
 * params, seed and state.  Asynchronous. */
int dpd_step(dpd_box box, int64_t nsteps);

/* Capture, without running anything, the HIP graphs that dpd_step(box,
 * nsteps) would launch now (runs are replayed graphs of up to 64 steps plus
 * one graph of the remainder; the last few lengths stay cached until the
 * tile, flags or kernel choice change), so that a later dpd_step of that
 * length spends no time capturing.  Requires params, seed and state.
 * DPD_EDEVICE if a capture fails. */
int dpd_prepare_steps(dpd_box box, int64_t nsteps);

/* Time the pair-force kernel alone: `reps` (1..10000) back-to-back launches
 * on the box stream between two HIP events, after one untimed launch; *ms_out
 * is the mean ms per launch.  The forces are those of the current positions
 * (binned first if needed); the state does not advance, and afterwards the
 * box holds the cell list of its current state as after dpd_build_cells.
 * Synchronises. */
int dpd_time_force(dpd_box box, int32_t reps, double* ms_out);

/* Copy one quantity (DPD_POS, DPD_VEL, DPD_VEL_CENTRED, DPD_FORCE) to
 * out_n3 (n x 3 floats, row = id).  DPD_FORCE and DPD_VEL_CENTRED need at
 * least one step.  Synchronises. */
int dpd_read(dpd_box box, int what, float* out_n3, int where);

/* The cell list of the last binning: pos4 / vel4 (n x 4 floats, may be
 * NULL) in cell order, the 4th float of pos4 carrying the particle id as
 * int32 bits; cell_start (n_cells + 1 int32, may be NULL).  Synchronises. */
int dpd_read_raw(dpd_box box, float* pos4, float* vel4, int32_t* cell_start, int where);

/* Diagnostics; DPD_ENONFINITE when the nonfinite flag is set (stats are
 * still filled).  Synchronises. */
int dpd_get_stats(dpd_box box, dpd_stats* out);

/* Accumulated flow profile: sum of the time-centred flow-axis velocity and
 * particle count per slab along grad_axis, over the steps since the last
 * reset; nbins must equal params.profile_bins.  Synchronises. */
int dpd_get_profile(dpd_box box, double* sum_v, double* count, int32_t nbins);

/* Zero the accumulated sums (stats sums and the profile). */
int dpd_reset_accumulators(dpd_box box);

/* Destroy a box (NULL-safe).  Synchronises; the workspace may be freed after. */
int dpd_destroy(dpd_box box);

/* Run nsteps >= 1 steps eagerly (no graph) and return the mean device time
 * per step of each stage in ms_out[4]: binning (scan, scatter, gather),
 * pair forces (with the kick-drift, which is fused into the force kernel
 * except on the reference force path), virial (0 unless DPD_FLAG_VIRIAL),
 * integrate (0 when fused).  Each stage is timed by events that its first kernel records as it
 * starts and its last as it ends (hipExtLaunchKernel), so the times are the
 * kernels' own, from the first one's start to the last one's end.  The fold
 * of the reductions, which a graph runs inside the next step's gather, runs
 * after the timed stages.  The steps advance the box like dpd_step.
 * Synchronises. */
int dpd_profile_steps(dpd_box box, int64_t nsteps, double* ms_out);

/* ---- a run that allocates nothing -------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The box
 * lives in an array of DPD_STATIC_WS_BYTES that the library holds in device
 * memory (one per GPU it runs on, kept until the process ends), instead of a
 * caller workspace. */

/* Size of the library's static per-GPU machine array: boxes whose
 * dpd_workspace_bytes is at most this (a 48^3 box at density 3 needs 40 MB). */
#define DPD_STATIC_WS_BYTES (64u * 1024u * 1024u)

/* One whole run, equal bit for bit to dpd_create (on any workspace) +
 * dpd_set_params + dpd_set_seed + dpd_set_state(pos_n3, vel_n3, DPD_DEVICE)
 * + dpd_set_step(step0) + dpd_step(nsteps) + dpd_read(DPD_POS / DPD_VEL,
 * DPD_DEVICE) + dpd_get_stats + dpd_destroy, with the box in the static
 * array of the current GPU.
 *   pos_n3, vel_n3:          device, n x 3 floats, row = id (inputs; as for
 *                            dpd_set_state: pos in [0, L), rounded to the grid)
 *   pos_out_n3, vel_out_n3:  device, n x 3 floats: x^{step0+nsteps} and
 *                            v^{step0+nsteps-1/2}; may not overlap the inputs
 *   stats:                   host, may be NULL
 * One species, no frozen particles (walls set in params act on the fluid by
 * bounce-back alone), the default tile.  The steps are
 * launched directly on hip_stream (no graph), and the call synchronises it.
 * It calls no hipMalloc, hipFree or other allocating routine.  Errors:
 * DPD_EINVAL (geometry, params, null arrays, positions), DPD_ENOMEM when the
 * box needs more than DPD_STATIC_WS_BYTES (checked before any GPU call),
 * DPD_ENONFINITE as dpd_get_stats (outputs still written), DPD_EDEVICE.
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents (each call clears what must start at zero): calls that
 * overlap on one GPU, from several threads or streams, race and must not be
 * made. */
int dpd_run_static(const dpd_geom* geom, const dpd_params* params, uint64_t seed, uint64_t step0,
                   const float* pos_n3, const float* vel_n3, int64_t nsteps, float* pos_out_n3,
                   float* vel_out_n3, dpd_stats* stats, void* hip_stream);

/* ---- batches of independent boxes ------------------------------------------
 * A batch steps many boxes (uneven sizes, own parameters and seeds) with one
 * launch per kernel for all of them, and a run of up to 1024 steps is a
 * single launch of one captured HIP graph.  Each box computes exactly what it
 * would alone (same work partition, same bits): ids, step counters and seeds
 * are per box, so no random number depends on the batch. */
typedef struct dpd_batch_s* dpd_batch;

/* Device bytes of the batch tables (descriptors and work prefixes). */
int dpd_batch_workspace_bytes(int32_t nboxes, size_t* bytes);

/* Group existing boxes (1..65536, distinct) into a batch working on
 * `hip_stream` with its tables in `dev_ws` (256-byte aligned, caller-owned,
 * must outlive the batch).  The boxes stay owned by the caller and must
 * outlive the batch. */
int dpd_batch_create(const dpd_box* boxes, int32_t nboxes, void* dev_ws, size_t ws_bytes, void* hip_stream,
                     dpd_batch* out);

/* Batch autotuner: bins every box once and times the batched pair-force
 * launch (`reps` launches per configuration, HIP events on the batch stream)
 * for the boxes' current tiles and for each tile shape of the single-box
 * list applied to all boxes, each with 256, 512 and 1024 threads per
 * workgroup (skipping configurations whose LDS does not fit a CU for some
 * box); keeps the fastest.  tile_out receives the uniform tile, or
 * {0, 0, 0} when the boxes' own tiles were fastest, and every box the
 * winning workgroup size (one launch has one; a batch runs with its first
 * box's); *ms_out (may be NULL) the mean ms per batched launch.  The batch
 * is timed with the kernel its steps run (forces with the kick-drift fused);
 * every box's state, diagnostics and flow profile are put
 * back afterwards.  Boxes must have params, seed and
 * state and must not hold a bare cell list; afterwards every box holds its
 * cell list (dpd_batch_step then starts from it).  No position, velocity or
 * force changes: the state does not advance and the trajectory does not
 * depend on the tile.
 * Synchronises. */
int dpd_batch_tune(dpd_batch batch, int32_t reps, int32_t tile_out[3], double* ms_out);

/* Advance every box by nsteps.  Every box needs params, seed and state;
 * either no box or every box holds a bare cell list (dpd_build_cells,
 * dpd_tune_tile or dpd_batch_tune without a step since).  Picks up each box's current parameters and tile.  Waits for
 * work pending on the boxes' streams; later work on a box's stream waits for
 * the batch.  Runs of 64..1024 steps are one launch of a captured graph
 * (kept for the next call of the same length); shorter runs are launched
 * directly.  Asynchronous on the batch stream. */
int dpd_batch_step(dpd_batch batch, int64_t nsteps);

/* Destroy a batch (NULL-safe; the boxes are untouched).  Synchronises. */
int dpd_batch_destroy(dpd_batch batch);

/* ---- serving ------------------------------------------------------------------
 * A request server over one caller-owned device pool.  Requests are admitted
 * in arrival order when a slot is free and their footprint
 * (dpd_workspace_bytes) fits in the pool; admitted requests keep their state
 * resident; each pump queues one quantum of steps for all active requests,
 * as one batch per density class (rho <= 4.5 and above, each at its own
 * launch shape), on the server stream without waiting for it; requests that
 * finish with a quantum have their results copied to pinned host memory
 * behind it and are completed (memory freed) by a later pump or poll once
 * those copies are done; waiting requests are admitted (set up on a second
 * stream of the server's own) as slots and memory free up, so requests that
 * arrive while others run join the next quantum.  At most two quanta are in
 * flight.  A request's result is the same bits alone or in a mix.  A request is one species without frozen particles: its params may
 * name a wall (fluid particles then bounce off the SDF surface) but carry no
 * frozen layer; species and frozen layers need a box of one's own. */
typedef struct dpd_server_s* dpd_server;

typedef struct {
    dpd_geom geom;
    dpd_params params;
    uint64_t seed;           /* seed of the random term                                  */
    int64_t nsteps;          /* steps to run (>= 0)                                      */
    const float* pos_n3;     /* initial state, host, n x 3 (copied at submit); both NULL: */
    const float* vel_n3;     /*   generated on the device as by dpd_init_random           */
    double init_kT;          /* temperature of the generated velocities                  */
    uint64_t init_seed;      /* seed of the generated state                              */
} dpd_request;

typedef struct {
    dpd_stats stats;         /* diagnostics at the end of the run                        */
    int32_t status;          /* DPD_OK, DPD_ENONFINITE or the error that retired it       */
    int32_t reserved;
    double t_submit, t_admit, t_done;   /* seconds on the server's steady clock          */
} dpd_result;

/* Create a server on `dev_pool` (device, 256-byte aligned, caller-owned,
 * outlives the server) with at most max_slots (1..4096) active requests,
 * working on `hip_stream`.  A small part of the pool holds the batch tables. */
int dpd_server_create(void* dev_pool, size_t pool_bytes, int32_t max_slots, void* hip_stream, dpd_server* out);

/* Queue a request (never blocks; DPD_ENOMEM if it could never fit). */
int dpd_server_submit(dpd_server server, const dpd_request* req, uint64_t* ticket);

/* Complete requests whose result copies are done, admit, queue one quantum
 * of up to quantum_steps steps for all active requests (never past a
 * request's end) and the result copies of those it finishes.  *ran_steps
 * (may be NULL) receives the steps queued.  Waits only for the quantum
 * queued by the previous pump (at most two in flight), or, with no request
 * active or waiting, for the last result copies. */
int dpd_server_pump(dpd_server server, int32_t quantum_steps, int32_t* ran_steps);

/* DPD_EAGAIN until the request is done; then fills the result and, if not
 * NULL, the final state (n x 3 floats each, id order) and forgets the ticket
 * (DPD_ENOTFOUND afterwards). */
int dpd_server_poll(dpd_server server, uint64_t ticket, dpd_result* res, float* pos_n3, float* vel_n3);

/* Requests waiting, active, and particle-steps completed so far. */
int dpd_server_counts(dpd_server server, int32_t* queued, int32_t* active, int64_t* particle_steps);

/* Seconds since the server was created (the clock of dpd_result). */
double dpd_server_clock(dpd_server server);

/* Destroy (NULL-safe): active requests are dropped.  Synchronises. */
int dpd_server_destroy(dpd_server server);

/* Thread-local message of the last error (never NULL). */
const char* dpd_last_error(void);

/* ---- diagnostics of the random term (used by parity tests) -------------- */

/* Philox4x32-10 words of n (counter, key) tuples on the GPU:
 * ctr4 (n x 4 uint32), key2 (n x 2 uint32) -> out4 (n x 4 uint32).
 * All pointers are `where`.  Synchronises. */
int dpd_philox(const uint32_t* ctr4, const uint32_t* key2, int64_t n, uint32_t* out4, int where,
               void* hip_stream);

/* Box-Muller of n word pairs on the GPU, in the FP32 arithmetic of the
 * force kernel: xi = sqrt(-2 ln u1) cos(2 pi u2).  Synchronises. */
int dpd_box_muller(const uint32_t* w0, const uint32_t* w1, int64_t n, float* xi, int where,
                   void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* DPD_H */
