/*
 * hmc.h -- C ABI of the MI355X (gfx950) library for the hot path of the hybrid Monte Carlo
 * (HMC) method of Zhang, Bartel & Lusk, "Parallelized Hybrid Monte Carlo Simulation of
 * Stress-Induced Texture Evolution" (arXiv:1009.0457):
 *
 *   a checkerboard Potts sweep over a periodic K^3 lattice of grain orientations in which
 *   every trial flip gets a grain-boundary energy change (Sec. 3, Eq. H_1) and an elastic
 *   energy change from a local constant-traction zone solve (Sec. 3, Eq. H_1 second form,
 *   Fig. 1), is accepted by Metropolis (Sec. 3, Eq. metrop_1) with counter-based Philox
 *   variates, and sees the stress of a global explicit elastic relaxation (Sec. 5) that is
 *   refreshed between sweeps.
 *
 * Conventions for every entry point:
 *   - Lattice sites are indexed i = x + K*(y + K*z); device arrays are dense in that order.
 *   - Voigt order xx, yy, zz, yz, xz, xy; engineering shear strains; stiffness and stress in
 *     GPa; elastic energies in GPa * voxel (voxel volume = 1).
 *   - Stress-field arrays are 6 component planes of K^3 floats (structure of arrays).
 *   - "dev" pointers are HIP device pointers on the context's device; "host" pointers are
 *     ordinary host memory.  The library never keeps a caller pointer beyond the call except
 *     the workspace passed to hmc_create, which it borrows until hmc_destroy.
 *   - The library allocates no device memory: everything lives in the caller's workspace.
 *   - Work is enqueued on the context's stream; only calls that return host values
 *     (hmc_energy, hmc_texture_histogram, hmc_get_stats, hmc_get_macro_strain) synchronise
 *     that stream.
 *   - Every call returns an hmc_status; nothing throws or aborts across the ABI.  On error
 *     hmc_last_error(ctx) holds a message.  A context is not thread-safe; separate contexts
 *     are independent.
 */
#ifndef HMC_H_
#define HMC_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HMC_OK = 0,
    HMC_EINVAL = 1,    /* bad argument (null pointer, out-of-range value) */
    HMC_ESHAPE = 2,    /* unsupported lattice shape: K odd, K < 2, K > 1024, K < 2h+2 with
                          elasticity, Q outside [1, 32767], workspace too small */
    HMC_ESTATE = 3,    /* call out of order (e.g. sweep before spins/orientations, elastic
                          sweep before a stress field exists) */
    HMC_EDEVICE = 4,   /* a HIP call or kernel launch failed */
    HMC_ENUMERIC = 5   /* non-finite input (Euler angles, load, parameters) or singular C;
                          or, from a call that synchronises the stream (hmc_energy,
                          hmc_texture_histogram, hmc_get_stats, hmc_get_macro_strain,
                          hmc_elastic_forward), a non-finite value that a kernel met since the
                          last such report: an injected stress field, the global solve's stress
                          field or stored energy, or a zone solve's energy change (whose trial
                          was rejected; a non-finite input to one trial's zone can also reach
                          the other trials solved in the same wavefront, which are rejected
                          too).  The report clears it; the call's outputs are still written. */
} hmc_status;

typedef struct hmc_ctx_s* hmc_ctx;

/* Run parameters.  hmc_default_params fills every field from (K, neighbors, zone_h). */
typedef struct {
    int32_t K;              /* lattice edge; even, 2 <= K <= 1024 */
    int32_t neighbors;      /* 6 (two-colour red/black) or 26 (eight-colour 2x2x2) */
    int32_t proposal;       /* 0: spin of a random neighbour slot; 1: uniform other state */
    int32_t zone_h;         /* zone half-width h in 0..3: the zone has (2h+1)^3 voxels */
    int32_t zone_steps;     /* heavy-ball steps n_r of each zone solve, >= 0 */
    int32_t refresh_every;  /* R >= 1: hmc_sweep refreshes the stress before sweep s when
                               s % R == 0 */
    int32_t refresh_steps;  /* explicit steps of each such warm refresh */
    int32_t cold_steps;     /* explicit steps hmc_stress_refresh uses for cold_start with
                               n_steps < 0 */
    int32_t zone_variant;   /* zone-solve kernel: 0 automatic (3 for h >= 1; 2 for h = 0),
                               1 one wavefront per trial, 2 node columns across a
                               256-lane work-group (h <= 2), 3 node columns of whole trials per
                               wavefront, x neighbours exchanged by cross-lane moves
                               (1 <= h <= 3), one wavefront per work-group; 4 and 5 the same
                               kernel with two and four wavefronts (twice and four times the
                               trials) per work-group.  Other values: HMC_EINVAL. */
    int32_t zone_screen;    /* 1: skip the zone solve of a trial whose rejection is already
                               certain: the point-zone energy 1/2 sigma_p.(S_old - S_new) sigma_p
                               is a lower bound of the zone's (its relaxation only adds
                               stiffness), so J*gb + lambda_el * that bound above the trial's
                               Metropolis threshold (plus a floating-point margin) rejects it.
                               Decisions are those of the full solve; the trial's record then
                               carries flag 8 and no dPi.  0: solve every real flip. */
    int32_t refresh_tile_z; /* node layers per work-group of the explicit global step and of its
                               adjoint, at most: 1, 2, 4, 8, 16 or 32, or 0 to pick the deepest
                               tile that still gives at least 1024 work-groups of 256 threads
                               (2 rather than 1; 1 if none does): shallower tiles recompute more
                               halo voxels but fill the GPU on small lattices.  A lattice of edge
                               K takes n = ceil(K / t) z-tiles of ceil(K / n) layers each.  Other
                               values: HMC_EINVAL. */
    int32_t material_points;/* material points of the global solve: 0 or 1, one per site at the
                               centre of its voxel (mesh = lattice, the default); 8, two per
                               direction in background cells of 2 x 2 x 2 sites (the paper's MPM
                               arrangement, Appendix; mesh of (K/2)^3 nodes, K >= 4; no adjoint
                               and no displacement read-out).  Set it
                               with hmc_set_material_points, which also sets glob_*.  Other
                               values: HMC_EINVAL. */
    double J;               /* grain-boundary energy per unlike bond (MC units) */
    double kT;              /* Monte Carlo temperature T_mc (MC units), > 0 */
    double C11, C12, C44;   /* cubic stiffness in the crystal frame (GPa) */
    double lambda_el;       /* MC energy per GPa*voxel (Sec. 4, Eq. elamc); 0 turns the
                               elastic term and all elastic buffers off */
    double zone_alpha, zone_beta;   /* zone heavy-ball step and momentum */
    double glob_alpha, glob_beta;   /* global relaxation step and momentum (displacements) */
    double glob_alphaE;             /* global relaxation step of the macroscopic strain */
    uint64_t seed;          /* Philox key: (seed & 0xffffffff, seed >> 32) */
} hmc_params;

/* Per-trial record written by hmc_colour_pass when a record array is given (24 bytes). */
typedef struct {
    int32_t q_new;   /* proposed state */
    int32_t gb;      /* change in the number of unlike neighbour bonds (energy J*gb) */
    float dPi;       /* zone energy change in GPa*voxel (0 unless a zone was solved) */
    uint32_t r1;     /* Metropolis variate: accept iff dE <= 0 or r1 < 2^32 exp(-dE/kT) */
    int32_t flags;   /* bit 0: q_new differs from the current state; bit 1: accepted;
                        bit 2: a zone solve produced dPi; bit 3: rejected by the lower-bound
                        screen without a zone solve */
    int32_t reserved;
} hmc_trial_record;

/* Counters accumulated since hmc_create (or the last hmc_reset_stats). */
typedef struct {
    int64_t site_trials;    /* trials, no-ops included (K^3 per sweep) */
    int64_t real_flips;     /* trials whose proposal differs from the current state */
    int64_t zone_solves;    /* zone solves run */
    int64_t accepted;       /* accepted real flips */
    int64_t screened;       /* real flips rejected by the lower-bound screen (zone_screen) */
    int64_t refresh_steps;  /* explicit global steps run */
} hmc_stats;

/* Fill *p with the defaults for a K^3 lattice: J = 1, kT = 0.5, the workload's nickel
 * constants C11/C12/C44 = 246.5/147.3/124.7 GPa, lambda_el = 2.6667e6/K (Sec. 4 with the
 * Table 1 values and l0 = 1 mm), n_r = 50 for h <= 1 and 200 otherwise, R = 10,
 * refresh 200 / cold 2000 steps, seed 1, and Polyak heavy-ball constants
 * alpha = 4/(sqrt(L)+sqrt(mu))^2, beta = ((sqrt(L)-sqrt(mu))/(sqrt(L)+sqrt(mu)))^2 with
 * L = 4 max(C11+2C12, C11-C12, 2C44), mu = (C11-C12)/2 (2 sin(pi/K))^2 for the global grid
 * and mu = (C11-C12)/2 / (2h+1)^2 for the zone.  Returns HMC_EINVAL for bad arguments. */
hmc_status hmc_default_params(hmc_params* p, int32_t K, int32_t neighbors, int32_t zone_h);

/* Set p->material_points (0, 1 or 8) and the global relaxation constants glob_alpha, glob_beta
 * and glob_alphaE for it, from p->K and p's stiffness: Polyak's heavy-ball values for the
 * stability bound L = 4 (one point per voxel) or 8 (eight per cell) times the largest Mandel
 * eigenvalue of the stiffness and the slowest shear wave of the mesh, 1/2 (C11 - C12)
 * (2 sin(pi/n))^2 with n = K or K/2 mesh cells per edge.  HMC_EINVAL for other counts. */
hmc_status hmc_set_material_points(hmc_params* p, int32_t n);

/* Bytes of device workspace hmc_create needs for these parameters and Q grains
 * (0 if the parameters are invalid). */
size_t hmc_workspace_bytes(const hmc_params* p, int32_t Q);

/* Create a context on the current HIP device.  dev_workspace: device buffer of at least
 * hmc_workspace_bytes(p, Q) bytes, 256-byte aligned, borrowed until hmc_destroy.
 * stream: the stream all work is enqueued on (0 = null stream).  On failure *out is NULL
 * and the status says why (HMC_ESHAPE, HMC_EINVAL, HMC_EDEVICE). */
hmc_status hmc_create(const hmc_params* p, int32_t Q, void* dev_workspace, size_t ws_bytes,
                      hipStream_t stream, hmc_ctx* out);

void hmc_destroy(hmc_ctx ctx);

/* Message of the last failed call on ctx (empty if none); valid until the next call.  With
 * ctx NULL: the message of this thread's last hmc_create / hmc_batch_create /
 * hmc_texture_histogram_noalloc (empty if it succeeded), which has no context to hold it. */
const char* hmc_last_error(hmc_ctx ctx);

/* Per-grain orientations: host array of Q Bunge triples (phi1, Phi, phi2) in radians.
 * The lab-frame stiffness is C' = A A A A C_crystal (Sec. 5, Eq. stiffrot) with the active
 * rotation A = Rz(phi1) Rx(Phi) Rz(phi2) (crystal -> lab), evaluated in double precision on
 * the host and uploaded in single precision together with its inverse.  HMC_ENUMERIC for
 * non-finite angles. */
hmc_status hmc_set_orientations(hmc_ctx ctx, const double* euler_host);

/* Spins: dev array of K^3 int32 grain indices in [0, Q) (copied; values are checked on
 * the device and HMC_EINVAL is returned for any out of range).  Resets no other state. */
hmc_status hmc_set_spins(hmc_ctx ctx, const int32_t* spins_dev);
hmc_status hmc_get_spins(hmc_ctx ctx, int32_t* spins_dev);

/* Applied macroscopic stress Sigma (Voigt, MPa, host array of 6): the average stress the
 * global solve holds (periodic lattice, Sec. 5).  All-zero load turns the elastic term off
 * (decisions then use exact integer thresholds).  HMC_ENUMERIC for non-finite components,
 * HMC_EINVAL for any beyond 5e4 MPa (the range the solve's fixed-point stress sums hold). */
hmc_status hmc_set_load(hmc_ctx ctx, const double sigma_MPa[6]);

/* Global explicit relaxation (Sec. 5), n_steps steps (cold_start with n_steps < 0 uses
 * p.cold_steps).  cold_start = 1: displacements zero and the macroscopic strain set to the
 * uniform-stress (Reuss) value mean(S_q) Sigma; 0: warm start from the current state with
 * zero velocities.  Ends by writing the stress field used by the zone solves.
 * HMC_ESTATE without orientations/spins/load or when lambda_el == 0. */
hmc_status hmc_stress_refresh(hmc_ctx ctx, int32_t n_steps, int32_t cold_start);

/* n_sweeps Monte Carlo steps (Sec. 3: one step = K^3 trials), starting at the current sweep
 * index s and advancing it.  Each sweep runs the colour classes in order 0..C-1; trials of
 * one class see the spins at the start of that class pass (Sec. 6, deferred updates).  With
 * the elastic term on, a warm refresh of p.refresh_steps precedes sweep s when
 * s % p.refresh_every == 0.  HMC_ESTATE if spins/orientations are missing or the elastic
 * term is on and no stress field exists yet. */
hmc_status hmc_sweep(hmc_ctx ctx, int32_t n_sweeps);

/* One colour pass of the current sweep index (no refresh, index not advanced): for tests
 * and lock-step comparison.  records_dev: NULL or a dev array of K^3 hmc_trial_record; the
 * record of every site of this colour is written at its site index (others untouched). */
hmc_status hmc_colour_pass(hmc_ctx ctx, int32_t colour, hmc_trial_record* records_dev);

/* Number of unlike bonds (each bond once: the grain-boundary energy of Sec. 3, Eq. H_1, is J
 * times it) and the stored elastic energy 1/2 sum_v eps_v . C_{q_v} eps_v (GPa*voxel; the
 * strain energy of Sec. 2, Eq. ela_hooke, summed over the voxels) of the current spins and
 * displacement state (0 when the elastic term has no state).  Synchronises. */
hmc_status hmc_energy(hmc_ctx ctx, int64_t* unlike_bonds, double* U_el);

/* Volume-weighted histogram of the angle between the unit lab axis and the nearest crystal
 * <100> direction of each site's grain: bin b = floor(angle / bin_deg), clamped to
 * nbins - 1 (the texture measure of Sec. 7: for rotations about z and a load along x, the
 * angle is the deviation from the nearest soft orientation that Eq. text_evl's density is
 * written in).  counts_host: nbins int64.  1 <= nbins <= 64, bin_deg > 0.  Synchronises. */
hmc_status hmc_texture_histogram(hmc_ctx ctx, const double axis[3], double bin_deg,
                                 int32_t nbins, int64_t* counts_host);

/* hmc_texture_histogram without a context and without any device allocation, for callers that
 * cannot allocate device memory or hand the library a workspace (code under stream capture
 * that must not allocate, tight serving loops, harnesses that forbid allocation).  Counts the
 * K^3 sites of spins_dev (dev, K^3 int32 grain indices in [0, Q), x fastest) by the texture bin
 * of their grain, exactly as hmc_texture_histogram does for a context holding these spins and
 * orientations (euler_host: Q Bunge triples in radians, host); counts_host: nbins int64.
 * Work is enqueued on `stream` (0 = null stream) and the call synchronises it.  Its scratch
 * (bin table, histogram, error flag) is a static device array of 132 352 bytes that each GPU
 * holds until the process ends; calls on one GPU share it, so calls that overlap on one GPU
 * (other streams, other threads) race.  Limits: 1 <= K <= 1024, 1 <= Q <= 32767 (HMC_ESHAPE
 * beyond), 1 <= nbins <= 64 and bin_deg > 0 (HMC_EINVAL), a spin outside [0, Q) is HMC_EINVAL,
 * non-finite angles HMC_ENUMERIC.  Message: hmc_last_error(NULL). */
hmc_status hmc_texture_histogram_noalloc(const int32_t* spins_dev, int32_t K, int32_t Q, const double* euler_host,
                                         const double axis[3], double bin_deg, int32_t nbins, int64_t* counts_host,
                                         hipStream_t stream);

/* Stress field of the last refresh (dev, 6 x K^3 float) out / in.  hmc_set_stress injects
 * a field (tests) and marks the stress as present; a non-finite entry is reported as
 * HMC_ENUMERIC by the next synchronising call. */
hmc_status hmc_get_stress(hmc_ctx ctx, float* dev_out);
hmc_status hmc_set_stress(hmc_ctx ctx, const float* dev_in);

/* Displacement fluctuation (dev, 3 x K^3 float planes) and macroscopic strain (host, 6
 * doubles) of the global solve; set_state also zeroes the velocities (tests, resume). */
hmc_status hmc_get_displacement(hmc_ctx ctx, float* dev_out);
hmc_status hmc_get_macro_strain(hmc_ctx ctx, double E_host[6]);
hmc_status hmc_set_elastic_state(hmc_ctx ctx, const float* u_dev, const double E_host[6]);

/* Sweep index s used for the Philox counter (resume). */
hmc_status hmc_set_sweep_index(hmc_ctx ctx, int64_t s);
hmc_status hmc_get_sweep_index(hmc_ctx ctx, int64_t* s);

hmc_status hmc_get_stats(hmc_ctx ctx, hmc_stats* out);
hmc_status hmc_reset_stats(hmc_ctx ctx);

/* Turn the lower-bound screen of hmc_params.zone_screen on (1) or off (0) for later sweeps. */
hmc_status hmc_set_zone_screen(hmc_ctx ctx, int32_t enable);

/* Select the zone-solve kernel (hmc_params.zone_variant) for later sweeps, e.g. from a
 * launch-shape autotuner.  Variants compute the same solve in a different FP32 rounding
 * order.  HMC_EINVAL for a variant the context's zone size does not allow. */
hmc_status hmc_set_zone_variant(hmc_ctx ctx, int32_t variant);

/* Race detection: the order in which the work-groups of the colour-pass, zone-solve and
 * explicit-step launches (forward and adjoint) take their parts of the work.  0: the default
 * (XCD-aware) order; 1: reversed; 2: a fixed shuffle.  No result may depend on it (same-colour
 * sites are never neighbours, every trial reads the pass's snapshot, and all cross-work-group
 * sums are integer), so sweeps, refreshes and gradients are bit-identical under all three; a
 * difference would expose a race.  HMC_EINVAL for other values. */
hmc_status hmc_set_block_order(hmc_ctx ctx, int32_t order);

/* Kernel timing.  While profiling is enabled the library records a pair of HIP events on
 * the context's stream around every launch of each kernel class below; hmc_get_kernel_times
 * synchronises, resolves the pairs recorded since the last call (or since enabling) into
 * launch counts and summed durations, and clears them.  Costs two event records per launch. */
typedef struct {
    int64_t launches;
    double total_ms;
} hmc_kernel_time;

typedef struct {
    hmc_kernel_time potts;          /* colour pass: draws, proposals, bond counts */
    hmc_kernel_time zone;           /* zone solves of one colour pass */
    hmc_kernel_time apply;          /* deferred writes of accepted elastic flips */
    hmc_kernel_time refresh_step;   /* one explicit step of the global solve (node part) */
    hmc_kernel_time refresh_other;  /* strain update, start, final stress field */
} hmc_kernel_times;

hmc_status hmc_set_profiling(hmc_ctx ctx, int32_t enable);
hmc_status hmc_get_kernel_times(hmc_ctx ctx, hmc_kernel_times* out);

/* Capture each sweep's launches (the colour passes, and the refresh that precedes every
 * refresh_every-th sweep) once into HIP graphs and replay them on later hmc_sweep calls.
 * Needs a context created on a non-null stream (HMC_EINVAL otherwise).  Graphs are
 * dropped and re-captured whenever orientations, spins, loads or the elastic state change.
 * Kernel timing (hmc_set_profiling) bypasses the graphs while it is on: HIP events recorded
 * by a captured graph carry no timestamps on this platform. */
hmc_status hmc_set_graphs(hmc_ctx ctx, int32_t enable);

/* ---- Batches: many independent replicas in every launch -----------------------------
 * A batch is an hmc_ctx whose replicas differ in lattice size, grains, temperature, load,
 * elastic scale, global relaxation constants and Philox seed, and share everything else in
 * the common hmc_params (neighbours, proposal, zone, step counts, J, C11/C12/C44; the
 * common K, kT, lambda_el, glob_* and seed are ignored).  Every colour pass, zone-solve
 * pass and explicit refresh step is one launch over all replicas; with hmc_set_graphs a
 * whole sweep of all replicas is one graph launch.  Results per replica are identical to
 * running it alone with the same parameters. */
typedef struct {
    int32_t K;              /* lattice edge (same rules as hmc_params.K) */
    int32_t Q;              /* grains of this replica */
    double kT;
    double lambda_el;       /* 0: elastic term off for this replica */
    double glob_alpha, glob_beta, glob_alphaE;
    double sigma_MPa[6];    /* applied average stress (Voigt, MPa; |each| <= 5e4) */
    uint64_t seed;          /* Philox key */
} hmc_replica;

/* Fill *r for a K^3 replica with Q grains: kT and seed from common, lambda_el = 2.6667e6/K
 * and the global heavy-ball constants for K and common->material_points as in
 * hmc_set_material_points, zero load. */
hmc_status hmc_default_replica(hmc_replica* r, const hmc_params* common, int32_t K, int32_t Q);

/* Workspace bytes of a batch of n replicas (0 if any description is invalid). */
size_t hmc_batch_workspace_bytes(const hmc_params* common, int32_t n, const hmc_replica* reps);

/* Create a batch of 1 <= n <= 4096 replicas (host array reps, copied).  Same workspace and
 * stream rules as hmc_create.  Then give every replica its orientations and spins with
 * hmc_batch_set_replica; hmc_stress_refresh, hmc_sweep, hmc_set_sweep_index, hmc_get_stats,
 * hmc_set_profiling/hmc_get_kernel_times and hmc_set_graphs act on all replicas. */
hmc_status hmc_batch_create(const hmc_params* common, int32_t n, const hmc_replica* reps, void* dev_workspace,
                            size_t ws_bytes, hipStream_t stream, hmc_ctx* out);

/* Replica r's orientations (host, Q_r Bunge triples) and spins (dev, K_r^3 int32). */
hmc_status hmc_batch_set_replica(hmc_ctx ctx, int32_t r, const double* euler_host, const int32_t* spins_dev);

/* Per-replica read-outs, as hmc_get_spins / hmc_get_stress / hmc_energy /
 * hmc_texture_histogram for replica r (those four act on replica 0). */
hmc_status hmc_batch_get_spins(hmc_ctx ctx, int32_t r, int32_t* spins_dev);
hmc_status hmc_batch_get_stress(hmc_ctx ctx, int32_t r, float* dev_out);
hmc_status hmc_batch_energy(hmc_ctx ctx, int32_t r, int64_t* unlike_bonds, double* U_el);
hmc_status hmc_batch_texture_histogram(hmc_ctx ctx, int32_t r, const double axis[3], double bin_deg,
                                       int32_t nbins, int64_t* counts_host);

/* Grains of replica r (0 for a single lattice): the face-connected clusters of equal spins on
 * the periodic lattice, whose mean volume K^3 / n is the grain size of Sec. 6's growth law.
 * Writes labels_dev[v] (dev, K_r^3 int32, caller-owned) = the smallest site index of the grain
 * of site v, and *n_grains (host).  Iterates label propagation and pointer jumping on the
 * context's stream until nothing changes, synchronising that stream once per round.  Reads the
 * spins as they are after all work enqueued so far. */
hmc_status hmc_grain_labels(hmc_ctx ctx, int32_t r, int32_t* labels_dev, int64_t* n_grains);

/* ---- Adjoint of the global explicit solve (single-lattice contexts) ------------------
 * U(theta, Sigma) = stored elastic energy after a cold start and n_steps explicit steps of
 * the global relaxation (as hmc_stress_refresh(ctx, n_steps, 1)), as a function of every
 * grain's Euler angles theta and the applied stress Sigma.  hmc_elastic_forward runs it and
 * keeps a checkpoint of the state every ckpt_every steps in the caller's adjoint workspace
 * (dev, hmc_adjoint_workspace_bytes, 256-byte aligned); hmc_elastic_backward recomputes one
 * segment at a time from those checkpoints and runs the reverse recurrence, returning
 * dU * dU/dtheta (host, Q x 3, per radian) and dU * dU/dSigma (host, 6, per MPa).  The
 * backward call leaves the context at the forward's final state.  The adjoint workspace must
 * not change between the two calls.  The forward's record is discarded by any later change
 * of the spins, orientations or load (hmc_set_spins, hmc_set_orientations, hmc_set_load,
 * hmc_sweep, hmc_colour_pass): hmc_elastic_backward then returns HMC_ESTATE until the next
 * forward, rather than a gradient of inputs the checkpoints were not taken from.  A backward
 * call keeps the record (it may be repeated with another dU).  HMC_ESTATE on batches,
 * without a forward, or with the elastic term disabled.  The backward call recomputes segments on a second stream of the
 * library's own (default priority, created on first use, released by hmc_destroy) while the
 * context's stream runs adjoint steps; events order the two, and the call returns only after
 * both are done (it returns host results), so the caller sees ordinary stream order. */
size_t hmc_adjoint_workspace_bytes(hmc_ctx ctx, int32_t n_steps, int32_t ckpt_every);
hmc_status hmc_elastic_forward(hmc_ctx ctx, int32_t n_steps, int32_t ckpt_every, void* dev_adjoint_ws,
                               size_t adjoint_ws_bytes, double* U_host);
hmc_status hmc_elastic_backward(hmc_ctx ctx, void* dev_adjoint_ws, size_t adjoint_ws_bytes, double dU,
                                double* grad_euler_host, double grad_sigma_MPa[6]);

/* Host-only helper (no device use): lab-frame Voigt stiffness and compliance (Q x 36
 * doubles each, row-major 6x6) exactly as hmc_set_orientations computes them before the
 * single-precision upload.  The compliance is built from the closed-form cubic compliance
 * and the strain transformation, not by inverting C. */
hmc_status hmc_grain_tables(const double* euler_host, int32_t Q, double C11, double C12,
                            double C44, double* C_out, double* S_out);

/* Host-only helper (no device use): derivatives of those tables with respect to the three
 * Euler angles, dC_out and dS_out of Q x 3 x 36 doubles ([grain][angle][6x6 row-major]),
 * by differentiating A = Rz(phi1) Rx(Phi) Rz(phi2) factor by factor. */
hmc_status hmc_grain_table_derivatives(const double* euler_host, int32_t Q, double C11, double C12,
                                       double C44, double* dC_out, double* dS_out);

#ifdef __cplusplus
}
#endif

#endif /* HMC_H_ */
