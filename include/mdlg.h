/*
 * mdlg.h -- C ABI of the MI355X (gfx950) MDLG library.
 *
 * The library runs Lennard-Jones molecular dynamics in periodic boxes and
 * coarse-grains it on the fly into the Molecular-Dynamics lattice gas (MDLG)
 * of Parsa & Wagner, "Lattice Gas with Molecular Dynamics Collision Operator":
 *
 *   - MD (section "Lattice Gas with Molecular Dynamics collision operator",
 *     Newton's equations for N particles with a pair potential in a periodic
 *     container; section "MDLG for a two-dimensional Lennard-Jones gas", the
 *     LJ potential V(r) = 4 eps [(sigma/r)^12 - (sigma/r)^6]).  Velocity-Verlet
 *     integration, cut off at r_cut (the paper does not state the integrator or
 *     the cutoff).
 *   - MDLG binning (eq. MDni): every lattice time step Delta t, each particle's
 *     lattice cell at t - Delta t and at t gives its lattice velocity
 *     v_i = C(t) - C(t - Delta t); n_i(x,t) counts the particles arriving in
 *     site x with velocity v_i.  Per site the library accumulates sum_t n_i,
 *     the local number N(x,t), the lattice momentum N u = sum_i v_i n_i and the
 *     second moment sum_i v_i v_i n_i, all exact integers.
 *   - the equilibrium distribution f_i^eq = <n_i> (eq. fieq) as the site and
 *     time average, and the continuous displacement moments behind a^2
 *     (eq. eqn:a).
 *
 * Conventions
 *   - All entry points return mdlg_status (0 = MDLG_OK, negative = error) and
 *     never throw.  Config errors are found synchronously on the host.
 *   - Device-side failures (a particle leaving its MD cell between rebuilds
 *     by more than the stencil's reach, non-finite coordinates, a velocity
 *     so large that a particle crosses more than one cell per step) set a
 *     device error word; it is
 *     reported as MDLG_E_UNSTABLE by the next call that synchronises
 *     (mdlg_get_f, mdlg_get_state, mdlg_sync), and mdlg_last_error() explains.
 *   - The caller owns all device memory: one workspace of
 *     mdlg_workspace_bytes() bytes (256-byte aligned) that must outlive the
 *     handle, plus the input arrays of mdlg_create.  The library never
 *     allocates device memory.  The caller owns every host array it passes.
 *   - Work is enqueued asynchronously on the HIP stream given at creation.
 *     One handle must be used from one host thread at a time.
 *   - Lattice: a cubic lattice of spacing lattice_dx with lattice[r][a] sites
 *     along axis a of replica r; the periodic box side is lattice[r][a] *
 *     lattice_dx.  Internally each lattice cell is k x k (x k) MD cells of side
 *     s = float32(lattice_dx / k); when lattice_dx / k is not a float32 value
 *     the box is lattice[r][a] * k * s (mdlg_describe reports s).  A particle belongs to site c along an axis when
 *     c * dx <= x < (c+1) * dx (the paper writes the interval closed above;
 *     the two readings differ on a set of measure zero).
 *   - Velocities: lattice velocities with |v_a| <= vmax on every axis are
 *     binned into Q = (2 vmax + 1)^dim bins with index
 *     i = sum_a (v_a + vmax) (2 vmax + 1)^a (x fastest); other particles are
 *     counted as overflow at their arrival site.  N(x,t) and the moments include
 *     every particle.
 *   - Several independent replicas (boxes of different sizes) can share one
 *     handle; they run in the same kernel launches.  Particle arrays are the
 *     concatenation of the replicas in order; site arrays likewise.
 *   - Results are deterministic: the same inputs give the same results bit
 *     for bit, with or without graph replay (no floating-point sum depends on
 *     the order in which atomics land).
 */
#ifndef MDLG_H
#define MDLG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MDLG_OK = 0,
    MDLG_E_INVALID = -1,   /* bad argument or configuration */
    MDLG_E_DEVICE = -2,    /* a HIP runtime call failed */
    MDLG_E_NOMEM = -3,     /* workspace too small */
    MDLG_E_UNSTABLE = -4,  /* device error word set (see mdlg_last_error) */
    MDLG_E_STATE = -5      /* call not valid in the current state */
} mdlg_status;

typedef struct mdlg_system mdlg_system; /* opaque, library-owned host handle */

typedef struct {
    int32_t dim;                /* 2 or 3 */
    int32_t n_replicas;         /* >= 1 */
    const int32_t *n_particles; /* host [n_replicas], each >= 1 */
    const int32_t *lattice;     /* host [n_replicas][dim], sites per axis M >= 1 */
    double lattice_dx;          /* lattice spacing Delta x (> 0) */
    double epsilon;             /* LJ eps (> 0) */
    double sigma;               /* LJ sigma (> 0) */
    double mass;                /* particle mass m (> 0) */
    double r_cut;               /* cutoff radius (> 0); box sides must exceed 2 r_cut */
    int32_t forces_off;         /* 1: ideal gas (no interactions) */
    double dt;                  /* MD time step (> 0) */
    int32_t md_steps_per_lattice_step; /* Delta t / dt (>= 1) */
    int32_t vmax;               /* velocity window half-width V (0..7) */
    int32_t thermostat_every;   /* rescale velocities to kT every this many MD steps in
                                   mdlg_step (0 = off); never during mdlg_coarse_grain */
    double kT;                  /* thermostat target k_B T */
    int32_t md_cell_split;      /* k: MD cells of side s = dx / k per lattice cell;
                                   power of two 1..8, or 0 = choose automatically */
    int32_t sort_every;         /* cell-list rebuild interval in MD steps (>= 1),
                                   or 0 = choose from kT, mass and dt */
    int32_t brick_x;            /* force-kernel brick extent along x in MD cells, 0 = auto */
    int32_t brick_y;            /* along y, 0 = auto */
    int32_t brick_z;            /* along z (3D), 0 = auto */
    int32_t adjoint_window;     /* largest adjoint window in MD steps (0 = no adjoint buffers) */
    int32_t adjoint_every;      /* checkpoint interval the workspace is sized for (>= 1 when
                                   adjoint_window > 0) */
    int32_t no_pair_list;       /* 1: every MD step walks the neighbour cells; 0: per-particle
                                   pair lists of radius r_cut + 2 margin, built at each
                                   cell-list rebuild, are used when the rebuild interval is
                                   at least 2 (results agree to float rounding) */
    int32_t block_threads;      /* threads per block of the force and pair-list kernels:
                                   64, 128 or 256, or 0 = choose automatically */
    int32_t collision_stats;    /* 1: record the MDLG collision operator Xi (eq. Xi) of
                                   every pair of consecutive lattice steps (see
                                   mdlg_get_xi); 0: off */
    int32_t n_shifts;           /* extra lattices binned every lattice step (0..32), see
                                   mdlg_get_shifts */
    const double *shifts;       /* host [n_shifts][2][dim], copied at creation: per extra
                                   lattice an offset a (lattice spacings) and a drift b
                                   (lattice spacings per lattice step) along every axis */
} mdlg_config;

/* Particle state in particle-id order (id = index in the concatenated input).
 * Every pointer is a host array of n_total * dim elements, or NULL to skip.
 *   ucell:      unwrapped MD-cell index per axis: wrapped cell + Mc * image,
 *               with Mc = lattice * k MD cells per axis and image the number of
 *               periodic box crossings;
 *   off:        position inside that MD cell, in [0, s), s = dx / k;
 *               the unwrapped position is ucell * s + off;
 *   vel:        velocity at the current time;
 *   acc:        acceleration F/m at the current time (mdlg_get_state only);
 *   prev_ucell, prev_off: the same two quantities at the last lattice snapshot
 *               (the positions the next lattice step is binned against). */
typedef struct {
    int32_t *ucell;
    float *off;
    float *vel;
    float *acc;
    int32_t *prev_ucell;
    float *prev_off;
} mdlg_particles;

/* Derived parameters of a configuration (host only, no device needed). */
typedef struct {
    int32_t md_cell_split;      /* k actually used */
    int32_t sort_every;         /* rebuild interval actually used */
    int32_t stencil;            /* neighbour-cell half-width ceil(r_cut / s) */
    int32_t n_velocities;       /* Q */
    int32_t n_moments;          /* per-site moments: 2 + dim + dim(dim+1)/2 */
    int32_t brick[3];           /* force-kernel brick extent in MD cells */
    int64_t n_total;            /* particles over all replicas */
    int64_t n_sites;            /* lattice sites over all replicas */
    int64_t n_cells;            /* MD cells over all replicas */
    int64_t n_bricks;           /* force-kernel work units per MD step */
    double cell_side;           /* s */
    double margin;              /* design excursion outside the cell between rebuilds (eight
                                   thermal speeds per axis over the interval); it sets the
                                   automatic rebuild interval and bounds the skin */
    int32_t pair_slots;         /* pair-list entries per particle (0 = no pair lists) */
    int32_t block_threads;      /* threads per force / pair-list block actually used */
    double skin;                /* pair lists hold the pairs within r_cut + 2 skin (skin <=
                                   margin); past it the force launches walk the cells until
                                   the next rebuild (mdlg_get_list_fallbacks) */
    double reach;               /* stencil's reach (stencil * s - r_cut) / 2 >= margin: the
                                   cell walk is exact for any excursion outside the cell up to
                                   it; a particle beyond it between rebuilds is a device error */
} mdlg_layout;

/* Validate cfg and report the derived layout.  Host only.  MDLG_E_INVALID on
 * any inconsistent field, and on MD cells (lattice_dx / md_cell_split) that
 * hold more than 128 particles on average at the densest replica's density
 * (the counting sort ranks a particle among a bounded number of earlier
 * particles of its cell); *out untouched on error. */
mdlg_status mdlg_describe(const mdlg_config *cfg, mdlg_layout *out);

/* Workspace size in bytes for cfg.  Host only. */
mdlg_status mdlg_workspace_bytes(const mdlg_config *cfg, size_t *bytes);

/* Create a system.  workspace_dev: device buffer of at least
 * mdlg_workspace_bytes(cfg) bytes, 256-byte aligned, owned by the caller.
 * hip_stream: the hipStream_t all work is enqueued on (NULL = null stream).
 * pos_dev: device float [n_total][dim] positions in [0, box) (the initial x_i(0)
 * of the paper's problem statement); vel_dev: device float [n_total][dim]
 * initial velocities v_i(0).  Both are read before the call returns (the call
 * synchronises the stream once).  The initial positions become the first
 * lattice snapshot. */
mdlg_status mdlg_create(const mdlg_config *cfg, void *workspace_dev, size_t workspace_bytes,
                        void *hip_stream, const float *pos_dev, const float *vel_dev,
                        mdlg_system **out);

/* Size of the static workspace of mdlg_create_static. */
#define MDLG_STATIC_WORKSPACE_BYTES ((size_t)32 << 20)

/* mdlg_create without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  The workspace is a static device array of
 * MDLG_STATIC_WORKSPACE_BYTES (32 MiB) that the library holds on each GPU it
 * runs on until the process ends; the call allocates nothing.  Arguments and
 * the rest of the lifetime are those of mdlg_create, on the device current on
 * the calling thread (hip_stream must belong to it).  The array keeps the
 * last handle's contents; creation clears what must start at zero.  Every
 * handle made this way on one GPU would share that GPU's array, so only one
 * may be alive per device: a second call before mdlg_destroy of the first
 * returns MDLG_E_STATE instead of letting the two race.  MDLG_E_NOMEM when
 * mdlg_workspace_bytes(cfg) exceeds the array (about 65,000 particles in 2D;
 * use mdlg_create beyond that). */
mdlg_status mdlg_create_static(const mdlg_config *cfg, void *hip_stream, const float *pos_dev,
                               const float *vel_dev, mdlg_system **out);

/* Advance n_md_steps velocity-Verlet steps (asynchronous).  With
 * thermostat_every > 0 the velocities of every replica are rescaled after
 * every that many steps so that sum m v^2 = kT dim (N_r - 1) (equilibration;
 * the paper sets the temperature of its run by the kinetic energy).
 * Invalidates the lattice snapshot: the next mdlg_coarse_grain takes a fresh
 * one first. */
mdlg_status mdlg_step(mdlg_system *sys, int64_t n_md_steps);

/* Run n_lattice_steps lattice time steps (asynchronous): each is
 * md_steps_per_lattice_step MD steps (no thermostat) followed by binning of
 * every particle against the previous snapshot (eq. MDni) and accumulation of
 * n_i, N, N u, the second moment and the continuous displacement moments. */
mdlg_status mdlg_coarse_grain(mdlg_system *sys, int64_t n_lattice_steps);

/* Read back the averages (synchronises).  Every output is optional (NULL):
 *   f        [Q]      f_i^eq = sum over sites and lattice steps of n_i divided by
 *                     (lattice steps * sites), over all replicas (eq. fieq);
 *   f_site   [n_sites][Q]   per-site time average of n_i;
 *   mom_site [n_sites][n_moments] per-site time averages of
 *            (N, overflow, sum_i v_a n_i for each axis a, then sum_i v_a v_b n_i
 *             for a <= b in row-major order: xx, xy, [xz], yy, [yz], [zz]);
 *   counts   [Q]      the raw integer sums behind f (uint64);
 *   n_samples         lattice steps * sites;
 *   n_overflow        particle-steps outside the velocity window;
 *   disp     [2*dim]  sum of delta x_a and of delta x_a^2 of the continuous
 *                     displacement x(t) - x(t - Delta t) over particles and
 *                     lattice steps (divide by n_total * lattice steps for
 *                     <delta x_a> and <delta x_a^2>);
 *   n_lattice_steps   lattice steps accumulated.
 * Returns MDLG_E_UNSTABLE if the device error word is set. */
mdlg_status mdlg_get_f(mdlg_system *sys, double *f, double *f_site, double *mom_site,
                       uint64_t *counts, int64_t *n_samples, int64_t *n_overflow, double *disp,
                       int64_t *n_lattice_steps);

/* Kinetics per replica of the current state (FP64; a half-step state is first
 * completed by its finishing kick, as a lattice step's end would):
 * out[r][0..dim-1] = total momentum sum m v, out[r][dim] = kinetic energy
 * sum m v^2 / 2, summed in particle order (the same sums for a replica alone
 * and in a batch).  Synchronises.  out is host [n_replicas][dim + 1]. */
mdlg_status mdlg_get_kinetics(mdlg_system *sys, double *out);

/* Zero all accumulators (n_i sums, moments, displacement sums, lattice-step
 * count) and invalidate the snapshot.  Asynchronous. */
mdlg_status mdlg_reset_accumulators(mdlg_system *sys);

/* Copy the particle state at the current time to host arrays in id order
 * (synchronises).  Completes the pending half kick to report full-step
 * velocities and accelerations; the trajectory is unchanged. */
mdlg_status mdlg_get_state(mdlg_system *sys, mdlg_particles *out);

/* Replace the particle state from host arrays in id order (ucell, off and vel
 * required; prev_ucell and prev_off optional: when NULL the new positions become
 * the snapshot).  Offsets must lie in [0, s).  Accumulators are kept. */
mdlg_status mdlg_set_state(mdlg_system *sys, const mdlg_particles *in);

/* Losses of the adjoint window, on the continuous displacement
 * delta x_j = x_j(t0 + W dt) - x_j(t0) over the window (the displacement whose
 * second moment defines a^2 in eq. eqn:a):
 *   MDLG_LOSS_MSD:    L = (1 / (N dim)) sum_j |delta x_j|^2
 *   MDLG_LOSS_MEAN_X: L = (1 / N) sum_j delta x_jx                         */
typedef enum { MDLG_LOSS_MSD = 0, MDLG_LOSS_MEAN_X = 1 } mdlg_loss;

/* Adjoint of one MD window (not a passage of the paper: the gradients of its
 * displacement moments with respect to the potential and the initial
 * velocities).  From the current positions x(t0) and velocities v(t0) -- or
 * v0_dev when not NULL (device float [n_total][dim], id order) -- runs
 * window_steps velocity-Verlet steps with the cell list frozen (checkpoints of
 * the state every ckpt_every steps), then the reverse sweep, recomputing each
 * segment from its checkpoint.  Outputs (any may be NULL): *loss, dL/deps,
 * dL/dsigma (host doubles) and dL/dv0 into g_v0_dev (device float
 * [n_total][dim], id order).  The system is left at t0 + window_steps.
 * Requires window_steps <= adjoint_window of the configuration, window_steps a
 * multiple of ckpt_every, window_steps / ckpt_every + 1 checkpoints and
 * ckpt_every + 1 segment positions within the sizes the configuration
 * reserved.  Synchronises.  All replicas take part: N is the particle count
 * over all replicas. */
mdlg_status mdlg_adjoint(mdlg_system *sys, int32_t window_steps, int32_t ckpt_every, int32_t loss,
                         const float *v0_dev, double *out_loss, double *dL_deps, double *dL_dsigma,
                         float *g_v0_dev);

/* Checkpoints.  The paper's run discards its start as equilibration and
 * continues from the equilibrated state (section "MDLG for a two-dimensional
 * Lennard-Jones gas"); a checkpoint makes such a run resumable.  A blob holds
 * the complete state of a handle: the particle state in the library's own
 * order, the lattice snapshot, every accumulator (n_i sums, moments,
 * displacement sums, collision-operator and shifted-lattice sums), the
 * kinetics of the last thermostat or readout, and the sequencing counters
 * (MD steps, lattice steps, the position inside the rebuild interval and the
 * collision-operator chain); between cell-list rebuilds also the pair lists.
 * Loading it into a handle created with the same configuration (and the same
 * LJ parameters) continues the run exactly: T lattice steps give the same
 * results, bit for bit, as T/2, save, load, T/2.
 *   mdlg_checkpoint_bytes: size of the blob of the current state (it grows
 *                          between rebuilds, when the pair lists are saved).
 *   mdlg_checkpoint_save:  writes the blob into host_blob (bytes >= the size
 *                          above, else MDLG_E_NOMEM); synchronises; returns
 *                          MDLG_E_UNSTABLE without writing when the device
 *                          error word is set.
 *   mdlg_checkpoint_load:  replaces the state of sys from the blob (exactly
 *                          the size save wrote); synchronises.  MDLG_E_INVALID
 *                          for a blob of another configuration or a damaged
 *                          header.  The caller owns host_blob throughout. */
mdlg_status mdlg_checkpoint_bytes(mdlg_system *sys, size_t *bytes);
mdlg_status mdlg_checkpoint_save(mdlg_system *sys, void *host_blob, size_t bytes);
mdlg_status mdlg_checkpoint_load(mdlg_system *sys, const void *host_blob, size_t bytes);

/* Change the LJ parameters eps and sigma of an existing system (r_cut stays
 * fixed in absolute units).  Asynchronous. */
mdlg_status mdlg_set_potential(mdlg_system *sys, double epsilon, double sigma);

/* Kernel classes of the hot path, for mdlg_get_timing. */
typedef enum {
    MDLG_K_FORCE = 0,   /* LJ forces fused with the velocity-Verlet kicks and drift */
    MDLG_K_COUNT = 1,   /* cell-list rebuild: canonicalise and count per cell */
    MDLG_K_SCAN = 2,    /* cell-list rebuild: exclusive scan of the counts */
    MDLG_K_SCATTER = 3, /* cell-list rebuild: permute the particle state */
    MDLG_K_BIN = 4,     /* MDLG binning and per-site accumulation (eq. MDni) */
    MDLG_K_NLIST = 5,   /* cell-list rebuild: per-particle pair lists */
    MDLG_K_XI = 6,      /* collision operator of consecutive lattice steps (eq. Xi) */
    MDLG_K_SHIFT = 7,   /* binning on displaced and moving lattices */
    MDLG_K_ADJOINT = 8, /* reverse step of the adjoint window (mdlg_adjoint) */
    MDLG_K_ADJOINT_FORCE = 9, /* a reverse step launched together with a force step that
                                 recomputes an earlier checkpoint segment */
    MDLG_K_NCLASS = 10
} mdlg_kernel_class;

/* Enable (1) or disable (0) per-kernel timing with HIP events on the handle's
 * stream.  While enabled, lattice steps run as individual launches (no graph
 * replay) with an event pair around each launch.  Enabling resets the
 * counters.  This is a measurement aid for callers profiling the hot path. */
mdlg_status mdlg_set_timing(mdlg_system *sys, int enable);

/* Total event-timed milliseconds and launch counts per kernel class since
 * timing was enabled (synchronises).  Both arrays are host [MDLG_K_NCLASS]. */
mdlg_status mdlg_get_timing(mdlg_system *sys, double *total_ms, int64_t *launches);

/* The constant that an event pair adds to a kernel's time, in milliseconds,
 * measured on the handle's stream: reps launches (1..1000) of a one-wave
 * kernel that waits about 20 microseconds on the device's constant-rate wall
 * clock, each between its own event pair, as mdlg_set_timing records them;
 * *offset_ms = the median of (event time - the wait).  Subtracted from the
 * per-launch averages of mdlg_get_timing it gives each kernel's own duration.
 * Synchronises; leaves the timing counters as they are.  MDLG_E_INVALID for a
 * NULL argument or reps out of range, MDLG_E_DEVICE when the device reports
 * no wall clock rate or a launch fails.  A measurement aid. */
mdlg_status mdlg_timing_offset(mdlg_system *sys, int reps, double *offset_ms);

/* Enqueue on the handle's stream a one-wave kernel that waits the given time
 * (0..1e6 microseconds) on the device's wall clock.  The host meanwhile
 * enqueues the launches that follow, so that an event-timed pass after it runs
 * its kernels back to back rather than at the host's launch rate (event pairs
 * around kernels shorter than a launch would otherwise take in the gaps).
 * Asynchronous.  MDLG_E_INVALID for a time out of range, MDLG_E_DEVICE when
 * the device reports no wall clock rate or the launch fails.  A measurement
 * aid. */
mdlg_status mdlg_timing_head_start(mdlg_system *sys, double microseconds);

/* Force launches since creation that walked the cells because the pair
 * lists might have been stale: the pair lists hold the pairs within
 * r_cut + 2 skin of their build, and each MD step folds the largest
 * half-step speed into a bound on every particle's displacement since; a
 * launch whose bound passes the skin walks the cell rows instead (exact for
 * excursions outside the cell up to the stencil's reach), until the next
 * rebuild.  A measure of
 * how often the skin (sized from the expected largest speed of the
 * system's particles) is too small.  Synchronises; *launches is host. */
mdlg_status mdlg_get_list_fallbacks(mdlg_system *sys, int64_t *launches);

/* Wait for all work queued on the handle's stream; report the error word. */
mdlg_status mdlg_sync(mdlg_system *sys);

/* Human-readable description of the last error on sys (or of the last
 * creation failure when sys is NULL).  Never NULL. */
const char *mdlg_last_error(const mdlg_system *sys);

/* Release the handle (the caller still owns the workspace). */
void mdlg_destroy(mdlg_system *sys);

/* The MDLG collision operator (eq. Xi):
 *   Xi_i(x, t) = n_i(x + v_i, t + Delta t) - n_i(x, t),
 * with n_i of eq. (MDni) (arrival site x, lattice velocity v_i, periodic
 * wrap of x + v_i inside the site's replica).  With collision_stats on, every
 * mdlg_coarse_grain lattice step after the first of an unbroken chain (the
 * chain restarts whenever the snapshot is retaken: after mdlg_step,
 * mdlg_set_state or mdlg_reset_accumulators) evaluates Xi at the previous
 * lattice time and accumulates, all in exact integers:
 *   sums      host [5][Q]: over sites and samples, sum Xi_i, sum Xi_i^2,
 *             sum Xi_i n_i, sum n_i, sum n_i^2 (n_i = n_i(x, t), the
 *             populations Xi acts on); NULL to skip;
 *   xi_site   host [n_sites][Q]: per site, sum over samples of Xi_i; or NULL;
 *   xi_last   host [n_sites][Q]: Xi_i(x, t) of the latest sample; or NULL;
 *   n_steps   number of samples (lattice times t).
 * Sum_i Xi_i(x, t) = 0 (eq. Mom0) holds exactly when no particle leaves or
 * enters x with a displacement outside the velocity window.  Synchronises.
 * MDLG_E_STATE when collision_stats is off. */
mdlg_status mdlg_get_xi(mdlg_system *sys, int64_t *sums, int64_t *xi_site, int32_t *xi_last,
                        int64_t *n_steps);

/* Binning on displaced and moving lattices.  Extra lattice j places the cell
 * boundaries so that a particle at x lies in cell floor(x / dx + a_j + b_j k)
 * along each axis at lattice time k (cfg.shifts).  A drift b_j = u is the
 * Galilean transform x + u t of the positions, which the paper uses to obtain
 * the equilibrium distribution at mean velocity u from one trajectory
 * (section on the velocity dependence of f_i^eq, eq. fialpha); static
 * offsets a_j = m / K, m = 0..K-1, average over K lattice placements, which
 * the paper names as the way to make the lattice momentum exact (remarks
 * after the one-particle table).  Every mdlg_coarse_grain lattice step
 * accumulates, per extra lattice and summed over all sites, exact integers:
 *   counts   host [n_shifts][Q + 1]: window bins as in eq. (MDni) (same
 *            numbering), then the particles whose displacement left the
 *            window;
 *   moments  host [n_shifts][d + d(d+1)/2]: sum over all particles of the
 *            lattice displacement v_a, then v_a v_b for a <= b;
 *   n_steps  lattice steps accumulated since the last reset.
 * NULL skips an output.  Synchronises.  MDLG_E_STATE when n_shifts is 0. */
mdlg_status mdlg_get_shifts(mdlg_system *sys, uint64_t *counts, int64_t *moments, int64_t *n_steps);

/* Launch-shape autotuner for batched and single systems (the f_i^eq of
 * eq. fieq are ensemble averages, so the same configuration is typically run
 * for many lattice steps and its shapes are worth measuring).  Every field of
 * cfg left automatic (0) among md_cell_split, sort_every, brick_x/y/z and
 * block_threads is
 * tuned by timing candidate layouts on the device: first the automatic layout
 * with and without pair lists (unless cfg asks for none), then the other MD-cell
 * splits, then rebuild intervals that divide a lattice step into equal parts
 * and fit the stencil margin, then block sizes of 64, 128 and 256 threads
 * with force-brick extents around 3/4, 1 and 3/2 targets per thread; each
 * stage keeps the fastest so far.  A candidate runs two warm-up
 * lattice steps and then ceil(md_steps / md_steps_per_lattice_step) timed
 * lattice steps (HIP events on hip_stream) from pos_dev / vel_dev (device
 * [n_total][dim], as for mdlg_create; not modified).  Candidates that do not
 * fit the workspace, fail to create, or report a device error are skipped.
 * *best receives a copy of *cfg with the tuned fields set (pointers still the
 * caller's); *best_ms_per_md_step (optional) the time per MD step measured
 * for it.  Every candidate runs in workspace_dev, one after another: the
 * library still allocates nothing.  Synchronises the stream.
 * MDLG_E_INVALID for bad arguments, MDLG_E_DEVICE when no candidate ran. */
mdlg_status mdlg_autotune(const mdlg_config *cfg, void *workspace_dev, size_t workspace_bytes,
                          void *hip_stream, const float *pos_dev, const float *vel_dev,
                          int32_t md_steps, mdlg_config *best, double *best_ms_per_md_step);

/* Workspace that holds every candidate mdlg_autotune may try for cfg.
 * Host only. */
mdlg_status mdlg_autotune_workspace_bytes(const mdlg_config *cfg, size_t *bytes);

#ifdef __cplusplus
}
#endif

#endif /* MDLG_H */
