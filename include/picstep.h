/*
 * picstep.h -- C ABI of the MI355X particle-step library (libpicstep.so).
 *
 * The library advances charged macro-particles of the special-relativistic
 * curvilinear PIC method of arXiv 2511.17710 (Entity paper I) through the
 * particle part of one leap-frog step (Sec. 2.3, steps 3-8):
 *   3. interpolate the Yee-staggered contravariant E, B to each particle
 *      with the first-order shape;
 *   4. convert them to the global orthonormal Cartesian basis
 *      (eq. curvspace-tetradtrans, then the spherical rotation);
 *   5. relativistic Boris push of u^{n-1/2} -> u^{n+1/2}
 *      (eq. curvspace-equations-of-motion);
 *   6-7. move x^n -> x^{n+1} in Cartesian space and convert back to code
 *      coordinates (Sec. 2.4 coordinate maps, App. B);
 *   8. deposit the conformal current (eq. curvspace-chargecons-2) with the
 *      charge-conserving zig-zag scheme (Sec. 3.2, footnote).
 * Grids: 2D/3D Cartesian (periodic), 2D axisymmetric spherical and
 * quasi-spherical (Sec. 2.4).  Fields are static during a call (test-particle
 * mode) and taken as centred at t^n.  Particles are kept in a per-cell stable
 * order by a counting sort.  Reverse-mode (adjoint) steps give gradients of a
 * linear function of the final current and momenta with respect to the fields
 * and the initial momenta.
 *
 * Conventions
 *  - Code coordinates x^i in [0, N_i), cell size 1 (Sec. 2.4).
 *  - Field arrays: [6][np3][np2][np1], x fastest, components
 *    (E1,E2,E3,B1,B2,B3) = contravariant components at their own Yee points
 *    (App. A), 2 ghost cells per side of every active dimension
 *    (np_d = N_d + 4; in 2D np3 = 1).  Current arrays: [3][np3][np2][np1],
 *    the raw conformal current sum q w dx^i / dt on Yee edges in code units.
 *  - Four-velocities u (units of m c) are in the global Cartesian basis
 *    (Sec. 2.3); azimuth phi is tracked for axisymmetric grids (Sec. 2.4).
 *  - Storage/arithmetic precision is chosen per context (PIC_F32 / PIC_F64);
 *    "real" below means float or double accordingly.
 *
 * Ownership and streams
 *  - Every device buffer is allocated by the caller (e.g. torch tensors) and
 *    only borrowed; the library never allocates or frees device memory.
 *  - All device work is enqueued on the stream given to pic_set_stream
 *    (default: the null stream).  Calls return after enqueueing, except where
 *    noted (loads and host readbacks synchronize the stream).
 *  - A context is not thread-safe; distinct contexts are independent.
 *
 * Errors: every function returns a pic_status; pic_last_error() gives the
 * message of the last failure on that context.  Argument errors are detected
 * on the host before any device work is enqueued.
 */
#ifndef PICSTEP_H
#define PICSTEP_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct pic_ctx pic_ctx;

typedef enum {
  PIC_OK = 0,
  PIC_E_ARG = 1,         /* invalid argument */
  PIC_E_RANGE = 2,       /* particle or field value outside its valid range */
  PIC_E_STATE = 3,       /* call out of order (e.g. push before fields/particles) */
  PIC_E_HIP = 4,         /* HIP runtime error (message holds hipGetErrorString) */
  PIC_E_CAPACITY = 5,    /* particle capacity or buffer size exceeded */
  PIC_E_UNSUPPORTED = 6  /* valid but not supported configuration */
} pic_status;

typedef enum { PIC_CART = 0, PIC_SPH = 1, PIC_QSPH = 2 } pic_geom;
typedef enum { PIC_F32 = 0, PIC_F64 = 1 } pic_prec;
typedef enum { PIC_BASIS_CONTRAVARIANT = 0, PIC_BASIS_TETRAD = 1 } pic_basis;

#define PIC_MAX_SPECIES 8

/* Grid and run description (Sec. 2.4 metrics; Sec. 2.1 units). */
typedef struct {
  int32_t geom;            /* pic_geom */
  int32_t dim;             /* PIC_CART: 2 or 3; PIC_SPH/PIC_QSPH: 2 (axisymmetric) */
  int32_t n[3];            /* active cells per dimension (unused dims: 1) */
  double lo[3], hi[3];     /* PIC_CART: box extents; (Q)SPH: lo[0] = r_min, hi[0] = r_max,
                              theta spans [0, pi] (lo[1], hi[1] ignored) */
  double r0, vartheta;     /* PIC_QSPH: r = r0 + exp(R), theta(T) stretching, -1/2 < vartheta < 1 */
  int32_t periodic[3];     /* PIC_CART: must be 1 for each active dimension */
  double rho0;             /* fiducial Larmor radius: push coefficient k = q dt / (2 m rho0) */
  int32_t prec;            /* pic_prec of particles, fields and current */
  int32_t fp64_axis_cells; /* PIC_F32 (Q)SPH: particles within this many cells of theta = 0,
                              theta = pi or r_min use FP64 for metric and move (default 2) */
  int32_t sort_every;      /* per-cell sort before global steps that are multiples of this;
                              0 = only on explicit pic_sort */
  int32_t reserved;
  uint64_t max_particles;  /* capacity summed over species */
} pic_grid_desc;

/* Byte sizes of the caller-allocated buffers (pic_query_sizes). */
typedef struct {
  uint64_t fields_bytes;       /* [6][npts] real */
  uint64_t current_bytes;      /* [3][npts] real */
  uint64_t particle_set_bytes; /* one particle set (two are bound: the sort ping-pongs) */
  uint64_t prev_bytes;         /* positions before the last step of pic_push_deposit */
  uint64_t scratch_bytes;      /* sort keys/values/histograms, permutation, flags */
  uint64_t checkpoint_bytes;   /* one particle-state checkpoint (adjoint) */
  uint64_t field_points;       /* npts = np1*np2*np3 */
  int32_t np[3];               /* padded extents */
  int32_t elem_bytes;          /* 4 (PIC_F32) or 8 (PIC_F64) */
} pic_sizes;

/* Device buffers (borrowed). */
typedef struct {
  void *fields;       /* fields_bytes */
  void *current;      /* current_bytes */
  void *particles[2]; /* 2 x particle_set_bytes */
  void *prev;         /* prev_bytes */
  void *scratch;      /* scratch_bytes */
} pic_buffers;

/* Layout of one particle set: byte offsets of its SoA arrays (UINT64_MAX when
 * absent), each array holding `capacity` elements; species s occupies elements
 * [species_offset[s], species_offset[s] + species_capacity[s]).  cell is int32,
 * u, w and phi are real.  cell packs (i1 + 1) | i2 << shift2 | i3 << shift3; bit
 * 30 marks a dead particle.  Offsets are in [0, 1) (Sec. 3.1): double in a
 * PIC_F64 context, 32-bit unsigned fixed point (offset = value * 2^-32) in a
 * PIC_F32 context, where pic_particles_load rounds to the nearest such value
 * below 1. */
typedef struct {
  uint64_t cell, offs[3], u[3], w, phi;
  uint64_t capacity;
  uint64_t species_offset[PIC_MAX_SPECIES];
  uint64_t species_capacity[PIC_MAX_SPECIES];
  uint64_t species_count[PIC_MAX_SPECIES]; /* loaded particles (alive or dead) */
  int32_t nspecies;
  int32_t active_set;      /* which of the two bound sets holds the current state */
  int32_t shift2, shift3;  /* cell packing */
  uint64_t prev_cell, prev_offs[3]; /* byte offsets inside the prev buffer */
  uint64_t id;             /* int32 particle id: its index in the pic_particles_load call */
} pic_layout;

/* Host view of one species for pic_particles_get: arrays of n (x3 for cell,
 * offs and u; rows per particle) that the caller owns; any pointer may be NULL. */
typedef struct {
  uint64_t n;          /* in: capacity of the arrays; out: particles written */
  int32_t *cell;       /* n x 3 per-dimension cell index (unused dims 0) */
  double *offs;        /* n x 3 */
  double *u;           /* n x 3 */
  double *w;           /* n */
  double *phi;         /* n (axisymmetric) */
  int32_t *alive;      /* n */
  int32_t *cell_prev;  /* n x 3, positions before the last pushed step */
  double *offs_prev;   /* n x 3 */
  int32_t *perm;       /* n, permutation applied by the last sort (new i <- old perm[i]) */
  int32_t *id;         /* n, each particle's index in its pic_particles_load call */
} pic_particle_view;

/* ---- context and setup (Sec. 2.4, Sec. 3.1) ---- */

/* Validates the description (host only, no device call) and creates a
 * context.  PIC_E_ARG for an invalid description, PIC_E_UNSUPPORTED for a
 * non-periodic Cartesian grid.  *out is set only on PIC_OK. */
pic_status pic_grid_init(const pic_grid_desc *desc, pic_ctx **out);

/* Destroys a context; never frees caller memory. */
void pic_grid_destroy(pic_ctx *ctx);

/* Sizes of every caller-allocated buffer (depends on species added so far
 * only through the total capacity). Host only. */
pic_status pic_query_sizes(const pic_ctx *ctx, pic_sizes *out);

/* Registers the caller's device buffers (sizes from pic_query_sizes). */
pic_status pic_bind_buffers(pic_ctx *ctx, const pic_buffers *buf);

/* Stream for all later device work (a hipStream_t; NULL = null stream). */
pic_status pic_set_stream(pic_ctx *ctx, void *hip_stream);

/* dt = cfl * dx_min, dx_min = min over cell centres of (sum_i 1/h_ii)^(-1/2)
 * (Sec. 2.4, timestep paragraph).  Host only. */
pic_status pic_timestep_from_cfl(const pic_ctx *ctx, double cfl, double *dt);

/* Adds a species with charge and mass in fiducial units (Sec. 2.1) and a
 * capacity; species are laid out contiguously in order of addition.
 * PIC_E_CAPACITY when the capacities exceed max_particles, PIC_E_STATE
 * after particles were loaded.  Host only. */
pic_status pic_species_add(pic_ctx *ctx, double charge, double mass, uint64_t capacity,
                           int32_t *species_id);

/* Pushers of the momentum update (step 5).  The method leaves the choice to a
 * conventional pusher on the global Cartesian components (Sec. 2.2, citing
 * Boris 1970 and Vay 2008); for strongly magnetised plasma it adds a hybrid
 * that hands a particle over to the guiding-centre approximation (Sec. 5.2,
 * after Bacchini et al. 2020). */
typedef enum {
  PIC_PUSH_BORIS = 0, /* relativistic Boris rotation (default) */
  PIC_PUSH_VAY = 1,   /* Vay (2008): implicit mean velocity, solved in closed form */
  PIC_PUSH_GCA = 2    /* flag, with either: the guiding-centre hybrid */
} pic_pusher;

/* Sets the pusher of a species (default PIC_PUSH_BORIS).  With PIC_PUSH_GCA a
 * particle is advanced as its guiding centre on a step where |E| < e_ovr |B|
 * (0 < e_ovr < 1) and its nominal gyroradius |u| m rho0 / (|q| |B|) is below
 * larmor_max (> 0, code length units): its momentum across B is dropped, the
 * parallel four-velocity takes the full parallel kick, and it drifts with
 * E x B / B^2.  The regime test is taken in FP64 on the particle's fields and
 * momentum before the step.  e_ovr and larmor_max are ignored without the
 * flag.  PIC_E_ARG for an unknown pusher or bad thresholds.  The adjoint
 * entry points refuse (PIC_E_UNSUPPORTED) a context with a species that does
 * not use the Boris pusher.  Host only. */
pic_status pic_species_set_pusher(pic_ctx *ctx, int32_t species, int32_t pusher, double e_ovr,
                                  double larmor_max);

/* Sets the fields from a host FP64 array in `basis`.  Tetrad input is turned
 * into contravariant components F^i = F^i_hat / sqrt(h_ii) at each
 * component's own Yee point (eq. curvspace-tetradtrans), in FP64, then
 * rounded to the storage precision; on (quasi-)spherical grids E3 and B2 are
 * set to 0 on the axis nodes j = 0 and j = N2 (Sec. 2.6).  includes_ghosts =
 * 0: `EB` is the active region [6][n3][n2][n1] and periodic ghosts are filled
 * by copy; 1: `EB` is the padded array [6][np3][np2][np1] (required for
 * (quasi-)spherical grids).  Synchronizes the stream. */
pic_status pic_fields_set(pic_ctx *ctx, const double *EB, int32_t basis,
                          int32_t includes_ghosts);

/* Refills the periodic ghost cells of the bound field buffer from the active
 * region (after the caller wrote the buffer directly).  Asynchronous. */
pic_status pic_fields_fill_ghosts(pic_ctx *ctx);

/* Loads n particles of one species from host FP64 arrays (rows per particle):
 * cell n x dim int32 (per-dimension indices), offs n x dim in [0,1), u n x 3
 * global Cartesian, w n, phi n (axisymmetric only, else NULL).  Validates on
 * the host: PIC_E_RANGE for an index outside the grid, an offset outside
 * [0,1), or a non-finite value; PIC_E_CAPACITY when n exceeds the species
 * capacity.  Replaces the species' previous content.  Synchronizes. */
pic_status pic_particles_load(pic_ctx *ctx, int32_t species, uint64_t n, const int32_t *cell,
                              const double *offs, const double *u, const double *w,
                              const double *phi);

/* Stable per-cell counting sort of every species (dead particles last);
 * ties keep their order.  Cells are ordered brick by brick (4x4x4 in 3D,
 * 8x8 in 2D).  When the particles are still in the order of the previous
 * sort and the library's own steps since then cannot have moved any of them
 * by more than one brick per dimension, the sort takes the brick-neighbour
 * form (counts per neighbouring brick, then a counting sort inside each
 * brick); otherwise three radix passes.  Same permutation either way.
 * Asynchronous. */
pic_status pic_sort(pic_ctx *ctx);

/* pic_sort without any device allocation by anyone: for callers that cannot
 * allocate device memory at the time of the call (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).  Same
 * result as pic_sort (the permutation is stored in the bound scratch buffer
 * as usual), but the radix sort's temporaries (keys, values, tile histograms,
 * column sums) live in a static device array of the library, 66 MiB per GPU,
 * held until the process ends; no hipMalloc, hipFree or allocating routine is
 * called.  Limit: at most 4,194,304 (2^22) particles per species, else
 * PIC_E_CAPACITY before any device work.  The device current at the call must
 * be the one the context's buffers live on.  Every call on a GPU uses that
 * GPU's one array: calls that overlap on one GPU (several streams or host
 * threads) race.  Asynchronous. */
pic_status pic_sort_static(pic_ctx *ctx);

/* n_steps particle steps with static fields and step size dt.  Before each
 * step whose global index is a multiple of sort_every (> 0) the particles are
 * sorted.  J is zeroed at the start of every step; after the call it holds
 * the conformal current of the last step (periodic ghost contributions added
 * into their images, ghosts zero; (quasi-)spherical ghosts keep the current
 * of radially exiting particles).  Positions before the last step are kept
 * in the prev buffer.  A particle leaving r_min or r_max deposits its step
 * and is then dead.  Asynchronous. */
pic_status pic_push_deposit(pic_ctx *ctx, double dt, int32_t n_steps);

/* ---- field solver: the field update around the particle step (Sec. 2.3
 * steps 2, 9-11), in place on the bound field buffer, in the discretized
 * forms of App. A: covariant components F_i = h_ii F^i differenced over unit
 * code cells and divided by sqrt(h) = sqrt(h11 h22 h33) at the updated
 * component's Yee point; metric factors are computed on the fly in FP64.
 * Updated points: periodic Cartesian grids the active region (ghosts
 * refilled from their images); (quasi-)spherical grids the nodes 0..N
 * (integer-staggered components) or cells 0..N-1 (half-staggered) of each
 * dimension, the radial ghosts being the caller's boundary values.  On the
 * polar axis (j = 0 and j = N2) E3 and B2 are kept 0 and E1 takes the
 * update integrated over the half cell next to the axis (Sec. 2.6).  All
 * asynchronous; PIC_E_ARG for a step above the CFL limit. */

/* Faraday (eq. discretized-faraday): B^i -= f (curl E)^i / sqrt(h).  The loop
 * takes two half steps, f = dt / 2, around the particle step. */
pic_status pic_fields_advance_b(pic_ctx *ctx, double f);

/* Ampere (eq. discretized-ampere) with the bound current buffer (the
 * conformal current of the last particle step): E^i += dt ((curl B)^i -
 * coupling J^i) / sqrt(h).  coupling is the factor the method writes as 4 pi
 * (with fields in units of B0, lengths of rho0 and the macro-particle
 * weights of the current, the plasma frequency of a cold species of
 * charge q, mass m and weight per unit volume n is sqrt(coupling n q^2 / m)). */
pic_status pic_fields_advance_e(pic_ctx *ctx, double dt, double coupling);

/* passes of the digital filter of Sec. 2.5 on the bound current buffer:
 * each component on its own lattice, weights (1/2)^(D + |di| + |dj| + |dk|)
 * over its 3^D neighbours; periodic Cartesian grids wrap, (quasi-)spherical
 * grids mirror across the axes (J1 even, J2 odd, J3 zero on the axis,
 * Sec. 2.6) and read the stored radial ghosts.  work: device buffer of
 * current_bytes (caller-owned scratch). */
pic_status pic_current_filter(pic_ctx *ctx, int32_t passes, void *work);

/* n_steps of the whole loop of Sec. 2.3: Faraday dt/2; the particle step
 * (sort at the context's cadence, interpolation at B^n, E^n, push, deposit);
 * filter_passes of the current filter; Faraday dt/2; Ampere with the filtered
 * current.  work as for pic_current_filter (may be NULL without passes).
 * After the call the bound buffers hold B^{n+1/2}, E^{n+1}, the particles at
 * x^{n+1}, u^{n+1/2}, and the (filtered) current of the last step. */
pic_status pic_step_full(pic_ctx *ctx, double dt, int32_t n_steps, int32_t filter_passes,
                         double coupling, void *work);

/* Copies the current [3][npts] (storage precision) to dst, on the device
 * (dst_is_device = 1, asynchronous) or the host (synchronizes). */
pic_status pic_current_get(const pic_ctx *ctx, void *dst, int32_t dst_is_device);

/* Copies the contravariant fields [6][npts] (storage precision) likewise. */
pic_status pic_fields_get(const pic_ctx *ctx, void *dst, int32_t dst_is_device);

/* Copies one species to host FP64 arrays in the current (sorted) order.
 * Synchronizes. */
pic_status pic_particles_get(const pic_ctx *ctx, int32_t species, pic_particle_view *dst);

/* Byte layout of the particle sets (for zero-copy device views). Host only. */
pic_status pic_particle_layout(const pic_ctx *ctx, pic_layout *out);

/* Global step counter (number of steps pushed so far). Host only. */
pic_status pic_step_count(const pic_ctx *ctx, int64_t *step);

/* Kernel timing.  While enabled, HIP events recorded on the bound stream
 * bracket every launch of the fused particle-step kernel, every per-cell sort
 * and every adjoint step kernel.  pic_timing_read waits for the recorded
 * events, returns the accumulated times (ms) and launch counts, and clears
 * them. */
typedef struct {
  int64_t push_launches;
  double push_ms;
  int64_t sort_calls;
  double sort_ms;
  int64_t adjoint_launches;
  double adjoint_ms;
  int64_t push_blocks;           /* blocks of the fused kernel with live particles */
  int64_t push_global_particles; /* particles whose stencil left the LDS tile, deposited with
                                    global atomics */
  int64_t sort_brick_calls;      /* sorts that took the brick-neighbour form (counted whether
                                    or not timing is enabled) */
} pic_timing;
pic_status pic_timing_enable(pic_ctx *ctx, int32_t enable);
pic_status pic_timing_read(pic_ctx *ctx, pic_timing *out);

/* ---- adjoint (reverse-mode derivative of the discrete K-step map) ----
 *
 * L = sum(lamJ * J_K) + sum(lam_u . u_K) is a linear function of the current
 * of the last of K steps and of the final four-velocities.  The fields are
 * static, so dL/dF accumulates the transposed interpolation of every step.
 * Memory is bounded by checkpointing: the particle state is saved every m
 * steps and each segment is recomputed once during the reverse sweep. */

/* Workspace bytes for pic_forward_checkpointed / pic_backward with K, m. */
pic_status pic_adjoint_workspace(const pic_ctx *ctx, int32_t K, int32_t m, uint64_t *bytes);

/* K steps exactly as pic_push_deposit(dt, K) runs them, sorts included (a
 * sort before every step whose global index is a multiple of sort_every),
 * saving the state (cell, offsets, u, w, phi) at steps 0, m, 2m, ... before
 * that step's sort, and the permutation of every sort, into `workspace`
 * (device, pic_adjoint_workspace bytes, which covers ceil(K / sort_every)
 * sorts).  Leaves the context at step K with J of the last step, like
 * pic_push_deposit.  Asynchronous. */
pic_status pic_forward_checkpointed(pic_ctx *ctx, double dt, int32_t K, int32_t m,
                                    void *workspace);

/* Reverse sweep after pic_forward_checkpointed(dt, K, m, workspace), with the
 * same dt, K and m (PIC_E_STATE otherwise).  A context holds one checkpointed
 * forward at a time: a second pic_forward_checkpointed replaces the first.
 * lamJ: device [3][npts] real (dL/dJ_K; may be NULL = 0); lam_u: device
 * [3][capacity] real in the particle order at step K (may be NULL).
 * Outputs (device, overwritten): dEB [6][npts] real, dL/d(fields) with
 * periodic ghost contributions added into their images (ghosts 0);
 * du0 [3][capacity] real, dL/du at step 0 in the particle order at step 0
 * (before that step's sort).  Segments are recomputed from the checkpoints
 * replaying the stored permutations, and the adjoints of the particles
 * follow every sort backwards.  Restores the particle state of step 0.
 * Asynchronous. */
pic_status pic_backward(pic_ctx *ctx, double dt, int32_t K, int32_t m, void *workspace,
                        const void *lamJ, const void *lam_u, void *dEB, void *du0);

/* After pic_forward_checkpointed(..., workspace): for every particle slot i
 * (0 <= i < capacity, species ranges as in pic_particle_layout) of the order
 * at step K, the slot the same particle had at step 0, composed from the
 * stored sort permutations (identity outside the species' counts).  dst:
 * host int32[capacity].  Synchronizes the bound stream.  PIC_E_STATE without
 * a completed forward. */
pic_status pic_checkpointed_order(const pic_ctx *ctx, const void *workspace, int32_t *dst);

/* ---- lower-level adjoint pieces, for callers with their own checkpoint
 * schedule.  A checkpoint is the particle state (cell, offsets, u, w, phi)
 * of the whole capacity, pic_sizes.checkpoint_bytes in the device buffer
 * `slot`; the step counter is not part of it.  Asynchronous. */
pic_status pic_checkpoint_save(pic_ctx *ctx, void *slot);
pic_status pic_checkpoint_load(pic_ctx *ctx, const void *slot);

typedef struct {
  void *lam_u;     /* device [3][capacity] real: in dL/du after the step, out dL/du before */
  void *lam_offs;  /* device [3][capacity] real: likewise for the in-cell offsets (rows of
                      unused dimensions are left untouched, except that on (quasi-)spherical
                      grids row 2 carries dL/dphi, the adjoint of the azimuth) */
  void *dEB;       /* device [6][npts] real: the step's dL/d(fields) is added, periodic
                      ghost contributions folded into their images */
  void *lamJ_work; /* device [3][npts] real scratch, used when lamJ is given */
} pic_adjoint_buffers;

/* Reverse of one particle step from the current particle
 * state, the state before that step (e.g. just restored with
 * pic_checkpoint_load): lamJ (device [3][npts] real, dL/dJ of this step, may
 * be NULL) is gathered through the step's zig-zag, the adjoints of u and of
 * the offsets are carried back through the move and the Boris push, and the
 * interpolation's adjoint is scattered into dEB.  A sort that began the step
 * is not reversed here (pic_backward handles sorts; with sort_every = 0 there
 * are none).  The particle state is left unchanged.  Asynchronous. */
pic_status pic_adjoint_step(pic_ctx *ctx, double dt, const void *lamJ,
                            const pic_adjoint_buffers *io);

/* ---- failure detection ----
 * The kernels raise bits of a sticky device error word instead of trapping:
 *   PIC_DEVERR_NONFINITE  a push produced a non-finite four-velocity (NaN or
 *                         infinite fields, momenta or weights); the particle
 *                         is kept as computed;
 *   PIC_DEVERR_SORT_MOVE  at a sort, a particle had crossed more than one
 *                         brick of the sort order in some dimension since the
 *                         previous sort (its cell was changed through the
 *                         bound buffers without pic_particles_modified); that
 *                         sort kept the previous order (identity permutation).
 * pic_device_errors waits for the bound stream, returns the word in *flags
 * and, when clear != 0, clears it. */
#define PIC_DEVERR_NONFINITE 1
#define PIC_DEVERR_SORT_MOVE 2
pic_status pic_device_errors(pic_ctx *ctx, int32_t *flags, int32_t clear);

/* Tells the library that the particle arrays were written through the bound
 * buffers (not by its own calls): the next sort then makes no assumption
 * about how far particles moved since the previous one (Sec. 3.3.2 sort of
 * the particle arrays; the fast form assumes moves of at most one brick). */
pic_status pic_particles_modified(pic_ctx *ctx);

/* Debug launch mode of the fused step kernel (race detection): with on != 0
 * every push launches its blocks one at a time, each alone on the GPU, in
 * the plain block order.  Particle results are identical to the normal
 * launch (the current differs only by the order of its floating-point
 * additions across blocks).  Slow: for small test grids. */
pic_status pic_debug_serial(pic_ctx *ctx, int32_t on);

/* Message of the last failing call on this context (never NULL). */
const char *pic_last_error(const pic_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* PICSTEP_H */
