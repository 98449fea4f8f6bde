/*
 * empic.h -- C ABI of libempic, an MI355X (gfx950) implementation of the
 * explicit 3D electromagnetic particle-in-cell step of KEMPIC-3D
 * (arXiv 2609.16575): staggered trilinear gather of E and B, relativistic
 * Boris push, charge-conserving ZigZag current deposit and Yee FDTD curl
 * updates (Sec. 2.2 of the paper, Fig. "PIC algorithm").
 *
 * Conventions (all calls):
 *   - Units c = eps0 = mu0 = 1 (the bare "- dt J" of the Ampere-Maxwell
 *     update, Sec. 2.3).  Momenta are u = gamma v.
 *   - Time levels (Sec. 2.3, 2.4): E and particle positions at t^n, B and
 *     momenta at t^{n-1/2}.  empic_step advances all four by whole steps.
 *   - Grid arrays are [k][j][i] (x fastest) with ext[a] = n[a] + 1 on a
 *     walled (absorbing or PEC) axis, n[a] on a periodic one.  Component locations in cell
 *     units: Ex(i+1/2,j,k) Ey(i,j+1/2,k) Ez(i,j,k+1/2), Bx(i,j+1/2,k+1/2)
 *     By(i+1/2,j,k+1/2) Bz(i+1/2,j+1/2,k); J like E; rho at nodes.  On a
 *     walled axis the entry n of a half-cell component is padding and
 *     stays zero.
 *   - All device memory is owned by the caller (fields, particle buffers,
 *     workspace).  The library keeps raw pointers only; the caller keeps the
 *     memory alive and unmoved while the handle lives.  empic_destroy never
 *     frees caller memory.
 *   - Every kernel is launched on the hipStream_t given at creation.  Calls
 *     are asynchronous except empic_diagnostics, empic_sync,
 *     empic_particle_count and empic_kernel_times, which synchronise it.
 *   - Every call returns an empic_status; nothing throws across the ABI.
 *     After EMPIC_E_ARG, EMPIC_E_CFL, EMPIC_E_CAPACITY or
 *     EMPIC_E_UNSUPPORTED the handle is unchanged and usable.  After
 *     EMPIC_E_HIP the handle is poisoned: only empic_destroy and
 *     empic_last_error are allowed.  EMPIC_E_NONFINITE / EMPIC_E_STATE
 *     report a fault word raised by the kernels (bits EMPIC_FAULT_*), as
 *     does EMPIC_E_CAPACITY when empic_diagnostics returns it
 *     (EMPIC_FAULT_CAPACITY).
 *   - A handle is not thread-safe; use one handle per stream.
 */
#ifndef EMPIC_H
#define EMPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EMPIC_MAX_SPECIES 4

typedef enum {
    EMPIC_OK = 0,
    EMPIC_E_ARG = 1,         /* bad argument (null, size, range, order of calls) */
    EMPIC_E_STATE = 2,       /* kernel fault word reports corrupted particle state */
    EMPIC_E_HIP = 3,         /* a HIP runtime call failed; handle poisoned */
    EMPIC_E_CFL = 4,         /* dt violates the 3D CFL bound (Sec. 2.3, CFL eq.) */
    EMPIC_E_CAPACITY = 5,    /* particle count exceeds a buffer's capacity */
    EMPIC_E_NONFINITE = 6,   /* a non-finite momentum or field reached a particle */
    EMPIC_E_UNSUPPORTED = 7  /* valid request this build does not implement */
} empic_status;

/* Boundaries per axis.  ABSORBING: first-order Mur on tangential E of both
 * faces.  PEC: perfectly conducting walls (the waveguide of Sec. 3.2),
 * tangential E zero on both faces.  Particles leaving a walled axis are
 * removed. */
enum { EMPIC_BC_PERIODIC = 0, EMPIC_BC_ABSORBING = 1, EMPIC_BC_PEC = 2 };

/* Arithmetic of the step. */
enum {
    EMPIC_FP32_CELLREL = 0, /* FP32 fields; particles as packed cell + FP32
                               in-cell offset + FP32 u; cell-sorted, fused
                               gather/push/deposit with LDS tiles */
    EMPIC_FP64_PLAIN = 1    /* FP64 fields and global FP64 positions, unsorted,
                               one thread per particle, global atomics */
};

/* Fault bits raised by kernels (empic_diag.fault_word). */
enum {
    EMPIC_FAULT_NONFINITE = 1u,   /* non-finite gamma after the push */
    EMPIC_FAULT_FAST = 2u,        /* |dxi| >= 1 cell in one step (impossible under CFL) */
    EMPIC_FAULT_OFFSET = 4u,      /* stored in-cell offset outside [0,1) */
    EMPIC_FAULT_CELL = 8u,        /* stored cell index outside the grid */
    EMPIC_FAULT_FALLBACK = 16u,   /* info: a particle left its tile window and was
                                     handled through global memory (not an error) */
    EMPIC_FAULT_CAPACITY = 32u    /* moving-window injection would exceed the
                                     species' capacity: nothing was injected */
};

/* Grid and time step (Sec. 2.3).  dt must satisfy
 *   dt <= 1 / sqrt(1/d0^2 + 1/d1^2 + 1/d2^2)              (c = 1)
 * FP32_CELLREL additionally limits n to <= 2047 x 2047 x 1023 cells (the
 * packed cell index) unless the handle holds no particles (max_capacity 0).
 * sort_every = S > 0 re-sorts particles by tile and cell at the start of
 * every S-th step (FP32 path); 0 sorts only on request and once before the
 * first step; -1 sorts adaptively: when particles leave their tile's
 * windows faster than 2e-5 of the particle slots per step, or after 64
 * steps.  The count is read back two steps late: each step waits for the
 * step two before it, so the GPU always has a step queued.  The adaptive
 * mode keeps four pinned host words and four events per handle (freed by
 * empic_destroy). */
typedef struct {
    int32_t n[3];
    int32_t bc[3];      /* EMPIC_BC_* per axis */
    double d[3];        /* cell sizes */
    double dt;
    int32_t precision;  /* EMPIC_FP32_CELLREL or EMPIC_FP64_PLAIN */
    int32_t sort_every;
} empic_grid_desc;

/* A species (Sec. 2.1): a macro-particle of weight w stands for w physical
 * particles with charge q w and mass m w.  per_particle_w = 1 takes the weight
 * of each particle from its `w` buffer instead (q w_p, m w_p). */
typedef struct {
    double q;
    double m;
    double w;
    int32_t per_particle_w;
    int32_t pad;
} empic_species_desc;

/* Device buffers of one species.  FP32_CELLREL: cell = packed
 * i | j << 11 | k << 22 (or -1 for a removed particle), pos = in-cell
 * offsets in [0,1) (float), u (float), w (float, optional).  FP64_PLAIN: cell
 * unused (may be NULL), pos = global positions in [0, L) (double), u (double),
 * w (double, optional).  id (int32) travels with the particle through sorts. */
typedef struct {
    int32_t *cell;
    void *pos[3];
    void *u[3];
    int32_t *id;
    void *w;
} empic_particle_buffers;

/* Soft current-sheet laser source (READING of the paper's external-source
 * module, Sec. 2.5 and 3.2): J_y on x-node plane i_s radiating
 * E_inc = a0 exp(-r^2/w0^2) exp(-2 ln2 (t-t0)^2/tau^2) sin(omega0 (t-t0)),
 * r^2 = (y-yc)^2 + (z-zc)^2, in both directions.  slab = 1 drops the y term
 * (r^2 = (z-zc)^2): the spot of the two-dimensional runs of Sec. 4, whose y
 * axis is periodic and two cells wide. */
typedef struct {
    double a0, w0, tau, t0, omega0, yc, zc;
    int32_t i_s;
    int32_t enabled;
    int32_t slab;
    int32_t pad;
} empic_laser_desc;

/* Waveguide port (the excitation of the field-solver benchmark, Sec. 3.2):
 * a hard source on the node plane `plane` of axis `axis` that sets, after
 * every step,  E_comp = e0 sin(pi s / L) (1 - exp(-t/tau)) sin(omega t)  at
 * t = t^{n+1}, s being the component's position along prof_axis and L that
 * axis' length (the TE10 profile).  comp and prof_axis are transverse to
 * axis; tau > 0. */
typedef struct {
    int32_t enabled;
    int32_t axis;
    int32_t plane;
    int32_t comp;
    int32_t prof_axis;
    int32_t pad;
    double e0, omega, tau;
} empic_port_desc;

/* FP64 diagnostics of the current state (Sec. 3.3).  U_E = dV/2 sum |E^n|^2,
 * U_B = dV/2 sum B^{n-1/2}.B^{n+1/2} (B^{n+1/2} formed from the state),
 * K_minus / K_plus = sum w m (gamma - 1) at u^{n-1/2} / u^{n+1/2} (the latter
 * from a side-effect-free push), K = their mean, U_tot = U_E + U_B + sum K.
 * Gauss residual r = div E - rho - rho_bg at nodes (backward differences).
 * cont_max = max |rho^n - rho^{n-1} + dt div J^{n-1/2}| when the previous
 * call was made exactly one step earlier (cont_valid = 1), with rho_max the
 * largest |rho^n| of the particles for scale; the nodes on the faces of a
 * walled (absorbing or PEC) axis are left out of cont_max, since a particle
 * leaving through the wall takes its charge out of the grid there. */
typedef struct {
    int64_t step;
    double t;
    double U_E, U_B, U_tot;
    double K[EMPIC_MAX_SPECIES];
    double K_minus[EMPIC_MAX_SPECIES];
    double K_plus[EMPIC_MAX_SPECIES];
    double gauss_max, gauss_l2;
    double cont_max, rho_max;
    int32_t cont_valid;
    uint32_t fault_word;
    /* storage slots in use: the live particles and, on the FP32 path, those
     * removed (through an absorbing wall or behind the window) since the last
     * sort, which drops them */
    int64_t n_particles[EMPIC_MAX_SPECIES];
    int64_t fallback_particles; /* cumulative count of out-of-window particles */
} empic_diag;

typedef struct empic_sim empic_sim;

/* Bytes of device workspace the handle needs for this grid, up to
 * max_species species of at most max_capacity particles each. */
size_t empic_workspace_bytes(const empic_grid_desc *g, int32_t max_species,
                             int64_t max_capacity);

/* Validate the grid (sizes, CFL -> EMPIC_E_CFL), keep the stream and the
 * caller-owned workspace (>= empic_workspace_bytes, 256-byte aligned). */
empic_status empic_create(const empic_grid_desc *g, int32_t max_species, int64_t max_capacity,
                          void *hip_stream, void *workspace, size_t workspace_bytes,
                          empic_sim **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): empic_create with
 * the library's own static workspace in place of a caller's.  The workspace
 * is a device array of EMPIC_STATIC_SCRATCH_BYTES that every GPU the library
 * runs on holds until the process ends; it serves one live handle per device
 * at a time.  The handle itself sits in static host storage.  The call
 * allocates nothing (no hipMalloc, hipHostMalloc or heap); the caller still
 * owns and passes the fields and particle buffers.
 *   - Grid and sizes as empic_create; EMPIC_E_CAPACITY when
 *     empic_workspace_bytes(g, max_species, max_capacity) exceeds
 *     EMPIC_STATIC_SCRATCH_BYTES.
 *   - EMPIC_E_ARG when a handle of this call still lives on the current
 *     device (empic_destroy releases it), or when hip_stream belongs to
 *     another device than the current one.
 *   - EMPIC_E_UNSUPPORTED for the adaptive sort (sort_every = -1 on the FP32
 *     path), which needs pinned host memory; give a fixed cadence.
 *   - The handle uses the current device's array; the array keeps what the
 *     previous handle left in it, and the call clears what the kernels need
 *     zero, as empic_create does.  Calls on the handle from several threads
 *     at once race on the array (as on any handle). */
#define EMPIC_STATIC_SCRATCH_BYTES (64u << 20)
empic_status empic_create_static(const empic_grid_desc *g, int32_t max_species,
                                 int64_t max_capacity, void *hip_stream, empic_sim **out);

/* Bind the six field arrays and the current density, each ext0*ext1*ext2
 * elements of float (FP32_CELLREL) or double (FP64_PLAIN).  E = E^n,
 * B = B^{n-1/2}; J is written by every step (J^{n+1/2} of the last step). */
empic_status empic_bind_fields(empic_sim *s, void *const E[3], void *const B[3],
                               void *const J[3]);

/* Register a species with `capacity` slots in buffers buf0 and, for the FP32
 * path, a second set buf1 of the same capacity that the sort ping-pongs into
 * (buf1 may be NULL for FP64_PLAIN).  The species starts empty; fill it with
 * empic_load_particles_f64.  Up to EMPIC_MAX_SPECIES. */
empic_status empic_add_species(empic_sim *s, const empic_species_desc *desc, int64_t capacity,
                               const empic_particle_buffers *buf0,
                               const empic_particle_buffers *buf1, int32_t *species_id_out);

/* Fill species `sp` with `count` particles from device FP64 arrays: pos_xyz
 * and u_xyz are count x 3 (interleaved x,y,z), global positions in [0, L),
 * u = u^{-1/2}.  w (count, may be NULL) is the per-particle weight; ids
 * (count int32, may be NULL -> 0..count-1).  Converted on the device to the
 * species' storage (cell + FP32 offset for FP32_CELLREL). */
empic_status empic_load_particles_f64(empic_sim *s, int32_t sp, int64_t count,
                                      const double *pos_xyz, const double *u_xyz,
                                      const double *w, const int32_t *ids);

/* Write the live particles of `sp` as FP64 global positions and momenta
 * (count x 3 each, device) and their ids, in storage order; *count_out (host)
 * receives the number written.  Synchronises.  Capacity of the outputs must
 * be >= the species' capacity. */
empic_status empic_store_particles_f64(empic_sim *s, int32_t sp, double *pos_xyz,
                                       double *u_xyz, int32_t *ids, int64_t *count_out);

/* Which of the two buffer sets holds the species' particles now (0 or 1). */
empic_status empic_current_buffer(empic_sim *s, int32_t sp, int32_t *which);

/* Immobile neutralising background charge density (enters Gauss only). */
empic_status empic_set_background(empic_sim *s, double rho_bg);

/* External laser source (see empic_laser_desc); enabled = 0 removes it. */
empic_status empic_set_laser(empic_sim *s, const empic_laser_desc *laser);

/* Waveguide port (see empic_port_desc); enabled = 0 removes it.  EMPIC_E_ARG
 * for an axis, component or plane outside the grid. */
empic_status empic_set_port(empic_sim *s, const empic_port_desc *port);

/* Moving window (READING of the module of Sec. 2.2 used by the wakefield run
 * of Sec. 4).  FP32 path, along an absorbing axis.  At the start of a step,
 * once (t - t_start) velocity >= (shifts + 1) cells d[axis], E and B move
 * `cells` planes toward index 0 (zeros enter at the front), particles move
 * the same number of cells (those behind the window are removed), species
 * with an injection (empic_set_injection) receive cold particles in the new
 * cells, and the particles are re-sorted.  Sources stay fixed in the window
 * frame (start the window after a laser pulse has been injected).  A shift
 * of the tile size along the axis keeps sorts rare. */
typedef struct {
    int32_t enabled;
    int32_t axis;
    int32_t cells;
    int32_t pad;
    double velocity;
    double t_start;
} empic_window_desc;

empic_status empic_set_window(empic_sim *s, const empic_window_desc *w);

/* Cold plasma injected by the moving window into species sp: per_cell[a]
 * particles per axis at offsets (m + 1/2)/per_cell[a], u = 0, weight w (a
 * species without per-particle weights injects its own w); ids continue
 * from the loaded count.  per_cell = {0,0,0} turns it off.  A shift that
 * would exceed the species' capacity injects nothing (its ids are skipped)
 * and raises EMPIC_FAULT_CAPACITY.  Ids are int32: empic_step refuses a shift whose
 * injection would take them past 2^31 - 1 (EMPIC_E_CAPACITY before that
 * step; the handle stays usable). */
empic_status empic_set_injection(empic_sim *s, int32_t sp, const int32_t per_cell[3], double w);

/* Current filter (READING of the compensated smoothing module, Sec. 2.2):
 * after the deposit, along x, then y, then z, each J component on its own
 * sub-grid gets `passes` applications of the binomial stencil (1/4, 1/2,
 * 1/4) and, if compensate = 1, one of (-1/4, 3/2, -1/4).  Periodic axes wrap;
 * on a walled axis values beyond the array count as zero.  Charge is then
 * conserved for the filtered density.  passes = compensate = 0 (the default)
 * turns it off; EMPIC_E_ARG outside 0..16 / 0..1.  The step adjoint takes
 * the filter into account. */
empic_status empic_set_filter(empic_sim *s, int32_t passes, int32_t compensate);

/* Particle shape order (the shape-function equation of Sec. 2.4, B-spline
 * b_l of the cloud; the paper runs l = 0, Sec. 5 names higher orders).
 * order 1 (the default): CIC weighting (b_1), ZigZag current.  order 2: the
 * triangular cloud b_1 weighs the grid with the quadratic B-spline b_2 --
 * 27-point gather of every component from its own Yee sub-grid, b_2 charge
 * for the diagnostics, and the EZ current (Sec. 2.5): a move that crosses a
 * cell of the b_2 stencil (between half-integer planes) is split at the
 * ZigZag relay point and each part gets Esirkepov's decomposition.  Order 2:
 * FP32 path on periodic three-dimensional grids (else EMPIC_E_UNSUPPORTED);
 * empic_step_vjp refuses it.  EMPIC_E_ARG for other orders. */
empic_status empic_set_shape_order(empic_sim *s, int32_t order);

/* Advance the state by nsteps PIC cycles (Sec. 2.2): Faraday with temporal
 * centring of B -> gather, Boris, move, ZigZag deposit for every species ->
 * current filter -> Ampere-Maxwell -> laser source -> Mur faces -> PEC walls
 * -> port.  FP32 path: a moving-window shift when one is due, then the
 * counting sort when sort_every (or the adaptive policy) asks for it, before
 * the cycle.  Asynchronous, except that the adaptive policy waits for the step
 * two steps earlier.  EMPIC_E_CAPACITY: an injection would overflow the ids
 * (the steps before it were taken). */
empic_status empic_step(empic_sim *s, int32_t nsteps);

/* Sort (FP32 path) by tile and cell now, dropping removed particles. */
empic_status empic_sort(empic_sim *s);

/* CIC charge density at nodes (Sec. 2.5) of species sp (-1 = all), FP64,
 * ext0*ext1*ext2 doubles on the device, overwritten.  No background. */
empic_status empic_deposit_rho(empic_sim *s, int32_t sp, double *rho_out);

/* Compute the FP64 diagnostics of the current state; synchronises. */
empic_status empic_diagnostics(empic_sim *s, empic_diag *out);

/* Live particles of species sp; synchronises. */
empic_status empic_particle_count(empic_sim *s, int32_t sp, int64_t *n);

/* Wait for the stream; surface asynchronous HIP errors and the fault word. */
empic_status empic_sync(empic_sim *s);

/* Kernel timing with HIP events on the handle's stream: enable = 1 starts
 * recording every launch of the particle kernel ("push"), of the field
 * kernels ("field") and of the sort ("sort"); enable = 2 records the
 * particle kernel only, through events attached to its own dispatch (no
 * extra marker between kernels); 0 stops.  Other values: EMPIC_E_ARG.
 * empic_kernel_times returns the summed milliseconds and the launch counts
 * since enabling, and synchronises. */
empic_status empic_enable_timing(empic_sim *s, int32_t enable);
empic_status empic_kernel_times(empic_sim *s, double *push_ms, int64_t *push_launches,
                                double *field_ms, int64_t *field_launches,
                                double *sort_ms, int64_t *sort_launches);

/* ---- Differentiable runs (FP32 path, periodic grid) ------------------------
 * Not in the paper: the adjoint of the step, for gradients of a loss of the
 * final fields or particles with respect to the initial state.  A state is
 * everything a step reads: E^n, B^{n-1/2} and, per species, the particle
 * record in the current storage order (cell, in-cell offsets, u^{n-1/2}, id,
 * per-particle weight; arrays of the species' capacity) plus its tile
 * offsets and slot count (empic_state_tile_words int32).  An adjoint holds
 * d(loss)/d(state): fields like E and B, positions per unit length (global
 * coordinates), momenta.  All device arrays, owned by the caller, FP32 for
 * floating point. */
typedef struct {
    void *E[3], *B[3];
    int32_t *cell[EMPIC_MAX_SPECIES];
    void *pos[EMPIC_MAX_SPECIES][3];
    void *u[EMPIC_MAX_SPECIES][3];
    int32_t *id[EMPIC_MAX_SPECIES];
    void *w[EMPIC_MAX_SPECIES];        /* NULL for species without per-particle w */
    int32_t *tiles[EMPIC_MAX_SPECIES];
} empic_state;

typedef struct {
    void *E[3], *B[3];
    void *pos[EMPIC_MAX_SPECIES][3];
    void *u[EMPIC_MAX_SPECIES][3];
} empic_adjoint;

/* int32 words of a state's tiles[] array per species (tile count + 2). */
empic_status empic_state_tile_words(empic_sim *s, int64_t *words);

/* Copy the current state into dst / set the current state from src (device
 * copies on the handle's stream).  Saving needs particles that have been
 * sorted since they were loaded (EMPIC_E_ARG otherwise); a loaded state
 * must come from this handle. */
empic_status empic_save_state(empic_sim *s, const empic_state *dst);
empic_status empic_load_state(empic_sim *s, const empic_state *src);

/* One step (as empic_step, without a sort) from state src into state dst:
 * src's fields are copied into dst's field arrays and stepped there (the
 * handle's own E and B are untouched; its J receives the step's current),
 * particles are read from src's arrays and written to dst's (the handle's
 * own particle buffers are untouched), tile offsets and slot count are
 * carried over, ids and per-particle weights copied unless dst shares src's
 * arrays.
 * For re-computing the states between checkpoints without copying them.
 * src and dst must not share cell, offset or momentum arrays.  A state
 * carries no time: the handle's step count is left as it was, and a handle
 * with a laser, port or moving window (whose fields depend on the step's
 * time) gets EMPIC_E_UNSUPPORTED. */
empic_status empic_step_state(empic_sim *s, const empic_state *src, const empic_state *dst);

/* Vector-Jacobian product of one step taken from state st: lam holds the
 * adjoint of the state after the step on entry and that of st on return
 * (in place).  Transposed curls for the fields, deposit-as-gather of -dt
 * lam_E, reverse Boris, gather-as-scatter (float atomics).  Derivatives are
 * those of the current piece of each piecewise map.  EMPIC_E_UNSUPPORTED for
 * the FP64 path or a non-periodic grid. */
empic_status empic_step_vjp(empic_sim *s, const empic_state *st, const empic_adjoint *lam);

/* empic_sort that also writes, per species, perm[i][j] = the slot before the
 * sort of the particle in slot j after it (-1 for slots past the new count);
 * perm[i] holds the species' capacity of int32 (device).  For sorts inside a
 * differentiable run. */
empic_status empic_sort_recorded(empic_sim *s, int32_t *const perm[EMPIC_MAX_SPECIES]);

/* Adjoint of a recorded sort, in place on lam's particle arrays: moves each
 * slot's position and momentum adjoints back to the slot before the sort;
 * slots no particle came from (removed particles) get zero.  Entries of perm
 * outside [0, capacity) are ignored.  Uses the species' second buffer set as
 * scratch, whose contents no step reads between sorts. */
empic_status empic_sort_vjp(empic_sim *s, int32_t *const perm[EMPIC_MAX_SPECIES],
                            const empic_adjoint *lam);

/* FP64 sum over i < n of a[i] * b[i] for FP32 device arrays a, b (e.g. a
 * gradient's projection on a direction summed over all particles), in a
 * fixed order (the same result on every call); *out on the host.
 * Synchronizes the handle's stream. */
empic_status empic_dot_f64(empic_sim *s, const float *a, const float *b, int64_t n, double *out);

/* Cells per tile of the FP32 path's sort order and fused kernel (x, y, z):
 * particles are stored tile by tile (tiles x-fastest), cell by cell inside a
 * tile (x-fastest).  empic_tile_shape gives the shape of three-dimensional
 * grids (8 x 8 x 4); empic_grid_tile_shape the shape a grid gets, 16 x 2 x 8
 * when it is at most three cells thick along y (the two-dimensional runs of
 * Sec. 4).  Host-only; no handle needed. */
void empic_tile_shape(int32_t out[3]);
void empic_grid_tile_shape(const empic_grid_desc *g, int32_t out[3]);

/* Per-handle message for the last failed call; valid until the next call. */
const char *empic_last_error(const empic_sim *s);

void empic_destroy(empic_sim *s);

#ifdef __cplusplus
}
#endif

#endif /* EMPIC_H */
