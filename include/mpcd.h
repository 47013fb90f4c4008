/*
 * mpcd.h -- C ABI of libmpcd, a stochastic-rotation-dynamics (SRD) variant of
 * multiparticle collision dynamics (MPCD) for one AMD MI355X (gfx950) GPU.
 *
 * The method is that of Howard, Panagiotopoulos and Nikoubashman,
 * arXiv:1801.10187. One time step (sec. 3, flow diagram of Fig. 1) is:
 *   stream   r <- r + v dt in a periodic box                        (eq. 1)
 *   bin      random grid shift, cubic cells of edge a               (sec. 2, 3.4)
 *   collide  per-cell mass, momentum and kinetic energy (sec. 3.5, eq. 3),
 *            a random axis per cell (sec. 3.6), optional Maxwell-Boltzmann
 *            scale factor (sec. 2, 3.6), rotation v <- u + xi R(alpha)(v - u)
 *            (eq. 2, Alg. 1)
 *
 * Conventions for every entry point
 *  - Every call returns an mpcd_status; no C++ exception crosses the ABI.
 *    mpcd_last_error() returns a thread-local text for the last failure.
 *  - Positions and velocities cross the ABI as row-major N x 3 arrays of
 *    double, (x0, y0, z0, x1, ...). A flag says whether a pointer is host or
 *    device memory. The context copies what it is given and never keeps a
 *    caller pointer; outputs go to caller-owned buffers.
 *  - Particles are identified by their tag: the solvent particles are tags
 *    0 .. n_solvent-1 in the order given to mpcd_create, embedded particles
 *    follow. Every get_* returns data in tag order, whatever the internal
 *    (cell-sorted) order.
 *  - The box is [0, L)^3 with L = n_cells[d] * a, periodic.
 *  - Call order within a step is mpcd_stream -> mpcd_bin -> mpcd_collide;
 *    any other order returns MPCD_ESTATE. mpcd_step runs whole steps from the
 *    state after a collide (or after create).
 *  - All device work is enqueued on the context's HIP stream. Errors raised
 *    inside kernels (range checks) are reported by mpcd_sync and by any get_*.
 *  - A context is not thread-safe; use one per host thread.
 */
#ifndef MPCD_H
#define MPCD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPCD_ABI_VERSION 3

typedef struct mpcd_ctx_s* mpcd_ctx;

typedef enum {
  MPCD_OK = 0,
  MPCD_EINVAL = 1, /* bad argument: sizes, parameters, positions outside the box */
  MPCD_ENOMEM = 2, /* device or host allocation failed                            */
  MPCD_EHIP = 3,   /* a HIP runtime call failed                                   */
  MPCD_ERANGE = 4, /* a kernel range check failed: a particle moved a whole box    */
                   /* length in one step (FP64 form), a momentum outside the       */
                   /* fixed-point range, or the Gamma sampler hit its attempt cap  */
  MPCD_ESTATE = 5  /* call out of order                                           */
} mpcd_status;

/* Storage forms (sec. 4.1, mixed precision). Both compute the cell sums,
 * the draws and the rotation in FP64 and keep the cell sums in integer fixed
 * point, so results do not depend on the order the particles are summed in.
 *  MPCD_FP64  positions and velocities in double precision; two-limb sums of
 *             resolution 2^-72; every term (m v_d, and m |v - u|^2 with the
 *             thermostat, m dv_d under the AT rule) must satisfy
 *             |term| < 2^30, and every displacement |v_d dt| < L_d.
 *  MPCD_FP32  position = home cell (10 bits per axis: at most 1024 cells per
 *             axis) plus an FP32 offset inside it, FP32 velocities; one-limb
 *             sums of resolution 2^-40 with |term| < 2^11 = 2048. With unit
 *             mass that bounds a velocity component by 2048 (and
 *             |v - u| by 45 with the thermostat); a strongly boosted flow or
 *             heavy, fast embedded particles can exceed it in this form only.
 * A term outside its range makes the step report MPCD_ERANGE. */
typedef enum { MPCD_FP64 = 0, MPCD_FP32 = 1 } mpcd_precision;

/* Collision rule: stochastic rotation (eq. 2, Alg. 1), or the Andersen
 * thermostat (eq. 4, sec. 3.7): v_i <- u + dv_i - sum_j m_j dv_j / M_c with
 * dv_i ~ N(0, kT / m_i) per component, drawn per particle from Philox counter
 * (tag within the box, step, 3, 0) by Box-Muller: in double precision in the
 * FP64 form; in single precision in the FP32 form (sec. 4.1: the mixed
 * model keeps double precision for the cell sums and the rotation), from
 * uniforms u = (w / 2^9 + 1/2) 2^-23 and with the scale sqrt(kT / m) rounded
 * to FP32. The AT rule thermostats by itself: thermostat must be 0 with it. */
typedef enum { MPCD_SRD = 0, MPCD_AT = 1 } mpcd_collision;

/* Problem parameters as the paper states the problem (sec. 2, sec. 4). */
typedef struct {
  int32_t n_cells[3];  /* cells per axis (>= 1); FP32 form: <= 1024 per axis    */
  double a;            /* cell edge (> 0)                                        */
  double alpha;        /* SRD rotation angle in radians (eq. 2)                  */
  double dt;           /* collision time (>= 0) (eq. 1)                          */
  double kT;           /* thermostat temperature (>= 0)                          */
  uint64_t seed;       /* user seed of the per-cell random streams (sec. 3.6)    */
  double solvent_mass; /* mass m of every solvent particle (> 0) (sec. 3.2)      */
  int32_t precision;   /* mpcd_precision: storage form of positions/velocities   */
  int32_t thermostat;  /* 0 none, 1 Maxwell-Boltzmann cell scaling (sec. 2, 3.6) */
  int32_t grid_shift;  /* 1 random grid shift each step (sec. 2), 0 none         */
  int32_t flags;       /* MPCD_FLAG_* bits, and a MPCD_TILE_* shape (0: rule)   */
  int32_t collision;   /* mpcd_collision: MPCD_SRD (0) or MPCD_AT (1)            */
} mpcd_params;

/* Test-only layout flag: size the per-tile particle slabs to the initial
 * maximum occupancy (no headroom), so that the first steps overflow them
 * and the enlarge-and-replay path runs.
 * Results are unchanged. */
#define MPCD_FLAG_TIGHT_SLABS 1

/* Solute coupling through an external MD integrator (sec. 3.6): the embedded
 * particles are not streamed by MPCD; between collisions the caller moves
 * them (and changes their velocities) with its own equations of motion and
 * hands their state over with mpcd_set_embedded; the collision then mixes
 * them with the solvent and mpcd_get_embedded returns their new velocities.
 * Without this flag embedded particles stream ballistically like the
 * solvent. */
#define MPCD_FLAG_MD_SOLUTE 2

/* Test hook for the error paths: after `after` more successful device
 * allocations by the library (any context, any thread), the next `count`
 * fail as if the device were out of memory; after < 0 or count <= 0 turns
 * failures off. Not for production use. */
mpcd_status mpcd_debug_fail_allocs(int64_t after, int64_t count);

/* The MD side of the solute coupling (sec. 3.6; sec. 4.3 integrates its
 * bead-spring chains by velocity Verlet, 50 MD steps of 0.002 per collision):
 * nsteps velocity-Verlet steps of size dt for n_chains chains of chain_len
 * beads with harmonic bonds U = k_bond/2 (|r_{i+1} - r_i| - bond_length)^2
 * between consecutive beads (minimum image in the periodic box of edge
 * lengths box[3]), no other forces. pos, vel: device arrays of
 * n_chains * chain_len x 3 doubles, bead i of chain c in row
 * c * chain_len + i, positions in [0, box) (kept there: wrapped after each
 * drift); mass: n_chains * chain_len doubles (> 0). Updated in place,
 * enqueued on hip_stream (NULL: the null stream), not waited for: the
 * caller's mpcd_set_embedded on the same stream, or a synchronisation,
 * orders it before the handover. One block per chain, one thread per bead.
 * MPCD_EINVAL for chain_len outside 1..1024, negative counts, box lengths
 * <= 0 or dt < 0. */
mpcd_status mpcd_md_verlet_chains(double* pos, double* vel, const double* mass, int64_t n_chains,
                                  int32_t chain_len, const double box[3], double k_bond,
                                  double bond_length, double dt, int32_t nsteps, void* hip_stream);

/* Tile shape (the cells a block of the step kernel collides together and
 * whose particles share a slab), in bits 8-10 of flags: 0 chooses by the
 * box's mean density rho (a box alone, SRD rule: rho >= 12: 4x4x2 cells,
 * >= 7.5: 4x4x4, >= 3.75: 8x4x4, else 8x8x4, and so the FP32 form's AT rule;
 * the FP64 form's AT rule: >= 12: 4x4x2, >= 2.5: 4x4x4, else 8x8x4; a box of
 * a batch: >= 12: 4x4x2, >= 3.5: 4x4x4,
 * >= 1.75: 8x4x4, else 8x8x4); MPCD_TILE_4x4x2 .. MPCD_TILE_8x8x4 set it. Results do
 * not depend on it (only how fast they come). In a batch each box may set
 * its own; the other flags must match. Sec. 3.5 tunes the equivalent launch
 * parameters by timing; paper_1801_10187_amd.autotune does that here. */
#define MPCD_TILE_SHIFT 8
#define MPCD_TILE_MASK (7 << MPCD_TILE_SHIFT)
#define MPCD_TILE_4x4x2 (1 << MPCD_TILE_SHIFT)
#define MPCD_TILE_4x4x4 (2 << MPCD_TILE_SHIFT)
#define MPCD_TILE_8x4x4 (3 << MPCD_TILE_SHIFT)
#define MPCD_TILE_8x8x4 (4 << MPCD_TILE_SHIFT)

/* Create a context and upload the initial state (sec. 3.2 particle data).
 *  pos, vel      n_solvent x 3 doubles; positions inside [0, L) per axis.
 *  n_embedded    embedded (solute) particles that take part in collisions
 *                only and stream ballistically (sec. 2, sec. 3.6); 0 for none.
 *  emb_pos/vel   n_embedded x 3 doubles; emb_mass n_embedded doubles (> 0).
 *  pointers_on_device  0: all arrays are host memory; 1: device memory.
 *  hip_stream    hipStream_t to enqueue on, or NULL for a stream the context
 *                creates (default priority) and owns.
 * The step counter starts at 0. Errors: MPCD_EINVAL for bad parameters or a
 * position outside the box, MPCD_ENOMEM, MPCD_EHIP. On error *out is NULL. */
mpcd_status mpcd_create(const mpcd_params* params, int64_t n_solvent,
                        const double* pos, const double* vel,
                        int64_t n_embedded, const double* emb_pos,
                        const double* emb_vel, const double* emb_mass,
                        int32_t pointers_on_device, void* hip_stream,
                        mpcd_ctx* out);

/* Create a context of n_boxes independent boxes (a batch) that every entry
 * point below advances together, one kernel launch for all of them. Box b
 * has its own parameters params[b] (cells, cell size, angle, dt, kT, seed,
 * solvent mass) and n_particles[b] solvent particles, rows
 * [first_b, first_b + n_particles[b]) of the row-major pos/vel arrays
 * (first_b = the sum of the earlier counts). precision, thermostat,
 * grid_shift and flags must be the same in every params[b]. No embedded
 * particles. Tags run over the boxes in order (box b's particle i has tag
 * first_b + i); per-cell outputs (counts, cell properties, draws) are the
 * boxes' cell arrays one after the other, and cell_of_tag holds the cell
 * index inside the particle's box. mpcd_create is the batch of one box.
 * Errors as mpcd_create; the text names the first bad box. */
mpcd_status mpcd_create_batch(int32_t n_boxes, const mpcd_params* params,
                              const int64_t* n_particles, const double* pos,
                              const double* vel, int32_t pointers_on_device,
                              void* hip_stream, mpcd_ctx* out);

/* Number of boxes of a context (1 for mpcd_create). */
mpcd_status mpcd_get_n_boxes(mpcd_ctx ctx, int32_t* n_boxes);

/* Where box `box` lives in the batch: its first tag and particle count, its
 * first cell in per-cell outputs and cell count, and (if shift_of_step is
 * not NULL) its grid shift for step counter `step`. Any pointer may be NULL.
 * MPCD_EINVAL for a box out of range. */
mpcd_status mpcd_get_box(mpcd_ctx ctx, int32_t box, int64_t* first_tag,
                         int64_t* n_particles, int64_t* first_cell,
                         int64_t* n_cells, double shift_of_step[3],
                         uint64_t step);

/* Streaming (eq. 1): r <- r + v dt, wrapped into the box. Needs the state
 * after create or after a collide. */
mpcd_status mpcd_stream(mpcd_ctx ctx);

/* Binning (sec. 3.4): draw the grid shift of the current step counter n and
 * group the particles by the tile of their collision cell on the shifted
 * grid (tiles are blocks of 4x4x4 to 8x8x4 cells, each owning a fixed-size
 * slab of particle slots). Needs a preceding mpcd_stream. Waits for the
 * device at its end: if a tile's slab overflowed, the slabs are enlarged and
 * the binning redone before returning. */
mpcd_status mpcd_bin(mpcd_ctx ctx);

/* Collision (sec. 3.5, 3.6, eq. 2, Alg. 1): cell sums, per-cell axis and
 * thermostat factor drawn from counter n, rotation. Increments the step
 * counter. Needs a preceding mpcd_bin. */
mpcd_status mpcd_collide(mpcd_ctx ctx);

/* nsteps whole steps (stream, bin, collide), equivalent to calling the three
 * entry points nsteps times: one launch per step, each step's collision
 * fused with the next step's stream and binning. nsteps >= 0. Waits for the
 * device at its end (see mpcd_bin about slab overflow).
 * The last launch leaves the next step's stream and binning prepared (the
 * collided velocities, streamed and binned) beside the collided positions,
 * so that the next mpcd_step starts with its collision; every get_* reads the
 * collided state, joining the two copies where needed.
 * mpcd_stream, mpcd_set_embedded (except for the solutes of
 * MPCD_FLAG_MD_SOLUTE, which it moves into the prepared binning) and a
 * changed step counter give the prepared binning up (the next mpcd_step
 * then streams and bins first), as does a slab overflow in that launch.
 * Results never depend on how a run is split into calls.
 * If a slab overflows and cannot be enlarged (MPCD_ENOMEM), the context is
 * rolled back to the input of the launch that overflowed: the state before
 * the call, or step s streamed and binned but not yet collided (then
 * mpcd_get_step returns s and mpcd_collide completes it); the error text
 * says which. */
mpcd_status mpcd_step(mpcd_ctx ctx, int64_t nsteps);

/* For callers that cannot allocate (tight serving loops, harnesses that
 * forbid device allocation): mpcd_step without any allocation, the same
 * steps bit for bit. Differences from mpcd_step:
 *  - (nsteps + 1) * n_boxes must not exceed MPCD_NOALLOC_MAX_SHIFTS, else
 *    MPCD_EINVAL and nothing runs;
 *  - the grid shifts of the call are staged in a table of the library (one
 *    per GPU, MPCD_NOALLOC_MAX_SHIFTS entries of 40 bytes = 320 KiB, held
 *    until the process ends) instead of the context's own: calls on one GPU
 *    whose work overlaps (contexts on different streams or host threads)
 *    race on it and must be serialised by the caller;
 *  - kernel timing (mpcd_profile_enable) records nothing during the call;
 *  - a full particle slab cannot be enlarged: the call returns MPCD_ENOMEM
 *    with the context rolled back to the input of the launch that
 *    overflowed -- the state before the call, or step s streamed and binned
 *    but not yet collided (mpcd_get_step returns s; mpcd_collide completes
 *    it, after which mpcd_step, which enlarges slabs, can continue).
 * Synchronises at its end, as mpcd_step does. */
#define MPCD_NOALLOC_MAX_SHIFTS 8192
mpcd_status mpcd_step_noalloc(mpcd_ctx ctx, int64_t nsteps);

/* State of the embedded particles only (tags n_solvent .. n_total - 1, box 0):
 * pos, vel are n_embedded x 3 doubles, row i = embedded particle i as given to
 * mpcd_create. get: any state; synchronises. set: only between steps (after
 * create or a collide, else MPCD_ESTATE); positions must lie in [0, L)
 * (else MPCD_EINVAL, and nothing is guaranteed about which rows were taken);
 * the values are stored in the context's precision. The exchange with an
 * MD integrator (MPCD_FLAG_MD_SOLUTE; sec. 3.6). The context keeps the slot
 * of every embedded particle, so both calls cost O(n_embedded) work on the
 * device (a thread per particle), whatever the number of solvent particles.
 * With MPCD_FLAG_MD_SOLUTE and the next step's binning prepared (after
 * mpcd_step), set moves each solute into that binning at the cell its new
 * position falls in under the next step's grid shift: a solute that stays in
 * its tile is updated in place, one that changes tile leaves its old tile's
 * slab (the slab's last particles fill the gap) and takes a slot at the end
 * of its new tile's slab; the solvent's binning is kept, so the next
 * mpcd_step starts with its collision. If a destination slab is full, the
 * prepared binning is given up instead and the next step streams and bins
 * everything (results are the same). Otherwise the next binning moves each
 * particle to the tile of its new position. With device pointers and the
 * handover's small index arrays allocated (on its first use) they allocate
 * nothing. */
mpcd_status mpcd_get_embedded(mpcd_ctx ctx, double* pos, double* vel,
                              int32_t pointers_on_device);
mpcd_status mpcd_set_embedded(mpcd_ctx ctx, const double* pos, const double* vel,
                              int32_t pointers_on_device);

/* Solute handovers (mpcd_set_embedded with MPCD_FLAG_MD_SOLUTE) that kept
 * the prepared binning, and those that gave it up because a destination
 * slab was full. Either pointer may be NULL. */
mpcd_status mpcd_handover_stats(mpcd_ctx ctx, int64_t* kept, int64_t* given_up);

/* Copy the state out in tag order: pos, vel are n_total x 3 doubles, where
 * n_total = n_solvent + n_embedded. Synchronises the context's stream. */
mpcd_status mpcd_get_state(mpcd_ctx ctx, double* pos, double* vel,
                           int32_t pointers_on_device);

/* Cells of the most recent mpcd_bin (or binning inside mpcd_step):
 * cell_of_tag[n_total] the x-fastest cell index ix + nx*(iy + ny*iz) on the
 * shifted grid (inside the particle's box), counts[n_cells] the occupancy
 * (n_cells: all boxes). Either pointer may be NULL.
 * MPCD_ESTATE if nothing has been binned yet. Synchronises. */
mpcd_status mpcd_get_cells(mpcd_ctx ctx, int32_t* cell_of_tag, int32_t* counts,
                           int32_t pointers_on_device);

/* Cell properties (sec. 3.5) of the binned, not yet collided state:
 * mass[n_cells], momentum[n_cells x 3], ek[n_cells] (eq. 3, relative to the
 * centre-of-mass velocity). Only valid between mpcd_bin and mpcd_collide
 * (else MPCD_ESTATE). Any pointer may be NULL. Synchronises. */
mpcd_status mpcd_get_cell_props(mpcd_ctx ctx, double* mass, double* momentum,
                                double* ek, int32_t pointers_on_device);

/* Per-cell random draws of the binned state for the current step counter
 * (SRD rule only; MPCD_EINVAL under the AT rule, which draws per particle):
 * axis[n_cells x 3] (sec. 3.6, cylindrical projection) and xi[n_cells]
 * (thermostat scale; 1 when the thermostat is off or N_c < 2). Cells with no
 * particle get axis (0, 0, 0) and xi 1. Only valid between mpcd_bin and
 * mpcd_collide. Either pointer may be NULL. Synchronises. */
mpcd_status mpcd_get_cell_draws(mpcd_ctx ctx, double* axis, double* xi,
                                int32_t pointers_on_device);

/* Cell-averaged velocity field of the current state on the unshifted grid
 * (each particle in its home cell floor(r / a)): u[n_cells x 3] the
 * mass-weighted mean velocity sum(m v) / sum(m) of the cell's particles (0
 * for an empty cell, sec. 3.5 cell properties), mass[n_cells] the cell's
 * mass. n_cells covers all boxes, one after the other. The sums are exact
 * (fixed point), so the result does not depend on the particles' order.
 * Either pointer may be NULL. Any state. Synchronises. */
mpcd_status mpcd_get_velocity_field(mpcd_ctx ctx, double* u, double* mass,
                                    int32_t pointers_on_device);

/* Grid shift drawn for step counter n, s[3] in (-a/2, a/2) (zero when the
 * shift is off), of box 0 (mpcd_get_box gives any box's). Host-only
 * computation; any state. */
mpcd_status mpcd_get_shift(mpcd_ctx ctx, uint64_t n, double s[3]);

/* Step counter: read, or set (to resume from a checkpoint; only in the
 * state after create or after a collide). */
mpcd_status mpcd_get_step(mpcd_ctx ctx, uint64_t* n);
mpcd_status mpcd_set_step(mpcd_ctx ctx, uint64_t n);

/* Net properties (sec. 3.5): total momentum p[3], kinetic energy ke and the
 * kinetic temperature of the motion relative to the centre of mass,
 * 2 (ke - |p|^2 / 2M) / (3 (n_total - 1)), over all boxes. Synchronises. */
mpcd_status mpcd_totals(mpcd_ctx ctx, double p[3], double* ke, double* kT);

/* The same per box: p[3 * n_boxes], ke[n_boxes], kT[n_boxes] (any may be
 * NULL). Synchronises. */
mpcd_status mpcd_box_totals(mpcd_ctx ctx, double* p, double* ke, double* kT);

/* Wait for the context's work and report kernel range errors. */
mpcd_status mpcd_sync(mpcd_ctx ctx);

/* Counts and sizes: n_total particles, n_cells cells. */
mpcd_status mpcd_get_sizes(mpcd_ctx ctx, int64_t* n_total, int64_t* n_cells);

/* Particle storage layout: tile size in cells, number of tiles, slots per
 * tile slab, and how many times the slabs were enlarged. Any pointer may be
 * NULL. */
mpcd_status mpcd_get_layout(mpcd_ctx ctx, int32_t tile[3], int64_t* n_tiles,
                            int64_t* capacity, int64_t* regrows);

/* Device memory a context of one box with these parameters and
 * n_particles solvent particles would take from the stream-ordered memory
 * pool its allocations come from, for a run of nsteps-step calls:
 * peak_bytes the most it holds at any moment (the upload buffer of
 * mpcd_create, 48 bytes per particle when host_arrays is 1; the grid-shift
 * table of a stepping call; the temporaries of mpcd_get_velocity_field or
 * mpcd_get_state), held_bytes what it keeps between calls. An estimate for
 * particles spread like a uniform fluid: mpcd_create sizes the slabs from
 * the fullest tile of the actual input, taken here as a whole tile's mean
 * occupancy plus five standard deviations (Poisson); a very uneven input, and an
 * enlargement of the slabs during a step (old and new slabs held at once),
 * need more. Either pointer may be NULL. Host-only computation. */
mpcd_status mpcd_footprint(const mpcd_params* params, int64_t n_particles, int64_t nsteps,
                           int32_t host_arrays, int64_t* peak_bytes, int64_t* held_bytes);

/* Launch mode of the stepping calls (mpcd_step, mpcd_bin; sec. 3.5 names
 * launch parameters as a tuning choice). on = 1: the tile-kernel launches
 * of each call are captured into a HIP graph on the context's stream and
 * the graph is launched; the context keeps the executable graph and updates
 * it in place from the next call's capture (new step numbers and buffers)
 * when the capture has the same shape, else instantiates a new one. on = 0
 * (the default): one stream launch per kernel. Results are the same bit for
 * bit. While kernel timing (mpcd_profile_enable) is on, calls launch on the
 * stream. MPCD_EINVAL for on other than 0 or 1, or for on = 1 with a context
 * created on the null or per-thread stream (which cannot be captured). */
mpcd_status mpcd_set_graph(mpcd_ctx ctx, int32_t on);

/* Executable graphs instantiated and updated in place by the context's
 * graph launches so far. Either pointer may be NULL. */
mpcd_status mpcd_graph_stats(mpcd_ctx ctx, int64_t* instantiations, int64_t* updates);

/* Kernel timing with HIP events on the context's stream. which: 0 the
 * collision kernel (collide with its per-cell draws, stream and bin of the
 * next step), 1 the stream / stream+bin kernels; MPCD_EINVAL for any other
 * value. on = 0 disables; on = P >= 1 brackets the first launch of each
 * kind and then one in every P with two events (P = 1: every launch; each
 * bracketed launch costs a few microseconds of stream time, so a larger P
 * disturbs a timed run less). mpcd_profile_read synchronises, returns the
 * summed milliseconds and the number of bracketed launches since the last
 * read, and clears them. MPCD_EINVAL for on < 0. */
mpcd_status mpcd_profile_enable(mpcd_ctx ctx, int32_t on);
mpcd_status mpcd_profile_read(mpcd_ctx ctx, int32_t which, double* total_ms,
                              int64_t* launches);

void mpcd_destroy(mpcd_ctx ctx);

/* Thread-local text of the last failure in this thread ("" if none). */
const char* mpcd_last_error(void);

/* ---- building blocks exposed for tests and measurement ---------------- */

/* Philox4x32-10 (Salmon et al., SC'11; the counter-based generator family
 * of sec. 3.6) evaluated on the GPU: ctr is n x 4 uint32 counters, key the
 * 64-bit key (low word k0, high word k1), out n x 4 uint32. Host pointers.
 * Synchronous. */
mpcd_status mpcd_philox4x32_10(const uint32_t* ctr, int64_t n, uint64_t key,
                               uint32_t* out);

/* Plain device-to-device copy of `bytes` bytes with the library's streaming
 * kernel; used to measure the achievable HBM bandwidth and to calibrate
 * hardware byte counters. Device pointers; hip_stream may be NULL.
 * Asynchronous on the stream. */
mpcd_status mpcd_copy_kernel(const void* src, void* dst, int64_t bytes,
                             void* hip_stream);

/* The same copy with four 16-byte vectors per thread and iteration, all
 * loaded before any is stored; a second estimate of the achievable HBM
 * bandwidth. Same arguments and behaviour as mpcd_copy_kernel. */
mpcd_status mpcd_copy_kernel_unrolled(const void* src, void* dst, int64_t bytes,
                                      void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MPCD_H */
