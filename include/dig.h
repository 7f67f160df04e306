/*
 * dig.h -- C ABI of the MI355X (gfx950) DSMC + DIG hot-path library (libdig).
 *
 * Method: "Multiscale simulation of rarefied polyatomic gas flow via DIG
 * method" (Luo, Huang, Li, Wu; arXiv:2501.10965).  The library advances
 * simulation particles of a polyatomic gas (velocity v, rotational energy)
 * with the DSMC scheme of Section 2.2 and applies the DIG particle
 * modification of Section 3.2; the algorithm loop is the four-step DIG
 * iteration of Section 3 (initialise from a macroscopic field, N_s DSMC
 * steps with time averaging, synthetic solve, particle modification).
 *
 * Units (Section 2): lengths in L0, density in rho0, temperature in T0,
 * speed in sqrt(R T0); molecular mass 1.  Kn = mu(T0)/(p0 L0) sqrt(pi R T0/2),
 * so mu(T) = Kn sqrt(2/pi) T^omega.
 *
 * Conventions for every entry point:
 *  - Pointers named *_dev are device pointers (HBM) owned by the caller;
 *    pointers named *_host are host pointers.  The library never frees caller
 *    memory and allocates no device memory after dsmc_create returns, except
 *    synth_solve's host-side scratch.
 *  - Every call that takes a dig_stream_t enqueues its work on that HIP stream
 *    (NULL = the default stream) and returns without waiting, unless its
 *    comment says it synchronises.
 *  - Return value: DIG_OK or an error code; dig_last_error() returns a
 *    thread-local message for the last failure.  No entry point aborts or
 *    throws.  Invalid arguments are rejected before any device work.
 *  - Array layouts: "field-major [F][C]" means element (f, c) at f*C + c,
 *    C = total cell count of the context (cells of all instances,
 *    instance after instance, x fastest then y).
 */
#ifndef DIG_H
#define DIG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dig_ctx dig_ctx;
typedef void* dig_stream_t; /* a hipStream_t */

typedef enum {
  DIG_OK = 0,
  DIG_ERR_INVALID = 1,  /* bad argument or configuration */
  DIG_ERR_CAPACITY = 2, /* particle capacity would overflow */
  DIG_ERR_HIP = 3,      /* a HIP runtime call failed */
  DIG_ERR_STATE = 4,    /* call not valid in the context's current state */
  DIG_ERR_NUMERIC = 5   /* non-finite or non-positive target values */
} dig_status;

/* Boundary condition of one domain face.  FREESTREAM (annulus outer circle
 * only): particles that leave are removed and the gas of a reservoir shell
 * outside the circle (density rho, temperature T, velocity U) enters each
 * step. */
enum { DIG_BC_PERIODIC = 0, DIG_BC_DIFFUSE = 1, DIG_BC_SPECULAR = 2, DIG_BC_FREESTREAM = 3 };
typedef struct {
  int32_t type; /* DIG_BC_* ; both faces of an axis periodic or neither */
  double T;     /* wall / freestream temperature */
  double U[3];  /* wall velocity (its normal component must be 0) / freestream velocity */
  double rho;   /* freestream density */
} dig_bc;

/* Geometry of an instance.  BOX: uniform Cartesian cells, positions held in
 * grid units.  ANNULUS (dim 2, one instance per context): the region
 * r_in <= r <= r_out around the origin, nx cells in the angle (face i at
 * 2 pi i / nx) and ny cells in the radius with faces
 * r_j = r_in + (r_out - r_in) (q^j - 1) / (q^ny - 1) (q = 1: uniform);
 * cell (i, j) has index i + nx j; positions in physical units.  Faces:
 * bc[0] the inner circle (DIFFUSE or SPECULAR), bc[1] the outer circle
 * (DIFFUSE, SPECULAR or FREESTREAM); bc[2], bc[3] unused.  GRADED (dim 1
 * or 2): a box whose cells have different widths, the wall-refined grids of
 * the DIG runs of Section 4.1 (Table 1): cell (i, j) spans
 * [xfaces[i], xfaces[i+1]] x [yfaces[j], yfaces[j+1]]; the face tables are
 * strictly increasing from 0 to lx (ly); positions in physical units; faces
 * and walls as for BOX. */
enum { DIG_GEOM_BOX = 0, DIG_GEOM_ANNULUS = 1, DIG_GEOM_GRADED = 2 };

/* One simulation instance (Section 4 gas: VSS/VHS omega 0.74, alpha 1,
 * d_r = 2, constant Z; d_r up to 6 and alpha up to 2 are accepted).  Faces are
 * ordered x-, x+, y-, y+. */
typedef struct {
  int32_t dim;          /* 1 (slab, positions x) or 2 (positions x, y) */
  int32_t nx, ny;       /* cells per axis; ny = 1 when dim = 1 */
  double lx, ly;        /* box: domain lengths; cell volume (lx/nx)(ly/ny), 2D, or lx/nx, 1D */
  int32_t geometry;     /* DIG_GEOM_* */
  double r_in, r_out, q;  /* annulus radii and radial stretch ratio (q >= 1) */
  double kn;            /* Knudsen number (Section 2) */
  double omega, alpha;  /* viscosity index in [0.5, 1]; scattering alpha in [1, 2]
                          (1: VHS, isotropic; otherwise VSS) */
  int32_t dr;           /* rotational degrees of freedom, 2..6 (Borgnakke-Larsen with
                          Beta(d_r/2, 5/2 - omega) fractions, Gamma(d_r/2) energies) */
  double zrot;          /* rotational collision number Z; P_inelastic <= 1 */
  double dt, weight;    /* time step; particle weight N_eff (mass per particle) */
  dig_bc bc[4];
  uint64_t seed;        /* Philox key */
  uint32_t instance_id; /* Philox counter word 2, low 24 bits */
  double sgmax_init;    /* initial majorant of sigma_T g; <= 0: default below */
  double tref;          /* default majorant = C (6 sqrt(2 tref))^(2 - 2 omega) */
  const double* xfaces; /* GRADED: host array of nx + 1 face coordinates, 0 .. lx; read
                          during the call that takes the config (copied by
                          dsmc_create), not kept; NULL otherwise */
  const double* yfaces; /* GRADED, dim 2: ny + 1 face coordinates, 0 .. ly */
} dig_config;

/* Byte offsets of the device arrays inside the caller's workspace.  Particle
 * arrays hold `capacity` elements, cell arrays `ncell`.  Buffer `cur`
 * (returned by dsmc_query) holds the current, cell-sorted particle state.
 * total_bytes also covers the library's own scratch after these arrays (cell
 * group and scan tables, geometry tables, and one 16-byte record per
 * particle in which cell groups too large for on-chip memory collide). */
typedef struct {
  size_t total_bytes;
  int64_t capacity, ncell;
  size_t x[2], y[2], vx[2], vy[2], vz[2], er[2], id[2]; /* f32 (x, y: grid units on a uniform
                                                           box, physical units on a graded box
                                                           or the annulus), u32 id */
  size_t cell, rank, perm_raw, perm;                    /* i32 per particle */
  size_t start;      /* i32 [ncell + 1]: first particle of each cell */
  size_t count;      /* i32 [ncell] */
  size_t sgmax;      /* f32 [ncell]: majorant of sigma_T g */
  size_t acc;        /* f64 [ncell][17]: time-accumulated raw sums */
  size_t sums;       /* f64 [ncell][17]: scratch for instantaneous sums */
  size_t cell_inst;  /* i32 [ncell]: instance of each cell */
  size_t cvol;       /* f64 [ncell]: cell volume (area in 2D, length in 1D) */
  size_t counters;   /* dig_counters */
} dig_layout;

/* Device-side counters (read with dsmc_query). */
typedef struct {
  int64_t n;          /* particles in the current buffer */
  int64_t step;       /* DSMC steps taken (Philox step counter) */
  int64_t nsamp;      /* steps accumulated into acc since the last reset */
  int64_t next_id;    /* next particle id handed out by dig_adjust */
  int64_t candidates, accepted, inelastic, saturated, wall_hits;
  int64_t removed, injected;  /* open boundaries: particles that left / entered */
  uint32_t err;       /* DIG_EBIT_* */
  uint32_t cur;       /* current particle buffer (0 or 1) */
} dig_counters;

enum {
  DIG_EBIT_SORT_OVERFLOW = 1u, /* a cell group exceeded the run table (slow path used) */
  DIG_EBIT_GROUPS = 2u,        /* more cell groups than launched: state invalid */
  DIG_EBIT_TARGET = 4u,        /* dig_adjust target non-finite or non-positive */
  DIG_EBIT_CAPACITY = 8u,      /* dig_adjust or inflow would exceed the capacity */
  DIG_EBIT_INFLOW = 16u        /* a step's inflow would have exceeded the capacity: none of
                                  that step's inflow entered (the rest of the step ran) */
};

/* Workspace planning.  cfgs[n_inst] describe the instances advanced
 * together (batching; all must share dim).  capacity = particle capacity of
 * the whole batch.  Fills *out; no device work.  Errors: DIG_ERR_INVALID. */
dig_status dig_plan(const dig_config* cfgs_host, int32_t n_inst, int64_t capacity,
                    dig_layout* out_host);

/* Creates a context over a caller-owned device workspace of at least
 * layout.total_bytes bytes (256-byte aligned).  Zeroes counters, counts and
 * accumulators and sets every cell's majorant; enqueued on `stream`.
 * group_particles / group_cells: cell-group size used by the sort and collide
 * kernels (0 = defaults 1024 / 64; ranges [256, 16384] / [32, 256]); results
 * do not depend on them.  Errors: DIG_ERR_INVALID, DIG_ERR_HIP. */
dig_status dsmc_create(const dig_config* cfgs_host, int32_t n_inst, int64_t capacity,
                       void* workspace_dev, size_t workspace_bytes, int32_t group_particles,
                       int32_t group_cells, dig_stream_t stream, dig_ctx** out);

/* Initialisation, DIG step 1 (Section 3): particles from the local
 * equilibrium of fields_dev = field-major [6][C] (rho, ux, uy, uz, Tt, Tr).
 * ppc > 0: exactly ppc particles per cell; ppc = 0: Iround(rho V / N_eff).
 * Velocities Maxwellian (Box-Muller), rotational energy exponential with mean
 * Tr (d_r = 2), positions uniform in the cell.  Synchronises once to read the
 * particle count.  Errors: DIG_ERR_INVALID, DIG_ERR_CAPACITY (state untouched). */
dig_status dsmc_init(dig_ctx* ctx, const double* fields_dev, int32_t ppc, dig_stream_t stream);

/* State injection: the caller has written a cell-sorted state of n particles
 * into buffer `cur` and the matching start array (i32 [C+1]).  Sets the
 * particle count, the step counter and the next id; enqueued. */
dig_status dsmc_inject(dig_ctx* ctx, int64_t n, int64_t step, int64_t next_id,
                       dig_stream_t stream);

/* One DSMC step = move (free flight, walls) + cell index + stable counting
 * sort + collide (NTC, VHS, Borgnakke-Larsen) + accumulate raw sums, Section
 * 2.2.  dsmc_step runs nsteps of them; dsmc_stage runs the selected stages of
 * one step (DIG_STAGE_* mask, in order), for inspection.  Capture-safe. */
enum { DIG_STAGE_MOVE = 1, DIG_STAGE_SORT = 2, DIG_STAGE_COLLIDE = 4, DIG_STAGE_ALL = 7 };
dig_status dsmc_step(dig_ctx* ctx, int32_t nsteps, dig_stream_t stream);
dig_status dsmc_stage(dig_ctx* ctx, int32_t stage_mask, dig_stream_t stream);

/* Moment sampling, equation DSMC_macroscopic.  out_dev = field-major [20][C]:
 * rho, ux, uy, uz, Tt, Tr, sigma xx yy zz xy xz yz, q_t xyz, q_r xyz, T,
 * mean particle count.  Rotational energy is stored per unit mass, so
 * Tr = 2<er>/d_r and q_r = rho <c er>.  Modes: INSTANT (current state),
 * AVERAGE (raw sums pooled over the steps since the last RESET), RESET (zero
 * the accumulator; out_dev may be NULL).  Empty cells give all-zero fields. */
enum { DIG_SAMPLE_INSTANT = 0, DIG_SAMPLE_AVERAGE = 1, DIG_SAMPLE_RESET = 2 };
dig_status dsmc_sample(dig_ctx* ctx, int32_t mode, double* out_dev, dig_stream_t stream);

/* DIG particle modification, Section 3.2, single-instance contexts only.
 * target_dev = field-major [6][C] (rho, ux, uy, uz, Tt, Tr).  Per cell: target
 * count Iround(rho V / N_eff); random deletion (partial Fisher-Yates) or
 * clones of random existing particles at uniform positions (empty cells draw
 * from the target equilibrium); then v <- a v + b, er <- c er so that u, Tt,
 * Tr equal the target.  FP64 arithmetic, FP32 storage.  Synchronises once.
 * Errors: DIG_ERR_NUMERIC (bad target), DIG_ERR_CAPACITY; on error the
 * particle state is unchanged. */
dig_status dig_adjust(dig_ctx* ctx, const double* target_dev, uint32_t dig_iter,
                      dig_stream_t stream);

/* Closure assembly, Sections 2.3 and 3.1, single-instance contexts only.
 * fields_dev = [20][C] from dsmc_sample.  A_host = relaxation matrix
 * (Att, Atr, Art, Arr) of equation kappa_A.  Outputs: hot_dev [12][C]
 * (sigma xx yy zz xy xz yz, q_t xyz, q_r xyz) = DSMC - NSF, zeroed where
 * Kn_GLL < kn_ref or where the cell's mean particle count (row 19 of
 * fields_dev) is below n_min (terms extracted from so few samples are
 * sampling noise; n_min = 0 switches this off); mask_dev [C] (1 = equilibrium,
 * HoT zeroed); kngll_dev [C]; nsf_dev [12][C] or NULL.  Gradients: the
 * neighbours' difference over the distance between their centres, one-sided
 * at walls.  Errors: DIG_ERR_INVALID (null pointer, singular A, n_min < 0). */
dig_status closure_assemble(dig_ctx* ctx, const double* fields_dev, const double* A_host,
                            double kn_ref, double n_min, double* hot_dev, uint8_t* mask_dev,
                            double* kngll_dev, double* nsf_dev, dig_stream_t stream);

/* Synthetic-equation solve, DIG step 3 (Section 3): the steady equations of
 * mass, momentum, total energy and rotational energy (equation
 * macroscopic_equation) closed by NSF terms plus the higher-order terms hot_dev
 * ([12][C] as produced by closure_assemble; NULL = NSF only) zeroed where
 * mask_dev [C] is nonzero (NULL = no mask).  m_half_dev = the DSMC time
 * average [>=6][C] (rho, ux, uy, uz, Tt, Tr first), also the initial guess;
 * m_next_dev [6][C] receives the solution.  Finite volumes on the uniform grid
 * of cfg (single instance), HLLC inviscid fluxes, central viscous and heat
 * fluxes, Dirichlet walls (wall_mode 0: the config's wall temperature and
 * velocity; 1: slip and jump taken from the DSMC field's wall-adjacent cells),
 * and pseudo-time steps toward the steady state, either explicit steps
 * common to all cells (DIG_SYNTH_EXPLICIT: total mass conserved exactly) or
 * implicit LU-SGS steps (DIG_SYNTH_LUSGS, the scheme named in Section 4:
 * matrix-free, with viscous spectral radii in the diagonal and a
 * point-implicit rotational source; cells in two colours, (ix + iy) even
 * first, so that each sweep is two parallel passes; the state scaled to the
 * initial total mass after every step; a periodic axis needs an even cell
 * count).  Both reach the same steady discrete solution.
 * Stops after max_iter steps or when the largest relative change of
 * (rho, u, Tt, Tr) in one step falls below tol (checked every check_every
 * steps, default 32; synchronises at each check).  workspace_dev: at least
 * dig_synth_workspace_bytes(cfg) bytes, 256-byte aligned, caller-owned.
 * Errors: DIG_ERR_INVALID (bad arguments), DIG_ERR_NUMERIC (non-finite state). */
enum { DIG_SYNTH_EXPLICIT = 0, DIG_SYNTH_LUSGS = 1 };
typedef struct {
  double A[4];           /* heat-flux relaxation matrix Att, Atr, Art, Arr */
  double cfl;            /* pseudo-time step factor (explicit: stability below 1;
                            LU-SGS: local time step of cfl times the explicit bound) */
  int32_t wall_mode;     /* 0 wall values, 1 DSMC slip / jump */
  int32_t check_every;   /* convergence check period (0 = 32) */
  int32_t scheme;        /* DIG_SYNTH_EXPLICIT or DIG_SYNTH_LUSGS */
  int32_t reserved;      /* 0 */
} dig_synth_opts;
size_t dig_synth_workspace_bytes(const dig_config* cfg_host);
dig_status synth_solve(const dig_config* cfg_host, const dig_synth_opts* opts_host,
                       const double* m_half_dev, const double* hot_dev, const uint8_t* mask_dev,
                       double* m_next_dev, void* workspace_dev, size_t workspace_bytes,
                       int32_t max_iter, double tol, int32_t* iters_host, double* change_host,
                       dig_stream_t stream);

/* synth_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same solve, with its scratch in a static device array of
 * DIG_SYNTH_STATIC_BYTES (32 MiB) that the library holds on each GPU it runs
 * on until the process ends, instead of a caller workspace.  The caller still
 * passes the inputs and m_next_dev.  Calls no allocation routine.  Grids
 * whose dig_synth_workspace_bytes exceed DIG_SYNTH_STATIC_BYTES (about
 * 70,000 cells) give DIG_ERR_INVALID.  Every call on one GPU shares that
 * GPU's array, which keeps the last call's contents (each call initialises
 * what it reads): calls that overlap in time on one GPU (other host threads,
 * other streams) race and must be serialised by the caller. */
#define DIG_SYNTH_STATIC_BYTES (32u << 20)
dig_status synth_solve_static(const dig_config* cfg_host, const dig_synth_opts* opts_host,
                              const double* m_half_dev, const double* hot_dev,
                              const uint8_t* mask_dev, double* m_next_dev, int32_t max_iter,
                              double tol, int32_t* iters_host, double* change_host,
                              dig_stream_t stream);

/* Checkpoint and resume (restart of a long run).  dsmc_save writes an image
 * of the state that later steps read: the current cell-sorted particles
 * (positions, velocities, rotational energies, ids), the cell start table,
 * every cell's majorant, the time-average accumulator, the counters (particle
 * count, step, samples, next id, statistics, error bits), the tuning, and a
 * fingerprint of the instance parameters; a hash over the whole image closes
 * it.  host_buf = NULL: *bytes receives the size needed and nothing is
 * written; otherwise host_buf must hold *bytes >= that size (else
 * DIG_ERR_INVALID, *bytes = size needed) and *bytes receives the size
 * written.  Synchronises `stream`.  Errors: DIG_ERR_STATE (no state, or a
 * partial step pending), DIG_ERR_HIP.
 *
 * dsmc_load replaces the state of a context created with the same
 * configuration (any capacity that holds the saved particles) by the image
 * of `bytes` bytes at host_buf.  Stepping on from a loaded image gives the
 * same results, bit for bit, as stepping on from the saved state.  The image
 * is checked before any device work: wrong magic or version, another
 * configuration, a truncated or corrupted image, or a particle state that
 * does not match its cells give DIG_ERR_INVALID (more particles than the
 * capacity: DIG_ERR_CAPACITY), and the context's state is left unchanged.
 * Captured step graphs are dropped.  Synchronises `stream` (the copies read
 * host_buf). */
dig_status dsmc_save(dig_ctx* ctx, void* host_buf, size_t* bytes, dig_stream_t stream);
dig_status dsmc_load(dig_ctx* ctx, const void* host_buf, size_t bytes, dig_stream_t stream);

/* Synchronises and copies the device counters into *out. */
dig_status dsmc_query(dig_ctx* ctx, dig_counters* out_host, dig_stream_t stream);

/* Gas constants of instance `inst` as the library computes them:
 * out[0] = C (sigma_T g = C g^(2-2 omega)), out[1] = P_inelastic,
 * out[2] = mu0, out[3] = cell volume, out[4] = default majorant. */
dig_status dig_constants(dig_ctx* ctx, int32_t inst, double* out_host5);

/* Per-kernel timing with HIP events recorded on `stream` immediately before
 * and after every launch of the step and adjust kernels.  mode 1: enable and
 * reset; mode 0: disable; mode 2: synchronise and read the totals into
 * ms_host[DIG_NKERNELS] (milliseconds) and launches_host[DIG_NKERNELS].
 * Kinds: DIG_K_SCAN counts both scan kernels as one launch; DIG_K_ORDER is
 * the ordering pass of a sort stage run on its own (a full step orders each
 * cell group inside the collide); DIG_K_COLLIDE is the collide stage, the
 * small-group and the oversize-group kernels timed together as one launch. */
enum { DIG_K_MOVE = 0, DIG_K_SCAN = 1, DIG_K_PLACE = 2, DIG_K_ORDER = 3, DIG_K_COLLIDE = 4,
       DIG_K_ADJUST = 5, DIG_K_SAMPLE = 6, DIG_K_CLOSURE = 7, DIG_NKERNELS = 8 };
dig_status dsmc_profile(dig_ctx* ctx, int32_t mode, double* ms_host, int64_t* launches_host,
                        dig_stream_t stream);

/* Restricts dsmc_profile's events to the kernel kinds whose bit
 * (1u << DIG_K_*) is set in mask, and to one launch of each such kind in
 * every `every` (counted from dsmc_profile mode 1); other launches run without
 * events, so that timing perturbs the step as little as possible.  The
 * launches counts read by dsmc_profile are those timed.  The default (and
 * after dsmc_create) is every kind, every launch.  Host only; takes effect at
 * the next launch.  Errors: DIG_ERR_INVALID (bit beyond DIG_NKERNELS, every <
 * 1). */
dig_status dsmc_profile_kinds(dig_ctx* ctx, uint32_t mask, int32_t every);

/* Launch configuration of the step kernels.  group_particles / group_cells as
 * in dsmc_create; seq_max: cells with at most this many particles run their
 * collision candidates in order on one lane, larger cells in parallel rounds
 * (range [0, 4096]); big_stage_kib: LDS budget of the kernel that collides
 * the cell groups larger than the small-group stage (range [38, 150]; 38: four
 * workgroups per compute unit, groups above about 1280 particles collide in
 * HBM; larger budgets hold larger groups with fewer workgroups per unit).
 * Every choice gives bit-identical results; only the speed differs.
 * ms_per_step is filled by dsmc_autotune (0 otherwise). */
typedef struct {
  int32_t group_particles;
  int32_t group_cells;
  int32_t seq_max;
  int32_t big_stage_kib;
  double ms_per_step;
} dig_tuning;

/* Reads the current tuning into *out (if non-null), then applies *in (if
 * non-null).  Host only.  Errors: DIG_ERR_INVALID (range; nothing changed),
 * DIG_ERR_STATE (a partial step is pending). */
dig_status dsmc_tuning(dig_ctx* ctx, const dig_tuning* in_host, dig_tuning* out_host);

/* Autotuner for the step kernels: coordinate search over group_particles in
 * {512, 1024, 2048, 4096, 8192}, group_cells in {32, 64, 128, 256}, seq_max in
 * {0, 64, 128, 192, 384} and big_stage_kib in {38, 50, 76} (the last only for
 * contexts with open boundaries or at least 256 particles per cell on
 * average; two passes over the axes), timing steps_per_trial real steps per
 * candidate with HIP events on `stream` (one untimed step before each); each
 * candidate is compared with the best configuration timed again right after
 * it, so that a state that evolves during the search (a developing flow)
 * does not bias the choice toward the earlier trials.  The timed steps are
 * ordinary steps of the simulation: the state advances by every step taken,
 * exactly as dsmc_step would advance it, whichever configuration ran them.
 * cache_path (nullable): a text file of lines
 *   "<arch> <dim> <log2 particles> <log2 cells> <T> <Gc> <seq_max> <big_kib> <ms>";
 * a line matching this device and size class is applied without trials, and a
 * new choice is appended.  The choice is applied and copied into *out.
 * Synchronises.  Errors: DIG_ERR_STATE, DIG_ERR_HIP, DIG_ERR_INVALID. */
dig_status dsmc_autotune(dig_ctx* ctx, int32_t steps_per_trial, const char* cache_path,
                         dig_tuning* out_host, dig_stream_t stream);

/* nsteps DSMC steps as HIP graphs of at most 64 steps each, launched on
 * `stream`: the first use of a graph for a given (steps, buffer parity,
 * particle count rounded up to a 1/64 share of the capacity, tuning) captures
 * the step kernels on a stream of the library's own, later uses replay the
 * instantiated graph.  Results are identical to dsmc_step.  Not available
 * while dsmc_profile is enabled (per-kernel events need eager launches).
 * Errors: DIG_ERR_STATE, DIG_ERR_HIP. */
dig_status dsmc_step_graph(dig_ctx* ctx, int32_t nsteps, dig_stream_t stream);

/* ---- Learned closure network ------------------------------------------
 * A multilayer perceptron that predicts the higher-order constitutive terms
 * (the deviations of sigma and q from their NSF values, Section 3.1) from
 * local gradients and the local Knudsen number, in place of the noisy DSMC
 * extraction where the local Knudsen number lies in a band.  Four linear
 * layers: inputs 9 (padded to 32) -> 128 -> 128 -> 128 -> outputs 7 (padded
 * to 16), tanh on the hidden layers.  Products run on the matrix cores with
 * BF16 operands (inputs, weights, hidden activations and back-propagated
 * pre-activation gradients rounded to bfloat16, nearest even) and FP32
 * accumulation; master weights, biases and the Adam moments are FP32.
 *
 * Parameters live in the caller's workspace as one FP32 array of
 * DIG_MLP_NPARAM values: W0 [128][32], b0 [128], W1 [128][128], b1 [128],
 * W2 [128][128], b2 [128], W3 [16][128], b3 [16] (row-major [out][in]).
 * Padded entries (W0 columns 9..31, W3 rows 7..15, b3[7..15]) must be 0 and
 * stay 0 under training.  After writing parameters, call mlp_sync. */
enum { DIG_MLP_NPARAM = 39312, DIG_MLP_IN = 9, DIG_MLP_OUT = 7 };
typedef struct dig_mlp dig_mlp;
typedef struct {
  size_t total_bytes;
  int32_t max_batch;   /* training batch capacity (multiple of 64) */
  size_t params;       /* f32 [DIG_MLP_NPARAM] master parameters */
  size_t grads;        /* f32 [DIG_MLP_NPARAM] gradient of the last mlp_grad */
  size_t adam_m, adam_v;  /* f32 [DIG_MLP_NPARAM] Adam moments */
  size_t loss;         /* f32 [1]: loss of the last mlp_grad */
} dig_mlp_layout;

/* Workspace planning for a training batch of up to max_batch samples. */
dig_status mlp_plan(int32_t max_batch, dig_mlp_layout* out_host);

/* Creates a network over a caller-owned, 256-byte aligned device workspace
 * of at least layout.total_bytes; zeroes gradients and Adam moments (the
 * parameters are the caller's to write).  Enqueued.  Errors: INVALID, HIP. */
dig_status mlp_create(void* workspace_dev, size_t workspace_bytes, int32_t max_batch,
                      dig_stream_t stream, dig_mlp** out);

/* Refreshes the BF16 weight copies from the FP32 master parameters. */
dig_status mlp_sync(dig_mlp* mlp, dig_stream_t stream);

/* Inference: y_dev [n][7] = network(x_dev [n][9]), FP32 in and out, any n. */
dig_status mlp_forward(dig_mlp* mlp, const float* x_dev, float* y_dev, int64_t n,
                       dig_stream_t stream);

/* Loss (mean over n samples and 7 outputs of (y - t)^2, written to the
 * workspace's loss slot) and its gradient for every parameter (overwrites the
 * gradient array).  n <= max_batch.  Errors: INVALID. */
dig_status mlp_grad(dig_mlp* mlp, const float* x_dev, const float* t_dev, int64_t n,
                    dig_stream_t stream);

/* One Adam step (Kingma and Ba, with bias correction) at step number t >= 1
 * from the stored gradient, then the BF16 copies are refreshed. */
dig_status mlp_adam(dig_mlp* mlp, float lr, float beta1, float beta2, float eps, int64_t t,
                    dig_stream_t stream);

/* The result of mlp_grad followed by mlp_adam (beta1 0.9, beta2 0.999,
 * eps 1e-8), bit for bit: same loss, stored gradient, moments and parameters.
 * The loss, the gradient reduction and the update run as one launch.
 * Errors: INVALID (as mlp_grad, or t < 1 or lr < 0). */
dig_status mlp_train_step(dig_mlp* mlp, const float* x_dev, const float* t_dev, int64_t n,
                          float lr, int64_t t, dig_stream_t stream);

void mlp_destroy(dig_mlp* mlp);

/* Standardisation of the network's inputs and targets: z = (v - mean)/std. */
typedef struct {
  double x_mean[9], x_std[9];
  double y_mean[7], y_std[7];
} dig_mlp_scaling;

/* Network inputs (and optionally targets) of every cell from time-averaged
 * fields_dev [20][C] (dsmc_sample layout), kngll_dev [C] and, for targets,
 * hot_dev [12][C] (closure_assemble layout).  Inputs, standardised:
 * lambda/sqrt(Tt) (dux/dx, dux/dy, duy/dx, duy/dy), lambda/Tt (dTt/dx, dTt/dy),
 * lambda/Tt (dTr/dx, dTr/dy), Kn_GLL, with the gradients and lambda of
 * closure_assemble.  Targets, standardised: HoT sigma_xx/p, sigma_xy/p,
 * sigma_yy/p, HoT q_t,x, q_t,y, q_r,x, q_r,y over p sqrt(Tt).  Empty cells:
 * zeros.  x_dev [C][9] f32; t_dev [C][7] f32 or NULL. */
/* Empty cells of a time average, before the closure of a DIG cycle: every
 * cell of fields_dev [20][C] without a usable sample (mean particle count,
 * row 19, not positive; rho or Tt not positive; Tr negative; or a non-finite
 * value in rows 0..5) takes rho, u, Tt, Tr from fallback_dev [6][C] (the
 * previous macroscopic solution), zero stresses and heat fluxes, the total
 * temperature (3 Tt + d_r Tr) / (3 + d_r) of the fallback and N = 0, so that
 * closure_assemble with n_min > 0 keeps its NSF closure and the synthetic
 * solve starts from a state in every cell.  The thinnest cells of a
 * wall-refined grid (Section 4.1) can stay empty over a whole cycle.  In
 * place, on `stream`.  Errors: DIG_ERR_INVALID (null pointer). */
dig_status fields_fill_empty(dig_ctx* ctx, double* fields_dev, const double* fallback_dev,
                             dig_stream_t stream);

dig_status closure_features(dig_ctx* ctx, const double* fields_dev, const double* kngll_dev,
                            const double* hot_dev, const dig_mlp_scaling* scaling_host,
                            float* x_dev, float* t_dev, dig_stream_t stream);

/* Three-band adaptive closure (Section 3.1 with the learned terms): cells
 * with the equilibrium mask set keep HoT = 0 (NSF); cells with
 * kn_lo <= Kn_GLL < kn_hi take the network's prediction y_dev [C][7]
 * (de-standardised; sigma_zz = -(sigma_xx + sigma_yy), z components 0)
 * unless the DSMC-extracted terms, as judge, reject it: in some component
 * |prediction - DSMC| (in the targets' scaled units, sigma/p and
 * q/(p sqrt(Tt))) exceeds judge_sigma standard errors of the DSMC term plus
 * judge_rel |DSMC| (then the DSMC-extracted term stays).  The standard error
 * comes from the sampling noise of the cell's time average, taken as
 * M = N x judge_steps independent particle samples (N = the mean particle
 * count, row 19 of fields_dev; judge_steps = the averaged steps divided by
 * the correlation time in steps): per-particle standard deviations of the
 * moment sums of an equilibrium cell (sqrt(4/3), 1, sqrt(4/3) for
 * sigma xx, xy, yy; sqrt(5/2) for q_t; 1 for q_r) over sqrt(M), combined
 * with the noise the NSF terms take from the central differences of the
 * neighbours' mean velocity (variance Tt/M), Tt (2 Tt^2/(3 M)) and
 * Tr (Tr^2/M), with mu and kappa from A_host (as closure_assemble).  All
 * other cells keep the DSMC-extracted term.  hot_dev [12][C] is updated in
 * place; src_dev [C] (nullable) receives 0 NSF, 1 DSMC, 2 network,
 * 3 network rejected.  Errors: DIG_ERR_INVALID (null pointer, kn_lo > kn_hi,
 * negative tolerance, judge_steps <= 0, singular A). */
dig_status closure_blend(dig_ctx* ctx, const double* fields_dev, const double* kngll_dev,
                         const uint8_t* mask_dev, const float* y_dev,
                         const dig_mlp_scaling* scaling_host, const double* A_host, double kn_lo,
                         double kn_hi, double judge_sigma, double judge_rel, double judge_steps,
                         double* hot_dev, uint8_t* src_dev, dig_stream_t stream);

const char* dig_last_error(void);
void dsmc_destroy(dig_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
