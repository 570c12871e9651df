/*
 * sph.h -- C ABI of libsph.so: one time step of weakly-compressible SPH
 * coupled two-way with boid agents, on one AMD Instinct MI355X (gfx950).
 *
 * The problem statement follows "A GPU-based Hydrodynamic Simulator with Boid
 * Interactions" (Liu, Kayar, Perlin): particles carry position, velocity and a
 * common mass (Section "Boid Motion and Agent Fluid Interaction", the particle
 * structure); the constants are the smoothing length ("radius"), the rest
 * density and gas constant of the equation of state p = k (rho - rho0)
 * (Section "Pressure and Viscosity"), the viscosity coefficient, and the boid
 * ranges / weights of the separation, alignment and cohesion rules (Section
 * "Boid Motion and Agent Fluid Interaction").  One step (the frame overview in
 * Section "Governing Equations") is:
 *   cell keys + counting sort        (Sections "Neighborhood Search",
 *                                     "Neighbor Search with Sorting")
 *   density + equation of state      (Sections "Smoothed Particle
 *                                     Hydrodynamics", "Pressure and Viscosity")
 *   pressure + viscosity forces      (Section "Pressure and Viscosity")
 *   boid steering, agent<->fluid coupling (Section "Boid Motion and Agent
 *                                     Fluid Interaction")
 *   symplectic (Euler-Cromer) integration with reflecting box walls.
 *
 * Conventions
 *  - Vectors cross the boundary as float32 AoS [n][3] in creation-id order.
 *    Pointers may be host or device memory (the library copies with
 *    hipMemcpyDefault).  The library copies inputs at create time and owns
 *    all device state; callers own every buffer they pass.
 *  - All work is enqueued on the stream given at create time (NULL = the
 *    null stream).  sph_step is asynchronous.  sph_read into host memory
 *    synchronises that stream; into device memory it is enqueued.
 *  - A context is not thread-safe.  No exception crosses the ABI; every
 *    failure returns a negative sph_status and sph_last_error() describes it.
 */
#ifndef SPH_H
#define SPH_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sph_ctx sph_ctx;

typedef enum {
  SPH_OK = 0,
  SPH_EINVAL = -1,     /* invalid argument (NULL pointer, size, parameter) */
  SPH_ENOMEM = -2,     /* device allocation failed */
  SPH_EHIP = -3,       /* a HIP runtime call failed */
  SPH_ECAPACITY = -4,  /* the cell grid exceeds n_buckets, or a count exceeds 2^31 */
  SPH_ENONFINITE = -5, /* non-finite state detected (with SPH_FLAG_CHECK_FINITE) */
  SPH_ESTATE = -6,     /* call not valid in the context's current state */
  SPH_ENOTIMPL = -7
} sph_status;

/* Flags (sph_params.flags). */
#define SPH_FLAG_DIAGNOSTICS 1u  /* keep per-particle / per-agent diagnostics of the last step */
#define SPH_FLAG_CHECK_FINITE 2u /* sph_step synchronises and rejects non-finite state */
#define SPH_FLAG_FUSED 4u        /* one persistent launch per step (grid-wide barriers between phases) */
#define SPH_FLAG_FEATURES 8u     /* compute the closure's agent features every step (SPH_AGENT_FEATURES) */

typedef struct sph_params {
  /* smoothing length h (> 0), rest density rho0, gas constant k, viscosity mu,
     particle mass m, time step dt (Section "Pressure and Viscosity"). */
  float h, rest_density, gas_k, viscosity, mass, dt;
  float gravity[3];        /* body acceleration, e.g. (0, 0, -9.81) */
  float box_min[3], box_max[3]; /* bounding box = grid extent = reflecting walls */
  float wall_restitution;  /* normal velocity is scaled by -e at a wall */
  /* boid rules: separation ("protect range"), alignment and cohesion
     ("visual range") radii and weights */
  float r_sep, r_ali, r_coh, w_sep, w_ali, w_coh;
  /* coupling radius and factor of the agent<->fluid pair force; speed limits */
  float r_couple, couple_factor, v_min, v_max;
  uint32_t n_buckets;      /* 0 = any grid size; else the cell table may hold at most this many cells */
  int32_t kernel_norm;     /* 0 = 3-D normalised spiky / viscosity kernels; 1 = constants as printed */
  uint32_t flags;          /* SPH_FLAG_* */
} sph_params;

/* Fields for sph_read.  Vectors are float32 [n][3]; counts are uint32. */
typedef enum {
  SPH_POS = 0,          /* fluid position, id order, after the last step */
  SPH_VEL = 1,          /* fluid velocity, id order */
  SPH_AGENT_POS = 2,    /* agent position, id order */
  SPH_AGENT_VEL = 3,    /* agent velocity, id order */
  SPH_DENSITY = 4,      /* density of the last step, id order, float32 [n] */
  SPH_NBR_COUNT = 5,    /* |{j != i : r_ij^2 < h^2}| of the last step, id order, uint32 [n] */
  SPH_CELL_KEY = 6,     /* cell key of the last step, id order, uint32 [n] */
  SPH_ACC_INT = 7,      /* internal (pressure + viscosity) acceleration, id order   [diagnostics] */
  SPH_ACC_COUPLE = 8,   /* acceleration from agents, id order                      [diagnostics] */
  SPH_TOUCHED = 9,      /* number of agents within r_couple, id order, uint32 [n]  [diagnostics] */
  SPH_AGENT_FORCE = 10, /* coupling force on each agent, id order                  [diagnostics] */
  SPH_AGENT_STEER = 11, /* steering acceleration, id order                         [diagnostics] */
  SPH_AGENT_COUNTS = 12,/* uint32 [a][4]: separation, alignment, cohesion, fluid-coupling counts [diagnostics] */
  SPH_SORTED_IDS = 13,  /* fluid ids in (key, id) order of the last step, uint32 [n] */
  SPH_CELL_OFFSETS = 14,/* first sorted slot of each cell, uint32 [cells + 1] */
  SPH_AGENT_KEY = 15,   /* agent cell key, id order, uint32 [a] */
  SPH_AGENT_SORTED_IDS = 16,
  SPH_AGENT_CELL_OFFSETS = 17,
  SPH_PAIR_COUNT = 18,  /* uint64 [1]: sum of SPH_NBR_COUNT over all steps since create */
  SPH_AGENT_FEATURES = 19,   /* bfloat16 bits, uint16 [a][256]: closure features of the last step */
  SPH_AGENT_FORCE_MODEL = 20, /* float32 [a][3]: closure (surrogate) force of the last step */
  /* neighbour-list forms only (sph_search_set), sorted order of the last step,
     entries are sorted indices and every list includes the particle itself */
  SPH_NBR_LIST_COUNTS = 21,  /* uint32 [n]: entries of each particle's list */
  SPH_NBR_LIST_OFFSETS = 22, /* uint32 [n + 1]: first entry of each list (sorted list only) */
  SPH_NBR_LIST = 23,         /* uint32 [list capacity]: the list buffer (bucket list: 27 x capacity
                                entries per particle, the first SPH_NBR_LIST_COUNTS of them valid) */
  SPH_VOXEL_FIELD = 24       /* float32 [nz][ny][nx]: voxel density at the cube corners (sph_voxel_enable) */
} sph_field;

typedef struct sph_info {
  int64_t n, n_agents;
  int32_t dims[3], agent_dims[3];
  int64_t cells, agent_cells;
  float cell, agent_cell;  /* cell edge lengths */
  int64_t steps;           /* steps taken since create */
  int64_t device_bytes;    /* device memory held by the context */
} sph_info;

/* Create a context holding n fluid particles and n_agents boid agents
   (either may be 0).  pos/vel: [n][3]; agent_pos/agent_vel: [n_agents][3].
   hip_stream: a hipStream_t (NULL = null stream).  On success *out owns all
   device state; release it with sph_destroy. */
sph_status sph_create(const sph_params* params, int64_t n, const float* pos, const float* vel,
                      int64_t n_agents, const float* agent_pos, const float* agent_vel, void* hip_stream,
                      sph_ctx** out);

/* Create a context holding n_scenes independent scenes, advanced together by
   every sph_step.  Scene s has its own parameters per_scene[s] and owns
   particles [part_off[s], part_off[s+1]) of pos/vel ([*][3], concatenated in
   scene order) and agents [agent_off[s], agent_off[s+1]) of agent_pos /
   agent_vel; part_off and agent_off hold n_scenes + 1 non-decreasing entries
   starting at 0.  Flags are taken from per_scene[0].  Per-element fields read
   back concatenated in scene order (ids restart at 0 in each scene); cell
   offset fields hold cells + 1 entries per scene. */
sph_status sph_create_batch(const sph_params* per_scene, int32_t n_scenes, const int64_t* part_off,
                            const int64_t* agent_off, const float* pos, const float* vel, const float* agent_pos,
                            const float* agent_vel, void* hip_stream, sph_ctx** out);

/* Advance n_steps >= 0 time steps (asynchronous).  Replays the captured
   graph when one of n_steps steps exists (see sph_capture).  Returns
   SPH_EHIP, and enqueues nothing, once an earlier fused step is known to have
   aborted (a grid barrier of the persistent step kernel timed out: the state
   is then half-updated and every later fused launch leaves at once); the
   knowledge arrives asynchronously, with the flag's copy that follows every
   fused launch, so the call that enqueued the aborted step may still return
   SPH_OK.  sph_read reports it without fail. */
sph_status sph_step(sph_ctx* ctx, int32_t n_steps);

/* Copy a field (sph_field) into dst (host or device), which must hold at
   least the field's size in bytes; dst_bytes is checked.  A host dst
   synchronises the stream; a device dst is enqueued, except on a context
   that has run fused steps, where the call first waits for the stream and
   returns SPH_EHIP (copying nothing) if any fused step aborted. */
sph_status sph_read(sph_ctx* ctx, int32_t field, void* dst, int64_t dst_bytes);

/* Raise (raise != 0) or clear (raise == 0) the fused step's sticky abort
   flag on the device, waiting for the stream first.  Raised, it acts like a
   timed-out grid barrier: every later fused launch leaves at entry, without
   touching the state, and sph_step / sph_read report SPH_EHIP.  Cleared, it
   re-arms fused steps (and resets the barrier's arrival count); the caller
   must restore a valid state itself (e.g. a fresh context from a saved one).
   Lets a caller exercise its handling of that failure; per-phase launches
   never read the flag. */
sph_status sph_abort_set(sph_ctx* ctx, int32_t raise);

/* Size in bytes of a field, or a negative status. */
int64_t sph_field_bytes(const sph_ctx* ctx, int32_t field);

sph_status sph_info_get(const sph_ctx* ctx, sph_info* out);

/* Capture n_steps steps into a HIP graph; later sph_step(ctx, n_steps) calls
   replay it.  n_steps = 0 drops the graph. */
sph_status sph_capture(sph_ctx* ctx, int32_t n_steps);

/* Execution form of a step, chosen by sph_autotune or set directly.
   fused = 0: one launch per phase (variant = block size / own particles per
   thread / LDS capacity of the fluid passes); fused = 1: one persistent
   launch per step (variant = LDS capacities).  tile_x = grid cells along x
   that one workgroup of the fluid passes takes at a time (1 ..
   sph_variant_tile_max: 32, or 64 for the variants with tables that wide).
   Every form gives bit-identical results; only the speed differs.  A context
   starts with fused = 0, variant 1 (256-thread blocks in both fluid passes),
   tile_x = 32. */
typedef struct sph_tuning {
  int32_t fused, variant, tile_x;
  float ms_per_step; /* measured by sph_autotune (0 when set by hand) */
} sph_tuning;

/* Time steps_per_trial steps of every execution form on the context's own
   state (two warm-up steps, then the faster of two timed runs; the state and
   every readable field are restored after each trial, so the simulation does
   not advance), keep the fastest and store it in *best (may be NULL).  When the
   environment variable SPH_AUTOTUNE_CACHE names a file, a result for the
   same device and problem shape is reused from it and new results appended.
   Drops a captured graph.  Synchronises the stream. */
sph_status sph_autotune(sph_ctx* ctx, int32_t steps_per_trial, sph_tuning* best);
sph_status sph_tuning_set(sph_ctx* ctx, const sph_tuning* t); /* drops a captured graph */
sph_status sph_tuning_get(const sph_ctx* ctx, sph_tuning* out);
/* Number of kernel variants of a form, and the name of one (NULL if out of range). */
int32_t sph_variant_count(int32_t fused);
const char* sph_variant_name(int32_t fused, int32_t variant);
/* Widest tile_x a variant accepts (0 if out of range). */
int32_t sph_variant_tile_max(int32_t fused, int32_t variant);

/* Neighbour search of the fluid passes.  The paper describes two list-based
   searches: a hash grid of fixed-capacity cell buckets filled through an
   atomic slot per particle, with a fixed-capacity list per particle over the
   27 surrounding cells ("Neighbor Search" section), and a search on the
   counting-sorted particles that counts each particle's neighbours, scans
   the counts into offsets and fills a packed list ("Neighbor Search with
   Sorting" section).  This library's own form gathers candidates cell row by
   cell row into LDS and keeps no list; the two list forms are kept beside it
   as ablations and run the density and force passes over their lists.
     mode 0  tiled cell gather (default; bucket_capacity, list_per_particle unused)
     mode 1  sorted list: list_per_particle entries per particle are reserved
             (0: 64), 2^32 - 1 in all at most
     mode 2  bucket list: bucket_capacity particles per cell (0: 32); the list
             holds 27 x bucket_capacity entries per particle
   The sorted list takes each particle's candidates in the tiled form's order,
   so every result is bit-identical to mode 0; the bucket list takes a cell's
   particles in the order its atomics gave, so sums may differ by rounding.
   A list form allocates its buffers here (the context owns them) and runs one
   launch per phase; sph_autotune then returns SPH_ESTATE.  sph_step,
   sph_step_profiled and sph_step_timed synchronise the stream at their end in
   a list form and return SPH_ECAPACITY if a bucket or the list buffer was too
   small in any of their steps; the state is then not valid (entries past the
   capacity were left out, never written out of bounds).  Drops a captured
   graph.  Synchronises the stream. */
sph_status sph_search_set(sph_ctx* ctx, int32_t mode, int32_t bucket_capacity, int32_t list_per_particle);

/* Voxel density at cube corners ("Voxel Density" section).  At corner
   x_c = box_min + c * spacing (per axis fl32(box_min + fl32(c * spacing)),
   c = 0 .. floor((box_max - box_min) / spacing), x fastest),
     phi(x) = |x - xbar| - r,  xbar = sum_i w_i x_i,
     w_i = k(|x - x_i| / R) / sum_j k(|x - x_j| / R),  k(s) = (1 - s^2)^3,
   over the particles with fl32 |x - x_i|^2 < fl32(R^2); a corner with none
   has phi = +inf.  Every particle has radius r (particle_radius), so the
   paper's weighted mean radius is r.  Once enabled, each step computes the
   field of the state it starts from (the positions its density pass uses),
   readable as SPH_VOXEL_FIELD; before the first step it holds zeros.
   spacing <= 0 turns the field off.  dims (may be NULL) receives the corners
   per axis (0 when off).  Single-scene contexts only (SPH_ENOTIMPL
   otherwise); at most 2^31 corners (SPH_ECAPACITY).  Runs the step as one
   launch per phase.  Drops a captured graph.  Synchronises the stream. */
sph_status sph_voxel_enable(sph_ctx* ctx, float spacing, float radius, float particle_radius, int32_t* dims);

/* Obstacle Grid and obstacle avoidance ("Underwater Agent Behaviors" and
   "Boid Motion and Agent Fluid Interaction" sections).  boxes[n_boxes][6]
   (min x, y, z, max x, y, z; host memory) are axis-aligned obstacles.  A box's
   mesh is its six faces, each a lattice of (n_u + 1) x (n_v + 1) vertices,
   n = max(1, ceil(extent / vertex_spacing)), at min + ((max - min) i) / n in
   double rounded to float, each carrying the face's outward normal.  Each
   vertex goes to the agent-grid cell of its position; a cell's obstacle normal
   is the mean of its vertices' normals.  Every step, a boid then adds
     weight * sum over the 27 agent cells c around its own of omega_c n_c
   to its steering, omega_c = 2 if the centre of c (min + (c + 1/2) d) is
   within r_sep of the boid, 1 if within r_ali, else 0 (float32 squared
   distances).  n_boxes = 0 removes the obstacles.  The grid is built on the
   host here (obstacles are static); single-scene contexts only (SPH_ENOTIMPL
   otherwise); at most 2^26 vertices (SPH_ECAPACITY).  Drops a captured graph.
   Synchronises the stream. */
sph_status sph_obstacles_set(sph_ctx* ctx, int32_t n_boxes, const float* boxes, float vertex_spacing, float weight);

/* ---------------------------------------------------------------------------
   Learned coupling closure.  A small MLP (256 -> 128 -> 128 -> 3, GELU after
   the hidden layers; bfloat16 operands, float32 accumulation) maps an agent's
   neighbourhood histogram to its fluid coupling force.  Features: the 4 x 4 x
   4 block of fluid-grid cells starting at round((y - box_min) / cell) - 2 on
   each axis, x fastest; per cell count / 8 and (mean fluid velocity - agent
   velocity) / 0.5, zero for an empty cell; rounded to bfloat16.  Weights are
   float32, flat order W1 [256][128], b1 [128], W2 [128][128], b2, W3 [128][3],
   b3 (49,795 values); the network predicts F / force_scale.
   ------------------------------------------------------------------------- */
typedef struct sph_closure sph_closure;
#define SPH_CLOSURE_PARAMS 49795
#define SPH_CLOSURE_FEATURES 256
/* floats in a closure checkpoint (sph_closure_io): weights, Adam first and
   second moments (SPH_CLOSURE_PARAMS each, flat order), force scale, Adam
   step count */
#define SPH_CLOSURE_STATE_FLOATS (3 * SPH_CLOSURE_PARAMS + 2)

typedef struct sph_train_params {
  int32_t epochs, batch;   /* e.g. 20, 4096 */
  float lr, beta1, beta2, eps; /* Adam: 1e-3, 0.9, 0.999, 1e-8 */
  float val_fraction;      /* held-out fraction of the pairs, e.g. 0.1 */
  uint32_t seed;           /* seeds the split and the shuffles */
} sph_train_params;

typedef struct sph_train_report {
  float train_loss;        /* mean loss of the last epoch (normalised forces) */
  float val_rel_rms;       /* sqrt(sum |F_pred - F|^2 / sum |F|^2) on the held-out pairs */
  float force_scale;       /* root mean square training force component */
  int32_t steps;           /* optimiser steps taken */
  double seconds;          /* wall time of the call */
} sph_train_report;

typedef struct sph_closure_stats {
  int32_t mode;            /* 1: the surrogate is in use between checks */
  float last_rel_rms;      /* error of the last check */
  int64_t checks, fallbacks, surrogate_steps, exact_steps;
} sph_closure_stats;

/* weights: SPH_CLOSURE_PARAMS float32 (host or device) or NULL (zeros). */
sph_status sph_closure_create(const float* weights, float force_scale, void* hip_stream, sph_closure** out);
/* Train with Adam on n (feature, exact force) pairs held in device memory:
   features uint16 bfloat16 bits [n][256], forces float32 [n][3].  Sets the
   force scale, keeps the weights in the closure; synchronises. */
sph_status sph_closure_train(sph_closure* cl, const uint16_t* features, const float* forces, int64_t n,
                             const sph_train_params* params, sph_train_report* report);
/* forces [n][3] = MLP(features) * force_scale (device pointers; asynchronous). */
sph_status sph_closure_predict(sph_closure* cl, const uint16_t* features, int64_t n, float* forces);
/* sph_closure_predict without any allocation, for callers that cannot
   allocate device memory (code under HIP graph capture, tight serving loops,
   harnesses that forbid hipMalloc): the forward pass's activations live in a
   fixed device array of the library (33.6 MB on every device the library
   runs on, held until the process ends) instead of the closure's work
   buffers, which sph_closure_predict grows with hipMalloc.  n <= 65,536 rows
   per call (SPH_ECAPACITY beyond; split larger inputs).  Same arguments and
   the same results as sph_closure_predict.  Every call on one device shares
   that array, so calls that overlap on one device (different streams, or
   several host threads) race; serialise them. */
sph_status sph_closure_predict_static(sph_closure* cl, const uint16_t* features, int64_t n, float* forces);
/* Gradient of the mean squared error between MLP(features) and forces /
   force_scale with respect to the weights (flat order), and that loss;
   device pointers for the inputs, host or device for grad / loss; synchronises. */
sph_status sph_closure_gradient(sph_closure* cl, const uint16_t* features, const float* forces, int64_t n,
                                float* grad, float* loss);
/* One Adam step (t >= 1) with the given gradient (host or device); the moments persist in the closure. */
sph_status sph_closure_adam_step(sph_closure* cl, const float* grad, int32_t t, float lr, float beta1, float beta2,
                                 float eps);
/* write = 0: copy the weights / scale out; 1: load them (either pointer may be NULL). */
sph_status sph_closure_weights(sph_closure* cl, int32_t write, float* weights, float* force_scale);
/* Save (dir = 0) or load (dir = 1) the closure's whole training state, so
   that training can stop and resume (section 5's checkpoint of the learned
   part): buf (host or device) holds SPH_CLOSURE_STATE_FLOATS float32 values,
   bytes is checked.  The step count is the t of the last Adam step
   (sph_closure_train's last step or the t given to sph_closure_adam_step); a
   resumed run passes t + 1, t + 2, ... to sph_closure_adam_step.  Loading
   rejects a non-positive scale or a step count that is not a whole number in
   [0, 2^24].  Synchronises. */
sph_status sph_closure_io(sph_closure* cl, int32_t dir, float* buf, int64_t bytes);
void sph_closure_destroy(sph_closure* cl);
const char* sph_closure_last_error(const sph_closure* cl);
/* Use cl for the agents' coupling force: every check_every steps (starting
   with the next step) both the surrogate and the exact gather run and
   rel_rms = sqrt(sum |F_pred - F|^2 / sum |F|^2) is measured on the device;
   the steps until the next check use the surrogate only if rel_rms <=
   max_rel_rms, the exact gather otherwise.  The fluid side always feels the
   exact reaction.  cl = NULL detaches.  The context does not own cl; it must
   outlive the attachment.  Drops a captured graph; steps run as per-phase
   launches while a closure is attached. */
sph_status sph_closure_attach(sph_ctx* ctx, sph_closure* cl, int32_t check_every, float max_rel_rms);
sph_status sph_closure_stats_get(sph_ctx* ctx, sph_closure_stats* out);

/* Profiling: run n_steps steps launched directly (never from a captured
   graph) and store in phase_ms[p] the summed duration in milliseconds of
   phase p over the n_steps steps.  The density and force kernels are timed by
   HIP events recorded at the kernel's own start and end (hipExtLaunchKernel);
   every other phase by HIP events recorded on the context's stream before and
   after it, which include the gap between launches.  Events are read back
   every 25 steps while the next 25 run.  n_phases must be >=
   SPH_STEP_PHASES; sph_phase_name(p) names phase p. */
#define SPH_STEP_PHASES 8
sph_status sph_step_profiled(sph_ctx* ctx, int32_t n_steps, double* phase_ms, int32_t n_phases);
/* Timing with the least disturbance: run n_steps steps launched directly,
   with HIP events only at the density and force kernels' own start and end
   (no event between phases, so the phases follow each other as in
   sph_step).  kernel_ms[0] receives the summed density time and kernel_ms[1]
   the summed force + integration time, in milliseconds (both 0 when the
   context has no fluid).  kernel_ms is a host array of 2 doubles. */
sph_status sph_step_timed(sph_ctx* ctx, int32_t n_steps, double* kernel_ms);
const char* sph_phase_name(int32_t phase);

void sph_destroy(sph_ctx* ctx);

/* Message of the last failure on ctx (or of the last failed create when ctx
   is NULL).  The pointer stays valid until the next call on ctx. */
const char* sph_last_error(const sph_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
