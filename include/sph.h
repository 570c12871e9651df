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
  SPH_PAIR_COUNT = 18   /* uint64 [1]: sum of SPH_NBR_COUNT over all steps since create */
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
   graph when one of n_steps steps exists (see sph_capture). */
sph_status sph_step(sph_ctx* ctx, int32_t n_steps);

/* Copy a field (sph_field) into dst (host or device), which must hold at
   least the field's size in bytes; dst_bytes is checked. */
sph_status sph_read(sph_ctx* ctx, int32_t field, void* dst, int64_t dst_bytes);

/* Size in bytes of a field, or a negative status. */
int64_t sph_field_bytes(const sph_ctx* ctx, int32_t field);

sph_status sph_info_get(const sph_ctx* ctx, sph_info* out);

/* Capture n_steps steps into a HIP graph; later sph_step(ctx, n_steps) calls
   replay it.  n_steps = 0 drops the graph. */
sph_status sph_capture(sph_ctx* ctx, int32_t n_steps);

/* Profiling: run n_steps steps eagerly (never from a captured graph),
   recording a HIP event on the context's stream before the first kernel and
   after every kernel; synchronises, then stores in phase_ms[p] the summed
   duration in milliseconds of kernel p over the n_steps steps.  n_phases must
   be >= SPH_STEP_PHASES; sph_phase_name(p) names kernel p. */
#define SPH_STEP_PHASES 9
sph_status sph_step_profiled(sph_ctx* ctx, int32_t n_steps, double* phase_ms, int32_t n_phases);
const char* sph_phase_name(int32_t phase);

void sph_destroy(sph_ctx* ctx);

/* Message of the last failure on ctx (or of the last failed create when ctx
   is NULL).  The pointer stays valid until the next call on ctx. */
const char* sph_last_error(const sph_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
