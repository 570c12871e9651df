/*
 * sph_oracle.h -- plain CPU reference for one SPH + boid time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP library: it derives every
 * constant itself from the parameters it is given.
 *
 * Arithmetic: physics in IEEE double from the float32 state; discrete
 * decisions (cell coordinates, "is j a neighbour of i") in IEEE single,
 * evaluated in a fixed order with no fused multiply-add, so that they are an
 * exact, portable definition.  Neighbour sets are brute force over all pairs
 * by definition (nbr_mode 0); nbr_mode 1 gathers the same sets from a cell
 * list (tests pin the two to be identical) and is only there to reach large
 * particle counts.
 *
 * All per-element arrays are in creation-id order and AoS ([n][3] for
 * vectors).  Any output pointer may be NULL.  Entries outside a sample are
 * left as NaN (doubles) or 0xFFFFFFFF (counts).
 */
#ifndef SPH_ORACLE_H
#define SPH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  /* Section "Pressure and Viscosity": smoothing length, rest density,
     gas constant of the equation of state, viscosity; particle mass; time step */
  double h, rest_density, gas_k, viscosity, mass, dt;
  double gravity[3], box_min[3], box_max[3], wall_restitution;
  /* Section "Boid Motion and Agent Fluid Interaction": ranges and weights */
  double r_sep, r_ali, r_coh, w_sep, w_ali, w_coh;
  double r_couple, couple_factor, v_min, v_max;
  int32_t kernel_norm; /* 0: 3-D normalised spiky / viscosity kernels; 1: the paper's printed constants */
  int32_t nbr_mode;    /* 0: brute force (definition); 1: cell list (identical sets) */
} orc_params;

typedef struct {
  /* fluid, id order */
  uint32_t *key, *nbr, *touched;          /* cell key, |N_i| (self excluded), #agents within r_couple */
  double *rho, *a_int, *a_coup, *x1, *v1; /* density, internal and coupling acceleration, new state */
  /* fluid cell table (full, never sampled) */
  uint32_t *cnt, *off, *sorted;           /* cnt[C], off[C+1], sorted ids [n] in (key, id) order */
  /* agents, id order */
  uint32_t *akey, *n_sep, *n_ali, *n_coh, *n_cpl;
  double *steer, *force, *y1, *u1;        /* steering accel, coupling force F_a, new state */
  uint32_t *acnt, *aoff, *asorted;
  /* the new state before the walls act (after the position update): lets a
     comparison tell a reflection decided on a value within rounding of a wall */
  double *x1f, *v1f, *y1f, *u1f;
} orc_out;

/* Grid derived from the parameters: cell size d = fl32(R (1 + 2^-10)) with
   R = h (fluid grid) or max(r_sep, r_ali, r_coh, r_couple) (agent grid);
   inv_d = fl32(1/d); dims = ceil((max - min) / d) in double.
   Returns the number of cells, or -1 on invalid input. */
int64_t orc_grid(const orc_params* p, int agent_grid, int32_t dims[3], float* cell, float* inv_cell);

/* One time step.  fsample / asample: ids to evaluate (NULL = all). */
int orc_step(const orc_params* p, int64_t n, const float* x, const float* v, int64_t na, const float* y,
             const float* u, const int64_t* fsample, int64_t n_fs, const int64_t* asample, int64_t n_as,
             orc_out* out);

/* orc_step with a further steering acceleration per agent (agent_acc[na][3],
   id order, may be NULL), added to the boid rules before the integration. */
int orc_step_ex(const orc_params* p, int64_t n, const float* x, const float* v, int64_t na, const float* y,
                const float* u, const int64_t* fsample, int64_t n_fs, const int64_t* asample, int64_t n_as,
                const double* agent_acc, orc_out* out);

/* orc_step_ex with the densities of the force terms given (rho_in[n], id
   order, may be NULL): the pressure, viscosity and coupling terms use
   rho_in[i] in place of the computed density of particle i, while out->rho
   still receives the computed one.  Lets a comparison separate the force
   arithmetic from the density it is fed. */
int orc_step_rho(const orc_params* p, int64_t n, const float* x, const float* v, int64_t na, const float* y,
                 const float* u, const int64_t* fsample, int64_t n_fs, const int64_t* asample, int64_t n_as,
                 const double* agent_acc, const double* rho_in, orc_out* out);

/* Number of OpenMP threads the oracle runs with, and a way to change it
   (n <= 0 leaves it). */
int orc_threads(void);
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
