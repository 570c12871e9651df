/*
 * sph_oracle.c -- plain CPU reference for one SPH + boid time step.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline of the bench).
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 *
 * The step follows the paper's frame (Section "Governing Equations", the
 * frame overview): neighbour search over a uniform grid sorted by cell
 * (Sections "Neighborhood Search", "Neighbor Search with Sorting"), density
 * and the equation of state, pressure and viscosity forces (Sections
 * "Smoothed Particle Hydrodynamics", "Pressure and Viscosity"), boid steering
 * and agent/fluid coupling (Section "Boid Motion and Agent Fluid
 * Interaction"), then Euler-Cromer (symplectic Euler) integration.  Every force
 * is evaluated from the start-of-step state, then fluid and agents are moved.
 *
 * Each per-particle sum runs over neighbours in ascending id, independently
 * per particle, so results do not depend on the thread count.
 */
#include "sph_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---------------------------------------------------------------- grid --- */

/* Section "Neighborhood Search": get_cell(p) = floor((p - m) / d) and the
   linear hash c_x + dim_x (c_y + dim_y c_z).  The cell is a hair larger than
   the search radius so that the 27-cell stencil provably holds every pair the
   single-precision distance test accepts. */
int64_t orc_grid(const orc_params* p, int agent_grid, int32_t dims[3], float* cell, float* inv_cell) {
  double r = p->h;
  if (agent_grid) {
    r = p->r_sep;
    if (p->r_ali > r) r = p->r_ali;
    if (p->r_coh > r) r = p->r_coh;
    if (p->r_couple > r) r = p->r_couple;
  }
  if (!(r > 0.0)) return -1;
  float d = (float)(r * (1.0 + 1.0 / 1024.0));
  float inv = (float)(1.0 / (double)d);
  int64_t total = 1;
  for (int k = 0; k < 3; ++k) {
    double ext = (double)(float)p->box_max[k] - (double)(float)p->box_min[k];
    if (!(ext > 0.0)) return -1;
    double nd = ceil(ext / (double)d);
    if (nd < 1.0) nd = 1.0;
    if (nd > 2147483647.0) return -1;
    dims[k] = (int32_t)nd;
    total *= dims[k];
  }
  if (cell) *cell = d;
  if (inv_cell) *inv_cell = inv;
  return total;
}

typedef struct {
  int32_t dims[3];
  float minv[3], inv;
  int64_t ncells;
} grid_t;

static int make_grid(const orc_params* p, int agent_grid, grid_t* g) {
  float d;
  g->ncells = orc_grid(p, agent_grid, g->dims, &d, &g->inv);
  for (int k = 0; k < 3; ++k) g->minv[k] = (float)p->box_min[k];
  return g->ncells > 0 ? 0 : -1;
}

/* Integer cell coordinates, in single precision: fl(fl(x - min) * inv_d),
   floored, clamped into the grid (a particle on the max wall belongs to the
   last cell). */
static void cell_of(const grid_t* g, const float* q, int32_t c[3]) {
  for (int k = 0; k < 3; ++k) {
    float t = q[k] - g->minv[k];
    t = t * g->inv;
    float f = floorf(t);
    int32_t ci;
    if (!(f >= 0.0f)) ci = 0;
    else if (f >= (float)g->dims[k]) ci = g->dims[k] - 1;
    else ci = (int32_t)f;
    if (ci > g->dims[k] - 1) ci = g->dims[k] - 1;
    c[k] = ci;
  }
}

static uint32_t hash_of(const grid_t* g, const int32_t c[3]) {
  return (uint32_t)((int64_t)c[0] + (int64_t)g->dims[0] * ((int64_t)c[1] + (int64_t)g->dims[1] * c[2]));
}

/* Single-precision squared distance: dx = fl(b - a) per axis, then
   fl(dz^2 + fl(dy^2 + fl(dx^2))) where the two outer steps are fused
   multiply-adds (C99 fmaf: the exact product plus sum, rounded once).
   Compiled without contraction, so nothing else is fused. */
static float dist2_f32(const float* a, const float* b) {
  float dx = b[0] - a[0];
  float dy = b[1] - a[1];
  float dz = b[2] - a[2];
  float s = dx * dx;
  s = fmaf(dy, dy, s);
  s = fmaf(dz, dz, s);
  return s;
}

static double dist2_f64(const float* a, const float* b) {
  double dx = (double)a[0] - (double)b[0];
  double dy = (double)a[1] - (double)b[1];
  double dz = (double)a[2] - (double)b[2];
  return dx * dx + dy * dy + dz * dz;
}

/* ------------------------------------------------- counting sort (order) --- */

/* Section "Neighbor Search with Sorting": per-cell counts, an exclusive prefix
   sum giving each cell's first slot, and a placement of every particle into its
   cell's range.  Visiting ids in ascending order makes the order within a cell
   ascending id, so the result is the (key, id) order. */
static void counting_order(const grid_t* g, int64_t n, const float* x, uint32_t* key, uint32_t* cnt,
                           uint32_t* off, uint32_t* sorted) {
  memset(cnt, 0, sizeof(uint32_t) * (size_t)g->ncells);
  for (int64_t i = 0; i < n; ++i) {
    int32_t c[3];
    cell_of(g, x + 3 * i, c);
    key[i] = hash_of(g, c);
    cnt[key[i]] += 1;
  }
  uint64_t run = 0;
  for (int64_t c = 0; c < g->ncells; ++c) {
    off[c] = (uint32_t)run;
    run += cnt[c];
  }
  off[g->ncells] = (uint32_t)run;
  uint32_t* fill = (uint32_t*)calloc((size_t)g->ncells, sizeof(uint32_t));
  for (int64_t i = 0; i < n; ++i) {
    uint32_t k = key[i];
    sorted[off[k] + fill[k]] = (uint32_t)i;
    fill[k] += 1;
  }
  free(fill);
}

/* ------------------------------------------------------ neighbour sets --- */

typedef struct {
  int64_t* v;
  int64_t len, cap;
} ilist;

static void il_push(ilist* l, int64_t a) {
  if (l->len == l->cap) {
    l->cap = l->cap ? 2 * l->cap : 256;
    l->v = (int64_t*)realloc(l->v, sizeof(int64_t) * (size_t)l->cap);
  }
  l->v[l->len++] = a;
}

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

typedef struct {
  int mode; /* 0 brute, 1 cells */
  int64_t n;
  const float* x;
  const grid_t* g;
  const uint32_t *off, *sorted;
} finder_t;

/* All j != self with fl32 dist2(q, x_j) < r2, ascending j.  Brute force visits
   every j; the cell variant visits the (2 ns + 1)^3 cells around q's cell. */
static void find(const finder_t* f, const float* q, float r2, int ns, int64_t self, ilist* out) {
  out->len = 0;
  if (f->mode == 0) {
    for (int64_t j = 0; j < f->n; ++j) {
      if (j == self) continue;
      if (dist2_f32(q, f->x + 3 * j) < r2) il_push(out, j);
    }
    return;
  }
  int32_t c[3];
  cell_of(f->g, q, c);
  for (int dz = -ns; dz <= ns; ++dz)
    for (int dy = -ns; dy <= ns; ++dy)
      for (int dx = -ns; dx <= ns; ++dx) {
        int32_t cc[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
        if (cc[0] < 0 || cc[1] < 0 || cc[2] < 0 || cc[0] >= f->g->dims[0] || cc[1] >= f->g->dims[1] ||
            cc[2] >= f->g->dims[2])
          continue;
        uint32_t k = hash_of(f->g, cc);
        for (uint32_t s = f->off[k]; s < f->off[k + 1]; ++s) {
          int64_t j = f->sorted[s];
          if (j == self) continue;
          if (dist2_f32(q, f->x + 3 * j) < r2) il_push(out, j);
        }
      }
  qsort(out->v, (size_t)out->len, sizeof(int64_t), cmp_i64);
}

/* ------------------------------------------------------------- physics --- */

typedef struct {
  double h, h2, m, rho0, k, mu;
  double c6;      /* poly6: 315 / (64 pi h^9) */
  double cp, cv;  /* pair-term constants of the pressure and viscosity kernels */
  double rc, cpc, cvc; /* the same at the coupling radius */
  float h2_32, rc2_32, rsep2_32, rali2_32, rcoh2_32;
} consts_t;

/* Section "Pressure and Viscosity".  The combined pair term is
     (m / rho_j) (1 - q) [ Cp k (rho_i + rho_j - 2 rho0) (1 - q) r_ij / q - Cv mu v_ij ].
   kernel_norm 0 uses the 3-D normalised spiky gradient -45/(pi h^6)(h - r)^2 r^
   and viscosity Laplacian 45/(pi h^6)(h - r): Cp = 45/(2 pi h^5), Cv = 45/(pi h^5).
   kernel_norm 1 uses the constants as printed (15/(pi h^4) and 40/(pi h^4)),
   which normalise in two dimensions. */
static void pair_consts(int norm, double h, double* cp, double* cv) {
  if (norm == 1) {
    *cp = 15.0 / (PI * h * h * h * h);
    *cv = 40.0 / (PI * h * h * h * h);
  } else {
    double h5 = h * h * h * h * h;
    *cp = 45.0 / (2.0 * PI * h5);
    *cv = 45.0 / (PI * h5);
  }
}

static void make_consts(const orc_params* p, consts_t* c) {
  c->h = (double)(float)p->h;
  c->h2 = c->h * c->h;
  c->m = (double)(float)p->mass;
  c->rho0 = (double)(float)p->rest_density;
  c->k = (double)(float)p->gas_k;
  c->mu = (double)(float)p->viscosity;
  double h9 = c->h2 * c->h2 * c->h2 * c->h2 * c->h;
  c->c6 = 315.0 / (64.0 * PI * h9);
  pair_consts(p->kernel_norm, c->h, &c->cp, &c->cv);
  c->rc = (double)(float)p->r_couple;
  pair_consts(p->kernel_norm, c->rc, &c->cpc, &c->cvc);
  c->h2_32 = (float)(c->h * c->h);
  double rs = (double)(float)p->r_sep, ra = (double)(float)p->r_ali, rh = (double)(float)p->r_coh;
  c->rc2_32 = (float)(c->rc * c->rc);
  c->rsep2_32 = (float)(rs * rs);
  c->rali2_32 = (float)(ra * ra);
  c->rcoh2_32 = (float)(rh * rh);
}

/* Density: rho_i = m W_poly6 summed over N_i plus the particle itself
   (Sections "Smoothed Particle Hydrodynamics" and "Neighborhood Search"). */
static double density_of(const consts_t* c, const float* x, int64_t i, const ilist* nb) {
  double s = c->h2 * c->h2 * c->h2; /* self: W(0) */
  for (int64_t t = 0; t < nb->len; ++t) {
    double r2 = dist2_f64(x + 3 * i, x + 3 * nb->v[t]);
    double d = c->h2 - r2;
    if (d > 0.0) s += d * d * d;
  }
  return c->m * c->c6 * s;
}

/* Pair term of particle i with partner at position xj, velocity vj, density
   rhoj; rho_i is the density of i.  Coincident pairs contribute nothing. */
static void pair_term(double h, double cp, double cv, double k, double mu, double rho0, double mj, const float* xi,
                      const float* vi, double rhoi, const float* xj, const float* vj, double rhoj, double acc[3]) {
  double r2 = dist2_f64(xi, xj);
  if (r2 == 0.0) return;
  double r = sqrt(r2);
  double q = r / h;
  double w = 1.0 - q;
  if (w < 0.0) w = 0.0;
  double pres = cp * k * (rhoi + rhoj - 2.0 * rho0) * w / q;
  double s = mj / rhoj * w;
  for (int a = 0; a < 3; ++a) {
    double rij = (double)xi[a] - (double)xj[a];
    double vij = (double)vi[a] - (double)vj[a];
    acc[a] += s * (pres * rij - cv * mu * vij);
  }
}

/* Walls: reflect a coordinate that left [lo, hi] and scale that velocity
   component by -e; finally clamp into the box. */
static void walls(const orc_params* p, double xn[3], double vn[3]) {
  for (int a = 0; a < 3; ++a) {
    double lo = (double)(float)p->box_min[a], hi = (double)(float)p->box_max[a];
    double e = (double)(float)p->wall_restitution;
    if (xn[a] < lo) {
      xn[a] = 2.0 * lo - xn[a];
      vn[a] = -e * vn[a];
    } else if (xn[a] > hi) {
      xn[a] = 2.0 * hi - xn[a];
      vn[a] = -e * vn[a];
    }
    if (xn[a] < lo) xn[a] = lo;
    if (xn[a] > hi) xn[a] = hi;
  }
}

static void fill_nan(double* a, int64_t m) {
  if (!a) return;
  for (int64_t i = 0; i < m; ++i) a[i] = NAN;
}
static void fill_ones(uint32_t* a, int64_t m) {
  if (!a) return;
  for (int64_t i = 0; i < m; ++i) a[i] = 0xFFFFFFFFu;
}

int orc_step(const orc_params* p, int64_t n, const float* x, const float* v, int64_t na, const float* y,
             const float* u, const int64_t* fsample, int64_t n_fs, const int64_t* asample, int64_t n_as,
             orc_out* out) {
  return orc_step_ex(p, n, x, v, na, y, u, fsample, n_fs, asample, n_as, NULL, out);
}

int orc_step_ex(const orc_params* p, int64_t n, const float* x, const float* v, int64_t na, const float* y,
                const float* u, const int64_t* fsample, int64_t n_fs, const int64_t* asample, int64_t n_as,
                const double* agent_acc, orc_out* out) {
  return orc_step_rho(p, n, x, v, na, y, u, fsample, n_fs, asample, n_as, agent_acc, NULL, out);
}

int orc_step_rho(const orc_params* p, int64_t n, const float* x, const float* v, int64_t na, const float* y,
                 const float* u, const int64_t* fsample, int64_t n_fs, const int64_t* asample, int64_t n_as,
                 const double* agent_acc, const double* rho_in, orc_out* out) {
  if (n < 0 || na < 0 || (n > 0 && (!x || !v)) || (na > 0 && (!y || !u))) return -1;
  grid_t g, ga;
  if (make_grid(p, 0, &g) || make_grid(p, 1, &ga)) return -1;
  if (g.ncells >= (int64_t)0xFFFFFFFF || ga.ncells >= (int64_t)0xFFFFFFFF) return -1;
  consts_t c;
  make_consts(p, &c);

  /* ---- ordering (always full) ---- */
  uint32_t* key = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
  uint32_t* cnt = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)g.ncells);
  uint32_t* off = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(g.ncells + 1));
  uint32_t* sorted = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
  counting_order(&g, n, x, key, cnt, off, sorted);
  uint32_t* akey = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(na > 0 ? na : 1));
  uint32_t* acnt = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)ga.ncells);
  uint32_t* aoff = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(ga.ncells + 1));
  uint32_t* asorted = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(na > 0 ? na : 1));
  counting_order(&ga, na, y, akey, acnt, aoff, asorted);

  finder_t ff = {p->nbr_mode, n, x, &g, off, sorted};
  /* agent-side finders are always brute force over agents (A is small) */
  finder_t fa = {0, na, y, &ga, aoff, asorted};
  /* stencil half-width on the fluid grid for the coupling radius */
  float dcell;
  int32_t dtmp[3];
  orc_grid(p, 0, dtmp, &dcell, NULL);
  int ns_c = (int)ceil((double)(float)p->r_couple / (double)dcell);
  if (ns_c < 1) ns_c = 1;

  /* ---- which particles need a density ---- */
  int64_t nfs = fsample ? n_fs : n, nas = asample ? n_as : na;
  unsigned char* need = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
  double* rho = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  fill_nan(rho, n);
  if (!fsample && !asample) {
    memset(need, 1, (size_t)n);
  } else {
#pragma omp parallel
    {
      ilist nb = {0, 0, 0};
#pragma omp for schedule(dynamic, 16)
      for (int64_t t = 0; t < nfs; ++t) {
        int64_t i = fsample ? fsample[t] : t;
        need[i] = 1;
        find(&ff, x + 3 * i, c.h2_32, 1, i, &nb);
        for (int64_t q = 0; q < nb.len; ++q) need[nb.v[q]] = 1;
      }
#pragma omp for schedule(dynamic, 4)
      for (int64_t t = 0; t < nas; ++t) {
        int64_t a = asample ? asample[t] : t;
        find(&ff, y + 3 * a, c.rc2_32, ns_c, -1, &nb);
        for (int64_t q = 0; q < nb.len; ++q) need[nb.v[q]] = 1;
      }
      free(nb.v);
    }
  }

  /* ---- density and neighbour counts ---- */
#pragma omp parallel
  {
    ilist nb = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
      if (!need[i]) continue;
      find(&ff, x + 3 * i, c.h2_32, 1, i, &nb);
      rho[i] = density_of(&c, x, i, &nb);
    }
    free(nb.v);
  }
  /* densities given by the caller replace the computed ones in every force
     term (the density output keeps the computed value) */
  double* rho_own = NULL;
  if (rho_in) {
    rho_own = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    memcpy(rho_own, rho, sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
      if (need[i]) rho[i] = rho_in[i];
  }

  /* ---- fluid outputs for the sample ---- */
  if (out) {
    fill_nan(out->rho, n);
    fill_nan(out->a_int, 3 * n);
    fill_nan(out->a_coup, 3 * n);
    fill_nan(out->x1, 3 * n);
    fill_nan(out->v1, 3 * n);
    fill_nan(out->x1f, 3 * n);
    fill_nan(out->v1f, 3 * n);
    fill_ones(out->nbr, n);
    fill_ones(out->touched, n);
  }
  const double dt = (double)(float)p->dt;
  const double gvec[3] = {(double)(float)p->gravity[0], (double)(float)p->gravity[1], (double)(float)p->gravity[2]};
#pragma omp parallel
  {
    ilist nb = {0, 0, 0}, ab = {0, 0, 0};
#pragma omp for schedule(dynamic, 16)
    for (int64_t t = 0; t < nfs; ++t) {
      int64_t i = fsample ? fsample[t] : t;
      const float* xi = x + 3 * i;
      const float* vi = v + 3 * i;
      find(&ff, xi, c.h2_32, 1, i, &nb);
      /* internal acceleration: a_i = (1/rho_i) sum_j pair term */
      double acc[3] = {0, 0, 0};
      for (int64_t q = 0; q < nb.len; ++q) {
        int64_t j = nb.v[q];
        pair_term(c.h, c.cp, c.cv, c.k, c.mu, c.rho0, c.m, xi, vi, rho[i], x + 3 * j, v + 3 * j, rho[j], acc);
      }
      for (int a = 0; a < 3; ++a) acc[a] /= rho[i];
      /* coupling: agents a with |y_a - x_i| < r_couple push on i with -G_ai / m */
      find(&fa, xi, c.rc2_32, 1, -1, &ab);
      double ac[3] = {0, 0, 0};
      for (int64_t q = 0; q < ab.len; ++q) {
        int64_t a = ab.v[q];
        /* G_ai = (m / rho_a) * pair term of the agent (a particle of mass m
           at rest density, so p_a = 0) with fluid particle i; i feels -G_ai / m */
        double t_ai[3] = {0, 0, 0};
        pair_term(c.rc, c.cpc, c.cvc, c.k, c.mu, c.rho0, c.m, y + 3 * a, u + 3 * a, c.rho0, xi, vi, rho[i], t_ai);
        for (int k = 0; k < 3; ++k) {
          double G = c.m / c.rho0 * t_ai[k];
          ac[k] -= G / c.m;
        }
      }
      if (out) {
        if (out->rho) out->rho[i] = rho_own ? rho_own[i] : rho[i];
        if (out->nbr) out->nbr[i] = (uint32_t)nb.len;
        if (out->touched) out->touched[i] = (uint32_t)ab.len;
        double vn[3], xn[3];
        for (int k = 0; k < 3; ++k) {
          if (out->a_int) out->a_int[3 * i + k] = acc[k];
          if (out->a_coup) out->a_coup[3 * i + k] = ac[k];
          vn[k] = (double)vi[k] + dt * (acc[k] + ac[k] + gvec[k]);
          xn[k] = (double)xi[k] + dt * vn[k];
        }
        for (int k = 0; k < 3; ++k) {
          if (out->x1f) out->x1f[3 * i + k] = xn[k];
          if (out->v1f) out->v1f[3 * i + k] = vn[k];
        }
        walls(p, xn, vn);
        for (int k = 0; k < 3; ++k) {
          if (out->x1) out->x1[3 * i + k] = xn[k];
          if (out->v1) out->v1[3 * i + k] = vn[k];
        }
      }
    }
    free(nb.v);
    free(ab.v);
  }

  /* ---- agents ---- */
  if (out) {
    fill_nan(out->steer, 3 * na);
    fill_nan(out->force, 3 * na);
    fill_nan(out->y1, 3 * na);
    fill_nan(out->u1, 3 * na);
    fill_nan(out->y1f, 3 * na);
    fill_nan(out->u1f, 3 * na);
    fill_ones(out->n_sep, na);
    fill_ones(out->n_ali, na);
    fill_ones(out->n_coh, na);
    fill_ones(out->n_cpl, na);
  }
  const double rsep = (double)(float)p->r_sep;
#pragma omp parallel
  {
    ilist sb = {0, 0, 0}, vb = {0, 0, 0}, cb = {0, 0, 0}, kb = {0, 0, 0};
#pragma omp for schedule(dynamic, 4)
    for (int64_t t = 0; t < nas; ++t) {
      int64_t a = asample ? asample[t] : t;
      const float* ya = y + 3 * a;
      const float* ua = u + 3 * a;
      /* separation: sum over b in S_a of (1 - |d|/r_sep) d, d = y_a - y_b */
      find(&fa, ya, c.rsep2_32, 1, a, &sb);
      double sep[3] = {0, 0, 0};
      for (int64_t q = 0; q < sb.len; ++q) {
        const float* yb = y + 3 * sb.v[q];
        double d[3] = {(double)ya[0] - yb[0], (double)ya[1] - yb[1], (double)ya[2] - yb[2]};
        double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double wgt = 1.0 - len / rsep;
        if (wgt < 0.0) wgt = 0.0;
        for (int k = 0; k < 3; ++k) sep[k] += wgt * d[k];
      }
      /* alignment: mean velocity of V_a minus own; cohesion: mean position of C_a minus own */
      find(&fa, ya, c.rali2_32, 1, a, &vb);
      find(&fa, ya, c.rcoh2_32, 1, a, &cb);
      double ali[3] = {0, 0, 0}, coh[3] = {0, 0, 0};
      if (vb.len > 0) {
        double mv[3] = {0, 0, 0};
        for (int64_t q = 0; q < vb.len; ++q)
          for (int k = 0; k < 3; ++k) mv[k] += (double)u[3 * vb.v[q] + k];
        for (int k = 0; k < 3; ++k) ali[k] = mv[k] / (double)vb.len - (double)ua[k];
      }
      if (cb.len > 0) {
        double mp[3] = {0, 0, 0};
        for (int64_t q = 0; q < cb.len; ++q)
          for (int k = 0; k < 3; ++k) mp[k] += (double)y[3 * cb.v[q] + k];
        for (int k = 0; k < 3; ++k) coh[k] = mp[k] / (double)cb.len - (double)ya[k];
      }
      double st[3];
      for (int k = 0; k < 3; ++k)
        st[k] = (double)(float)p->w_sep * sep[k] + (double)(float)p->w_ali * ali[k] + (double)(float)p->w_coh * coh[k];
      /* further steering given per agent (obstacle avoidance), added to the rules */
      if (agent_acc)
        for (int k = 0; k < 3; ++k) st[k] += agent_acc[3 * a + k];
      /* coupling force on the agent: F_a = sum_j G_aj over fluid within r_couple */
      find(&ff, ya, c.rc2_32, ns_c, -1, &kb);
      double F[3] = {0, 0, 0};
      for (int64_t q = 0; q < kb.len; ++q) {
        int64_t j = kb.v[q];
        /* G_aj = (m / rho_a) * pair term, rho_a = rest density */
        double t_aj[3] = {0, 0, 0};
        pair_term(c.rc, c.cpc, c.cvc, c.k, c.mu, c.rho0, c.m, ya, ua, c.rho0, x + 3 * j, v + 3 * j, rho[j], t_aj);
        for (int k = 0; k < 3; ++k) F[k] += c.m / c.rho0 * t_aj[k];
      }
      /* integrate: u' = u + dt (steer + couple_factor F / m); clamp speed; y' = y + dt u' */
      double un[3], yn[3];
      double cf = (double)(float)p->couple_factor;
      for (int k = 0; k < 3; ++k) un[k] = (double)ua[k] + dt * (st[k] + cf * F[k] / c.m);
      double sp = sqrt(un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
      double vmax = (double)(float)p->v_max, vmin = (double)(float)p->v_min;
      if (sp > vmax) {
        for (int k = 0; k < 3; ++k) un[k] *= vmax / sp;
      } else if (sp > 0.0 && sp < vmin) {
        for (int k = 0; k < 3; ++k) un[k] *= vmin / sp;
      }
      for (int k = 0; k < 3; ++k) yn[k] = (double)ya[k] + dt * un[k];
      if (out)
        for (int k = 0; k < 3; ++k) {
          if (out->y1f) out->y1f[3 * a + k] = yn[k];
          if (out->u1f) out->u1f[3 * a + k] = un[k];
        }
      walls(p, yn, un);
      if (out) {
        if (out->n_sep) out->n_sep[a] = (uint32_t)sb.len;
        if (out->n_ali) out->n_ali[a] = (uint32_t)vb.len;
        if (out->n_coh) out->n_coh[a] = (uint32_t)cb.len;
        if (out->n_cpl) out->n_cpl[a] = (uint32_t)kb.len;
        for (int k = 0; k < 3; ++k) {
          if (out->steer) out->steer[3 * a + k] = st[k];
          if (out->force) out->force[3 * a + k] = F[k];
          if (out->y1) out->y1[3 * a + k] = yn[k];
          if (out->u1) out->u1[3 * a + k] = un[k];
        }
      }
    }
    free(sb.v);
    free(vb.v);
    free(cb.v);
    free(kb.v);
  }

  if (out) {
    if (out->key) memcpy(out->key, key, sizeof(uint32_t) * (size_t)n);
    if (out->cnt) memcpy(out->cnt, cnt, sizeof(uint32_t) * (size_t)g.ncells);
    if (out->off) memcpy(out->off, off, sizeof(uint32_t) * (size_t)(g.ncells + 1));
    if (out->sorted) memcpy(out->sorted, sorted, sizeof(uint32_t) * (size_t)n);
    if (out->akey) memcpy(out->akey, akey, sizeof(uint32_t) * (size_t)na);
    if (out->acnt) memcpy(out->acnt, acnt, sizeof(uint32_t) * (size_t)ga.ncells);
    if (out->aoff) memcpy(out->aoff, aoff, sizeof(uint32_t) * (size_t)(ga.ncells + 1));
    if (out->asorted) memcpy(out->asorted, asorted, sizeof(uint32_t) * (size_t)na);
  }
  free(key);
  free(cnt);
  free(off);
  free(sorted);
  free(akey);
  free(acnt);
  free(aoff);
  free(asorted);
  free(need);
  free(rho);
  free(rho_own);
  return 0;
}
