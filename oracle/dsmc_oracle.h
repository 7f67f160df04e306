/*
 * FP64 CPU oracle for the DSMC + DIG hot path of "Multiscale simulation of
 * rarefied polyatomic gas flow via DIG method" (Luo, Huang, Li, Wu,
 * arXiv:2501.10965).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plainly written
 * reference that the HIP path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never calls it.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * Units are the paper's (Section 2): length L0, density rho0, temperature T0,
 * speed sqrt(R T0); molecular mass = 1, so rho is the number density times
 * the particle weight.  In a uniform box, positions are held in grid units
 * (x/dx, y/dy) so that the cell index is floor() of the position; an annulus
 * and a graded box (cells of different widths between per-axis face tables)
 * hold them in physical units.
 */
#ifndef DSMC_ORACLE_H
#define DSMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_PERIODIC = 0, ORC_BC_DIFFUSE = 1, ORC_BC_SPECULAR = 2, ORC_BC_FREESTREAM = 3 };
enum { ORC_GEOM_BOX = 0, ORC_GEOM_ANNULUS = 1, ORC_GEOM_GRADED = 2 };

/* Philox stream tags (third counter word, high byte). */
enum {
  ORC_TAG_INIT = 1, ORC_TAG_INIT_N = 2, ORC_TAG_WALL = 3, ORC_TAG_NCAND = 4,
  ORC_TAG_COLL = 5, ORC_TAG_DIG_N = 6, ORC_TAG_DIG_DEL = 7, ORC_TAG_DIG_SRC = 8,
  ORC_TAG_DIG_EMPTY = 9, ORC_TAG_INFLOW = 10,
  ORC_TAG_ER = 11, /* extra words of a rotational energy with d_r > 2 */
  ORC_TAG_BL = 12  /* Borgnakke-Larsen fraction by rejection for d_r > 2 */
};

typedef struct {
  int32_t  dim;          /* 1 or 2 */
  int32_t  nx, ny;       /* cells per axis (ny = 1 for dim 1) */
  double   lx, ly;       /* domain lengths (ly ignored for dim 1) */
  int32_t  geometry;     /* ORC_GEOM_*; annulus: nx angular x ny radial cells */
  double   r_in, r_out, q; /* annulus radii, radial stretch ratio */
  double   kn, omega, alpha;
  int32_t  dr;           /* rotational degrees of freedom, 2..6 */
  double   zrot;         /* rotational collision number Z */
  double   dt, weight;   /* time step; particle weight N_eff (mass per particle) */
  int32_t  bc_type[4];   /* faces x-, x+, y-, y+ */
  double   bc_T[4];
  double   bc_U[4][3];
  double   bc_rho[4];    /* freestream density */
  uint64_t seed;
  uint32_t instance;
  /* graded box: face coordinates along x (nx + 1) and y (ny + 1, dim 2),
   * strictly increasing from 0 to lx (ly) */
  const double* xf;
  const double* yf;
} orc_config;

typedef struct {
  int64_t candidates, accepted, inelastic, saturated;
} orc_collide_stats;

/* Philox4x32-10 block (Salmon et al., SC'11). */
void     orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void     orc_draw(const orc_config* c, uint32_t entity, uint32_t step, uint32_t tag,
                  uint32_t draw, uint32_t out[4]);
double   orc_u01(uint32_t r);
uint32_t orc_pick(uint32_t r, uint32_t n);

double orc_mu0(const orc_config* c);
double orc_csigma(const orc_config* c);
double orc_pinelastic(const orc_config* c);
double orc_cell_volume(const orc_config* c);
/* Volume (area, length) of one cell; the annulus cell (i, j) spans the angle
 * 2 pi / nx and the radii of faces j and j + 1. */
double orc_cell_volume_at(const orc_config* c, int32_t cell);
/* Annulus radial face j: r_in + (r_out - r_in)(q^j - 1)/(q^ny - 1). */
double orc_annulus_face(const orc_config* c, int32_t j);
/* Freestream inflow at the outer circle of an annulus: appends the
 * reservoir-shell particles of this step at index n; returns their number
 * (or -1 if the capacity would be exceeded). */
int64_t orc_inject(const orc_config* c, int64_t n, int64_t cap, double* x, double* y,
                   double* vx, double* vy, double* vz, double* er, uint32_t* id,
                   uint32_t step, uint64_t next_id);

/* start (nullable, [ncell + 1]) receives the first particle of every cell. */
int64_t orc_init(const orc_config* c, const double* fields, int32_t ppc, int64_t cap,
                 double* x, double* y, double* vx, double* vy, double* vz, double* er,
                 uint32_t* id, int64_t* start);

int64_t orc_move(const orc_config* c, int64_t n, double* x, double* y, double* vx,
                 double* vy, double* vz, double* er, const uint32_t* id, uint32_t step);

/* Cell of every particle; -1 for a particle outside a freestream boundary. */
void orc_cell_index(const orc_config* c, int64_t n, const double* x, const double* y,
                    int32_t* cell);

/* Stable counting sort; particles with a negative cell are dropped (the
 * sorted count is start[ncell]). */
void orc_sort(int64_t n, const int32_t* cell, int32_t ncell, int64_t* perm, int64_t* start);

void orc_collide(const orc_config* c, int32_t ncell, const int64_t* start, double* vx,
                 double* vy, double* vz, double* er, float* sgmax, uint32_t step,
                 orc_collide_stats* st, double* obs_out, double* margin_out);

void orc_sample_sums(int32_t ncell, const int64_t* start, const double* vx,
                     const double* vy, const double* vz, const double* er, double* sums);

void orc_sums_to_fields(const orc_config* c, int32_t ncell, const double* sums,
                        double nsteps, double* fields);

int orc_adjust(const orc_config* c, int32_t ncell, const int64_t* start, const double* x,
               const double* y, const double* vx, const double* vy, const double* vz,
               const double* er, const uint32_t* id, const double* target, uint32_t dig_iter,
               uint64_t next_id, int64_t cap, double* ox, double* oy, double* ovx,
               double* ovy, double* ovz, double* oer, uint32_t* oid, int64_t* ostart,
               int64_t* n_out, uint64_t* next_id_out);

void orc_closure(const orc_config* c, const double* fields, const double A[4], double kn_ref,
                 double n_min, double* hot, uint8_t* mask, double* kn_gll, double* nsf);

#ifdef __cplusplus
}
#endif
#endif
