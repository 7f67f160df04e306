/*
 * FP64 CPU oracle for the DSMC + DIG hot path (arXiv:2501.10965).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Written for
 * readability, single threaded, in the order the paper states the steps.
 *
 * Readings where the paper is silent are the ones listed in the design notes
 * of the repository (NTC candidate count by Iround, sgmax frozen within a
 * step, rotational energy stored per unit mass, Bird's double relaxation in
 * pick order, Beta(1, 5/2 - omega) energy split for two rotational degrees of
 * freedom, survivors-then-clones particle order after the DIG count change).
 */
#include "dsmc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two
 * 32x32->64 multiplies and xors, with a Weyl key schedule between rounds. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* Counter layout: (entity, step, tag << 24 | instance, draw); key = seed. */
void orc_draw(const orc_config* c, uint32_t entity, uint32_t step, uint32_t tag,
              uint32_t draw, uint32_t out[4]) {
  uint32_t ctr[4] = {entity, step, (tag << 24) | (c->instance & 0xFFFFFFu), draw};
  uint32_t key[2] = {(uint32_t)(c->seed & 0xFFFFFFFFu), (uint32_t)(c->seed >> 32)};
  orc_philox(ctr, key, out);
}

/* Uniform in (0,1): the top 23 bits centred in their interval; exactly
 * representable in single precision, so both precisions see the same value. */
double orc_u01(uint32_t r) { return ((double)(r >> 9) + 0.5) * (1.0 / 8388608.0); }

/* Uniform integer in [0, n). */
uint32_t orc_pick(uint32_t r, uint32_t n) { return (uint32_t)(((uint64_t)r * n) >> 32); }

/* ------------------------------------------------------------------------ */
/* Gas constants.  The Knudsen number definition of Section 2 gives
 * mu(T0) = Kn sqrt(2/pi) in paper units; mu = mu0 T^omega. */
double orc_mu0(const orc_config* c) { return c->kn * sqrt(2.0 / M_PI); }

/* VHS: sigma_T * g = C g^(2 - 2 omega).  C is fixed so that the equilibrium
 * collision frequency n <sigma_T g> equals the VHS value
 * 30 p / ((5 - 2w)(7 - 2w) mu), which ties the collision rate to the
 * viscosity mu0 T^omega above. */
double orc_csigma(const orc_config* c) {
  double w = c->omega, a = c->alpha;
  double num = 15.0 * M_PI;
  double den = sqrt(2.0) * (5.0 - 2.0 * w) * (7.0 - 2.0 * w) * pow(4.0, 1.0 - w) *
               tgamma(2.5 - w) * c->kn;
  /* VSS: the same viscosity takes a cross-section (a + 1)(a + 2) / (6 a)
   * times the VHS one (collision frequency 5 (a+1)(a+2) p / (a (5-2w)(7-2w) mu)) */
  return num / den * ((a + 1.0) * (a + 2.0) / (6.0 * a));
}

/* Fraction of inelastic collisions, equation P_inelastic (Section 2.2). */
double orc_pinelastic(const orc_config* c) {
  double w = c->omega, a = c->alpha;
  return a * (5.0 - 2.0 * w) * (7.0 - 2.0 * w) / (5.0 * (a + 1.0) * (a + 2.0) * c->zrot);
}

double orc_cell_volume(const orc_config* c) {
  double dx = c->lx / c->nx;
  if (c->dim == 1) return dx;
  return dx * (c->ly / c->ny);
}

double orc_annulus_face(const orc_config* c, int32_t j) {
  if (c->q == 1.0) return c->r_in + (c->r_out - c->r_in) * (double)j / (double)c->ny;
  return c->r_in +
         (c->r_out - c->r_in) * (pow(c->q, (double)j) - 1.0) / (pow(c->q, (double)c->ny) - 1.0);
}

double orc_cell_volume_at(const orc_config* c, int32_t cell) {
  if (c->geometry == ORC_GEOM_GRADED) {
    int32_t i = cell % c->nx, j = cell / c->nx;
    double w = c->xf[i + 1] - c->xf[i];
    if (c->dim == 1) return w;
    return w * (c->yf[j + 1] - c->yf[j]);
  }
  if (c->geometry != ORC_GEOM_ANNULUS) return orc_cell_volume(c);
  int32_t j = cell / c->nx;
  double ra = orc_annulus_face(c, j), rb = orc_annulus_face(c, j + 1);
  return 0.5 * (2.0 * M_PI / (double)c->nx) * (rb * rb - ra * ra);
}

static double iround(double x, double u) {
  double f = floor(x);
  return f + ((u < x - f) ? 1.0 : 0.0);
}

static void box_muller(double ua, double ub, double* z0, double* z1) {
  double r = sqrt(-2.0 * log(ua));
  *z0 = r * cos(2.0 * M_PI * ub);
  *z1 = r * sin(2.0 * M_PI * ub);
}

/* Rotational energy of a particle in equilibrium at temperature T with d_r
 * rotational degrees of freedom: T times a Gamma(d_r/2) variate, the sum of
 * d_r/2 (rounded down) exponential variates plus, for odd d_r, half the
 * square of a normal one.  u0: the first uniform (the only one for d_r = 2);
 * the other words come from one extra draw (entity, step, ORC_TAG_ER, idx):
 * further exponentials from its words 0 and 1, the normal from words 2, 3. */
static double rot_energy(const orc_config* c, double T, double u0, uint32_t entity,
                         uint32_t step, uint32_t idx) {
  double g = -log(u0);
  if (c->dr > 2) {
    uint32_t w[4];
    orc_draw(c, entity, step, ORC_TAG_ER, idx, w);
    if (c->dr >= 4) g += -log(orc_u01(w[0]));
    if (c->dr >= 6) g += -log(orc_u01(w[1]));
    if (c->dr % 2 == 1) {
      double z0, z1;
      box_muller(orc_u01(w[2]), orc_u01(w[3]), &z0, &z1);
      g += 0.5 * z0 * z0;
    }
  }
  return T * g;
}

/* ------------------------------------------------------------------------ */
/* Initialisation (DIG step 1, Section 3): particles drawn from the local
 * equilibrium of fields [rho, ux, uy, uz, Tt, Tr] (each an array of ncell).
 * ppc > 0 puts exactly ppc particles in every cell; otherwise the count is
 * Iround(rho V / N_eff) as in the particle-number rule of Section 3.2. */
int64_t orc_init(const orc_config* c, const double* fields, int32_t ppc, int64_t cap,
                 double* x, double* y, double* vx, double* vy, double* vz, double* er,
                 uint32_t* id, int64_t* start) {
  int32_t ncell = c->nx * c->ny;
  const double *rho = fields, *ux = fields + ncell, *uy = fields + 2 * ncell,
               *uz = fields + 3 * ncell, *tt = fields + 4 * ncell, *tr = fields + 5 * ncell;
  int64_t n = 0;
  for (int32_t cell = 0; cell < ncell; ++cell) {
    int64_t cnt;
    if (ppc > 0) {
      cnt = ppc;
    } else {
      uint32_t w[4];
      orc_draw(c, (uint32_t)cell, 0, ORC_TAG_INIT_N, 0, w);
      cnt = (int64_t)iround(rho[cell] * orc_cell_volume_at(c, cell) / c->weight, orc_u01(w[0]));
    }
    if (n + cnt > cap) return -1;
    if (start) start[cell] = n;
    int32_t ix = cell % c->nx, iy = cell / c->nx;
    double st = sqrt(tt[cell]);
    for (int64_t k = 0; k < cnt; ++k, ++n) {
      uint32_t a[4], b[4];
      orc_draw(c, (uint32_t)n, 0, ORC_TAG_INIT, 0, a);
      orc_draw(c, (uint32_t)n, 0, ORC_TAG_INIT, 1, b);
      double z0, z1, z2, z3;
      box_muller(orc_u01(a[2]), orc_u01(a[3]), &z0, &z1);
      box_muller(orc_u01(b[0]), orc_u01(b[1]), &z2, &z3);
      if (c->geometry == ORC_GEOM_ANNULUS) {
        /* uniform over the cell's area: r^2 uniform between the face radii */
        double ra = orc_annulus_face(c, iy), rb = orc_annulus_face(c, iy + 1);
        double r = sqrt(ra * ra + orc_u01(a[0]) * (rb * rb - ra * ra));
        double th = (2.0 * M_PI / (double)c->nx) * ((double)ix + orc_u01(a[1]));
        x[n] = r * cos(th);
        y[n] = r * sin(th);
      } else if (c->geometry == ORC_GEOM_GRADED) {
        /* uniform over the cell between its faces */
        x[n] = c->xf[ix] + orc_u01(a[0]) * (c->xf[ix + 1] - c->xf[ix]);
        y[n] = (c->dim == 2) ? c->yf[iy] + orc_u01(a[1]) * (c->yf[iy + 1] - c->yf[iy]) : 0.0;
      } else {
        x[n] = ix + orc_u01(a[0]);
        y[n] = (c->dim == 2) ? iy + orc_u01(a[1]) : 0.0;
      }
      vx[n] = ux[cell] + st * z0;
      vy[n] = uy[cell] + st * z1;
      vz[n] = uz[cell] + st * z2;
      er[n] = rot_energy(c, tr[cell], orc_u01(b[2]), (uint32_t)n, 0, 0);
      id[n] = (uint32_t)n;
    }
  }
  if (start) start[ncell] = n;
  return n;
}

/* ------------------------------------------------------------------------ */
/* Free flight with fully diffuse (or specular) walls, Section 2.2 and the
 * gas-surface model stated in Section 4.  Wall events are taken in time
 * order; a tie goes to the x face.  Periodic axes wrap at the end. */
#define ORC_MAXHIT 8

static int is_wall(int t) { return t == ORC_BC_DIFFUSE || t == ORC_BC_SPECULAR; }

/* Free flight in an annulus (positions in physical units): reflections at
 * the inner circle, and at the outer circle when it is a wall, in time order;
 * diffuse re-emission about the normal into the gas. */
static int64_t move_annulus(const orc_config* c, int64_t n, double* x, double* y, double* vx,
                            double* vy, double* vz, double* er, const uint32_t* id,
                            uint32_t step) {
  int64_t hits_total = 0;
  double ri = orc_annulus_face(c, 0), ro = orc_annulus_face(c, c->ny);
  int outer_wall = c->bc_type[1] != ORC_BC_FREESTREAM;
  for (int64_t p = 0; p < n; ++p) {
    double t = c->dt;
    for (int hit = 0; hit < ORC_MAXHIT; ++hit) {
      double A = vx[p] * vx[p] + vy[p] * vy[p];
      if (!(A > 0.0)) break;
      double B = x[p] * vx[p] + y[p] * vy[p];
      double R2 = x[p] * x[p] + y[p] * y[p];
      double th = t;
      int face = -1;
      if (B < 0.0) {
        double D = B * B - A * (R2 - ri * ri);
        if (D >= 0.0) {
          double tf = (-B - sqrt(D)) / A;
          if (tf >= 0.0 && tf <= th) { th = tf; face = 0; }
        }
      }
      if (outer_wall) {
        double D = B * B - A * (R2 - ro * ro);
        if (D >= 0.0) {
          double tf = (-B + sqrt(D)) / A;
          if (tf >= 0.0 && tf < th) { th = tf; face = 1; }
        }
      }
      if (face < 0) break;
      x[p] += vx[p] * th;
      y[p] += vy[p] * th;
      t -= th;
      double rr = sqrt(x[p] * x[p] + y[p] * y[p]);
      double sgn = face == 0 ? 1.0 : -1.0;
      double nx = sgn * x[p] / rr, ny = sgn * y[p] / rr;
      double Rw = face == 0 ? ri : ro;
      x[p] = Rw * (x[p] / rr);
      y[p] = Rw * (y[p] / rr);
      if (c->bc_type[face] == ORC_BC_SPECULAR) {
        double vn = vx[p] * nx + vy[p] * ny;
        vx[p] -= 2.0 * vn * nx;
        vy[p] -= 2.0 * vn * ny;
      } else {
        uint32_t w[4];
        orc_draw(c, id[p], step, ORC_TAG_WALL, (uint32_t)hit, w);
        double T = c->bc_T[face];
        double vn = sqrt(-2.0 * T * log(orc_u01(w[0])));
        double z0, z1;
        box_muller(orc_u01(w[1]), orc_u01(w[2]), &z0, &z1);
        double vt = sqrt(T) * z0;
        vx[p] = vn * nx - vt * ny;
        vy[p] = vn * ny + vt * nx;
        vz[p] = sqrt(T) * z1;
        er[p] = rot_energy(c, T, orc_u01(w[3]), id[p], step, (uint32_t)hit);
      }
      ++hits_total;
    }
    x[p] += vx[p] * t;
    y[p] += vy[p] * t;
  }
  return hits_total;
}

int64_t orc_move(const orc_config* c, int64_t n, double* x, double* y, double* vx,
                 double* vy, double* vz, double* er, const uint32_t* id, uint32_t step) {
  if (c->geometry == ORC_GEOM_ANNULUS) return move_annulus(c, n, x, y, vx, vy, vz, er, id, step);
  /* uniform box: grid units; graded box: physical units (the walls at 0 and
   * lx, ly; periodic axes wrap over lx, ly) */
  int graded = c->geometry == ORC_GEOM_GRADED;
  double dx = graded ? 1.0 : c->lx / c->nx, dy = graded ? 1.0 : (c->dim == 2) ? c->ly / c->ny : 1.0;
  double gx = graded ? c->lx : c->nx, gy = graded ? c->ly : c->ny;
  int64_t hits_total = 0;
  for (int64_t p = 0; p < n; ++p) {
    double t = c->dt;
    int hit = 0;
    for (;;) {
      double sx = vx[p] / dx, sy = (c->dim == 2) ? vy[p] / dy : 0.0;
      int face = -1;
      double th = t;
      double xe = x[p] + sx * t;
      if (xe < 0.0 && is_wall(c->bc_type[0])) {
        double tf = (0.0 - x[p]) / sx;
        if (tf <= th) { th = tf; face = 0; }
      } else if (xe > gx && is_wall(c->bc_type[1])) {
        double tf = (gx - x[p]) / sx;
        if (tf <= th) { th = tf; face = 1; }
      }
      if (c->dim == 2) {
        double ye = y[p] + sy * t;
        if (ye < 0.0 && is_wall(c->bc_type[2])) {
          double tf = (0.0 - y[p]) / sy;
          if (face < 0 ? tf <= th : tf < th) { th = tf; face = 2; }
        } else if (ye > gy && is_wall(c->bc_type[3])) {
          double tf = (gy - y[p]) / sy;
          if (face < 0 ? tf <= th : tf < th) { th = tf; face = 3; }
        }
      }
      if (face < 0 || hit >= ORC_MAXHIT) {
        x[p] += sx * t;
        if (c->dim == 2) y[p] += sy * t;
        if (hit >= ORC_MAXHIT) { /* pathological: clamp into the box */
          if (is_wall(c->bc_type[0]) && x[p] < 0.0) x[p] = 0.0;
          if (is_wall(c->bc_type[1]) && x[p] > gx) x[p] = gx;
          if (c->dim == 2) {
            if (is_wall(c->bc_type[2]) && y[p] < 0.0) y[p] = 0.0;
            if (is_wall(c->bc_type[3]) && y[p] > gy) y[p] = gy;
          }
        }
        break;
      }
      /* advance to the wall and put the particle exactly on it */
      x[p] += sx * th;
      if (c->dim == 2) y[p] += sy * th;
      if (face == 0) x[p] = 0.0;
      if (face == 1) x[p] = gx;
      if (face == 2) y[p] = 0.0;
      if (face == 3) y[p] = gy;
      t -= th;
      int axis = face / 2;
      double inward = (face % 2 == 0) ? 1.0 : -1.0;
      if (c->bc_type[face] == ORC_BC_SPECULAR) {
        if (axis == 0) vx[p] = -vx[p]; else vy[p] = -vy[p];
      } else {
        uint32_t w[4];
        orc_draw(c, id[p], step, ORC_TAG_WALL, (uint32_t)hit, w);
        double T = c->bc_T[face];
        double vn = sqrt(-2.0 * T * log(orc_u01(w[0])));
        double z0, z1;
        box_muller(orc_u01(w[1]), orc_u01(w[2]), &z0, &z1);
        double s = sqrt(T);
        if (axis == 0) {
          vx[p] = inward * vn;
          vy[p] = c->bc_U[face][1] + s * z0;
        } else {
          vy[p] = inward * vn;
          vx[p] = c->bc_U[face][0] + s * z0;
        }
        vz[p] = c->bc_U[face][2] + s * z1;
        er[p] = rot_energy(c, T, orc_u01(w[3]), id[p], step, (uint32_t)hit);
      }
      ++hit;
      ++hits_total;
    }
    if (c->bc_type[0] == ORC_BC_PERIODIC) x[p] -= gx * floor(x[p] / gx);
    if (c->dim == 2 && c->bc_type[2] == ORC_BC_PERIODIC) y[p] -= gy * floor(y[p] / gy);
  }
  return hits_total;
}

/* Cell of a grid-unit position: floor, clamped to the last cell when a
 * particle sits exactly on the upper face. */
/* Annulus cell of a position, decided in single precision (the position as
 * stored in FP32): the squared radius against the FP32 squared face radii
 * (rf2, ny + 1 entries), and the angular sector as the unique i with
 * d_i x p >= 0 > d_{i+1} x p for the FP32 face directions
 * d_i = (cos 2 pi i/nx, sin 2 pi i/nx) (dir, nx + 1 pairs, the last equal to
 * the first); the search for it starts at the sector of atan2.  Outside a
 * freestream outer circle: -1. */
static int32_t annulus_cell(const orc_config* c, const float* rf2, const float* dir, double xd,
                            double yd) {
  float x = (float)xd, y = (float)yd;
  float r2 = x * x + y * y;
  if (c->bc_type[1] == ORC_BC_FREESTREAM && r2 >= rf2[c->ny]) return -1;
  int32_t lo = 0, hi = c->ny - 1; /* largest j <= ny - 1 with rf2[j] <= r2, else 0 */
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) / 2;
    if (rf2[mid] <= r2) lo = mid; else hi = mid - 1;
  }
  double th = atan2((double)y, (double)x);
  if (th < 0.0) th += 2.0 * M_PI;
  int32_t i = (int32_t)(th / (2.0 * M_PI) * c->nx);
  if (i < 0) i = 0;
  if (i >= c->nx) i = c->nx - 1;
  for (int32_t it = 0; it <= c->nx; ++it) {
    float c0 = dir[2 * i] * y - dir[2 * i + 1] * x;
    float c1 = dir[2 * i + 2] * y - dir[2 * i + 3] * x;
    if (c0 < 0.0f) i = (i == 0) ? c->nx - 1 : i - 1;
    else if (c1 >= 0.0f) i = (i == c->nx - 1) ? 0 : i + 1;
    else return i + c->nx * lo;
  }
  return -2; /* no sector: cannot happen for nx >= 3 */
}

void orc_cell_index(const orc_config* c, int64_t n, const double* x, const double* y,
                    int32_t* cell) {
  if (c->geometry == ORC_GEOM_ANNULUS) {
    float* rf2 = (float*)malloc(sizeof(float) * (size_t)(c->ny + 1));
    float* dir = (float*)malloc(sizeof(float) * 2 * (size_t)(c->nx + 1));
    for (int32_t j = 0; j <= c->ny; ++j) {
      double r = orc_annulus_face(c, j);
      rf2[j] = (float)(r * r);
    }
    for (int32_t i = 0; i <= c->nx; ++i) {
      double t = 2.0 * M_PI * (double)(i % c->nx) / (double)c->nx;
      dir[2 * i] = (float)cos(t);
      dir[2 * i + 1] = (float)sin(t);
    }
    for (int64_t p = 0; p < n; ++p) cell[p] = annulus_cell(c, rf2, dir, x[p], y[p]);
    free(rf2);
    free(dir);
    return;
  }
  if (c->geometry == ORC_GEOM_GRADED) {
    /* the cell whose faces bracket the position, decided in single
     * precision (the position as stored in FP32) against the FP32 faces:
     * the largest i <= n - 1 with face[i] <= x, else 0 */
    float* fx = (float*)malloc(sizeof(float) * (size_t)(c->nx + 1));
    float* fy = (float*)malloc(sizeof(float) * (size_t)(c->ny + 1));
    for (int32_t i = 0; i <= c->nx; ++i) fx[i] = (float)c->xf[i];
    for (int32_t j = 0; j <= c->ny; ++j) fy[j] = (c->dim == 2) ? (float)c->yf[j] : 0.0f;
    for (int64_t p = 0; p < n; ++p) {
      int32_t ix = 0, iy = 0;
      float xs = (float)x[p];
      for (int32_t i = 1; i < c->nx; ++i)
        if (fx[i] <= xs) ix = i;
      if (c->dim == 2) {
        float ys = (float)y[p];
        for (int32_t j = 1; j < c->ny; ++j)
          if (fy[j] <= ys) iy = j;
      }
      cell[p] = ix + c->nx * iy;
    }
    free(fx);
    free(fy);
    return;
  }
  for (int64_t p = 0; p < n; ++p) {
    int32_t ix = (int32_t)floor(x[p]);
    if (ix < 0) ix = 0;
    if (ix > c->nx - 1) ix = c->nx - 1;
    int32_t iy = 0;
    if (c->dim == 2) {
      iy = (int32_t)floor(y[p]);
      if (iy < 0) iy = 0;
      if (iy > c->ny - 1) iy = c->ny - 1;
    }
    cell[p] = ix + c->nx * iy;
  }
}

/* Stable counting sort: new slot k holds old particle perm[k]; particles of a
 * cell keep their previous relative order. */
void orc_sort(int64_t n, const int32_t* cell, int32_t ncell, int64_t* perm, int64_t* start) {
  int64_t* fill = (int64_t*)calloc((size_t)ncell, sizeof(int64_t));
  for (int32_t c = 0; c <= ncell; ++c) start[c] = 0;
  for (int64_t p = 0; p < n; ++p)
    if (cell[p] >= 0) start[cell[p] + 1] += 1;
  for (int32_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
  for (int64_t p = 0; p < n; ++p) {
    int32_t c = cell[p];
    if (c < 0) continue;
    perm[start[c] + fill[c]] = p;
    fill[c] += 1;
  }
  free(fill);
}

/* ------------------------------------------------------------------------ */
/* Collisions in every cell (Section 2.2): no-time-counter candidate pairs,
 * VHS acceptance, Borgnakke-Larsen exchange with double relaxation, then
 * scattering: isotropic for alpha = 1, otherwise the VSS deflection
 * cos(chi) = 2 u^(1/alpha) - 1 from the pre-collision relative velocity with a
 * uniform azimuth (Bird's rotation of the relative velocity).  The state
 * arrays are in cell order. */
/* Fraction x = er' / E_c given to the internal mode of one particle in an
 * inelastic collision: a Beta(d_r/2, 5/2 - omega) variate (Borgnakke-Larsen
 * with d_r internal degrees of freedom).  d_r = 2: the inverse distribution
 * function, 1 - u^(1/(5/2 - omega)) with the word u.  Otherwise
 * acceptance-rejection with uniform proposals against the density at its
 * mode x* = (a - 1)/(a + b - 2): attempt t takes the words 2(t mod 2) and
 * 2(t mod 2) + 1 of draw (cell, step, ORC_TAG_BL, 64 (2k + p) + t/2) as the
 * proposal x and the test u, accepting when u < (x/x*)^(a-1)
 * ((1-x)/(1-x*))^(b-1), all in FP64; after 64 rejections (probability below
 * 1e-30) x* itself.  k: candidate, p: 0 first particle, 1 second.  The
 * decisions enter the margin. */
static double bl_fraction(const orc_config* c, uint32_t u, uint32_t cell, uint32_t step,
                          int64_t k, int p, double* margin) {
  double b = 2.5 - c->omega;
  if (c->dr == 2) return 1.0 - pow(orc_u01(u), 1.0 / b);
  double a = 0.5 * c->dr;
  double xm = (a - 1.0) / (a + b - 2.0);
  for (uint32_t t = 0; t < 64; ++t) {
    uint32_t w[4];
    orc_draw(c, cell, step, ORC_TAG_BL, (uint32_t)(64 * (2 * k + p)) + t / 2, w);
    double x = orc_u01(w[2 * (t % 2)]);
    double ut = orc_u01(w[2 * (t % 2) + 1]);
    double ratio = pow(x / xm, a - 1.0) * pow((1.0 - x) / (1.0 - xm), b - 1.0);
    if (margin && fabs(ut - ratio) < *margin) *margin = fabs(ut - ratio);
    if (ut < ratio) return x;
  }
  return xm;
}

void orc_collide(const orc_config* c, int32_t ncell, const int64_t* start, double* vx,
                 double* vy, double* vz, double* er, float* sgmax, uint32_t step,
                 orc_collide_stats* st, double* obs_out, double* margin_out) {
  double csig = orc_csigma(c);
  double pin = orc_pinelastic(c);
  double expo = 1.0 - c->omega;            /* sigma g = C (g^2)^(1 - omega) */
  for (int32_t cell = 0; cell < ncell; ++cell) {
    int64_t b = start[cell];
    int64_t N = start[cell + 1] - b;
    double sgm = (double)sgmax[cell];
    double obs = 0.0;
    double margin = INFINITY; /* smallest |u - threshold| of the cell's decisions */
    int64_t ncand = 0;
    if (N >= 2) {
      uint32_t w[4];
      orc_draw(c, (uint32_t)cell, step, ORC_TAG_NCAND, 0, w);
      double xc = 0.5 * (double)N * (double)(N - 1) * c->weight * sgm * c->dt /
                  orc_cell_volume_at(c, cell);
      ncand = (int64_t)iround(xc, orc_u01(w[0]));
    }
    for (int64_t k = 0; k < ncand; ++k) {
      uint32_t r0[4], r1[4], r2[4];
      orc_draw(c, (uint32_t)cell, step, ORC_TAG_COLL, (uint32_t)(3 * k), r0);
      int64_t i = orc_pick(r0[0], (uint32_t)N);
      int64_t j = orc_pick(r0[1], (uint32_t)(N - 1));
      if (j >= i) j += 1;
      i += b;
      j += b;
      double gxv = vx[i] - vx[j], gyv = vy[i] - vy[j], gzv = vz[i] - vz[j];
      double g2 = gxv * gxv + gyv * gyv + gzv * gzv;
      double sg = csig * pow(g2, expo);
      if (sg > obs) obs = sg;
      double ratio = sg / sgm;
      if (st) st->candidates += 1;
      if (ratio > 1.0 && st) st->saturated += 1;
      if (fabs(orc_u01(r0[2]) - ratio) < margin) margin = fabs(orc_u01(r0[2]) - ratio);
      if (!(orc_u01(r0[2]) < ratio)) continue;
      if (st) st->accepted += 1;
      orc_draw(c, (uint32_t)cell, step, ORC_TAG_COLL, (uint32_t)(3 * k + 1), r1);
      orc_draw(c, (uint32_t)cell, step, ORC_TAG_COLL, (uint32_t)(3 * k + 2), r2);
      double et = 0.25 * g2; /* relative translational energy, reduced mass 1/2 */
      double pk = pin;
      if (fabs(orc_u01(r0[3]) - pk) < margin) margin = fabs(orc_u01(r0[3]) - pk);
      if (fabs(orc_u01(r1[1]) - pk) < margin) margin = fabs(orc_u01(r1[1]) - pk);
      /* first picked particle, then the second: Bird's double relaxation */
      if (orc_u01(r0[3]) < pk) {
        double ec = et + er[i];
        double frac = bl_fraction(c, r1[0], (uint32_t)cell, step, k, 0, &margin);
        er[i] = frac * ec;
        et = ec - er[i];
        if (st) st->inelastic += 1;
      }
      if (orc_u01(r1[1]) < pk) {
        double ec = et + er[j];
        double frac = bl_fraction(c, r1[2], (uint32_t)cell, step, k, 1, &margin);
        er[j] = frac * ec;
        et = ec - er[j];
        if (st) st->inelastic += 1;
      }
      double gp = 2.0 * sqrt(et);
      double nx, ny, nz;
      if (c->alpha == 1.0) {
        double ct = 2.0 * orc_u01(r1[3]) - 1.0;
        double stt = sqrt(1.0 - ct * ct);
        double ph = 2.0 * M_PI * orc_u01(r2[0]);
        nx = ct;
        ny = stt * cos(ph);
        nz = stt * sin(ph);
      } else {
        /* VSS: deflection chi about the unit relative velocity u with a
         * uniform azimuth.  The azimuth is measured from the coordinate axis
         * least aligned with u (first on ties), taken as the first of three
         * cyclically ordered components (a, b, c); then
         * n = cc u + sc (se p e_a' + ...) in Bird's rotation form with
         * p = sqrt(b^2 + c^2) >= sqrt(2/3), so the rotation is well
         * conditioned for every direction of u.  The choice of axis is a
         * decision taken in floating point: its gap enters the margin. */
        double gm = sqrt(g2);
        double u3[3] = {gxv / gm, gyv / gm, gzv / gm};
        double m0 = fabs(u3[0]), m1 = fabs(u3[1]), m2 = fabs(u3[2]);
        int k = 0;
        if (m1 < m0) k = 1;
        if (m2 < (k == 0 ? m0 : m1)) k = 2;
        double lo = fabs(u3[k]), next = INFINITY;
        for (int q = 0; q < 3; ++q)
          if (q != k && fabs(u3[q]) < next) next = fabs(u3[q]);
        if (next - lo < margin) margin = next - lo;
        double ua = u3[k], ub = u3[(k + 1) % 3], uc = u3[(k + 2) % 3];
        double cc = 2.0 * pow(orc_u01(r1[3]), 1.0 / c->alpha) - 1.0;
        double sc = sqrt(fmax(0.0, 1.0 - cc * cc));
        double eps = 2.0 * M_PI * orc_u01(r2[0]);
        double se = sin(eps), ce = cos(eps);
        double pp = sqrt(ub * ub + uc * uc);
        double n3[3];
        n3[k] = cc * ua + sc * se * pp;
        n3[(k + 1) % 3] = cc * ub + sc * (ce * uc - ua * ub * se) / pp;
        n3[(k + 2) % 3] = cc * uc - sc * (ce * ub + ua * uc * se) / pp;
        nx = n3[0];
        ny = n3[1];
        nz = n3[2];
      }
      double cx = 0.5 * (vx[i] + vx[j]), cy = 0.5 * (vy[i] + vy[j]), cz = 0.5 * (vz[i] + vz[j]);
      vx[i] = cx + 0.5 * gp * nx;
      vy[i] = cy + 0.5 * gp * ny;
      vz[i] = cz + 0.5 * gp * nz;
      vx[j] = cx - 0.5 * gp * nx;
      vy[j] = cy - 0.5 * gp * ny;
      vz[j] = cz - 0.5 * gp * nz;
    }
    if (obs_out) obs_out[cell] = obs;
    if (margin_out) margin_out[cell] = margin;
    if (obs > sgm) {
      float f = (float)obs;
      if ((double)f < obs) f = nextafterf(f, INFINITY);
      sgmax[cell] = f;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Raw per-cell sums behind the sampled moments of equation DSMC_macroscopic:
 * [N, Sv(3), Svv(xx,yy,zz,xy,xz,yz), Sv|v|^2(3), Ser, Sv er(3)]. */
void orc_sample_sums(int32_t ncell, const int64_t* start, const double* vx,
                     const double* vy, const double* vz, const double* er, double* sums) {
  for (int32_t c = 0; c < ncell; ++c) {
    double* s = sums + 17 * (int64_t)c;
    for (int f = 0; f < 17; ++f) s[f] = 0.0;
    for (int64_t p = start[c]; p < start[c + 1]; ++p) {
      double a = vx[p], b = vy[p], d = vz[p], e = er[p];
      double v2 = a * a + b * b + d * d;
      s[0] += 1.0;
      s[1] += a;
      s[2] += b;
      s[3] += d;
      s[4] += a * a;
      s[5] += b * b;
      s[6] += d * d;
      s[7] += a * b;
      s[8] += a * d;
      s[9] += b * d;
      s[10] += a * v2;
      s[11] += b * v2;
      s[12] += d * v2;
      s[13] += e;
      s[14] += a * e;
      s[15] += b * e;
      s[16] += d * e;
    }
  }
}

/* Sums pooled over nsteps steps -> fields [20][ncell]:
 * rho, ux, uy, uz, Tt, Tr, sxx, syy, szz, sxy, sxz, syz, qtx, qty, qtz,
 * qrx, qry, qrz, T, mean particle count.  Equation DSMC_macroscopic, with the
 * rotational energy per unit mass er = I_r / 2 (so Tr = 2<er>/d_r and
 * q_r = rho <c er>). */
void orc_sums_to_fields(const orc_config* c, int32_t ncell, const double* sums,
                        double nsteps, double* fields) {
  for (int32_t cell = 0; cell < ncell; ++cell) {
    double V = orc_cell_volume_at(c, cell);
    const double* s = sums + 17 * (int64_t)cell;
    double out[20];
    for (int f = 0; f < 20; ++f) out[f] = 0.0;
    double N = s[0];
    if (N > 0.0) {
      double rho = c->weight * N / (V * nsteps);
      double u[3] = {s[1] / N, s[2] / N, s[3] / N};
      /* central second moments <c_i c_j> */
      double m2[3][3];
      m2[0][0] = s[4] / N - u[0] * u[0];
      m2[1][1] = s[5] / N - u[1] * u[1];
      m2[2][2] = s[6] / N - u[2] * u[2];
      m2[0][1] = m2[1][0] = s[7] / N - u[0] * u[1];
      m2[0][2] = m2[2][0] = s[8] / N - u[0] * u[2];
      m2[1][2] = m2[2][1] = s[9] / N - u[1] * u[2];
      double tr = m2[0][0] + m2[1][1] + m2[2][2];
      double Tt = tr / 3.0;
      double Tr = 2.0 * (s[13] / N) / c->dr;
      /* raw second moments <v_i v_j> */
      double r2[3][3] = {{s[4] / N, s[7] / N, s[8] / N},
                         {s[7] / N, s[5] / N, s[9] / N},
                         {s[8] / N, s[9] / N, s[6] / N}};
      double rtr = r2[0][0] + r2[1][1] + r2[2][2];
      double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
      out[0] = rho;
      out[1] = u[0];
      out[2] = u[1];
      out[3] = u[2];
      out[4] = Tt;
      out[5] = Tr;
      out[6] = rho * (m2[0][0] - tr / 3.0);
      out[7] = rho * (m2[1][1] - tr / 3.0);
      out[8] = rho * (m2[2][2] - tr / 3.0);
      out[9] = rho * m2[0][1];
      out[10] = rho * m2[0][2];
      out[11] = rho * m2[1][2];
      for (int i = 0; i < 3; ++i) {
        /* <c_i |c|^2> expanded in raw moments */
        double m3 = s[10 + i] / N;
        double ru = r2[i][0] * u[0] + r2[i][1] * u[1] + r2[i][2] * u[2];
        double cc = m3 - 2.0 * ru - u[i] * rtr + 2.0 * u[i] * uu;
        out[12 + i] = 0.5 * rho * cc;
        out[15 + i] = rho * (s[14 + i] / N - u[i] * (s[13] / N));
      }
      out[18] = (3.0 * Tt + c->dr * Tr) / (3.0 + c->dr);
      out[19] = N / nsteps;
    }
    for (int f = 0; f < 20; ++f) fields[f * (int64_t)ncell + cell] = out[f];
  }
}

/* A point of cell (ix, iy) at fractions (ua, ub) of its extent, in the
 * position units of the geometry (grid units or physical units). */
static void cell_point(const orc_config* c, int32_t ix, int32_t iy, double ua, double ub,
                       double* x, double* y) {
  if (c->geometry == ORC_GEOM_GRADED) {
    *x = c->xf[ix] + ua * (c->xf[ix + 1] - c->xf[ix]);
    *y = (c->dim == 2) ? c->yf[iy] + ub * (c->yf[iy + 1] - c->yf[iy]) : 0.0;
  } else {
    *x = ix + ua;
    *y = (c->dim == 2) ? iy + ub : 0.0;
  }
}

/* ------------------------------------------------------------------------ */
/* DIG particle modification (Section 3.2): target count by Iround, random
 * deletion (partial Fisher-Yates) or cloning of random existing particles at
 * uniform positions, then the linear transform v <- a v + b, er <- c er that
 * makes u, Tt, Tr of the cell equal to the target [rho, ux, uy, uz, Tt, Tr].
 * Returns 0, 1 for an invalid target, 2 when the capacity would overflow; on
 * an error nothing is written. */
int orc_adjust(const orc_config* c, int32_t ncell, const int64_t* start, const double* x,
               const double* y, const double* vx, const double* vy, const double* vz,
               const double* er, const uint32_t* id, const double* target, uint32_t dig_iter,
               uint64_t next_id, int64_t cap, double* ox, double* oy, double* ovx,
               double* ovy, double* ovz, double* oer, uint32_t* oid, int64_t* ostart,
               int64_t* n_out, uint64_t* next_id_out) {
  const double *trho = target, *tux = target + ncell, *tuy = target + 2 * ncell,
               *tuz = target + 3 * ncell, *ttt = target + 4 * ncell, *ttr = target + 5 * ncell;
  /* validation and target counts */
  int64_t* nt = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ncell > 0 ? ncell : 1));
  int64_t total = 0;
  for (int32_t cell = 0; cell < ncell; ++cell) {
    double r = trho[cell];
    if (!isfinite(r) || r < 0.0 || !isfinite(tux[cell]) || !isfinite(tuy[cell]) ||
        !isfinite(tuz[cell]) || !isfinite(ttt[cell]) || !isfinite(ttr[cell]) ||
        (r > 0.0 && (ttt[cell] <= 0.0 || ttr[cell] < 0.0))) {
      free(nt);
      return 1;
    }
    uint32_t w[4];
    orc_draw(c, (uint32_t)cell, dig_iter, ORC_TAG_DIG_N, 0, w);
    nt[cell] = (int64_t)iround(r * orc_cell_volume_at(c, cell) / c->weight, orc_u01(w[0]));
    total += nt[cell];
  }
  if (total > cap) {
    free(nt);
    return 2;
  }
  int64_t pos = 0;
  uint64_t created = 0;
  for (int32_t cell = 0; cell < ncell; ++cell) {
    int64_t b = start[cell], N = start[cell + 1] - b, Nt = nt[cell];
    int32_t ix = cell % c->nx, iy = cell / c->nx;
    int64_t begin = pos;
    ostart[cell] = begin;
    if (Nt <= N) {
      int64_t D = N - Nt;
      int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
      unsigned char* del = (unsigned char*)calloc((size_t)(N > 0 ? N : 1), 1);
      for (int64_t k = 0; k < N; ++k) idx[k] = k;
      for (int64_t k = 0; k < D; ++k) {
        uint32_t w[4];
        orc_draw(c, (uint32_t)cell, dig_iter, ORC_TAG_DIG_DEL, (uint32_t)(k >> 2), w);
        int64_t j = k + orc_pick(w[k & 3], (uint32_t)(N - k));
        int64_t t = idx[k];
        idx[k] = idx[j];
        idx[j] = t;
      }
      for (int64_t k = 0; k < D; ++k) del[idx[k]] = 1;
      for (int64_t k = 0; k < N; ++k) {
        if (del[k]) continue;
        int64_t p = b + k;
        ox[pos] = x[p]; oy[pos] = y[p];
        ovx[pos] = vx[p]; ovy[pos] = vy[p]; ovz[pos] = vz[p];
        oer[pos] = er[p]; oid[pos] = id[p];
        ++pos;
      }
      free(idx);
      free(del);
    } else if (N > 0) {
      for (int64_t k = 0; k < N; ++k) {
        int64_t p = b + k;
        ox[pos] = x[p]; oy[pos] = y[p];
        ovx[pos] = vx[p]; ovy[pos] = vy[p]; ovz[pos] = vz[p];
        oer[pos] = er[p]; oid[pos] = id[p];
        ++pos;
      }
      for (int64_t k = 0; k < Nt - N; ++k) {
        uint32_t w[4];
        orc_draw(c, (uint32_t)cell, dig_iter, ORC_TAG_DIG_SRC, (uint32_t)k, w);
        int64_t src = b + orc_pick(w[0], (uint32_t)N);
        cell_point(c, ix, iy, orc_u01(w[1]), orc_u01(w[2]), &ox[pos], &oy[pos]);
        ovx[pos] = vx[src]; ovy[pos] = vy[src]; ovz[pos] = vz[src];
        oer[pos] = er[src];
        oid[pos] = (uint32_t)(next_id + created);
        ++created;
        ++pos;
      }
    } else {
      /* empty cell: draw the new particles from the target equilibrium */
      double st = sqrt(ttt[cell]);
      for (int64_t k = 0; k < Nt; ++k) {
        uint32_t a[4], bb[4];
        orc_draw(c, (uint32_t)cell, dig_iter, ORC_TAG_DIG_EMPTY, (uint32_t)(2 * k), a);
        orc_draw(c, (uint32_t)cell, dig_iter, ORC_TAG_DIG_EMPTY, (uint32_t)(2 * k + 1), bb);
        double z0, z1, z2, z3;
        box_muller(orc_u01(a[2]), orc_u01(a[3]), &z0, &z1);
        box_muller(orc_u01(bb[0]), orc_u01(bb[1]), &z2, &z3);
        cell_point(c, ix, iy, orc_u01(a[0]), orc_u01(a[1]), &ox[pos], &oy[pos]);
        ovx[pos] = tux[cell] + st * z0;
        ovy[pos] = tuy[cell] + st * z1;
        ovz[pos] = tuz[cell] + st * z2;
        oer[pos] = rot_energy(c, ttr[cell], orc_u01(bb[2]), (uint32_t)(next_id + created), dig_iter,
                              0);
        oid[pos] = (uint32_t)(next_id + created);
        ++created;
        ++pos;
      }
    }
    /* step iii: temporary moments of the current particles; step iv: transform */
    int64_t m = pos - begin;
    if (m > 0) {
      double su[3] = {0, 0, 0}, se = 0.0;
      for (int64_t p = begin; p < pos; ++p) {
        su[0] += ovx[p];
        su[1] += ovy[p];
        su[2] += ovz[p];
        se += oer[p];
      }
      double us[3] = {su[0] / m, su[1] / m, su[2] / m};
      double sc = 0.0;
      for (int64_t p = begin; p < pos; ++p) {
        double a = ovx[p] - us[0], bq = ovy[p] - us[1], d = ovz[p] - us[2];
        sc += a * a + bq * bq + d * d;
      }
      double tts = sc / (3.0 * m);
      double trs = 2.0 * (se / m) / c->dr;
      double a = (m >= 2 && tts > 0.0) ? sqrt(ttt[cell] / tts) : 1.0;
      double bx = tux[cell] - a * us[0], by = tuy[cell] - a * us[1], bz = tuz[cell] - a * us[2];
      double cr = (trs > 0.0) ? ttr[cell] / trs : 1.0;
      for (int64_t p = begin; p < pos; ++p) {
        ovx[p] = a * ovx[p] + bx;
        ovy[p] = a * ovy[p] + by;
        ovz[p] = a * ovz[p] + bz;
        oer[p] = cr * oer[p];
      }
    }
  }
  ostart[ncell] = pos;
  *n_out = pos;
  *next_id_out = next_id + created;
  free(nt);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Closure assembly (Sections 2.3 and 3.1).  fields = [20][ncell] as produced
 * by orc_sums_to_fields.  Outputs hot = [12][ncell] (sigma xx,yy,zz,xy,xz,yz,
 * q_t xyz, q_r xyz) = DSMC - NSF, zeroed where Kn_GLL < kn_ref (mask = 1);
 * cells whose mean particle count (fields row 19) is below n_min also count
 * as in equilibrium: terms extracted from so few samples are noise;
 * nsf (optional) = the NSF terms themselves. */
/* Cell-centre coordinate of cell i along `axis` (graded box), and the
 * distance between the centres of cells a and b = a + 1 (mod n across a
 * periodic axis: the wrapped distance). */
static double centre(const orc_config* c, int axis, int32_t i) {
  const double* f = (axis == 0) ? c->xf : c->yf;
  return 0.5 * (f[i] + f[i + 1]);
}

static double centre_gap(const orc_config* c, int axis, int32_t a, int32_t b) {
  int32_t n = (axis == 0) ? c->nx : c->ny;
  double L = (axis == 0) ? c->lx : c->ly;
  if (c->geometry != ORC_GEOM_GRADED) return L / n;
  double d = centre(c, axis, b) - centre(c, axis, a);
  if (b < a) d += L; /* across the periodic seam */
  (void)n;
  return d;
}

/* Derivative of f along `axis` at cell (ix, iy): the difference of the two
 * neighbours over the distance between their centres (central), the
 * one-sided difference at a wall; across a periodic seam the neighbours
 * wrap.  Exact for linear fields on any grid. */
static double grad_axis(const orc_config* c, const double* f, int32_t ix, int32_t iy, int axis) {
  int32_t n = (axis == 0) ? c->nx : c->ny;
  if (axis == 1 && c->dim == 1) return 0.0;
  if (n < 2) return 0.0;
  int32_t i = (axis == 0) ? ix : iy;
  int periodic = c->bc_type[2 * axis] == ORC_BC_PERIODIC;
#define AT(ii) ((axis == 0) ? f[(ii) + c->nx * iy] : f[ix + c->nx * (ii)])
  if (i > 0 && i < n - 1)
    return (AT(i + 1) - AT(i - 1)) / (centre_gap(c, axis, i - 1, i) + centre_gap(c, axis, i, i + 1));
  if (periodic) {
    int32_t ip = (i + 1) % n, im = (i - 1 + n) % n;
    return (AT(ip) - AT(im)) / (centre_gap(c, axis, im, i) + centre_gap(c, axis, i, ip));
  }
  if (i == 0) return (AT(1) - AT(0)) / centre_gap(c, axis, 0, 1);
  return (AT(n - 1) - AT(n - 2)) / centre_gap(c, axis, n - 2, n - 1);
#undef AT
}

void orc_closure(const orc_config* c, const double* fields, const double A[4], double kn_ref,
                 double n_min, double* hot, uint8_t* mask, double* kn_gll, double* nsf) {
  int32_t ncell = c->nx * c->ny;
  const double *rho = fields, *ux = fields + ncell, *uy = fields + 2 * ncell,
               *uz = fields + 3 * ncell, *tt = fields + 4 * ncell, *tr = fields + 5 * ncell;
  double* speed = (double*)malloc(sizeof(double) * (size_t)ncell);
  for (int32_t k = 0; k < ncell; ++k)
    speed[k] = sqrt(ux[k] * ux[k] + uy[k] * uy[k] + uz[k] * uz[k]);
  double mu0 = orc_mu0(c);
  double det = A[0] * A[3] - A[1] * A[2];
  double gam = (5.0 + c->dr) / (3.0 + c->dr);
  for (int32_t k = 0; k < ncell; ++k) {
    int32_t ix = k % c->nx, iy = k / c->nx;
    double out_nsf[12] = {0};
    double h[12] = {0};
    double kn = INFINITY;
    if (rho[k] > 0.0 && tt[k] > 0.0) {
      double dux[2] = {grad_axis(c, ux, ix, iy, 0), grad_axis(c, ux, ix, iy, 1)};
      double duy[2] = {grad_axis(c, uy, ix, iy, 0), grad_axis(c, uy, ix, iy, 1)};
      double duz[2] = {grad_axis(c, uz, ix, iy, 0), grad_axis(c, uz, ix, iy, 1)};
      double dtt[2] = {grad_axis(c, tt, ix, iy, 0), grad_axis(c, tt, ix, iy, 1)};
      double dtr[2] = {grad_axis(c, tr, ix, iy, 0), grad_axis(c, tr, ix, iy, 1)};
      double drho[2] = {grad_axis(c, rho, ix, iy, 0), grad_axis(c, rho, ix, iy, 1)};
      double dsp[2] = {grad_axis(c, speed, ix, iy, 0), grad_axis(c, speed, ix, iy, 1)};
      double mu = mu0 * pow(tt[k], c->omega);
      double div = dux[0] + duy[1];
      /* equation ns_constitutive (d/dz = 0) */
      out_nsf[0] = -mu * (2.0 * dux[0] - 2.0 / 3.0 * div);
      out_nsf[1] = -mu * (2.0 * duy[1] - 2.0 / 3.0 * div);
      out_nsf[2] = -mu * (0.0 - 2.0 / 3.0 * div);
      out_nsf[3] = -mu * (dux[1] + duy[0]);
      out_nsf[4] = -mu * (duz[0]);
      out_nsf[5] = -mu * (duz[1]);
      /* equation kappa_A: [kt, kr] = mu/2 A^-1 [5, dr] */
      double kt = 0.5 * mu * (A[3] * 5.0 - A[1] * c->dr) / det;
      double kr = 0.5 * mu * (-A[2] * 5.0 + A[0] * c->dr) / det;
      out_nsf[6] = -kt * dtt[0];
      out_nsf[7] = -kt * dtt[1];
      out_nsf[8] = 0.0;
      out_nsf[9] = -kr * dtr[0];
      out_nsf[10] = -kr * dtr[1];
      out_nsf[11] = 0.0;
      /* equation hot_constitutive: HoT = DSMC - NSF */
      for (int f = 0; f < 12; ++f) h[f] = fields[(6 + f) * (int64_t)ncell + k] - out_nsf[f];
      /* gradient-length local Knudsen number, Section 3.1 */
      double lam = mu / (rho[k] * tt[k]) * sqrt(M_PI * tt[k] / 2.0);
      double g = sqrt(drho[0] * drho[0] + drho[1] * drho[1]) / rho[k];
      double us = speed[k];
      double cs = sqrt(gam * tt[k]);
      double gu = sqrt(dsp[0] * dsp[0] + dsp[1] * dsp[1]) / (us > cs ? us : cs);
      double gt = sqrt(dtt[0] * dtt[0] + dtt[1] * dtt[1]) / tt[k];
      double gr = (tr[k] > 0.0) ? sqrt(dtr[0] * dtr[0] + dtr[1] * dtr[1]) / tr[k] : 0.0;
      double m = g;
      if (gu > m) m = gu;
      if (gt > m) m = gt;
      if (gr > m) m = gr;
      kn = lam * m;
    }
    uint8_t eq = (kn < kn_ref || fields[19 * (int64_t)ncell + k] < n_min) ? 1 : 0;
    for (int f = 0; f < 12; ++f) {
      hot[f * (int64_t)ncell + k] = (eq || !(rho[k] > 0.0 && tt[k] > 0.0)) ? 0.0 : h[f];
      if (nsf) nsf[f * (int64_t)ncell + k] = out_nsf[f];
    }
    mask[k] = eq;
    kn_gll[k] = kn;
  }
  free(speed);
}

/* ------------------------------------------------------------------------ */
/* Freestream inflow (open outer circle of an annulus).  The shell between the
 * outer circle and r_res = r_out + (|U| + 6 sqrt(T)) dt is filled every step
 * with freestream gas: Iround(rho A / N_eff) particles per angular sector of
 * area A, positions uniform in the sector (r^2 uniform, angle uniform),
 * Maxwellian velocities about U, exponential rotational energies.  The shell
 * radii are taken as the single-precision squares the kernels hold.  Ids
 * follow next_id in (sector, k) order. */
int64_t orc_inject(const orc_config* c, int64_t n, int64_t cap, double* x, double* y,
                   double* vx, double* vy, double* vz, double* er, uint32_t* id,
                   uint32_t step, uint64_t next_id) {
  const double T = c->bc_T[1];
  const double* U = c->bc_U[1];
  double Um = sqrt(U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
  double rr = c->r_out + (Um + 6.0 * sqrt(T)) * c->dt;
  double dth = 2.0 * M_PI / (double)c->nx;
  double mean = c->bc_rho[1] * (0.5 * dth * (rr * rr - c->r_out * c->r_out)) / c->weight;
  double ro = orc_annulus_face(c, c->ny);
  double ra2 = (double)(float)(ro * ro), rb2 = (double)(float)(rr * rr);
  int64_t total = 0;
  for (int32_t f = 0; f < c->nx; ++f) {
    uint32_t w[4];
    orc_draw(c, (uint32_t)f, step, ORC_TAG_INFLOW, 0, w);
    total += (int64_t)iround(mean, orc_u01(w[0]));
  }
  if (n + total > cap) return -1;
  int64_t q = 0;
  double sT = sqrt(T);
  for (int32_t f = 0; f < c->nx; ++f) {
    uint32_t w[4];
    orc_draw(c, (uint32_t)f, step, ORC_TAG_INFLOW, 0, w);
    int64_t k_f = (int64_t)iround(mean, orc_u01(w[0]));
    for (int64_t k = 0; k < k_f; ++k, ++q) {
      uint32_t a[4], b[4];
      orc_draw(c, (uint32_t)f, step, ORC_TAG_INFLOW, (uint32_t)(1 + 2 * k), a);
      orc_draw(c, (uint32_t)f, step, ORC_TAG_INFLOW, (uint32_t)(2 + 2 * k), b);
      double r = sqrt(ra2 + orc_u01(a[0]) * (rb2 - ra2));
      double th = dth * ((double)f + orc_u01(a[1]));
      double z0, z1, z2, z3;
      box_muller(orc_u01(a[2]), orc_u01(a[3]), &z0, &z1);
      box_muller(orc_u01(b[0]), orc_u01(b[1]), &z2, &z3);
      int64_t p = n + q;
      x[p] = r * cos(th);
      y[p] = r * sin(th);
      vx[p] = U[0] + sT * z0;
      vy[p] = U[1] + sT * z1;
      vz[p] = U[2] + sT * z2;
      er[p] = rot_energy(c, T, orc_u01(b[2]), (uint32_t)(next_id + (uint64_t)q), step, 0);
      id[p] = (uint32_t)(next_id + (uint64_t)q);
    }
  }
  return total;
}
