/* Drives every entry point of the C oracle through a few DSMC steps and one
 * DIG modification on small workloads (a lid-driven cavity, a VSS slab
 * between walls at different temperatures, a cylinder annulus with
 * freestream inflow), for builds with AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Exit status 0 when every case ran; a
 * sanitizer report aborts the program. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "dsmc_oracle.h"

static double* dz(int64_t n) { return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

typedef struct {
  double *x, *y, *vx, *vy, *vz, *er;
  uint32_t* id;
} parts;

static parts alloc_parts(int64_t cap) {
  parts p = {dz(cap), dz(cap), dz(cap), dz(cap), dz(cap), dz(cap),
             (uint32_t*)calloc((size_t)cap, sizeof(uint32_t))};
  return p;
}

static void free_parts(parts* p) {
  free(p->x); free(p->y); free(p->vx); free(p->vy); free(p->vz); free(p->er); free(p->id);
}

static void permute(parts* p, parts* tmp, const int64_t* perm, int64_t n) {
  for (int64_t i = 0; i < n; ++i) {
    const int64_t s = perm[i];
    tmp->x[i] = p->x[s]; tmp->y[i] = p->y[s]; tmp->vx[i] = p->vx[s];
    tmp->vy[i] = p->vy[s]; tmp->vz[i] = p->vz[s]; tmp->er[i] = p->er[s];
    tmp->id[i] = p->id[s];
  }
  parts t = *p;
  *p = *tmp;
  *tmp = t;
}

static orc_config base(int dim, int nx, int ny, double kn) {
  orc_config c;
  memset(&c, 0, sizeof(c));
  c.dim = dim; c.nx = nx; c.ny = ny; c.lx = 1.0; c.ly = 1.0;
  c.geometry = ORC_GEOM_BOX; c.q = 1.0;
  c.kn = kn; c.omega = 0.74; c.alpha = 1.0; c.dr = 2; c.zrot = 5.0;
  c.dt = 0.2 * 0.5167738723407999 * kn;
  for (int f = 0; f < 4; ++f) { c.bc_type[f] = ORC_BC_DIFFUSE; c.bc_T[f] = 1.0; }
  c.seed = 12345; c.instance = 0;
  return c;
}

static double run_case(const char* name, orc_config* c, int ppc, int64_t cap, int nsteps,
                       int open) {
  const int32_t nc = c->nx * c->ny;
  parts p = alloc_parts(cap), tmp = alloc_parts(cap), out = alloc_parts(cap);
  double* fields = dz(6 * (int64_t)nc);
  for (int32_t k = 0; k < nc; ++k) {
    fields[k] = 1.0;
    fields[4 * nc + k] = 1.0;
    fields[5 * nc + k] = 1.0;
  }
  int64_t* start = (int64_t*)calloc((size_t)nc + 1, sizeof(int64_t));
  int64_t* ostart = (int64_t*)calloc((size_t)nc + 1, sizeof(int64_t));
  int64_t* perm = (int64_t*)calloc((size_t)cap, sizeof(int64_t));
  int32_t* cell = (int32_t*)calloc((size_t)cap, sizeof(int32_t));
  float* sgmax = (float*)calloc((size_t)nc, sizeof(float));
  double* obs = dz(nc);
  double* margin = dz(nc);
  double* sums = dz(17 * (int64_t)nc);
  double* acc = dz(17 * (int64_t)nc);
  double* avg = dz(20 * (int64_t)nc);
  double* hot = dz(12 * (int64_t)nc);
  double* nsf = dz(12 * (int64_t)nc);
  double* kn = dz(nc);
  uint8_t* mask = (uint8_t*)calloc((size_t)nc, 1);
  int64_t n = orc_init(c, fields, ppc, cap, p.x, p.y, p.vx, p.vy, p.vz, p.er, p.id, start);
  if (n < 0) { fprintf(stderr, "%s: init over capacity\n", name); exit(2); }
  const double g = 6.0 * sqrt(2.0);
  const float sg0 = (float)(orc_csigma(c) * pow(g, 2.0 - 2.0 * c->omega));
  for (int32_t k = 0; k < nc; ++k) sgmax[k] = sg0;
  uint64_t next_id = (uint64_t)n;
  orc_collide_stats st = {0, 0, 0, 0};
  for (int s = 0; s < nsteps; ++s) {
    if (open) {
      const int64_t k = orc_inject(c, n, cap, p.x, p.y, p.vx, p.vy, p.vz, p.er, p.id,
                                   (uint32_t)s, next_id);
      if (k < 0) { fprintf(stderr, "%s: inflow over capacity\n", name); exit(2); }
      n += k;
      next_id += (uint64_t)k;
    }
    orc_move(c, n, p.x, p.y, p.vx, p.vy, p.vz, p.er, p.id, (uint32_t)s);
    orc_cell_index(c, n, p.x, p.y, cell);
    orc_sort(n, cell, nc, perm, start);
    n = start[nc];
    permute(&p, &tmp, perm, n);
    orc_collide(c, nc, start, p.vx, p.vy, p.vz, p.er, sgmax, (uint32_t)s, &st, obs, margin);
    orc_sample_sums(nc, start, p.vx, p.vy, p.vz, p.er, sums);
    for (int64_t k = 0; k < 17 * (int64_t)nc; ++k) acc[k] += sums[k];
  }
  orc_sums_to_fields(c, nc, acc, (double)nsteps, avg);
  const double A[4] = {2.0 / 3.0, 0.0, 0.0, 5.0 / (7.0 - 2.0 * c->omega)};
  orc_closure(c, avg, A, 0.01, 1.0, hot, mask, kn, nsf);
  int64_t n_out = 0;
  uint64_t nid_out = 0;
  int rc = -1;
  if (c->geometry == ORC_GEOM_BOX) {
    /* target: the average fields with the density raised by 2 % */
    for (int32_t k = 0; k < nc; ++k) avg[k] *= 1.02;
    rc = orc_adjust(c, nc, start, p.x, p.y, p.vx, p.vy, p.vz, p.er, p.id, avg, 1, next_id, cap,
                    out.x, out.y, out.vx, out.vy, out.vz, out.er, out.id, ostart, &n_out,
                    &nid_out);
  }
  double chk = 0.0;
  for (int64_t i = 0; i < n; ++i) chk += p.vx[i] + 0.5 * p.er[i];
  for (int32_t k = 0; k < nc; ++k) chk += hot[k] + kn[k] * (isfinite(kn[k]) ? 1.0 : 0.0);
  printf("%s: %lld particles, %lld candidates, %lld collisions, adjust rc %d -> %lld, "
         "checksum %.6e\n", name, (long long)n, (long long)st.candidates,
         (long long)st.accepted, rc, (long long)n_out, chk);
  free_parts(&p); free_parts(&tmp); free_parts(&out);
  free(fields); free(start); free(ostart); free(perm); free(cell); free(sgmax); free(obs);
  free(margin); free(sums); free(acc); free(avg); free(hot); free(nsf); free(kn); free(mask);
  return chk;
}

int main(void) {
  /* lid-driven cavity, 10 x 10 cells, 30 particles per cell */
  orc_config cav = base(2, 10, 10, 0.05);
  cav.bc_U[3][0] = 0.35;
  cav.weight = 0.01 / 30.0;
  run_case("cavity", &cav, 30, 10 * 10 * 30 * 3, 20, 0);

  /* VSS slab between walls at 1.0 and 1.5, 30 cells, 40 particles per cell */
  orc_config slab = base(1, 30, 1, 0.05);
  slab.alpha = 1.5;
  slab.bc_T[1] = 1.5;
  slab.bc_type[2] = slab.bc_type[3] = ORC_BC_PERIODIC;
  slab.weight = (1.0 / 30.0) / 40.0;
  run_case("vss slab", &slab, 40, 30 * 40 * 3, 20, 0);

  /* cylinder annulus with a Mach 2 freestream entering at the outer circle */
  orc_config ann = base(2, 24, 10, 0.05);
  ann.geometry = ORC_GEOM_ANNULUS;
  ann.r_in = 0.5; ann.r_out = 2.5; ann.q = 1.1;
  ann.bc_type[1] = ORC_BC_FREESTREAM;
  ann.bc_rho[1] = 1.0;
  ann.bc_U[1][0] = 2.0 * sqrt(1.4);
  ann.bc_type[2] = ann.bc_type[3] = ORC_BC_PERIODIC;
  ann.weight = M_PI * (2.5 * 2.5 - 0.5 * 0.5) / 20000.0;
  ann.dt = 0.002;
  run_case("annulus", &ann, 0, 200000, 15, 1);
  return 0;
}
