// Host side of libdig: validation, workspace layout, launches, errors.
#include <math.h>
#include <stddef.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "dig_internal.h"

using namespace dig;

namespace {

thread_local std::string g_err;

dig_status fail(dig_status s, const std::string& m) {
  g_err = m;
  return s;
}

}  // namespace

// Error reporting for the other translation units of the library.
dig_status dig::report(dig_status s, const char* msg) { return fail(s, msg); }

namespace {

dig_status hip_fail(hipError_t e, const char* where) {
  return fail(DIG_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                 \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Internal {
  size_t gfirst, inst_pstart, params, newcount, ccount, newstart, cstart, bsum, lastcnt,
      xsum, stats, rf2, dir, inj_off, done, big_list, big_count, fc32, fc64, vstage;
  int64_t gfirst_len;
};

// Gas constants in paper units (Section 2): mu0 from the Knudsen number, the
// cross-section constant that gives the collision frequency
// 5 (a+1)(a+2) p / (a (5-2w)(7-2w) mu) (30 p / ((5-2w)(7-2w) mu) for VHS,
// a = 1), and P_inelastic of equation P_inelastic.
double vhs_constant(const dig_config& c) {
  const double w = c.omega, a = c.alpha;
  return 15.0 * M_PI /
         (sqrt(2.0) * (5.0 - 2.0 * w) * (7.0 - 2.0 * w) * pow(4.0, 1.0 - w) * tgamma(2.5 - w) *
          c.kn) *
         ((a + 1.0) * (a + 2.0) / (6.0 * a));
}
double p_inelastic(const dig_config& c) {
  const double w = c.omega, a = c.alpha;
  return a * (5.0 - 2.0 * w) * (7.0 - 2.0 * w) / (5.0 * (a + 1.0) * (a + 2.0) * c.zrot);
}
double cell_volume(const dig_config& c) {
  const double dx = c.lx / c.nx;
  return c.dim == 1 ? dx : dx * (c.ly / c.ny);
}

// Annulus geometry: radius of radial face j, FP32 squared face radii,
// angular face directions and cell areas, all from FP64 values.
double annulus_face(const dig_config& c, int j) {
#pragma clang fp contract(off)
  if (c.q == 1.0) return c.r_in + (c.r_out - c.r_in) * (double)j / (double)c.ny;
  return c.r_in + (c.r_out - c.r_in) * (pow(c.q, (double)j) - 1.0) / (pow(c.q, (double)c.ny) - 1.0);
}
double annulus_dtheta(const dig_config& c) { return 2.0 * M_PI / (double)c.nx; }
double annulus_cell_area(const dig_config& c, int j) {
#pragma clang fp contract(off)
  const double ra = annulus_face(c, j), rb = annulus_face(c, j + 1);
  return 0.5 * annulus_dtheta(c) * (rb * rb - ra * ra);
}
// Freestream reservoir shell: outer radius and mean particles per sector.
double reservoir_radius(const dig_config& c) {
#pragma clang fp contract(off)
  const dig_bc& b = c.bc[1];
  const double U = sqrt(b.U[0] * b.U[0] + b.U[1] * b.U[1] + b.U[2] * b.U[2]);
  return c.r_out + (U + 6.0 * sqrt(b.T)) * c.dt;
}
double reservoir_mean(const dig_config& c) {
#pragma clang fp contract(off)
  const double rr = reservoir_radius(c);
  return c.bc[1].rho * (0.5 * annulus_dtheta(c) * (rr * rr - c.r_out * c.r_out)) / c.weight;
}
double default_majorant(const dig_config& c) {
  if (c.sgmax_init > 0.0) return c.sgmax_init;
  return vhs_constant(c) * pow(6.0 * sqrt(2.0 * c.tref), 2.0 - 2.0 * c.omega);
}

// Graded box: what is wrong with the face tables ("" when nothing): each
// table present, finite, strictly increasing (also in FP32, so that every
// cell can be located), from exactly 0 to the domain length.
std::string faces_problem(const dig_config& c) {
  for (int axis = 0; axis < c.dim; ++axis) {
    const double* f = axis == 0 ? c.xfaces : c.yfaces;
    const int n = axis == 0 ? c.nx : c.ny;
    const double L = axis == 0 ? c.lx : c.ly;
    const char* name = axis == 0 ? "xfaces" : "yfaces";
    if (!f) return std::string("graded box needs ") + name;
    if (!(f[0] == 0.0) || !(f[n] == L))
      return std::string(name) + " must run from 0 to the domain length";
    for (int i = 0; i < n; ++i)
      if (!std::isfinite(f[i + 1]) || !(f[i + 1] > f[i]) || !((float)f[i + 1] > (float)f[i]))
        return std::string(name) + " must be finite and strictly increasing (also in FP32)";
  }
  return "";
}

double graded_volume(const dig_config& c, int k) {
  const int i = k % c.nx, j = k / c.nx;
  const double w = c.xfaces[i + 1] - c.xfaces[i];
  return c.dim == 1 ? w : w * (c.yfaces[j + 1] - c.yfaces[j]);
}

// Entries of the face tables of a set of instances (graded boxes only).
int64_t face_entries(const dig_config* cfgs, int32_t n_inst) {
  int64_t n = 0;
  for (int i = 0; i < n_inst; ++i)
    if (cfgs[i].geometry == DIG_GEOM_GRADED)
      n += (cfgs[i].nx + 1) + (cfgs[i].dim == 2 ? cfgs[i].ny + 1 : 0);
  return n;
}

dig_status validate(const dig_config* cfgs, int32_t n_inst, int64_t capacity, int64_t* ncell) {
  if (!cfgs) return fail(DIG_ERR_INVALID, "null config");
  if (n_inst < 1) return fail(DIG_ERR_INVALID, "n_inst must be >= 1");
  if (capacity < 1 || capacity > (int64_t)INT32_MAX - 1024)
    return fail(DIG_ERR_INVALID, "capacity out of range");
  int64_t C = 0;
  for (int i = 0; i < n_inst; ++i) {
    const dig_config& c = cfgs[i];
    const std::string at = "instance " + std::to_string(i) + ": ";
    if (c.dim != 1 && c.dim != 2) return fail(DIG_ERR_INVALID, at + "dim must be 1 or 2");
    bool finite = std::isfinite(c.lx) && std::isfinite(c.ly) && std::isfinite(c.r_in) &&
                  std::isfinite(c.r_out) && std::isfinite(c.q) && std::isfinite(c.kn) &&
                  std::isfinite(c.omega) && std::isfinite(c.alpha) && std::isfinite(c.zrot) &&
                  std::isfinite(c.dt) && std::isfinite(c.weight) &&
                  std::isfinite(c.sgmax_init) && std::isfinite(c.tref);
    for (int f = 0; f < 4; ++f)
      finite = finite && std::isfinite(c.bc[f].T) && std::isfinite(c.bc[f].rho) &&
               std::isfinite(c.bc[f].U[0]) && std::isfinite(c.bc[f].U[1]) &&
               std::isfinite(c.bc[f].U[2]);
    if (!finite) return fail(DIG_ERR_INVALID, at + "every real parameter must be finite");
    if (c.dim != cfgs[0].dim) return fail(DIG_ERR_INVALID, at + "all instances must share dim");
    if (c.nx < 1 || c.ny < 1 || (c.dim == 1 && c.ny != 1))
      return fail(DIG_ERR_INVALID, at + "bad cell counts");
    if (c.geometry != DIG_GEOM_BOX && c.geometry != DIG_GEOM_ANNULUS &&
        c.geometry != DIG_GEOM_GRADED)
      return fail(DIG_ERR_INVALID, at + "unknown geometry");
    if (c.geometry == DIG_GEOM_GRADED) {
      const std::string why = faces_problem(c);
      if (!why.empty()) return fail(DIG_ERR_INVALID, at + why);
    }
    if (c.geometry == DIG_GEOM_ANNULUS) {
      if (c.dim != 2 || n_inst != 1)
        return fail(DIG_ERR_INVALID, at + "an annulus is 2D and alone in its context");
      if (!(c.r_in > 0.0) || !(c.r_out > c.r_in) || !(c.q >= 1.0) || c.nx < 3)
        return fail(DIG_ERR_INVALID, at + "annulus needs 0 < r_in < r_out, q >= 1, nx >= 3");
      const int ti = c.bc[0].type, to = c.bc[1].type;
      if (ti != DIG_BC_DIFFUSE && ti != DIG_BC_SPECULAR)
        return fail(DIG_ERR_INVALID, at + "inner circle must be a wall");
      if (to != DIG_BC_DIFFUSE && to != DIG_BC_SPECULAR && to != DIG_BC_FREESTREAM)
        return fail(DIG_ERR_INVALID, at + "outer circle must be a wall or freestream");
      for (int f = 0; f < 2; ++f)
        if (c.bc[f].type == DIG_BC_DIFFUSE &&
            (!(c.bc[f].T > 0.0) || c.bc[f].U[0] != 0.0 || c.bc[f].U[1] != 0.0))
          return fail(DIG_ERR_INVALID, at + "annulus walls are at rest with T > 0");
      if (to == DIG_BC_FREESTREAM && (!(c.bc[1].T > 0.0) || !(c.bc[1].rho > 0.0)))
        return fail(DIG_ERR_INVALID, at + "freestream needs rho > 0 and T > 0");
    } else if (!(c.lx > 0.0) || (c.dim == 2 && !(c.ly > 0.0))) {
      return fail(DIG_ERR_INVALID, at + "bad domain size");
    }
    if (!(c.kn > 0.0)) return fail(DIG_ERR_INVALID, at + "Kn must be > 0");
    if (!(c.omega >= 0.5 && c.omega <= 1.0))
      return fail(DIG_ERR_INVALID, at + "omega must lie in [0.5, 1]");
    if (!(c.alpha >= 1.0 && c.alpha <= 2.0))
      return fail(DIG_ERR_INVALID, at + "alpha must lie in [1, 2] (1: VHS, else VSS)");
    if (c.dr < 2 || c.dr > 6) return fail(DIG_ERR_INVALID, at + "d_r must lie in [2, 6]");
    if (!(c.zrot > 0.0) || p_inelastic(c) > 1.0)
      return fail(DIG_ERR_INVALID, at + "Z must give P_inelastic <= 1");
    if (!(c.dt > 0.0) || !(c.weight > 0.0))
      return fail(DIG_ERR_INVALID, at + "dt and weight must be > 0");
    if (c.instance_id > 0xFFFFFFu) return fail(DIG_ERR_INVALID, at + "instance_id >= 2^24");
    if (!(c.sgmax_init > 0.0) && !(c.tref > 0.0))
      return fail(DIG_ERR_INVALID, at + "need sgmax_init > 0 or tref > 0");
    const int nf = c.geometry == DIG_GEOM_ANNULUS ? 0 : (c.dim == 1 ? 2 : 4);
    for (int f = 0; f < nf; ++f) {
      const dig_bc& b = c.bc[f];
      if (b.type < 0 || b.type > 2) return fail(DIG_ERR_INVALID, at + "bad bc type for a box");
      if (b.type == DIG_BC_DIFFUSE) {
        if (!(b.T > 0.0)) return fail(DIG_ERR_INVALID, at + "diffuse wall needs T > 0");
        if (b.U[f / 2] != 0.0)
          return fail(DIG_ERR_INVALID, at + "wall velocity must be tangential");
      }
    }
    for (int ax = 0; ax < nf / 2; ++ax)
      if ((c.bc[2 * ax].type == DIG_BC_PERIODIC) != (c.bc[2 * ax + 1].type == DIG_BC_PERIODIC))
        return fail(DIG_ERR_INVALID, at + "periodic faces must come in pairs");
    C += (int64_t)c.nx * c.ny;
  }
  if (C > (int64_t)INT32_MAX / 32) return fail(DIG_ERR_INVALID, "too many cells");
  *ncell = C;
  return DIG_OK;
}

void plan_layout(int64_t cap, int64_t C, int32_t n_inst, int32_t geo_nx, int32_t geo_ny,
                 int64_t nfaces, dig_layout* L, Internal* I) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  memset(L, 0, sizeof(*L));
  L->capacity = cap;
  L->ncell = C;
  for (int b = 0; b < 2; ++b) {
    L->x[b] = take(4 * cap);
    L->y[b] = take(4 * cap);
    L->vx[b] = take(4 * cap);
    L->vy[b] = take(4 * cap);
    L->vz[b] = take(4 * cap);
    L->er[b] = take(4 * cap);
    L->id[b] = take(4 * cap);
  }
  L->cell = take(4 * cap);
  L->rank = take(4 * cap);
  L->perm_raw = take(4 * cap);
  L->perm = take(4 * cap);
  L->start = take(4 * (C + 1));
  L->count = take(4 * C);
  L->sgmax = take(4 * C);
  L->acc = take(8 * 17 * C);
  L->sums = take(8 * 17 * C);
  L->cell_inst = take(4 * C);
  L->cvol = take(8 * C);
  L->counters = take(sizeof(dig_counters));
  I->gfirst_len = cap / kMinGroupParticles + C / kMinGroupCells + 4;
  I->gfirst = take(4 * I->gfirst_len);
  I->inst_pstart = take(8 * (n_inst + 1));
  I->params = take(sizeof(InstParam) * n_inst);
  I->newcount = take(4 * C);
  I->ccount = take(4 * C);
  I->newstart = take(4 * (C + 1));
  I->cstart = take(4 * (C + 1));
  I->bsum = take(8 * (scan_blocks((int)C) + 1));
  I->lastcnt = take(4 * (scan_blocks((int)C) + 1));
  I->xsum = take(8 * 2 * (exscan_chunks((int)C) + 1));
  I->stats = take(sizeof(unsigned long long) * kStatSlots * ST_N);
  I->done = take(sizeof(uint32_t));
  I->big_list = take(4 * I->gfirst_len);
  I->big_count = take(sizeof(uint32_t));
  I->rf2 = take(4 * (geo_ny + 1));
  I->dir = take(8 * (geo_nx + 1));
  I->inj_off = take(4 * (geo_nx + 2));
  I->fc32 = take(4 * nfaces);
  I->fc64 = take(8 * nfaces);
  I->vstage = take(16 * cap);
  L->total_bytes = o;
}

// Table sizes of the annulus geometry (0 for boxes).
int32_t geo_dims(const dig_config* cfgs, int axis) {
  if (cfgs[0].geometry != DIG_GEOM_ANNULUS) return 0;
  return axis == 0 ? cfgs[0].nx : cfgs[0].ny;
}

InstParam make_param(const dig_config& c, int32_t cell0, int32_t face0) {
  InstParam p;
  memset(&p, 0, sizeof(p));
  p.face0 = -1;
  p.dim = c.dim;
  p.nx = c.nx;
  p.ny = c.ny;
  p.cell0 = cell0;
  p.ncell = c.nx * c.ny;
  p.dr = c.dr;
  for (int f = 0; f < 4; ++f) {
    const bool used = c.dim == 2 || f < 2;
    p.bc_type[f] = used ? c.bc[f].type : DIG_BC_PERIODIC;
    p.bc_T[f] = (float)c.bc[f].T;
    for (int k = 0; k < 3; ++k) p.bc_U[f][k] = (float)c.bc[f].U[k];
  }
  p.dx = c.lx / c.nx;
  p.dy = c.dim == 2 ? c.ly / c.ny : 1.0;
  p.inv_dx = (float)(1.0 / p.dx);
  p.inv_dy = (float)(1.0 / p.dy);
  p.gx = (float)c.nx;
  p.gy = (float)c.ny;
  p.dtf = (float)c.dt;
  p.csig = (float)vhs_constant(c);
  p.expo = (float)(1.0 - c.omega);
  p.beta_inv = (float)(1.0 / (2.5 - c.omega));
  p.key0 = (uint32_t)(c.seed & 0xFFFFFFFFu);
  p.key1 = (uint32_t)(c.seed >> 32);
  p.inst = c.instance_id;
  p.pin = p_inelastic(c);
  p.vss = c.alpha != 1.0 ? 1u : 0u;
  p.ainv = 1.0 / c.alpha;
  p.weight = c.weight;
  p.dt = c.dt;
  p.vol = cell_volume(c);
  p.mu0 = c.kn * sqrt(2.0 / M_PI);
  p.omega = c.omega;
  p.geom = (uint32_t)c.geometry;
  if (c.geometry == DIG_GEOM_GRADED) {
    // physical units: unit scale, walls at the domain lengths
    p.face0 = face0;
    p.dx = p.dy = 1.0;
    p.inv_dx = p.inv_dy = 1.0f;
    p.gx = (float)c.lx;
    p.gy = c.dim == 2 ? (float)c.ly : 1.0f;
    p.vol = graded_volume(c, 0);
  }
  if (c.geometry == DIG_GEOM_ANNULUS) {
    const double ri = annulus_face(c, 0), ro = annulus_face(c, c.ny);
    p.rin2 = (float)(ri * ri);
    p.rout2 = (float)(ro * ro);
    p.rin = (float)ri;
    p.rout = (float)ro;
    p.dthf = (float)annulus_dtheta(c);
    // inverse of the face radii r_j = r_in + (r_out - r_in) (q^j - 1) / (q^ny - 1)
    if (c.q == 1.0) {
      p.rk = (float)((double)c.ny / (c.r_out - c.r_in));
      p.rlq = 0.0f;
    } else {
      p.rk = (float)((pow(c.q, (double)c.ny) - 1.0) / (c.r_out - c.r_in));
      p.rlq = (float)(1.0 / log2(c.q));
    }
    p.vol = annulus_cell_area(c, 0);
    p.bc_type[2] = p.bc_type[3] = DIG_BC_PERIODIC;
    if (c.bc[1].type == DIG_BC_FREESTREAM) {
      const double rr = reservoir_radius(c);
      p.res2 = (float)(rr * rr);
      p.res_mean = reservoir_mean(c);
      p.rho_inf = c.bc[1].rho;
    }
  }
  return p;
}

}  // namespace

struct dig_ctx {
  std::vector<dig_config> cfg;
  std::vector<InstParam> params;
  std::vector<int32_t> cell_inst_host;
  std::vector<double> cvol_host;
  std::vector<float> rf2_host, dir_host;
  std::vector<float> fc32_host;   // graded boxes: face tables, instance after instance
  std::vector<double> fc64_host;
  dig_layout L;
  Internal I;
  unsigned char* ws = nullptr;
  int32_t n_inst = 0, ncell = 0, dim = 1;
  int64_t capacity = 0, n_host = 0;
  int cur = 0;
  int32_t T = 1024, Gc = 64, Lp = 1536;
  int32_t Lbig = 0;  // particle stage of the oversize-group collide
  bool has_state = false;
  int phase = 0;  // 0: ready to move, 1: moved (cells reserved), 2: sorted
  int32_t seq_max = kSeqMaxDefault;
  int32_t big_kib = (int32_t)(kBigLdsBytes / 1024);  // oversize-group stage budget
  int32_t inj_sectors = 0;  // angular sectors with freestream inflow
  // event pairs (start, stop) bracketing launches, with the kernel kind of each
  struct EvPool {
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;
    size_t used = 0;
  };
  // captured step graphs, keyed by what the captured launches depend on
  struct Graph {
    int32_t nsteps, cur, T, Gc, seq, big;
    int64_t n;
    hipGraph_t g;
    hipGraphExec_t x;
    hipEvent_t done;  // recorded after the latest launch of this graph
  };
  std::vector<Graph> graphs;
  hipStream_t cap = nullptr;  // capture stream, default priority
  // event profiling
  bool prof = false;
  uint32_t prof_mask = ~0u;  // kernel kinds timed while profiling
  int32_t prof_every = 1;     // time one launch of a kind in every prof_every
  int64_t prof_seen[DIG_NKERNELS] = {};
  EvPool eager;
  double prof_ms[DIG_NKERNELS] = {0};
  int64_t prof_n[DIG_NKERNELS] = {0};
};

namespace {

StepArgs args(const dig_ctx* c) {
  StepArgs a;
  memset(&a, 0, sizeof(a));
  unsigned char* w = c->ws;
  const dig_layout& L = c->L;
  const int s = c->cur, d = 1 - c->cur;
  a.A = DevState{(float*)(w + L.x[s]), (float*)(w + L.y[s]), (float*)(w + L.vx[s]),
                 (float*)(w + L.vy[s]), (float*)(w + L.vz[s]), (float*)(w + L.er[s]),
                 (uint32_t*)(w + L.id[s])};
  a.B = DevState{(float*)(w + L.x[d]), (float*)(w + L.y[d]), (float*)(w + L.vx[d]),
                 (float*)(w + L.vy[d]), (float*)(w + L.vz[d]), (float*)(w + L.er[d]),
                 (uint32_t*)(w + L.id[d])};
  a.cell = (int32_t*)(w + L.cell);
  a.rank = (int32_t*)(w + L.rank);
  a.perm_raw = (int32_t*)(w + L.perm_raw);
  a.perm = (int32_t*)(w + L.perm);
  a.start = (int32_t*)(w + L.start);
  a.count = (int32_t*)(w + L.count);
  a.cell_inst = (int32_t*)(w + L.cell_inst);
  a.gfirst = (int32_t*)(w + c->I.gfirst);
  a.sgmax = (float*)(w + L.sgmax);
  a.acc = (double*)(w + L.acc);
  a.sums = (double*)(w + L.sums);
  a.inst_pstart = (int64_t*)(w + c->I.inst_pstart);
  a.bsum = (int64_t*)(w + c->I.bsum);
  a.lastcnt = (int32_t*)(w + c->I.lastcnt);
  a.stats = (unsigned long long*)(w + c->I.stats);
  a.done = (uint32_t*)(w + c->I.done);
  a.big_list = (int32_t*)(w + c->I.big_list);
  a.big_count = (uint32_t*)(w + c->I.big_count);
  a.lds_big = c->Lbig;
  a.ext_any = 0;
  a.dr_any = 0;
  for (const InstParam& q : c->params) {
    a.ext_any |= (q.vss || q.dr != 2) ? 1 : 0;
    a.dr_any |= q.dr != 2 ? 1 : 0;
  }
  a.big_runs = big_run_slots(c->Lbig, c->Gc);
  a.params = (const InstParam*)(w + c->I.params);
  a.ctr = (dig_counters*)(w + L.counters);
  a.n_inst = c->n_inst;
  a.ncell = c->ncell;
  a.dim = c->dim;
  a.group_particles = c->T;
  a.group_cells = c->Gc;
  a.lds_particles = c->Lp;
  a.seq_max = c->seq_max;
  // launch bound for the particle kernels (they read the exact count on the
  // device): the host count rounded up to a 1/64 share of the capacity, so
  // that the small count changes of a DIG adjustment keep captured graphs valid
  const int64_t q = std::max<int64_t>(4096, c->capacity / 64);
  a.n_upper = std::max<int64_t>(1, std::min<int64_t>(c->capacity, (c->n_host + q - 1) / q * q));
  // with inflow and outflow the count changes every step on the device
  if (c->inj_sectors > 0) a.n_upper = c->capacity;
  a.cvol = (const double*)(w + L.cvol);
  a.fc32 = (const float*)(w + c->I.fc32);
  a.fc64 = (const double*)(w + c->I.fc64);
  a.vstage = (float4*)(w + c->I.vstage);
  a.rf2 = (const float*)(w + c->I.rf2);
  a.dir = (const float2*)(w + c->I.dir);
  a.inj_off = (int32_t*)(w + c->I.inj_off);
  a.capacity = c->capacity;
  a.inj_sectors = c->inj_sectors;
  return a;
}

// Timing-only events: no system-scope fence at record (its cache write-back
// and invalidation would stall the next kernel for microseconds); the
// durations are read after a stream synchronisation.
hipError_t pool_grow(dig_ctx::EvPool* p, size_t pairs) {
  while (p->kind.size() < pairs) {
    hipEvent_t a, b;
    hipError_t e = hipEventCreateWithFlags(&a, hipEventDisableSystemFence);
    if (e != hipSuccess) return e;
    e = hipEventCreateWithFlags(&b, hipEventDisableSystemFence);
    if (e != hipSuccess) return e;
    p->ev.push_back(a);
    p->ev.push_back(b);
    p->kind.push_back(0);
  }
  return hipSuccess;
}

void pool_free(dig_ctx::EvPool* p) {
  for (auto& e : p->ev) (void)hipEventDestroy(e);
  p->ev.clear();
  p->kind.clear();
  p->used = 0;
}

hipError_t pool_fold(dig_ctx* c, const dig_ctx::EvPool& p) {
  for (size_t k = 0; k < p.used; ++k) {
    float ms = 0.0f;
    hipError_t e = hipEventElapsedTime(&ms, p.ev[2 * k], p.ev[2 * k + 1]);
    if (e != hipSuccess) return e;
    c->prof_ms[p.kind[k]] += ms;
    c->prof_n[p.kind[k]] += 1;
  }
  return hipSuccess;
}

// Folds the recorded event pairs into the per-kernel totals; synchronises
// `s`, where all of them were enqueued.
hipError_t prof_fold(dig_ctx* c, hipStream_t s) {
  if (c->eager.used == 0) return hipSuccess;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  e = pool_fold(c, c->eager);
  c->eager.used = 0;
  return e;
}

// Runs one launch, bracketed by events when profiling is on.
template <class F>
hipError_t timed(dig_ctx* c, int kind, hipStream_t s, F&& launch) {
  if (!c->prof || !((c->prof_mask >> kind) & 1u)) return launch();
  if (c->prof_seen[kind]++ % c->prof_every != 0) return launch();
  dig_ctx::EvPool* p = &c->eager;
  if (p->used == p->kind.size()) {
    hipError_t e = prof_fold(c, s);
    if (e != hipSuccess) return e;
  }
  const size_t k = p->used++;
  p->kind[k] = kind;
  hipError_t e = hipEventRecord(p->ev[2 * k], s);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  return hipEventRecord(p->ev[2 * k + 1], s);
}

__global__ void k_counts_from_start(const int32_t* start, int32_t* counts, int C) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < C) counts[c] = start[c + 1] - start[c];
}

__global__ void k_add_i64(int64_t* p, int64_t v) { *p += v; }
__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }
__global__ void k_clear_err(uint32_t* p, uint32_t bits) { *p &= ~bits; }

dig_status check_ctx(dig_ctx* c) {
  if (!c) return fail(DIG_ERR_INVALID, "null context");
  return DIG_OK;
}

// Largest LDS particle stage for group size T: the group target plus room for
// its last cell, within 48 KiB of LDS; larger groups go to the oversize-group
// collide.  At least 512 (the collide keeps its candidate words in the stage's
// source arrays).
int32_t lds_particles_for(int32_t T, int32_t Gc) {
  int32_t Lp = T + 256;
  while (Lp > 512 && collide_lds_bytes(Lp, Gc) > 48 * 1024) Lp -= 256;
  return Lp;
}

// Stage of the oversize-group collide: the largest multiple of 256 particles
// whose layout fits its LDS budget (about 5900 particles); 0 if none does.
int32_t lds_big_for(int32_t Gc, int32_t kib) {
  const size_t budget = (size_t)kib * 1024;
  int32_t Lb = (int32_t)(budget / 24 / 256 * 256);
  while (Lb > 0 && !big_stage_fits(Lb, Gc, budget)) Lb -= 256;
  return Lb;
}

dig_status check_tuning(int32_t T, int32_t Gc, int32_t seq, int32_t big) {
  if (big < (int32_t)(kBigLdsBytes / 1024) || big > (int32_t)(kBigLdsMax / 1024))
    return fail(DIG_ERR_INVALID, "big_stage_kib must lie in [38, 150]");
  if (T < kMinGroupParticles || T > 16384)
    return fail(DIG_ERR_INVALID, "group_particles must lie in [256, 16384]");
  if (Gc < kMinGroupCells || Gc > 256)
    return fail(DIG_ERR_INVALID, "group_cells must lie in [32, 256]");
  if (seq < 0 || seq > 4096) return fail(DIG_ERR_INVALID, "seq_max must lie in [0, 4096]");
  return DIG_OK;
}

void apply_tuning(dig_ctx* c, int32_t T, int32_t Gc, int32_t seq, int32_t big) {
  c->big_kib = big;
  c->T = T;
  c->Gc = Gc;
  c->seq_max = seq;
  c->Lp = lds_particles_for(T, Gc);
  c->Lbig = lds_big_for(Gc, big);
}

// Destroys the captured graphs.  A replay may still be in flight on the
// stream it was launched on: wait for each graph's own completion event (not
// for the whole device).
void drop_graphs(dig_ctx* c) {
  for (auto& g : c->graphs) {
    (void)hipEventSynchronize(g.done);
    (void)hipEventDestroy(g.done);
    (void)hipGraphExecDestroy(g.x);
    (void)hipGraphDestroy(g.g);
  }
  c->graphs.clear();
}

// Stages must run in order (move, sort, collide): the sort consumes the
// reservations of the move and the collide consumes the sorted permutation.
dig_status run_stages(dig_ctx* c, int mask, hipStream_t s) {
  StepArgs a = args(c);
  if (mask & DIG_STAGE_MOVE) {
    if (c->phase != 0) return fail(DIG_ERR_STATE, "move needs a completed previous step");
    if (c->inj_sectors > 0) HIP_TRY(launch_inject(a, s));
    HIP_TRY(timed(c, DIG_K_MOVE, s, [&] { return launch_move(a, s); }));
    c->phase = 1;
  }
  // When the sort and the collide run together, the collide kernels put each
  // cell group in stable order themselves (k_collide the groups that fit its
  // stage, k_collide_big the others); the sort stage alone orders the whole
  // permutation in a pass of its own so that it can be inspected.
  const bool fused = (mask & DIG_STAGE_SORT) && (mask & DIG_STAGE_COLLIDE);
  if (mask & DIG_STAGE_SORT) {
    if (c->phase != 1) return fail(DIG_ERR_STATE, "sort needs the move stage first");
    HIP_TRY(timed(c, DIG_K_SCAN, s, [&] { return launch_scan(a, a.count, false, s); }));
    HIP_TRY(timed(c, DIG_K_PLACE, s, [&] { return launch_place(a, s); }));
    if (!fused) HIP_TRY(timed(c, DIG_K_ORDER, s, [&] { return launch_order(a, s); }));
    c->phase = 2;
  }
  if (mask & DIG_STAGE_COLLIDE) {
    if (c->phase != 2) return fail(DIG_ERR_STATE, "collide needs the sort stage first");
    HIP_TRY(timed(c, DIG_K_COLLIDE, s,
                  [&] { return launch_collide(a, true, true, true, fused, s); }));
    c->cur ^= 1;
    c->phase = 0;
  }
  return DIG_OK;
}

}  // namespace

extern "C" {

const char* dig_last_error(void) { return g_err.c_str(); }

dig_status dig_plan(const dig_config* cfgs, int32_t n_inst, int64_t capacity, dig_layout* out) {
  if (!out) return fail(DIG_ERR_INVALID, "null layout");
  int64_t C = 0;
  dig_status st = validate(cfgs, n_inst, capacity, &C);
  if (st != DIG_OK) return st;
  Internal I;
  plan_layout(capacity, C, n_inst, geo_dims(cfgs, 0), geo_dims(cfgs, 1),
              face_entries(cfgs, n_inst), out, &I);
  return DIG_OK;
}

dig_status dsmc_create(const dig_config* cfgs, int32_t n_inst, int64_t capacity, void* ws,
                       size_t ws_bytes, int32_t group_particles, int32_t group_cells,
                       dig_stream_t stream, dig_ctx** out) {
  if (!out) return fail(DIG_ERR_INVALID, "null output");
  *out = nullptr;
  int64_t C = 0;
  dig_status st = validate(cfgs, n_inst, capacity, &C);
  if (st != DIG_OK) return st;
  if (!ws) return fail(DIG_ERR_INVALID, "null workspace");
  if (((uintptr_t)ws) % kAlign) return fail(DIG_ERR_INVALID, "workspace not 256-byte aligned");
  const int32_t T = group_particles > 0 ? group_particles : 1024;
  const int32_t Gc = group_cells > 0 ? group_cells : 64;
  st = check_tuning(T, Gc, kSeqMaxDefault, (int32_t)(kBigLdsBytes / 1024));
  if (st != DIG_OK) return st;
  dig_ctx* c = new dig_ctx;
  c->cfg.assign(cfgs, cfgs + n_inst);
  c->n_inst = n_inst;
  c->ncell = (int32_t)C;
  c->dim = cfgs[0].dim;
  c->capacity = capacity;
  c->n_host = capacity;
  apply_tuning(c, T, Gc, kSeqMaxDefault, (int32_t)(kBigLdsBytes / 1024));
  plan_layout(capacity, C, n_inst, geo_dims(cfgs, 0), geo_dims(cfgs, 1),
              face_entries(cfgs, n_inst), &c->L, &c->I);
  if (ws_bytes < c->L.total_bytes) {
    const std::string msg =
        "workspace too small: need " + std::to_string(c->L.total_bytes) + " bytes";
    delete c;
    return fail(DIG_ERR_INVALID, msg);
  }
  c->ws = (unsigned char*)ws;
  {
    // dynamic LDS allowance of the oversize-group collide
    const hipError_t e = collide_setup();
    if (e != hipSuccess) {
      delete c;
      return hip_fail(e, "collide_setup");
    }
  }
  int32_t cell0 = 0;
  for (int i = 0; i < n_inst; ++i) {
    const dig_config& g = cfgs[i];
    const int32_t face0 = (int32_t)c->fc64_host.size();
    c->params.push_back(make_param(g, cell0, face0));
    for (int k = 0; k < g.nx * g.ny; ++k) {
      c->cell_inst_host.push_back(i);
      c->cvol_host.push_back(g.geometry == DIG_GEOM_ANNULUS  ? annulus_cell_area(g, k / g.nx)
                             : g.geometry == DIG_GEOM_GRADED ? graded_volume(g, k)
                                                             : cell_volume(g));
    }
    if (g.geometry == DIG_GEOM_GRADED) {
      // the context keeps its own copy of the face tables
      for (int k = 0; k <= g.nx; ++k) c->fc64_host.push_back(g.xfaces[k]);
      if (g.dim == 2)
        for (int k = 0; k <= g.ny; ++k) c->fc64_host.push_back(g.yfaces[k]);
    }
    cell0 += g.nx * g.ny;
  }
  for (double f : c->fc64_host) c->fc32_host.push_back((float)f);
  for (int i = 0; i < n_inst; ++i) {
    dig_config& g = c->cfg[i];
    if (g.geometry == DIG_GEOM_GRADED) {
      g.xfaces = c->fc64_host.data() + c->params[i].face0;
      g.yfaces = g.dim == 2 ? g.xfaces + g.nx + 1 : nullptr;
    } else {
      g.xfaces = g.yfaces = nullptr;
    }
  }
  if (cfgs[0].geometry == DIG_GEOM_ANNULUS) {
    const dig_config& g = cfgs[0];
    for (int j = 0; j <= g.ny; ++j) {
      const double r = annulus_face(g, j);
      c->rf2_host.push_back((float)(r * r));
    }
    for (int i = 0; i <= g.nx; ++i) {
      const double th = 2.0 * M_PI * (double)(i % g.nx) / (double)g.nx;
      c->dir_host.push_back((float)cos(th));
      c->dir_host.push_back((float)sin(th));
    }
    if (g.bc[1].type == DIG_BC_FREESTREAM) c->inj_sectors = g.nx;
  }
  hipStream_t s = (hipStream_t)stream;
  StepArgs a = args(c);
  hipError_t e = hipMemcpyAsync((void*)a.params, c->params.data(),
                                sizeof(InstParam) * n_inst, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(a.cell_inst, c->cell_inst_host.data(), 4 * C, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync((void*)a.cvol, c->cvol_host.data(), 8 * C, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !c->rf2_host.empty())
    e = hipMemcpyAsync((void*)a.rf2, c->rf2_host.data(), 4 * c->rf2_host.size(),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !c->dir_host.empty())
    e = hipMemcpyAsync((void*)a.dir, c->dir_host.data(), 4 * c->dir_host.size(),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !c->fc64_host.empty())
    e = hipMemcpyAsync((void*)a.fc64, c->fc64_host.data(), 8 * c->fc64_host.size(),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !c->fc32_host.empty())
    e = hipMemcpyAsync((void*)a.fc32, c->fc32_host.data(), 4 * c->fc32_host.size(),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_fill_i32(a.count, C, 0, s);
  if (e == hipSuccess) e = launch_fill_i32((int32_t*)a.done, 1, 0, s);
  if (e == hipSuccess) e = launch_fill_i32((int32_t*)a.big_count, 1, 0, s);
  if (e == hipSuccess) e = launch_fill_f64(a.acc, 17 * C, 0.0, s);
  for (int i = 0; i < n_inst && e == hipSuccess; ++i)
    e = launch_fill_f32(a.sgmax + c->params[i].cell0, c->params[i].ncell,
                        (float)default_majorant(cfgs[i]), s);
  if (e == hipSuccess) e = launch_set_counters(a.ctr, 0, 0, 0, true, s);
  if (e == hipSuccess)
    e = launch_fill_f64((double*)a.stats, (int64_t)kStatSlots * ST_N, 0.0, s);
  // the host copies above read host vectors owned by the context: wait for them
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "dsmc_create");
  }
  *out = c;
  return DIG_OK;
}

dig_status dsmc_init(dig_ctx* c, const double* fields, int32_t ppc, dig_stream_t stream) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (!fields) return fail(DIG_ERR_INVALID, "null fields");
  if (ppc < 0) return fail(DIG_ERR_INVALID, "ppc must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  c->cur = 0;
  c->phase = 0;
  c->n_host = c->capacity;
  StepArgs a = args(c);
  HIP_TRY(launch_set_counters(a.ctr, 0, 0, 0, true, s));
  HIP_TRY(launch_fill_f64((double*)a.stats, (int64_t)kStatSlots * ST_N, 0.0, s));
  HIP_TRY(launch_init(a, fields, ppc, s, 0));
  HIP_TRY(launch_scan(a, a.count, true, s));
  int32_t total = 0;
  HIP_TRY(hipMemcpyAsync(&total, a.start + c->ncell, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (total > c->capacity) {
    c->has_state = false;
    return fail(DIG_ERR_CAPACITY, "initial particle count " + std::to_string(total) +
                                      " exceeds capacity");
  }
  c->n_host = total;
  a = args(c);
  HIP_TRY(launch_init(a, fields, ppc, s, 1));
  HIP_TRY(launch_set_counters(a.ctr, total, 0, total, false, s));
  c->has_state = true;
  return DIG_OK;
}

dig_status dsmc_inject(dig_ctx* c, int64_t n, int64_t step, int64_t next_id,
                       dig_stream_t stream) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (n < 0 || n > c->capacity) return fail(DIG_ERR_CAPACITY, "n outside [0, capacity]");
  hipStream_t s = (hipStream_t)stream;
  c->n_host = n > 0 ? n : 1;
  c->phase = 0;
  StepArgs a = args(c);
  hipLaunchKernelGGL(k_counts_from_start, dim3((c->ncell + 255) / 256), dim3(256), 0, s,
                     a.start, a.count, c->ncell);
  HIP_TRY(hipGetLastError());
  HIP_TRY(launch_scan(a, a.count, false, s));
  HIP_TRY(launch_set_counters(a.ctr, n, step, next_id, false, s));
  c->n_host = n;
  c->has_state = true;
  return DIG_OK;
}

dig_status dsmc_step(dig_ctx* c, int32_t nsteps, dig_stream_t stream) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (!c->has_state) return fail(DIG_ERR_STATE, "no particle state (call dsmc_init)");
  if (nsteps < 0) return fail(DIG_ERR_INVALID, "nsteps < 0");
  if (c->phase != 0) return fail(DIG_ERR_STATE, "a partial step is pending (dsmc_stage)");
  for (int k = 0; k < nsteps; ++k) {
    dig_status st = run_stages(c, DIG_STAGE_ALL, (hipStream_t)stream);
    if (st != DIG_OK) return st;
  }
  return DIG_OK;
}

dig_status dsmc_stage(dig_ctx* c, int32_t mask, dig_stream_t stream) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (!c->has_state) return fail(DIG_ERR_STATE, "no particle state");
  if (mask & ~DIG_STAGE_ALL) return fail(DIG_ERR_INVALID, "bad stage mask");
  return run_stages(c, mask, (hipStream_t)stream);
}

dig_status dsmc_sample(dig_ctx* c, int32_t mode, double* out, dig_stream_t stream) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  StepArgs a = args(c);
  if (mode == DIG_SAMPLE_RESET) {
    HIP_TRY(launch_fill_f64(a.acc, 17 * (int64_t)c->ncell, 0.0, s));
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, &a.ctr->nsamp, (int64_t)0);
    HIP_TRY(hipGetLastError());
    return DIG_OK;
  }
  if (!out) return fail(DIG_ERR_INVALID, "null output");
  if (mode == DIG_SAMPLE_INSTANT) {
    if (!c->has_state) return fail(DIG_ERR_STATE, "no particle state");
    HIP_TRY(timed(c, DIG_K_SAMPLE, s, [&] { return launch_sample_state(a, s); }));
    HIP_TRY(launch_convert(a, a.sums, false, out, s));
    return DIG_OK;
  }
  if (mode == DIG_SAMPLE_AVERAGE) {
    HIP_TRY(launch_convert(a, a.acc, true, out, s));
    return DIG_OK;
  }
  return fail(DIG_ERR_INVALID, "bad sample mode");
}

dig_status dig_adjust(dig_ctx* c, const double* target, uint32_t iter, dig_stream_t stream) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (!target) return fail(DIG_ERR_INVALID, "null target");
  if (c->n_inst != 1) return fail(DIG_ERR_INVALID, "dig_adjust needs a single-instance context");
  if (c->cfg[0].geometry == DIG_GEOM_ANNULUS)
    return fail(DIG_ERR_INVALID, "dig_adjust supports boxes only (uniform or graded)");
  if (!c->has_state) return fail(DIG_ERR_STATE, "no particle state");
  if (c->phase != 0) return fail(DIG_ERR_STATE, "a partial step is pending (dsmc_stage)");
  hipStream_t s = (hipStream_t)stream;
  StepArgs a = args(c);
  unsigned char* w = c->ws;
  int32_t* newcount = (int32_t*)(w + c->I.newcount);
  int32_t* ccount = (int32_t*)(w + c->I.ccount);
  int32_t* newstart = (int32_t*)(w + c->I.newstart);
  int32_t* cstart = (int32_t*)(w + c->I.cstart);
  HIP_TRY(launch_adjust_count(a, target, iter, newcount, ccount, s));
  HIP_TRY(launch_exscan2(newcount, newstart, ccount, cstart, c->ncell,
                         (int64_t*)(w + c->I.xsum), s));
  int32_t tot[2] = {0, 0};
  uint32_t err = 0;
  HIP_TRY(hipMemcpyAsync(&tot[0], newstart + c->ncell, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&tot[1], cstart + c->ncell, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&err, &a.ctr->err, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (err & DIG_EBIT_TARGET) {
    hipLaunchKernelGGL(k_clear_err, dim3(1), dim3(1), 0, s, &a.ctr->err,
                       (uint32_t)DIG_EBIT_TARGET);
    HIP_TRY(hipGetLastError());
    return fail(DIG_ERR_NUMERIC, "dig_adjust: non-finite or non-positive target");
  }
  if (tot[0] > c->capacity)
    return fail(DIG_ERR_CAPACITY, "dig_adjust: " + std::to_string(tot[0]) +
                                      " particles exceed the capacity");
  HIP_TRY(timed(c, DIG_K_ADJUST, s,
                [&] { return launch_adjust_build(a, target, iter, newstart, cstart, s); }));
  c->cur ^= 1;
  c->n_host = tot[0] > 0 ? tot[0] : 1;
  a = args(c);
  HIP_TRY(launch_scan(a, newcount, true, s));
  hipLaunchKernelGGL(k_add_i64, dim3(1), dim3(1), 0, s, &a.ctr->next_id, (int64_t)tot[1]);
  HIP_TRY(hipGetLastError());
  c->n_host = tot[0];
  return DIG_OK;
}

dig_status closure_assemble(dig_ctx* c, const double* fields, const double* A, double kn_ref,
                            double n_min, double* hot, uint8_t* mask, double* kngll,
                            double* nsf, dig_stream_t stream) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (!fields || !A || !hot || !mask || !kngll) return fail(DIG_ERR_INVALID, "null argument");
  const double det = A[0] * A[3] - A[1] * A[2];
  if (!(fabs(det) > 0.0)) return fail(DIG_ERR_INVALID, "singular relaxation matrix A");
  if (!(n_min >= 0.0)) return fail(DIG_ERR_INVALID, "n_min must be >= 0");
  for (const auto& g : c->cfg)
    if (g.geometry == DIG_GEOM_ANNULUS)
      return fail(DIG_ERR_INVALID, "closure_assemble supports boxes only (uniform or graded)");
  StepArgs a = args(c);
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(timed(c, DIG_K_CLOSURE, s, [&] {
    return launch_closure(a, fields, A[0], A[1], A[2], A[3], kn_ref, n_min, hot, mask, kngll,
                          nsf, s);
  }));
  return DIG_OK;
}

static dig_status scaling_of(const dig_mlp_scaling* in, MlpScale* out) {
  if (!in) return fail(DIG_ERR_INVALID, "null scaling");
  for (int k = 0; k < 9; ++k) {
    out->x_mean[k] = in->x_mean[k];
    out->x_std[k] = in->x_std[k];
    if (!(in->x_std[k] > 0.0)) return fail(DIG_ERR_INVALID, "scaling std must be > 0");
  }
  for (int k = 0; k < 7; ++k) {
    out->y_mean[k] = in->y_mean[k];
    out->y_std[k] = in->y_std[k];
    if (!(in->y_std[k] > 0.0)) return fail(DIG_ERR_INVALID, "scaling std must be > 0");
  }
  return DIG_OK;
}

dig_status fields_fill_empty(dig_ctx* c, double* fields, const double* fallback,
                             dig_stream_t stream) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (!fields || !fallback) return fail(DIG_ERR_INVALID, "null argument");
  HIP_TRY(launch_fill_empty(args(c), fields, fallback, (hipStream_t)stream));
  return DIG_OK;
}

dig_status closure_features(dig_ctx* c, const double* fields, const double* kngll,
                            const double* hot, const dig_mlp_scaling* scaling, float* x, float* t,
                            dig_stream_t stream) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (!fields || !kngll || !x || (t && !hot)) return fail(DIG_ERR_INVALID, "null argument");
  if (c->cfg[0].geometry == DIG_GEOM_ANNULUS)
    return fail(DIG_ERR_INVALID, "boxes only (uniform or graded)");
  MlpScale sc;
  dig_status st = scaling_of(scaling, &sc);
  if (st != DIG_OK) return st;
  HIP_TRY(launch_learn_features(args(c), fields, kngll, hot, sc, x, t, (hipStream_t)stream));
  return DIG_OK;
}

dig_status closure_blend(dig_ctx* c, const double* fields, const double* kngll,
                         const uint8_t* mask, const float* y, const dig_mlp_scaling* scaling,
                         const double* A, double kn_lo, double kn_hi, double judge_sigma,
                         double judge_rel, double judge_steps, double* hot, uint8_t* src,
                         dig_stream_t stream) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (!fields || !kngll || !mask || !y || !hot || !A)
    return fail(DIG_ERR_INVALID, "null argument");
  if (!(kn_lo <= kn_hi) || !(judge_sigma >= 0.0) || !(judge_rel >= 0.0) || !(judge_steps > 0.0))
    return fail(DIG_ERR_INVALID, "bad band or judge tolerance");
  const double det = A[0] * A[3] - A[1] * A[2];
  if (!(fabs(det) > 0.0)) return fail(DIG_ERR_INVALID, "singular relaxation matrix A");
  MlpScale sc;
  dig_status st = scaling_of(scaling, &sc);
  if (st != DIG_OK) return st;
  const JudgeGas J{A[0], A[1], A[2], A[3], det};
  HIP_TRY(launch_learn_blend(args(c), fields, kngll, mask, y, sc, J, kn_lo, kn_hi, judge_sigma,
                             judge_rel, judge_steps, hot, src, (hipStream_t)stream));
  return DIG_OK;
}

dig_status dsmc_query(dig_ctx* c, dig_counters* out, dig_stream_t stream) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (!out) return fail(DIG_ERR_INVALID, "null output");
  hipStream_t s = (hipStream_t)stream;
  StepArgs a = args(c);
  unsigned long long slots[kStatSlots * ST_N];
  HIP_TRY(hipMemcpyAsync(out, a.ctr, sizeof(dig_counters), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(slots, a.stats, sizeof(slots), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  out->cur = (uint32_t)c->cur;
  int64_t sum[ST_N] = {0};
  for (int k = 0; k < kStatSlots; ++k)
    for (int f = 0; f < ST_N; ++f) sum[f] += (int64_t)slots[k * ST_N + f];
  out->candidates = sum[ST_CAND];
  out->accepted = sum[ST_ACC];
  out->inelastic = sum[ST_INEL];
  out->saturated = sum[ST_SAT];
  out->wall_hits = sum[ST_HITS];
  out->removed = sum[ST_REMOVED];
  out->injected = sum[ST_INJECTED];
  return DIG_OK;
}

dig_status dig_constants(dig_ctx* c, int32_t inst, double* out) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (!out || inst < 0 || inst >= c->n_inst) return fail(DIG_ERR_INVALID, "bad instance");
  const dig_config& g = c->cfg[inst];
  out[0] = vhs_constant(g);
  out[1] = p_inelastic(g);
  out[2] = g.kn * sqrt(2.0 / M_PI);
  out[3] = g.geometry == DIG_GEOM_GRADED ? graded_volume(g, 0) : cell_volume(g);
  out[4] = default_majorant(g);
  return DIG_OK;
}

dig_status dsmc_profile(dig_ctx* c, int32_t mode, double* ms, int64_t* launches,
                        dig_stream_t stream) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (mode == 1) {
    HIP_TRY(pool_grow(&c->eager, 4096));
    c->eager.used = 0;
    for (int k = 0; k < DIG_NKERNELS; ++k) {
      c->prof_ms[k] = 0.0;
      c->prof_n[k] = 0;
    }
    for (int k = 0; k < DIG_NKERNELS; ++k) c->prof_seen[k] = 0;
    c->prof = true;
    return DIG_OK;
  }
  if (mode == 0) {
    HIP_TRY(prof_fold(c, s));
    c->prof = false;
    return DIG_OK;
  }
  if (mode == 2) {
    if (!ms || !launches) return fail(DIG_ERR_INVALID, "null output");
    HIP_TRY(prof_fold(c, s));
    for (int k = 0; k < DIG_NKERNELS; ++k) {
      ms[k] = c->prof_ms[k];
      launches[k] = c->prof_n[k];
    }
    return DIG_OK;
  }
  return fail(DIG_ERR_INVALID, "bad profile mode");
}

dig_status dsmc_profile_kinds(dig_ctx* c, uint32_t mask, int32_t every) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (mask >> DIG_NKERNELS) return fail(DIG_ERR_INVALID, "unknown kernel kind in mask");
  if (every < 1) return fail(DIG_ERR_INVALID, "every must be >= 1");
  c->prof_mask = mask;
  c->prof_every = every;
  return DIG_OK;
}

dig_status dsmc_tuning(dig_ctx* c, const dig_tuning* in, dig_tuning* out) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (out) {
    out->group_particles = c->T;
    out->group_cells = c->Gc;
    out->seq_max = c->seq_max;
    out->big_stage_kib = c->big_kib;
    out->ms_per_step = 0.0;
  }
  if (in) {
    if (c->phase != 0) return fail(DIG_ERR_STATE, "a partial step is pending (dsmc_stage)");
    dig_status st =
        check_tuning(in->group_particles, in->group_cells, in->seq_max, in->big_stage_kib);
    if (st != DIG_OK) return st;
    apply_tuning(c, in->group_particles, in->group_cells, in->seq_max, in->big_stage_kib);
  }
  return DIG_OK;
}

}  // extern "C"

namespace {

// Steps per captured graph: longer runs replay it (graph size stays bounded).
constexpr int32_t kGraphSteps = 64;

// Launches k <= kGraphSteps steps as one graph, capturing it on first use.
dig_status graph_steps(dig_ctx* c, int32_t k, hipStream_t stream) {
  const int cur0 = c->cur;
  const int64_t nup = args(c).n_upper;
  dig_ctx::Graph* hit = nullptr;
  for (auto& g : c->graphs)
    if (g.nsteps == k && g.cur == cur0 && g.n == nup && g.T == c->T && g.Gc == c->Gc &&
        g.seq == c->seq_max && g.big == c->big_kib)
      hit = &g;
  if (!hit) {
    if (c->graphs.size() >= 8) drop_graphs(c);
    if (!c->cap) HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    dig_status st = DIG_OK;
    for (int i = 0; i < k && st == DIG_OK; ++i) st = run_stages(c, DIG_STAGE_ALL, c->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap, &g);
    // nothing ran during capture: the host view of the state is unchanged
    c->cur = cur0;
    c->phase = 0;
    if (st != DIG_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return st != DIG_OK ? st : hip_fail(e, "hipStreamEndCapture");
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_fail(e, "hipGraphInstantiate");
    }
    hipEvent_t done = nullptr;
    e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (e != hipSuccess) {
      (void)hipGraphExecDestroy(x);
      (void)hipGraphDestroy(g);
      return hip_fail(e, "hipEventCreateWithFlags");
    }
    c->graphs.push_back({k, cur0, c->T, c->Gc, c->seq_max, c->big_kib, nup, g, x, done});
    hit = &c->graphs.back();
  }
  HIP_TRY(hipGraphLaunch(hit->x, stream));
  HIP_TRY(hipEventRecord(hit->done, stream));
  c->cur = cur0 ^ (k & 1);
  return DIG_OK;
}

}  // namespace

extern "C" {

dig_status dsmc_step_graph(dig_ctx* c, int32_t nsteps, dig_stream_t stream) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (!c->has_state) return fail(DIG_ERR_STATE, "no particle state (call dsmc_init)");
  if (nsteps < 0) return fail(DIG_ERR_INVALID, "nsteps < 0");
  if (c->phase != 0) return fail(DIG_ERR_STATE, "a partial step is pending (dsmc_stage)");
  if (c->prof) return fail(DIG_ERR_STATE, "graph steps need dsmc_profile disabled");
  for (int32_t done = 0; done < nsteps;) {
    const int32_t k = nsteps - done < kGraphSteps ? nsteps - done : kGraphSteps;
    const dig_status st = graph_steps(c, k, (hipStream_t)stream);
    if (st != DIG_OK) return st;
    done += k;
  }
  return DIG_OK;
}

dig_status dsmc_autotune(dig_ctx* c, int32_t steps_per_trial, const char* cache_path,
                         dig_tuning* out, dig_stream_t stream) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (!c->has_state) return fail(DIG_ERR_STATE, "no particle state (call dsmc_init)");
  if (c->phase != 0) return fail(DIG_ERR_STATE, "a partial step is pending (dsmc_stage)");
  if (steps_per_trial < 1) return fail(DIG_ERR_INVALID, "steps_per_trial must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  std::string arch(prop.gcnArchName);
  arch = arch.substr(0, arch.find(':'));
  auto lg2 = [](int64_t v) {
    int r = 0;
    while (v > 1) {
      v >>= 1;
      ++r;
    }
    return r;
  };
  const int ln = lg2(c->n_host), lc = lg2(c->ncell);
  dig_tuning best{c->T, c->Gc, c->seq_max, c->big_kib, 0.0};
  if (cache_path) {
    if (FILE* f = fopen(cache_path, "r")) {
      char a[64];
      int d, n, cl, T, Gc, sq, bk;
      double ms;
      bool found = false;
      while (fscanf(f, "%63s %d %d %d %d %d %d %d %lf", a, &d, &n, &cl, &T, &Gc, &sq, &bk, &ms) ==
             9)
        if (arch == a && d == c->dim && n == ln && cl == lc &&
            check_tuning(T, Gc, sq, bk) == DIG_OK) {
          best = dig_tuning{T, Gc, sq, bk, ms};
          found = true;
        }
      fclose(f);
      if (found) {
        apply_tuning(c, best.group_particles, best.group_cells, best.seq_max,
                     best.big_stage_kib);
        if (out) *out = best;
        return DIG_OK;
      }
    }
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  dig_status st = DIG_OK;
  auto trial = [&](const dig_tuning& t, double* ms) -> dig_status {
    apply_tuning(c, t.group_particles, t.group_cells, t.seq_max, t.big_stage_kib);
    dig_status r = run_stages(c, DIG_STAGE_ALL, s);
    if (r != DIG_OK) return r;
    if (hipEventRecord(e0, s) != hipSuccess) return fail(DIG_ERR_HIP, "event record");
    for (int k = 0; k < steps_per_trial; ++k)
      if ((r = run_stages(c, DIG_STAGE_ALL, s)) != DIG_OK) return r;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      return fail(DIG_ERR_HIP, "event synchronise");
    float f = 0.0f;
    if (hipEventElapsedTime(&f, e0, e1) != hipSuccess) return fail(DIG_ERR_HIP, "event time");
    *ms = (double)f / steps_per_trial;
    return DIG_OK;
  };
  st = trial(best, &best.ms_per_step);
  const int32_t Ts[] = {512, 1024, 2048, 4096, 8192};
  const int32_t Gcs[] = {32, 64, 128, 256};
  const int32_t Sqs[] = {0, 64, 128, 192, 384};
  const int32_t Bks[] = {38, 50, 76};
  // two passes over the four axes (the best group size can depend on the
  // others); each new configuration is timed once, beside a fresh timing of
  // the best so far
  std::vector<dig_tuning> tried{best};
  auto seen = [&](const dig_tuning& t) {
    for (const dig_tuning& u : tried)
      if (u.group_particles == t.group_particles && u.group_cells == t.group_cells &&
          u.seq_max == t.seq_max && u.big_stage_kib == t.big_stage_kib)
        return true;
    return false;
  };
  for (int pass = 0; pass < 2 && st == DIG_OK; ++pass) {
    for (int axis = 0; axis < 4 && st == DIG_OK; ++axis) {
      const int32_t* vals = axis == 0 ? Ts : axis == 1 ? Gcs : axis == 2 ? Sqs : Bks;
      const int nv = axis == 1 ? 4 : axis == 3 ? 3 : 5;
      // the stage of oversize groups matters only where some group exceeds
      // the small-group stage
      if (axis == 3 && c->inj_sectors == 0 && c->n_host / c->ncell < 256) continue;
      const dig_tuning base = best;
      for (int k = 0; k < nv && st == DIG_OK; ++k) {
        dig_tuning t = base;
        int32_t* field = axis == 0   ? &t.group_particles
                         : axis == 1 ? &t.group_cells
                         : axis == 2 ? &t.seq_max
                                     : &t.big_stage_kib;
        *field = vals[k];
        if (seen(t)) continue;
        tried.push_back(t);
        st = trial(t, &t.ms_per_step);
        // the state keeps evolving (a developing flow slows or speeds every
        // step), so the best configuration is timed again right after the
        // candidate and the two are compared at the same point of the run
        double ms_best = 0.0;
        if (st == DIG_OK) st = trial(best, &ms_best);
        if (st == DIG_OK && t.ms_per_step < ms_best) {
          best = t;
        } else if (st == DIG_OK) {
          best.ms_per_step = ms_best;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  apply_tuning(c, best.group_particles, best.group_cells, best.seq_max, best.big_stage_kib);
  if (st != DIG_OK) return st;
  if (cache_path) {
    if (FILE* f = fopen(cache_path, "a")) {
      fprintf(f, "%s %d %d %d %d %d %d %d %.6f\n", arch.c_str(), c->dim, ln, lc,
              best.group_particles, best.group_cells, best.seq_max, best.big_stage_kib,
              best.ms_per_step);
      fclose(f);
    }
  }
  if (out) *out = best;
  return DIG_OK;
}

}  // extern "C"

namespace {

// Checkpoint image: a header, then the current particle state and the
// per-cell state that later steps read.
struct SaveHeader {
  char magic[8];  // "DIGSAVE1"
  uint32_t version;
  int32_t dim, n_inst, ncell;
  int64_t n;
  uint64_t cfg_hash;       // instance parameters as the kernels see them
  uint64_t payload_bytes;  // bytes after the header
  dig_counters ctr;
  int32_t T, Gc, seq, big;  // tuning at the time of the save
  uint64_t hash;            // over the header up to this field and the payload
};
constexpr uint32_t kSaveVersion = 1;

// Word-wise multiplicative hash: detects truncation and corruption (not an
// authentication code).
uint64_t mix_hash(const unsigned char* p, size_t n, uint64_t h) {
  const uint64_t P = 0x100000001b3ULL;
  size_t k = 0;
  for (; k + 8 <= n; k += 8) {
    uint64_t w;
    memcpy(&w, p + k, 8);
    h = (h ^ w) * P;
    h ^= h >> 29;
  }
  for (; k < n; ++k) h = (h ^ p[k]) * P;
  return h;
}

uint64_t cfg_hash(const dig_ctx* c) {
  uint64_t h = 0xcbf29ce484222325ULL;
  h = mix_hash((const unsigned char*)c->params.data(), sizeof(InstParam) * c->params.size(), h);
  const int32_t dims[3] = {c->dim, c->n_inst, c->ncell};
  h = mix_hash((const unsigned char*)dims, sizeof(dims), h);
  return mix_hash((const unsigned char*)c->fc64_host.data(), 8 * c->fc64_host.size(), h);
}

// Payload: x, y, vx, vy, vz, er (f32), id (u32) of n particles; start
// (i32, C + 1); majorant (f32, C); accumulator (f64, 17 C); statistics slots.
size_t payload_bytes(int64_t n, int64_t C) {
  return (size_t)n * 28 + 4 * (size_t)(C + 1) + 4 * (size_t)C + 8 * 17 * (size_t)C +
         sizeof(unsigned long long) * kStatSlots * ST_N;
}

uint64_t image_hash(const SaveHeader& h, const unsigned char* payload) {
  uint64_t v = mix_hash((const unsigned char*)&h, offsetof(SaveHeader, hash),
                        0x84222325cbf29ce4ULL);
  return mix_hash(payload, h.payload_bytes, v);
}

// Host-side checks of a checkpoint's particle state against the context:
// start is a non-decreasing table from 0 to n, and every box particle lies
// in the cell its position maps to.
// Cell of a position along one graded axis: the largest i <= n - 1 with
// f[i] <= v (FP32 faces), else 0 -- the kernels' rule.
int32_t host_face_cell(const float* f, int32_t n, float v) {
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) / 2;
    if (f[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

bool image_state_ok(const dig_ctx* c, const unsigned char* p, int64_t n) {
  const float *x = (const float*)p, *y = x + n;
  const int32_t* start = (const int32_t*)(p + (size_t)n * 28);
  if (start[0] != 0 || start[c->ncell] != n) return false;
  for (int32_t k = 0; k < c->ncell; ++k)
    if (start[k + 1] < start[k]) return false;
  for (int i = 0; i < c->n_inst; ++i) {
    const InstParam& q = c->params[i];
    for (int32_t k = q.cell0; k < q.cell0 + q.ncell; ++k)
      for (int32_t e = start[k]; e < start[k + 1]; ++e) {
        if (!std::isfinite(x[e]) || (q.dim == 2 && !std::isfinite(y[e]))) return false;
        if (q.geom == DIG_GEOM_ANNULUS) continue;
        // inside the domain, in the cell the kernels would place it in
        const float yv = q.dim == 2 ? y[e] : 0.0f;
        if (x[e] < 0.0f || x[e] > q.gx || (q.dim == 2 && (yv < 0.0f || yv > q.gy))) return false;
        int32_t ix, iy = 0;
        if (q.geom == DIG_GEOM_GRADED) {
          const float* fx = c->fc32_host.data() + q.face0;
          ix = host_face_cell(fx, q.nx, x[e]);
          if (q.dim == 2) iy = host_face_cell(fx + q.nx + 1, q.ny, yv);
        } else {
          ix = std::min((int32_t)floorf(x[e]), q.nx - 1);
          if (q.dim == 2) iy = std::min((int32_t)floorf(yv), q.ny - 1);
        }
        if (q.cell0 + ix + q.nx * iy != k) return false;
      }
  }
  return true;
}

}  // namespace

extern "C" {

dig_status dsmc_save(dig_ctx* c, void* host_buf, size_t* bytes, dig_stream_t stream) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (!bytes) return fail(DIG_ERR_INVALID, "null size");
  if (!c->has_state) return fail(DIG_ERR_STATE, "no particle state");
  if (c->phase != 0) return fail(DIG_ERR_STATE, "a partial step is pending (dsmc_stage)");
  hipStream_t s = (hipStream_t)stream;
  StepArgs a = args(c);
  SaveHeader h;
  memset(&h, 0, sizeof(h));
  HIP_TRY(hipMemcpyAsync(&h.ctr, a.ctr, sizeof(dig_counters), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t n = h.ctr.n;
  const int64_t C = c->ncell;
  const size_t need = sizeof(SaveHeader) + payload_bytes(n, C);
  if (!host_buf) {
    *bytes = need;
    return DIG_OK;
  }
  if (*bytes < need) {
    *bytes = need;
    return fail(DIG_ERR_INVALID, "checkpoint buffer too small: need " + std::to_string(need));
  }
  unsigned char* p = (unsigned char*)host_buf + sizeof(SaveHeader);
  const void* src[7] = {a.A.x, a.A.y, a.A.vx, a.A.vy, a.A.vz, a.A.er, a.A.id};
  for (int k = 0; k < 7; ++k)
    HIP_TRY(hipMemcpyAsync(p + (size_t)k * 4 * n, src[k], 4 * (size_t)n, hipMemcpyDeviceToHost,
                           s));
  unsigned char* q = p + (size_t)n * 28;
  HIP_TRY(hipMemcpyAsync(q, a.start, 4 * (C + 1), hipMemcpyDeviceToHost, s));
  q += 4 * (C + 1);
  HIP_TRY(hipMemcpyAsync(q, a.sgmax, 4 * C, hipMemcpyDeviceToHost, s));
  q += 4 * C;
  HIP_TRY(hipMemcpyAsync(q, a.acc, 8 * 17 * C, hipMemcpyDeviceToHost, s));
  q += 8 * 17 * C;
  HIP_TRY(hipMemcpyAsync(q, a.stats, sizeof(unsigned long long) * kStatSlots * ST_N,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  memcpy(h.magic, "DIGSAVE1", 8);
  h.version = kSaveVersion;
  h.dim = c->dim;
  h.n_inst = c->n_inst;
  h.ncell = c->ncell;
  h.n = n;
  h.cfg_hash = cfg_hash(c);
  h.payload_bytes = payload_bytes(n, C);
  h.ctr.cur = 0;
  h.T = c->T;
  h.Gc = c->Gc;
  h.seq = c->seq_max;
  h.big = c->big_kib;
  h.hash = image_hash(h, p);
  memcpy(host_buf, &h, sizeof(h));
  *bytes = need;
  return DIG_OK;
}

dig_status dsmc_load(dig_ctx* c, const void* host_buf, size_t bytes, dig_stream_t stream) {
  if (check_ctx(c)) return DIG_ERR_INVALID;
  if (!host_buf) return fail(DIG_ERR_INVALID, "null checkpoint");
  if (c->phase != 0) return fail(DIG_ERR_STATE, "a partial step is pending (dsmc_stage)");
  if (bytes < sizeof(SaveHeader)) return fail(DIG_ERR_INVALID, "checkpoint truncated");
  SaveHeader h;
  memcpy(&h, host_buf, sizeof(h));
  if (memcmp(h.magic, "DIGSAVE1", 8) != 0 || h.version != kSaveVersion)
    return fail(DIG_ERR_INVALID, "not a checkpoint of this library version");
  if (h.dim != c->dim || h.n_inst != c->n_inst || h.ncell != c->ncell ||
      h.cfg_hash != cfg_hash(c))
    return fail(DIG_ERR_INVALID, "checkpoint of a different configuration");
  if (h.n < 0 || h.n > c->capacity)
    return fail(DIG_ERR_CAPACITY, "checkpoint holds more particles than the capacity");
  const int64_t n = h.n, C = c->ncell;
  if (h.payload_bytes != payload_bytes(n, C) || bytes != sizeof(SaveHeader) + h.payload_bytes)
    return fail(DIG_ERR_INVALID, "checkpoint truncated or of the wrong size");
  const unsigned char* p = (const unsigned char*)host_buf + sizeof(SaveHeader);
  if (image_hash(h, p) != h.hash) return fail(DIG_ERR_INVALID, "checkpoint corrupted");
  if (!image_state_ok(c, p, n))
    return fail(DIG_ERR_INVALID, "checkpoint particle state inconsistent with its cells");
  if (check_tuning(h.T, h.Gc, h.seq, h.big) != DIG_OK)
    return fail(DIG_ERR_INVALID, "checkpoint tuning out of range");
  // valid: replace the state (the particles go to buffer 0)
  hipStream_t s = (hipStream_t)stream;
  drop_graphs(c);
  apply_tuning(c, h.T, h.Gc, h.seq, h.big);
  c->cur = 0;
  c->phase = 0;
  c->n_host = n > 0 ? n : 1;
  StepArgs a = args(c);
  void* dst[7] = {a.A.x, a.A.y, a.A.vx, a.A.vy, a.A.vz, a.A.er, a.A.id};
  for (int k = 0; k < 7; ++k)
    HIP_TRY(hipMemcpyAsync(dst[k], p + (size_t)k * 4 * n, 4 * (size_t)n, hipMemcpyHostToDevice,
                           s));
  const unsigned char* q = p + (size_t)n * 28;
  HIP_TRY(hipMemcpyAsync(a.start, q, 4 * (C + 1), hipMemcpyHostToDevice, s));
  q += 4 * (C + 1);
  HIP_TRY(hipMemcpyAsync(a.sgmax, q, 4 * C, hipMemcpyHostToDevice, s));
  q += 4 * C;
  HIP_TRY(hipMemcpyAsync(a.acc, q, 8 * 17 * C, hipMemcpyHostToDevice, s));
  q += 8 * 17 * C;
  HIP_TRY(hipMemcpyAsync(a.stats, q, sizeof(unsigned long long) * kStatSlots * ST_N,
                         hipMemcpyHostToDevice, s));
  // cell counts, groups and instance ranges from the start table, as after
  // dsmc_inject; then the counters of the saved state
  hipLaunchKernelGGL(k_counts_from_start, dim3((c->ncell + 255) / 256), dim3(256), 0, s,
                     a.start, a.count, c->ncell);
  HIP_TRY(hipGetLastError());
  HIP_TRY(launch_scan(a, a.count, false, s));
  HIP_TRY(launch_fill_i32((int32_t*)a.done, 1, 0, s));
  HIP_TRY(launch_fill_i32((int32_t*)a.big_count, 1, 0, s));
  HIP_TRY(hipMemcpyAsync(a.ctr, &h.ctr, sizeof(dig_counters), hipMemcpyHostToDevice, s));
  // the copies read the caller's buffer and the local header
  HIP_TRY(hipStreamSynchronize(s));
  c->n_host = n;
  c->has_state = true;
  return DIG_OK;
}

void dsmc_destroy(dig_ctx* c) {
  if (!c) return;
  drop_graphs(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  pool_free(&c->eager);
  delete c;
}

}  // extern "C"
