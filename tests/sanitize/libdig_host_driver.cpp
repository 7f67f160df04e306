// Host-side logic of libdig under AddressSanitizer and
// UndefinedBehaviorSanitizer: workspace planning of valid and invalid
// configurations (box, batch, annulus), the synthetic-solve and network
// workspace sizes, and the argument checks of every entry point that must
// reject a call before any device work.  Nothing here touches a GPU: every
// call either plans on the host or fails its argument checks.  Exit status 0
// when every expectation held; a sanitizer report aborts the program.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "dig.h"

static int failures = 0;

static void expect(bool ok, const char* what) {
  if (!ok) {
    fprintf(stderr, "FAILED: %s (last error: %s)\n", what, dig_last_error());
    ++failures;
  }
}

static void expect_invalid(dig_status s, const char* what) {
  expect(s == DIG_ERR_INVALID, what);
  const char* m = dig_last_error();
  expect(m != nullptr && strlen(m) > 0, "an error leaves a message");
}

static dig_config box(int dim, int nx, int ny) {
  dig_config c;
  memset(&c, 0, sizeof(c));
  c.dim = dim;
  c.nx = nx;
  c.ny = dim == 2 ? ny : 1;
  c.lx = c.ly = 1.0;
  c.geometry = DIG_GEOM_BOX;
  c.q = 1.0;
  c.kn = 0.05;
  c.omega = 0.74;
  c.alpha = 1.0;
  c.dr = 2;
  c.zrot = 5.0;
  c.dt = 0.005;
  c.weight = 1e-4;
  for (int f = 0; f < 4; ++f) {
    c.bc[f].type = DIG_BC_DIFFUSE;
    c.bc[f].T = 1.0;
  }
  c.seed = 7;
  c.tref = 1.0;
  return c;
}

static dig_config annulus() {
  dig_config c = box(2, 48, 20);
  c.geometry = DIG_GEOM_ANNULUS;
  c.r_in = 0.5;
  c.r_out = 5.5;
  c.q = 1.05;
  c.bc[1].type = DIG_BC_FREESTREAM;
  c.bc[1].U[0] = 5.9;
  c.bc[1].rho = 1.0;
  c.bc[2].type = c.bc[3].type = DIG_BC_PERIODIC;
  return c;
}

int main() {
  dig_layout L;
  // valid plans
  dig_config cav = box(2, 64, 48);
  expect(dig_plan(&cav, 1, 100000, &L) == DIG_OK, "cavity plan");
  expect(L.total_bytes > 0 && L.ncell == 64 * 48 && L.capacity >= 100000, "cavity layout");
  dig_config batch[5];
  for (int i = 0; i < 5; ++i) {
    batch[i] = box(1, 10 + 7 * i, 1);
    batch[i].instance_id = (uint32_t)i;
  }
  expect(dig_plan(batch, 5, 20000, &L) == DIG_OK, "batch plan");
  expect(L.ncell == 10 + 17 + 24 + 31 + 38, "batch cell count");
  dig_config ann = annulus();
  expect(dig_plan(&ann, 1, 500000, &L) == DIG_OK, "annulus plan");

  // invalid plans
  expect_invalid(dig_plan(nullptr, 1, 1000, &L), "null configs");
  expect_invalid(dig_plan(&cav, 0, 1000, &L), "no instances");
  expect_invalid(dig_plan(&cav, 1, 0, &L), "zero capacity");
  expect_invalid(dig_plan(&cav, 1, -5, &L), "negative capacity");
  expect_invalid(dig_plan(&cav, 1, (int64_t)1 << 62, &L), "capacity beyond 32-bit indices");
  expect_invalid(dig_plan(&cav, 1, 1000, nullptr), "null layout");
  struct Bad {
    const char* what;
    void (*edit)(dig_config*);
  };
  const Bad bad[] = {
      {"dim 3", [](dig_config* c) { c->dim = 3; }},
      {"no cells", [](dig_config* c) { c->nx = 0; }},
      {"negative ny", [](dig_config* c) { c->ny = -4; }},
      {"kn NaN", [](dig_config* c) { c->kn = NAN; }},
      {"kn negative", [](dig_config* c) { c->kn = -1.0; }},
      {"omega above 1", [](dig_config* c) { c->omega = 1.2; }},
      {"alpha above 2", [](dig_config* c) { c->alpha = 2.5; }},
      {"d_r 7", [](dig_config* c) { c->dr = 7; }},
      {"d_r 1", [](dig_config* c) { c->dr = 1; }},
      {"Z below P_inelastic = 1", [](dig_config* c) { c->zrot = 0.1; }},
      {"dt zero", [](dig_config* c) { c->dt = 0.0; }},
      {"dt infinite", [](dig_config* c) { c->dt = INFINITY; }},
      {"weight zero", [](dig_config* c) { c->weight = 0.0; }},
      {"lx negative", [](dig_config* c) { c->lx = -1.0; }},
      {"one periodic face", [](dig_config* c) { c->bc[0].type = DIG_BC_PERIODIC; }},
      {"unknown face type", [](dig_config* c) { c->bc[2].type = 17; }},
      {"freestream on a box", [](dig_config* c) { c->bc[1].type = DIG_BC_FREESTREAM; }},
      {"wall temperature zero", [](dig_config* c) { c->bc[3].T = 0.0; }},
      {"wall moving along its normal", [](dig_config* c) { c->bc[0].U[0] = 0.3; }},
      {"unknown geometry", [](dig_config* c) { c->geometry = 9; }},
  };
  for (const Bad& b : bad) {
    dig_config c = box(2, 16, 16);
    b.edit(&c);
    expect_invalid(dig_plan(&c, 1, 10000, &L), b.what);
  }
  const Bad bad_ann[] = {
      {"annulus in 1D", [](dig_config* c) { c->dim = 1; c->ny = 1; }},
      {"annulus r_in 0", [](dig_config* c) { c->r_in = 0.0; }},
      {"annulus r_out below r_in", [](dig_config* c) { c->r_out = 0.4; }},
      {"annulus q below 1", [](dig_config* c) { c->q = 0.9; }},
      {"annulus freestream inner circle", [](dig_config* c) { c->bc[0].type = DIG_BC_FREESTREAM; }},
      {"annulus freestream density 0", [](dig_config* c) { c->bc[1].rho = 0.0; }},
  };
  for (const Bad& b : bad_ann) {
    dig_config c = annulus();
    b.edit(&c);
    expect_invalid(dig_plan(&c, 1, 10000, &L), b.what);
  }
  // graded boxes: valid tables, then broken ones
  double xf[9] = {0.0, 0.01, 0.03, 0.07, 0.5, 0.93, 0.97, 0.99, 1.0};
  double yf[5] = {0.0, 0.1, 0.5, 0.9, 1.0};
  dig_config gr = box(2, 8, 4);
  gr.geometry = DIG_GEOM_GRADED;
  gr.xfaces = xf;
  gr.yfaces = yf;
  expect(dig_plan(&gr, 1, 10000, &L) == DIG_OK, "graded plan");
  expect(dig_synth_workspace_bytes(&gr) > 0, "graded synth workspace");
  gr.yfaces = nullptr;
  expect_invalid(dig_plan(&gr, 1, 10000, &L), "graded box without y faces");
  gr.yfaces = yf;
  xf[3] = 0.02;
  expect_invalid(dig_plan(&gr, 1, 10000, &L), "graded faces not increasing");
  xf[3] = 0.07;
  xf[8] = 0.98;
  expect_invalid(dig_plan(&gr, 1, 10000, &L), "graded faces short of lx");
  xf[8] = 1.0;
  yf[2] = NAN;
  expect_invalid(dig_plan(&gr, 1, 10000, &L), "graded faces not finite");
  yf[2] = 0.5;
  xf[2] = 0.01 + 1e-12;
  expect_invalid(dig_plan(&gr, 1, 10000, &L), "graded faces equal in FP32");
  xf[2] = 0.03;
  expect(dig_plan(&gr, 1, 10000, &L) == DIG_OK, "graded plan after repair");
  dig_config two[2] = {annulus(), annulus()};
  expect_invalid(dig_plan(two, 2, 10000, &L), "two annulus instances");
  dig_config mixed[2] = {box(1, 10, 1), box(2, 10, 10)};
  expect_invalid(dig_plan(mixed, 2, 10000, &L), "instances of different dim");

  // synthetic-solve workspace and argument checks (no device pointers given)
  expect(dig_synth_workspace_bytes(&cav) > 0, "synth workspace of a box");
  expect(dig_synth_workspace_bytes(nullptr) == 0, "synth workspace of no config");
  dig_synth_opts so;
  memset(&so, 0, sizeof(so));
  so.A[0] = 2.0 / 3.0;
  so.A[3] = 5.0 / (7.0 - 1.48);
  so.cfl = 0.5;
  int32_t it = 0;
  double ch = 0.0;
  expect_invalid(synth_solve(&cav, &so, nullptr, nullptr, nullptr, nullptr, nullptr, 0, 10,
                             1e-5, &it, &ch, nullptr),
                 "synth_solve without buffers");
  expect_invalid(synth_solve(nullptr, &so, nullptr, nullptr, nullptr, nullptr, nullptr, 0, 10,
                             1e-5, &it, &ch, nullptr),
                 "synth_solve without config");
  expect_invalid(synth_solve_static(&cav, nullptr, nullptr, nullptr, nullptr, nullptr, 10, 1e-5,
                                    &it, &ch, nullptr),
                 "synth_solve_static without options");
  dig_config huge = box(2, 2000, 2000);
  expect_invalid(synth_solve_static(&huge, &so, nullptr, nullptr, nullptr, nullptr, 10, 1e-5,
                                    &it, &ch, nullptr),
                 "synth_solve_static on a grid beyond its static scratch");

  // network workspace planning
  dig_mlp_layout ml;
  expect(mlp_plan(1, &ml) == DIG_OK && ml.total_bytes > 0, "mlp plan of 1 sample");
  expect(mlp_plan(65536, &ml) == DIG_OK && ml.max_batch == 65536, "mlp plan of 65536");
  expect(mlp_plan(1 << 24, &ml) == DIG_OK, "mlp plan at the largest batch");
  expect_invalid(mlp_plan(0, &ml), "mlp plan of 0");
  expect_invalid(mlp_plan((1 << 24) + 1, &ml), "mlp plan beyond the largest batch");
  expect_invalid(mlp_plan(64, nullptr), "mlp plan without layout");
  dig_mlp* net = nullptr;
  expect_invalid(mlp_create(nullptr, 0, 64, nullptr, &net), "mlp_create without workspace");
  expect(net == nullptr, "mlp_create failure leaves no handle");
  expect_invalid(mlp_forward(nullptr, nullptr, nullptr, 10, nullptr), "mlp_forward null");
  expect_invalid(mlp_grad(nullptr, nullptr, nullptr, 10, nullptr), "mlp_grad null");
  expect_invalid(mlp_adam(nullptr, 1e-3f, 0.9f, 0.999f, 1e-8f, 1, nullptr), "mlp_adam null");
  expect_invalid(mlp_sync(nullptr, nullptr), "mlp_sync null");
  mlp_destroy(nullptr);

  // every context entry point rejects a null context before device work
  size_t bytes = 0;
  dig_counters cnt;
  dig_tuning tu;
  double c5[5];
  expect(dsmc_init(nullptr, nullptr, 10, nullptr) != DIG_OK, "dsmc_init null");
  expect(dsmc_step(nullptr, 1, nullptr) != DIG_OK, "dsmc_step null");
  expect(dsmc_step_graph(nullptr, 1, nullptr) != DIG_OK, "dsmc_step_graph null");
  expect(dsmc_stage(nullptr, 1, nullptr) != DIG_OK, "dsmc_stage null");
  expect(dsmc_sample(nullptr, 0, nullptr, nullptr) != DIG_OK, "dsmc_sample null");
  expect(dig_adjust(nullptr, nullptr, 0, nullptr) != DIG_OK, "dig_adjust null");
  expect(closure_assemble(nullptr, nullptr, nullptr, 0.01, 1.0, nullptr, nullptr, nullptr, nullptr,
                          nullptr) != DIG_OK,
         "closure_assemble null");
  expect(dsmc_save(nullptr, nullptr, &bytes, nullptr) != DIG_OK, "dsmc_save null");
  expect(dsmc_load(nullptr, nullptr, 0, nullptr) != DIG_OK, "dsmc_load null");
  expect(dsmc_query(nullptr, &cnt, nullptr) != DIG_OK, "dsmc_query null");
  expect(dig_constants(nullptr, 0, c5) != DIG_OK, "dig_constants null");
  expect(dsmc_tuning(nullptr, nullptr, &tu) != DIG_OK, "dsmc_tuning null");
  expect(dsmc_autotune(nullptr, 5, nullptr, &tu, nullptr) != DIG_OK, "dsmc_autotune null");
  expect(fields_fill_empty(nullptr, nullptr, nullptr, nullptr) != DIG_OK, "fields_fill_empty null");
  expect(closure_features(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                          nullptr) != DIG_OK,
         "closure_features null");
  expect(closure_blend(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0.0, 1.0,
                       3.0, 0.1, 10.0, nullptr, nullptr, nullptr) != DIG_OK,
         "closure_blend null");
  expect(dsmc_create(&cav, 1, 1000, nullptr, 0, 0, 0, nullptr, nullptr) != DIG_OK,
         "dsmc_create without output or workspace");
  dsmc_destroy(nullptr);

  if (failures) {
    fprintf(stderr, "%d expectations failed\n", failures);
    return 1;
  }
  printf("libdig host checks passed\n");
  return 0;
}
