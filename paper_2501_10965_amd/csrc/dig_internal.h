// Internal declarations of libdig shared by the kernels and the host API.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dig.h"

namespace dig {

// Philox stream tags (high byte of counter word 2).
enum : uint32_t {
  TAG_INIT = 1, TAG_INIT_N = 2, TAG_WALL = 3, TAG_NCAND = 4, TAG_COLL = 5,
  TAG_DIG_N = 6, TAG_DIG_DEL = 7, TAG_DIG_SRC = 8, TAG_DIG_EMPTY = 9
};

constexpr int kMaxHits = 8;      // wall events per particle and step
constexpr int kRunMax = 4096;    // run table of the sort kernel
constexpr int kCandChunk = 128;  // candidates staged per round set
constexpr int kRoundChunkMax = 256;  // large-cell round sets where the stage holds their words
constexpr int kSeqMaxDefault = 192;  // cells up to this size: one lane, candidates in order
constexpr int kMinGroupParticles = 256;
// Statistics counters are spread over kStatSlots cache lines (slot = block
// index mod kStatSlots) so that thousands of workgroups do not serialise on
// one address; dsmc_query sums the slots.
constexpr int kStatSlots = 64;
enum { ST_CAND = 0, ST_ACC = 1, ST_INEL = 2, ST_SAT = 3, ST_HITS = 4, ST_N = 8 };
constexpr int kMinGroupCells = 32;

// Per-instance constants, resident in the workspace.
struct InstParam {
  int32_t dim, nx, ny, cell0;
  int32_t ncell, dr;
  int32_t face0;  // graded box: offset of this instance's x faces in the face
                  // tables (nx + 1 entries, then ny + 1 y faces in 2D); -1 otherwise
  int32_t pad1;
  int32_t bc_type[4];
  float bc_T[4];
  float bc_U[4][3];
  float inv_dx, inv_dy, gx, gy;
  float dtf, csig, expo, beta_inv;
  uint32_t key0, key1, inst, geom;
  double pin;            // P_inelastic (decisions taken in double)
  double weight, dt, vol;
  double mu0, omega, dx, dy;
  // annulus: FP32 squared radii of the inner and outer circles (rounded from
  // FP64), their radii, the angular width of a cell; freestream reservoir:
  // outer radius squared, mean particle count per angular sector; the radial
  // index guess j ~ log2(1 + (r - r_in) rk) rlq (rlq = 0: j ~ (r - r_in) rk)
  float rin2, rout2, rin, rout;
  float res2, dthf, rk, rlq;
  double res_mean, rho_inf;
  // scattering: isotropic (vss = 0, alpha = 1) or VSS with 1/alpha (the
  // deflection angle is taken in FP64)
  uint32_t vss;
  double ainv;
};
enum : uint32_t { TAG_INFLOW = 10, TAG_ER = 11, TAG_BL = 12 };

struct DevState {
  float *x, *y, *vx, *vy, *vz, *er;
  uint32_t* id;
};

__device__ __forceinline__ uint4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32 -> 64-bit product per multiplier gives both halves
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint4 draw(const InstParam& P, uint32_t entity, uint32_t step,
                                      uint32_t tag, uint32_t idx) {
  return philox10(entity, step, (tag << 24) | (P.inst & 0xFFFFFFu), idx, P.key0, P.key1);
}

// (k + 1/2) 2^-23 for the top 23 bits k: exact in single precision.
__device__ __forceinline__ float u01f(uint32_t r) {
  return (float)(r >> 9) * 0x1p-23f + 0x1p-24f;
}
__device__ __forceinline__ double u01d(uint32_t r) {
  return (double)(r >> 9) * 0x1p-23 + 0x1p-24;
}
__device__ __forceinline__ uint32_t pick(uint32_t r, uint32_t n) { return __umulhi(r, n); }

// Launch plumbing implemented in dig_kernels.hip.
struct StepArgs {
  DevState A, B;
  int32_t *cell, *rank, *perm_raw, *perm, *start, *count, *cell_inst, *gfirst;
  float* sgmax;
  double *acc, *sums;
  int64_t* inst_pstart;
  int64_t* bsum;       // chunk sums of the cell scan
  int32_t* lastcnt;    // last count of each scan chunk
  unsigned long long* stats;  // [kStatSlots][ST_N]
  const InstParam* params;
  dig_counters* ctr;
  int32_t n_inst, ncell, dim;
  int32_t group_particles, group_cells, lds_particles;
  int32_t seq_max;  // cells with at most this many particles collide on one lane
  int64_t n_upper;
  const double* cvol;  // [ncell] cell volumes
  const float* fc32;   // graded boxes: FP32 face coordinates (cell location)
  const double* fc64;  // graded boxes: FP64 face coordinates (positions, distances)
  const float* rf2;    // annulus: [ny + 1] FP32 squared face radii
  const float2* dir;   // annulus: [nx + 1] FP32 (cos, sin) of the angular faces
  int32_t* inj_off;    // freestream: [nx + 2] inflow offsets per angular sector
  int64_t capacity;
  int32_t inj_sectors;  // angular sectors with inflow (0: closed domain)
  uint32_t* done;       // ticket of the workgroups that finished the collide
  int32_t lds_big;      // particle stage of the oversize-group collide
  int32_t big_runs;     // its run-table capacity
  int32_t* big_list;    // groups too large for the collide's stage, listed by it
  uint32_t* big_count;  // entries in big_list (emptied by k_collide_big)
  // velocities and rotational energies of the groups collided in global
  // memory, one record per particle at the destination slot
  float4* vstage;
  int32_t ext_any;      // some instance needs the extended model (alpha != 1 or d_r != 2)
  int32_t dr_any;       // some instance has d_r != 2
};
enum { ST_REMOVED = 5, ST_INJECTED = 6 };

hipError_t launch_inject(const StepArgs& a, hipStream_t s);

// Standardisation of the closure network's inputs and targets.
struct MlpScale {
  double x_mean[9], x_std[9], y_mean[7], y_std[7];
};
hipError_t launch_learn_features(const StepArgs& a, const double* F, const double* kn,
                                 const double* hot, const MlpScale& sc, float* x, float* t,
                                 hipStream_t s);
// Heat-flux relaxation matrix A of the judge's NSF noise (det = Att Arr - Atr Art).
struct JudgeGas {
  double Att, Atr, Art, Arr, det;
};
hipError_t launch_learn_blend(const StepArgs& a, const double* F, const double* kn,
                              const uint8_t* mask, const float* y, const MlpScale& sc,
                              const JudgeGas& J, double kn_lo, double kn_hi,
                              double judge_sigma, double judge_rel, double judge_steps,
                              double* hot, uint8_t* src, hipStream_t s);

// Sets the thread-local message returned by dig_last_error; returns s.
dig_status report(dig_status s, const char* msg);

int64_t group_launch(const StepArgs& a);
int scan_blocks(int ncell);
size_t collide_lds_bytes(int lds_particles, int group_cells);
// LDS of the oversize-group collide: the stage budget is a tuning choice
// (38 KiB: four workgroups per CU; larger stages hold larger cells with fewer
// workgroups per CU), at most kBigLdsMax.
constexpr size_t kBigLdsBytes = 38 * 1024;
constexpr size_t kBigLdsMax = 150 * 1024;
bool big_stage_fits(int lds_big, int group_cells, size_t budget);
int big_run_slots(int lds_big, int group_cells);
hipError_t collide_setup();
hipError_t launch_move(const StepArgs& a, hipStream_t s);
hipError_t launch_scan(const StepArgs& a, int32_t* counts, bool set_n, hipStream_t s);
hipError_t launch_place(const StepArgs& a, hipStream_t s);
hipError_t launch_order(const StepArgs& a, hipStream_t s);
hipError_t launch_collide(const StepArgs& a, bool collide, bool sample, bool end_step,
                          bool fuse_order, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);
hipError_t launch_set_counters(dig_counters* c, int64_t n, int64_t step, int64_t next_id,
                               bool reset_all, hipStream_t s);
hipError_t launch_init(const StepArgs& a, const double* fields, int32_t ppc, hipStream_t s,
                       int phase);
hipError_t launch_sample_state(const StepArgs& a, hipStream_t s);
hipError_t launch_convert(const StepArgs& a, const double* sums, bool average, double* out,
                          hipStream_t s);
hipError_t launch_adjust_count(const StepArgs& a, const double* target, uint32_t iter,
                               int32_t* newcount, int32_t* ccount, hipStream_t s);
// Exclusive scans out0 = scan(in0), out1 = scan(in1) of n counts each, with
// the totals in out0[n] and out1[n]; csum: 2 exscan_chunks(n) int64 of scratch.
int exscan_chunks(int n);
hipError_t launch_exscan2(const int32_t* in0, int32_t* out0, const int32_t* in1,
                          int32_t* out1, int32_t n, int64_t* csum, hipStream_t s);
hipError_t launch_adjust_build(const StepArgs& a, const double* target, uint32_t iter,
                               const int32_t* newstart, const int32_t* cstart,
                               hipStream_t s);
hipError_t launch_fill_empty(const StepArgs& a, double* fields, const double* fallback,
                             hipStream_t s);
hipError_t launch_closure(const StepArgs& a, const double* fields, double Att, double Atr,
                          double Art, double Arr, double kn_ref, double n_min, double* hot,
                          uint8_t* mask, double* kngll, double* nsf, hipStream_t s);

}  // namespace dig
