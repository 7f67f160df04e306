// HIP kernels of libdig for gfx950 (CDNA4, wave64).
//
// One DSMC step (Section 2.2 of arXiv:2501.10965) is six launches:
//   k_move          free flight + walls + cell index + wave-aggregated
//                   reservation of slots per destination cell
//   k_scan_reduce,  cell counts -> cell starts, cell groups, instance ranges
//   k_scan_apply
//   k_place         provisional placement by the reserved rank
//   k_collide       per cell group that fits its LDS stage: stable order of
//                   the group, gather into the other buffer, NTC/VHS/BL
//                   collisions, FP64 moment sums accumulated per cell; larger
//                   groups are listed
//   k_collide_big   the same for the listed groups, in a larger stage or in
//                   global memory; closes the step
// (k_order orders every group when the sort stage runs on its own.)  Every
// result is a deterministic function of (seed, step, state): no
// floating-point atomics, and the reservation atomics only decide the order
// of runs, which the ordering restores.
#include <math.h>

#include <algorithm>

#include "dig_internal.h"

namespace dig {

static __device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Instance of particle slot p (instance particle ranges are contiguous).
static __device__ __forceinline__ int find_inst(const int64_t* pstart, int n_inst, int64_t p) {
  int lo = 0, hi = n_inst - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (pstart[mid] <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Workgroups are dispatched to the eight XCDs round robin (block b to XCD
// b mod 8), each XCD with its own L2.  Cell groups next to each other share
// source particles (the gather of particles that changed cells), so give
// every XCD one contiguous range of groups: a bijection of [0, n).
constexpr int kXcds = 8;
static __device__ __forceinline__ int xcd_group(int b, int n) {
  const int x = b % kXcds, i = b / kXcds;
  const int q = n / kXcds, r = n % kXcds;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Largest i in [0, n) with a[i] <= v (a non-decreasing, a[0] <= v).
template <typename T>
static __device__ __forceinline__ int floor_index(const T* a, int n, T v) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (a[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Iround of Section 3.2 with the products taken in a fixed order and no
// contraction, so the host oracle and the device agree bit for bit.
static __device__ __noinline__ double ncand_mean(int N, double w, double sg, double dt,
                                                 double vol) {
#pragma clang fp contract(off)
  return 0.5 * (double)N * (double)(N - 1) * w * sg * dt / vol;
}
static __device__ __noinline__ double count_mean(double rho, double vol, double w) {
#pragma clang fp contract(off)
  return rho * vol / w;
}
static __device__ __forceinline__ int iround(double x, uint32_t r) {
  const double f = floor(x);
  return (int)f + ((u01d(r) < x - f) ? 1 : 0);
}

// Hardware transcendentals (about 1 ulp): x^e for x > 0, natural log, square
// root and reciprocal.
static __device__ __forceinline__ float fpow(float x, float e) {
  return __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(x));
}
static __device__ __forceinline__ float flog(float x) {
  return 0.69314718055994531f * __builtin_amdgcn_logf(x);
}
static __device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
static __device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

static __device__ __forceinline__ float keep_inside(float v, int cellidx) {
  // position ix + u rounded to float must stay below the upper cell face
  const float top = (float)(cellidx + 1);
  return v < top ? v : __uint_as_float(__float_as_uint(top) - 1u);  // largest float below top
}

// Graded box: the cell of a coordinate along one axis, the largest
// i <= n - 1 with f[i] <= v for the FP32 faces f (else 0).
static __device__ __forceinline__ int face_cell(const float* f, int n, float v) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (f[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Graded box: the point at fraction u of cell i along one axis,
// f[i] + u (f[i+1] - f[i]) in FP64, as an FP32 coordinate that lies in the
// cell (between its FP32 faces, below the upper one).
static __device__ __forceinline__ float graded_point(const double* f64, const float* f32, int i,
                                                     double u) {
  const float v = (float)(f64[i] + u * (f64[i + 1] - f64[i]));
  const float lo = f32[i], hi = f32[i + 1];
  if (v < lo) return lo;
  return v < hi ? v : __uint_as_float(__float_as_uint(hi) - 1u);
}

// Rotational energy in equilibrium at temperature T is T times a
// Gamma(d_r/2) variate: the exponential -log u0 of the word already drawn,
// and for d_r > 2 the rest from one extra draw (entity, step, TAG_ER, idx):
// further exponentials from its words 0 (d_r >= 4) and 1 (d_r = 6), half the
// square of a normal from words 2 and 3 (odd d_r).  This returns that rest
// (0 for d_r = 2), in FP64.
static __device__ double rot_extra(const InstParam& I, double T, uint32_t entity, uint32_t step,
                                   uint32_t idx) {
  if (I.dr <= 2) return 0.0;
  const uint4 w = draw(I, entity, step, TAG_ER, idx);
  double g = 0.0;
  if (I.dr >= 4) g += -log(u01d(w.x));
  if (I.dr >= 6) g += -log(u01d(w.y));
  if (I.dr & 1) {
    const double z = sqrt(-2.0 * log(u01d(w.z))) * cos(2.0 * M_PI * u01d(w.w));
    g += 0.5 * z * z;
  }
  return T * g;
}

// ---------------------------------------------------------------------------
// Annulus cell map.  The radial index is the largest j with rf2[j] <= r^2
// (clamped to the ring) for the FP32 squared radius and the FP32 table of
// squared face radii: a guess from the inverse of the face-radius formula,
// settled by comparisons with the table (one or two loads instead of a binary
// search).  The angular index starts from atan2 and is settled by the signs
// of FP32 cross products with the face directions.  The decisions are rounded
// comparisons without contraction, so the oracle takes the same ones from the
// same stored position.
static __device__ int annulus_cell(const StepArgs& a, const InstParam& I, float x, float y) {
#pragma clang fp contract(off)
  const float r2 = x * x + y * y;
  const int nr = I.ny, nt = I.nx;
  const float s = (fsqrt(r2) - I.rin) * I.rk;
  float gj = I.rlq > 0.0f ? __log2f(1.0f + s) * I.rlq : s;
  gj = fminf(fmaxf(gj, 0.0f), (float)(nr - 1));  // a NaN guess becomes 0
  int j = (int)gj;
  while (j > 0 && a.rf2[j] > r2) --j;
  while (j < nr - 1 && a.rf2[j + 1] <= r2) ++j;
  float th = atan2f(y, x);
  if (th < 0.0f) th += 6.28318530717958648f;
  int i = (int)(th * (float)nt * 0.15915494309189535f);
  i = i < 0 ? 0 : (i >= nt ? nt - 1 : i);
  for (int it = 0; it < 4; ++it) {
    const float2 d0 = a.dir[i], d1 = a.dir[i + 1];
    const float c0 = d0.x * y - d0.y * x;  // >= 0: at or past face i
    const float c1 = d1.x * y - d1.y * x;  // < 0: before face i + 1
    if (c0 < 0.0f) {
      i = i == 0 ? nt - 1 : i - 1;
    } else if (c1 >= 0.0f) {
      i = i == nt - 1 ? 0 : i + 1;
    } else {
      break;
    }
  }
  return I.cell0 + i + nt * j;
}

// Diffuse re-emission from a circular wall with unit normal (nx, ny) into the
// gas: normal speed from the flux-weighted Maxwellian, tangential and z
// components Gaussian, rotational energy exponential (d_r = 2).
static __device__ __forceinline__ void circle_diffuse(const InstParam& P, int face, uint4 w,
                                                      float nx, float ny, float* vx, float* vy,
                                                      float* vz, float* er) {
  const float T = P.bc_T[face];
  const float vn = fsqrt(-2.0f * T * flog(u01f(w.x)));
  const float r = fsqrt(-2.0f * flog(u01f(w.y)));
  const float ph = 6.28318530717958648f * u01f(w.z);
  const float sn = __sinf(ph), cs = __cosf(ph);
  const float sT = fsqrt(T);
  const float vt = sT * (r * cs);
  *vx = vn * nx - vt * ny;
  *vy = vn * ny + vt * nx;
  *vz = sT * (r * sn);
  *er = -T * flog(u01f(w.w));
}

// Free flight in the annulus: reflection at the inner circle (and at the outer
// circle when it is a wall); with a freestream outer boundary a particle that
// ends outside it has left (returns -1).  Wall events in time order.
template <bool EXT>
static __device__ int move_annulus(const StepArgs& a, const InstParam& P, int64_t p,
                                   uint32_t step, int* hits) {
  float x = a.A.x[p], y = a.A.y[p];
  float vx = a.A.vx[p], vy = a.A.vy[p];
  float vz = 0.0f;  // not needed: a diffuse wall redraws it, a specular wall keeps it
  float t = P.dtf;
  int hit = 0;
  bool vset = false, er_set = false;
  float er = 0.0f;
  const bool outer_wall = P.bc_type[1] != DIG_BC_FREESTREAM;
  while (hit < kMaxHits) {
    const float A = vx * vx + vy * vy;
    if (!(A > 0.0f)) break;
    const float B = x * vx + y * vy;  // half the linear coefficient
    const float R2 = x * x + y * y;
    float th = t;
    int face = -1;
    // inner circle, reached from outside while approaching it
    if (B < 0.0f) {
      const float D = B * B - A * (R2 - P.rin2);
      if (D >= 0.0f) {
        const float tf = (-B - fsqrt(D)) / A;
        if (tf >= 0.0f && tf <= th) { th = tf; face = 0; }
      }
    }
    if (outer_wall) {
      const float D = B * B - A * (R2 - P.rout2);
      if (D >= 0.0f) {
        const float tf = (-B + fsqrt(D)) / A;
        if (tf >= 0.0f && tf < th) { th = tf; face = 1; }
      }
    }
    if (face < 0) break;
    x += vx * th;
    y += vy * th;
    t -= th;
    // back onto the circle; unit normal into the gas
    const float rr = fsqrt(x * x + y * y);
    const float nx = (face == 0 ? 1.0f : -1.0f) * x / rr;
    const float ny = (face == 0 ? 1.0f : -1.0f) * y / rr;
    const float Rw = face == 0 ? P.rin : P.rout;
    x = Rw * (x / rr);
    y = Rw * (y / rr);
    if (P.bc_type[face] == DIG_BC_SPECULAR) {
      const float vn = vx * nx + vy * ny;
      vx -= 2.0f * vn * nx;
      vy -= 2.0f * vn * ny;
    } else {
      const uint4 w = draw(P, a.A.id[p], step, TAG_WALL, (uint32_t)hit);
      circle_diffuse(P, face, w, nx, ny, &vx, &vy, &vz, &er);
      if constexpr (EXT) {
        if (P.dr > 2) er += (float)rot_extra(P, P.bc_T[face], a.A.id[p], step, (uint32_t)hit);
      }
      er_set = true;
    }
    vset = true;
    ++hit;
  }
  x += vx * t;
  y += vy * t;
  a.A.x[p] = x;
  a.A.y[p] = y;
  if (vset) {
    a.A.vx[p] = vx;
    a.A.vy[p] = vy;
    if (er_set) {
      a.A.vz[p] = vz;
      a.A.er[p] = er;
    }
  }
  *hits = hit;
  if (!outer_wall) {
#pragma clang fp contract(off)
    const float r2 = x * x + y * y;
    if (r2 >= P.rout2) return -1;
  }
  return annulus_cell(a, P, x, y);
}

// ---------------------------------------------------------------------------
// Free flight with diffuse / specular walls for one particle; returns its cell.
template <bool EXT>
static __device__ __forceinline__ int move_particle(const StepArgs& a, const InstParam& P,
                                                    int64_t p, uint32_t step, int* hits) {
  if (P.geom == DIG_GEOM_ANNULUS) return move_annulus<EXT>(a, P, p, step, hits);
  const bool two = P.dim == 2;
  float x = a.A.x[p];
  float y = two ? a.A.y[p] : 0.0f;
  float vx = a.A.vx[p], vy = a.A.vy[p];
  float vz = 0.0f;  // not needed: a diffuse wall redraws it, a specular wall keeps it
  float t = P.dtf;
  int hit = 0;
  bool er_set = false;
  float er = 0.0f;
  for (;;) {
    const float sx = vx * P.inv_dx;
    const float sy = two ? vy * P.inv_dy : 0.0f;
    int face = -1;
    float th = t;
    const float xe = x + sx * t;
    const bool w0 = P.bc_type[0] != DIG_BC_PERIODIC, w1 = P.bc_type[1] != DIG_BC_PERIODIC;
    if (xe < 0.0f && w0) {
      const float tf = (0.0f - x) / sx;
      if (tf <= th) { th = tf; face = 0; }
    } else if (xe > P.gx && w1) {
      const float tf = (P.gx - x) / sx;
      if (tf <= th) { th = tf; face = 1; }
    }
    if (two) {
      const float ye = y + sy * t;
      const bool w2 = P.bc_type[2] != DIG_BC_PERIODIC, w3 = P.bc_type[3] != DIG_BC_PERIODIC;
      if (ye < 0.0f && w2) {
        const float tf = (0.0f - y) / sy;
        if (face < 0 ? tf <= th : tf < th) { th = tf; face = 2; }
      } else if (ye > P.gy && w3) {
        const float tf = (P.gy - y) / sy;
        if (face < 0 ? tf <= th : tf < th) { th = tf; face = 3; }
      }
    }
    if (face < 0 || hit >= kMaxHits) {
      x += sx * t;
      if (two) y += sy * t;
      if (hit >= kMaxHits) {
        if (w0 && x < 0.0f) x = 0.0f;
        if (w1 && x > P.gx) x = P.gx;
        if (two) {
          if (P.bc_type[2] != DIG_BC_PERIODIC && y < 0.0f) y = 0.0f;
          if (P.bc_type[3] != DIG_BC_PERIODIC && y > P.gy) y = P.gy;
        }
      }
      break;
    }
    x += sx * th;
    if (two) y += sy * th;
    if (face == 0) x = 0.0f;
    if (face == 1) x = P.gx;
    if (face == 2) y = 0.0f;
    if (face == 3) y = P.gy;
    t -= th;
    const int axis = face >> 1;
    const float inward = (face & 1) ? -1.0f : 1.0f;
    if (P.bc_type[face] == DIG_BC_SPECULAR) {
      if (axis == 0) vx = -vx; else vy = -vy;
    } else {
      const uint4 w = draw(P, a.A.id[p], step, TAG_WALL, (uint32_t)hit);
      const float T = P.bc_T[face];
      const float vn = fsqrt(-2.0f * T * flog(u01f(w.x)));
      const float r = fsqrt(-2.0f * flog(u01f(w.y)));
      const float ph = 6.28318530717958648f * u01f(w.z);
      const float sn = __sinf(ph), cs = __cosf(ph);
      const float sT = fsqrt(T);
      if (axis == 0) {
        vx = inward * vn;
        vy = P.bc_U[face][1] + sT * (r * cs);
      } else {
        vy = inward * vn;
        vx = P.bc_U[face][0] + sT * (r * cs);
      }
      vz = P.bc_U[face][2] + sT * (r * sn);
      er = -T * flog(u01f(w.w));
      if constexpr (EXT) {
        if (P.dr > 2) er += (float)rot_extra(P, T, a.A.id[p], step, (uint32_t)hit);
      }
      er_set = true;
    }
    ++hit;
  }
  if (P.bc_type[0] == DIG_BC_PERIODIC) x -= P.gx * floorf(x / P.gx);
  if (two && P.bc_type[2] == DIG_BC_PERIODIC) y -= P.gy * floorf(y / P.gy);
  a.A.x[p] = x;
  if (two) a.A.y[p] = y;
  if (hit) {
    a.A.vx[p] = vx;
    a.A.vy[p] = vy;
    if (er_set) {  // diffuse re-emission draws vz and er; specular keeps them
      a.A.vz[p] = vz;
      a.A.er[p] = er;
    }
  }
  *hits = hit;
  if (P.geom == DIG_GEOM_GRADED) {
    const float* f = a.fc32 + P.face0;
    const int ix = face_cell(f, P.nx, x);
    const int iy = two ? face_cell(f + P.nx + 1, P.ny, y) : 0;
    return P.cell0 + ix + P.nx * iy;
  }
  int ix = (int)floorf(x);
  ix = ix < 0 ? 0 : (ix > P.nx - 1 ? P.nx - 1 : ix);
  int iy = 0;
  if (two) {
    iy = (int)floorf(y);
    iy = iy < 0 ? 0 : (iy > P.ny - 1 ? P.ny - 1 : iy);
  }
  return P.cell0 + ix + P.nx * iy;
}

// Free flight, cell index and reservation of a slot in the destination cell.
// EXT: compiled with the Gamma(d_r/2) wall re-emission of d_r > 2, launched
// only where an instance has d_r != 2 (keeps the basic kernel within 64 VGPRs).
template <bool EXT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(EXT ? 4 : 8))) void k_move(StepArgs a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = a.ctr->n;
  const uint32_t step = (uint32_t)a.ctr->step;
  const bool valid = p < n;
  int cell = 0;
  int hits_here = 0;
  const int inst = valid ? find_inst(a.inst_pstart, a.n_inst, p) : 0;
  const int iu = __builtin_amdgcn_readfirstlane(inst);
  if (__all(!valid || inst == iu)) {
    if (valid) cell = move_particle<EXT>(a, a.params[iu], p, step, &hits_here);
  } else if (valid) {
    cell = move_particle<EXT>(a, a.params[inst], p, step, &hits_here);
  }
  // a particle that left through an open boundary reserves nothing
  const bool gone = valid && cell < 0;
  const bool keep = valid && !gone;
  // wave-aggregated reservation: one atomic per (wave, destination cell); the
  // lanes of a run get consecutive ranks in lane (= slot) order
  // The runs are found with ballots (no memory traffic); then every run
  // leader reserves its run with the same atomic instruction.
  unsigned long long todo = __ballot(keep);
  int my_leader = 0, in_run = 0, run_len = 0;
  while (todo) {
    const int leader = __ffsll(todo) - 1;  // wave-uniform: read the lane directly
    const int lc = __builtin_amdgcn_readlane(cell, leader);
    const unsigned long long m = __ballot(keep && cell == lc);
    if (keep && cell == lc) {
      my_leader = leader;
      in_run = __popcll(m & __lanemask_lt());
    }
    if (lane_id() == leader) run_len = __popcll(m);
    todo &= ~m;
  }
  int base = 0;
  if (run_len > 0) base = atomicAdd(&a.count[cell], run_len);
  base = __shfl(base, my_leader);
  if (valid) {
    a.cell[p] = cell;
    a.rank[p] = base + in_run;
  }
  // wall-hit and removal statistics: one atomic per wave into a spread slot
  if (__ballot(hits_here != 0)) {  // most waves have no wall hit
    int hsum = hits_here;
    for (int off = 32; off > 0; off >>= 1) hsum += __shfl_xor(hsum, off);
    if (lane_id() == 0)
      atomicAdd(&a.stats[(blockIdx.x % kStatSlots) * ST_N + ST_HITS], (unsigned long long)hsum);
  }
  const int ngone = __popcll(__ballot(gone));
  if (lane_id() == 0 && ngone)
    atomicAdd(&a.stats[(blockIdx.x % kStatSlots) * ST_N + ST_REMOVED], (unsigned long long)ngone);
}

// ---------------------------------------------------------------------------
// Cell counts -> cell starts in two passes over chunks of kScanChunk cells:
// chunk sums, then per-chunk exclusive scans offset by the preceding chunks.
// The second pass also zeroes the counts, writes the cell-group table (group
// key = floor(start/T) + floor(c/Gc)), the instance particle ranges and n.
constexpr int kScanPer = 2;
constexpr int kScanChunk = 256 * kScanPer;

__global__ __launch_bounds__(256) void k_scan_reduce(StepArgs a, const int32_t* counts) {
  __shared__ int s_w[4];
  const int C = a.ncell;
  const int c0 = blockIdx.x * kScanChunk + threadIdx.x * kScanPer;
  int sum = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k)
    if (c0 + k < C) sum += counts[c0 + k];
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
  if (lane_id() == 0) s_w[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    a.bsum[blockIdx.x] = (int64_t)s_w[0] + s_w[1] + s_w[2] + s_w[3];
    const int last = min(C, (int)(blockIdx.x + 1) * kScanChunk) - 1;
    a.lastcnt[blockIdx.x] = counts[last];
  }
}

__global__ __launch_bounds__(256) void k_scan_apply(StepArgs a, int32_t* counts, int32_t glaunch,
                                                    int set_n) {
  __shared__ int64_t s_off;
  __shared__ int s_w[4];
  __shared__ int s_last[256];
  const int C = a.ncell;
  const int b = blockIdx.x;
  const int nb = gridDim.x;
  const int tid = threadIdx.x;
  // offset of this chunk: sum of the preceding chunk sums
  int64_t o = 0;
  for (int k = tid; k < b; k += 256) o += a.bsum[k];
  for (int off = 32; off > 0; off >>= 1) o += __shfl_xor(o, off);
  if (lane_id() == 0) s_w[tid >> 6] = 0;
  __shared__ int64_t s_o[4];
  if (lane_id() == 0) s_o[tid >> 6] = o;
  __syncthreads();
  if (tid == 0) s_off = s_o[0] + s_o[1] + s_o[2] + s_o[3];
  const int c0 = b * kScanChunk + tid * kScanPer;
  int cnt[kScanPer];
  int mine = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    cnt[k] = (c0 + k < C) ? counts[c0 + k] : 0;
    mine += cnt[k];
  }
  s_last[tid] = cnt[kScanPer - 1];
  // block exclusive scan of the per-thread sums
  int incl = mine;
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off);
    if (lane_id() >= off) incl += v;
  }
  if (lane_id() == 63) s_w[tid >> 6] = incl;
  __syncthreads();
  int wpre = 0;
  for (int k = 0; k < (tid >> 6); ++k) wpre += s_w[k];
  const int64_t T = a.group_particles, G = a.group_cells;
  int64_t st = s_off + wpre + incl - mine;
  // start of the cell before this thread's first cell
  int64_t prev_start;
  if (tid > 0) prev_start = st - s_last[tid - 1];
  else prev_start = (b > 0) ? st - a.lastcnt[b - 1] : -1;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int c = c0 + k;
    if (c >= C) break;
    a.start[c] = (int32_t)st;
    counts[c] = 0;
    const int64_t key = st / T + c / G;
    const int64_t kp = (c == 0) ? -1 : (prev_start / T + (c - 1) / G);
    for (int64_t g = kp + 1; g <= key; ++g) {
      if (g <= glaunch) a.gfirst[g] = c;
      else atomicOr(&a.ctr->err, (uint32_t)DIG_EBIT_GROUPS);
    }
    const int ci = a.cell_inst[c];
    if (a.params[ci].cell0 == c) a.inst_pstart[ci] = st;
    prev_start = st;
    st += cnt[k];
  }
  if (b == nb - 1) {
    // the last chunk holds cell C-1: total, group tail, instance end
    __shared__ int64_t s_tot, s_klast;
    if (c0 <= C - 1 && C - 1 < c0 + kScanPer) {
      s_tot = st;
      const int64_t slast = st - cnt[(C - 1) - c0];
      s_klast = slast / T + (C - 1) / G;
    }
    __syncthreads();
    if (tid == 0) {
      a.start[C] = (int32_t)s_tot;
      a.inst_pstart[a.n_inst] = s_tot;
      if (set_n) a.ctr->n = s_tot;
    }
    for (int64_t g = s_klast + 1 + tid; g <= glaunch; g += 256) a.gfirst[g] = C;
  }
}

__global__ __launch_bounds__(256) void k_place(StepArgs a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.ctr->n) return;
  const int c = a.cell[p];
  if (c >= 0) a.perm_raw[a.start[c] + a.rank[p]] = (int32_t)p;
}

// ---------------------------------------------------------------------------
// Block-wide exclusive scan of one int per thread (blockDim a multiple of 64).
static __device__ __forceinline__ int block_exscan(int v, int* s_w, int* total) {
  int incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off);
    if (lane_id() >= off) incl += t;
  }
  if (lane_id() == 63) s_w[threadIdx.x >> 6] = incl;
  __syncthreads();
  int pre = 0, tot = 0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
    if (k < (int)(threadIdx.x >> 6)) pre += s_w[k];
    tot += s_w[k];
  }
  __syncthreads();
  *total = tot;
  return pre + incl - v;
}

// Restores (cell, slot) order inside each cell.  The provisional segment of a
// cell is a concatenation of runs, one per reserving wave; a run is increasing
// and the runs of different waves cover disjoint slot ranges, so ordering the
// runs by their first slot yields the stable counting-sort order.
constexpr int kOrderPer = 4;  // consecutive entries per thread, loaded together

// Stable order of one cell group in global memory: perm_raw -> perm.
// Tables in shared memory supplied by the caller: s_start[group_cells + 1],
// s_key and s_off[run_max], s_re[run_max + 1], s_w[16], s_nr.
static __device__ void order_group_global(const StepArgs& a, int g, int* s_start, uint32_t* s_key,
                                          uint32_t* s_re, uint32_t* s_off, int* s_w, int* s_nr,
                                          int run_max) {
  const int c_lo = a.gfirst[g], c_hi = a.gfirst[g + 1];
  if (c_lo >= c_hi) return;
  const int nc = c_hi - c_lo;
  const int e_lo = a.start[c_lo];
  const int ng = a.start[c_hi] - e_lo;
  for (int c = threadIdx.x; c <= nc; c += blockDim.x) s_start[c] = a.start[c_lo + c] - e_lo;
  if (threadIdx.x == 0) *s_nr = 0;
  __syncthreads();
  if (ng == 0) return;
  const int32_t* src = a.perm_raw + e_lo;
  int32_t* dst = a.perm + e_lo;
  const int chunk = kOrderPer * (int)blockDim.x;
  // runs: each thread flags run heads among kOrderPer consecutive entries
  bool overflow = false;
  for (int base = 0; base < ng; base += chunk) {
    const int e0 = base + kOrderPer * (int)threadIdx.x;
    uint32_t v[kOrderPer];
#pragma unroll
    for (int u = 0; u < kOrderPer; ++u) v[u] = e0 + u < ng ? (uint32_t)src[e0 + u] : 0u;
    uint32_t pv = (e0 > 0 && e0 < ng) ? (uint32_t)src[e0 - 1] : 0u;
    int c = e0 < ng ? floor_index(s_start, nc + 1, e0) : nc;
    bool head[kOrderPer];
    int cnt = 0;
#pragma unroll
    for (int u = 0; u < kOrderPer; ++u) {
      const int e = e0 + u;
      head[u] = false;
      if (e < ng) {
        while (s_start[c + 1] <= e) ++c;
        head[u] = (e == s_start[c]) || ((v[u] >> 6) != (pv >> 6));
      }
      pv = v[u];
      cnt += head[u];
    }
    int total;
    int r = *s_nr + block_exscan(cnt, s_w, &total);
#pragma unroll
    for (int u = 0; u < kOrderPer; ++u)
      if (head[u]) {
        if (r < run_max) {
          s_key[r] = v[u];
          s_re[r] = (uint32_t)(e0 + u);
        }
        ++r;
      }
    __syncthreads();
    if (threadIdx.x == 0) *s_nr += total;
    __syncthreads();
    if (*s_nr > run_max) { overflow = true; break; }
  }
  if (!overflow) {
    const int nr = *s_nr;
    if (threadIdx.x == 0) s_re[nr] = (uint32_t)ng;
    __syncthreads();
    for (int r = threadIdx.x; r < nr; r += blockDim.x) {
      const int e = (int)s_re[r];
      const int c = floor_index(s_start, nc + 1, e);
      // runs of cell c: those starting in [s_start[c], s_start[c+1])
      const int r0 = floor_index(s_re, nr + 1, (uint32_t)s_start[c]);
      const uint32_t key = s_key[r];
      uint32_t off = (uint32_t)s_start[c];
      for (int q = r0; q < nr && s_re[q] < (uint32_t)s_start[c + 1]; ++q)
        if (s_key[q] < key) off += s_re[q + 1] - s_re[q];
      s_off[r] = off;
    }
    __syncthreads();
    for (int base = 0; base < ng; base += chunk) {
      const int e0 = base + kOrderPer * (int)threadIdx.x;
      if (e0 >= ng) continue;
      int32_t v[kOrderPer];
#pragma unroll
      for (int u = 0; u < kOrderPer; ++u) v[u] = e0 + u < ng ? src[e0 + u] : 0;
      int r = floor_index(s_re, nr + 1, (uint32_t)e0);
#pragma unroll
      for (int u = 0; u < kOrderPer; ++u) {
        const int e = e0 + u;
        if (e < ng) {
          while (s_re[r + 1] <= (uint32_t)e) ++r;
          dst[s_off[r] + (uint32_t)e - s_re[r]] = v[u];
        }
      }
    }
  } else {
    // slow path: rank each entry against its cell by direct counting
    if (threadIdx.x == 0) atomicOr(&a.ctr->err, (uint32_t)DIG_EBIT_SORT_OVERFLOW);
    for (int e = threadIdx.x; e < ng; e += blockDim.x) {
      const int c = floor_index(s_start, nc + 1, e);
      const int32_t sv = src[e];
      int rank = 0;
      for (int q = s_start[c]; q < s_start[c + 1]; ++q) rank += (src[q] < sv);
      dst[s_start[c] + rank] = sv;
    }
  }
  __syncthreads();
}

// Ordering pass of a staged sort: every cell group, one workgroup each.
__global__ __launch_bounds__(256) void k_order(StepArgs a) {
  __shared__ int s_start[1025];
  __shared__ uint32_t s_key[kRunMax];
  __shared__ uint32_t s_re[kRunMax + 1];
  __shared__ uint32_t s_off[kRunMax];
  __shared__ int s_w[16];
  __shared__ int s_nr;
  order_group_global(a, xcd_group(blockIdx.x, gridDim.x), s_start, s_key, s_re, s_off, s_w,
                     &s_nr, kRunMax);
}

// ---------------------------------------------------------------------------
// Collisions.  Particle store in LDS (fast) or in the destination buffer.
struct LdsStore {
  float4* v;
  __device__ float4 ld(int i) const { return v[i]; }
  __device__ void st(int i, float4 q) const { v[i] = q; }
};
// A group's velocities and rotational energies in global memory, one
// 16-byte record per particle.
struct RecordStore {
  float4* v;
  __device__ float4 ld(int i) const { return v[i]; }
  __device__ void st(int i, float4 q) const { v[i] = q; }
};
struct GlobalStore {
  float *vx, *vy, *vz, *er;
  __device__ float4 ld(int i) const { return make_float4(vx[i], vy[i], vz[i], er[i]); }
  __device__ void st(int i, float4 q) const {
    vx[i] = q.x;
    vy[i] = q.y;
    vz[i] = q.z;
    er[i] = q.w;
  }
};

struct CollideShared {
  int* start;   // [Gc+1]
  int* coff;    // [Gc+1] candidate offsets of the large cells
  int* soff;    // [Gc+1] candidate offsets of the small cells
  uint4* words; // [2 KC] pre-drawn words of a chunk of small-cell candidates
  float* sgm;   // [Gc]
  uint32_t* obs;  // [Gc]
  int* inst;    // [Gc]
  int* stat;    // [4]
  int* wsum;    // [16]
};

// Candidate of a cell (Section 2.2): VHS acceptance of the pair against the
// majorant with the uniform word w2; returns sigma_T g and the squared
// relative speed.
static __device__ __forceinline__ bool vhs_accept(const InstParam& I, float sgm, uint32_t w2,
                                                  const float4& va, const float4& vb,
                                                  float* sg_out, float* g2_out) {
  // no contraction: every inlined copy (one-lane cells, rounds, LDS or
  // global stores) rounds alike, so results do not depend on the path
#pragma clang fp contract(off)
  const float gx = va.x - vb.x, gy = va.y - vb.y, gz = va.z - vb.z;
  const float g2 = gx * gx + gy * gy + gz * gz;
  const float sg = g2 > 0.0f ? I.csig * fpow(g2, I.expo) : 0.0f;
  *sg_out = sg;
  *g2_out = g2;
  return u01f(w2) < sg * frcp(sgm);
}

// Accepted collision: Borgnakke-Larsen exchange for the first then the
// second particle (double relaxation, tests w3 and r1.y, Beta(1, 5/2 - omega)
// splits r1.x and r1.z), then scattering that conserves momentum and the
// total energy: isotropic (cos theta from r1.w, phi from w8), or for VSS the
// deflection cos chi = 2 u^(1/alpha) - 1 (u from r1.w) about the
// pre-collision relative velocity with azimuth from w8 (Bird's rotation
// formulas, from the coordinate axis least aligned with that velocity).
// Borgnakke-Larsen fraction for d_r > 2: a Beta(d_r/2, 5/2 - omega) variate
// by acceptance-rejection in FP64 with uniform proposals against the density
// at its mode x* = (a - 1)/(a + b - 2); attempt t takes the words 2(t mod 2)
// and 2(t mod 2) + 1 of draw (cell, step, TAG_BL, 64 (2k + p) + t/2) as the
// proposal and the test; after 64 rejections (probability below 1e-30) x*.
// k: candidate of the cell, p: 0 first particle, 1 second.
static __device__ double bl_fraction(const InstParam& I, uint32_t ent, uint32_t step, uint32_t k,
                                     uint32_t p) {
  const double a = 0.5 * I.dr, b = 2.5 - I.omega;
  const double xm = (a - 1.0) / (a + b - 2.0);
  uint4 w = make_uint4(0u, 0u, 0u, 0u);
  for (uint32_t t = 0; t < 64; ++t) {
    if ((t & 1u) == 0) w = draw(I, ent, step, TAG_BL, 64u * (2u * k + p) + t / 2u);
    const double x = u01d((t & 1u) ? w.z : w.x);
    const double ut = u01d((t & 1u) ? w.w : w.y);
    const double ratio = pow(x / xm, a - 1.0) * pow((1.0 - x) / (1.0 - xm), b - 1.0);
    if (ut < ratio) return x;
  }
  return xm;
}

template <bool EXT>
static __device__ __forceinline__ void apply_collision(const InstParam& I, float g2, uint32_t w3,
                                                       uint4 r1, uint32_t w8, float4& va,
                                                       float4& vb, int* inel, uint32_t ent,
                                                       uint32_t step, uint32_t kk) {
#pragma clang fp contract(off)  // as in vhs_accept
  float et = 0.25f * g2;  // relative translational energy, reduced mass 1/2
  if (u01d(w3) < I.pin) {
    const float ec = et + va.w;
    float x = 0.0f;
    if constexpr (EXT) {
      if (I.dr != 2) x = (float)bl_fraction(I, ent, step, kk, 0u);
    }
    if (!EXT || I.dr == 2) x = 1.0f - fpow(u01f(r1.x), I.beta_inv);
    va.w = x * ec;
    et = ec - va.w;
    ++*inel;
  }
  if (u01d(r1.y) < I.pin) {
    const float ec = et + vb.w;
    float x = 0.0f;
    if constexpr (EXT) {
      if (I.dr != 2) x = (float)bl_fraction(I, ent, step, kk, 1u);
    }
    if (!EXT || I.dr == 2) x = 1.0f - fpow(u01f(r1.z), I.beta_inv);
    vb.w = x * ec;
    et = ec - vb.w;
    ++*inel;
  }
  const float hg = fsqrt(et);  // half of |g'| = 2 sqrt(et)
  float nx, ny, nz;
  bool iso = true;  // the basic kernels carry no VSS code
  if constexpr (EXT) iso = !I.vss;
  if (iso) {
    // ct = 2u - 1 is exact; sin theta from (1 - ct)(1 + ct), both factors
    // exact, keeps its relative accuracy near ct = +-1
    const float ct = 2.0f * u01f(r1.w) - 1.0f;
    const float st = fsqrt(fmaxf(0.0f, (1.0f - ct) * (1.0f + ct)));
    const float ph = 6.28318530717958648f * u01f(w8);
    const float sp = __sinf(ph), cp = __cosf(ph);
    nx = ct;
    ny = st * cp;
    nz = st * sp;
  } else {
    // azimuth from the coordinate axis least aligned with the relative
    // velocity (first on ties), in cyclic component order (a, b, c), so that
    // p = sqrt(b^2 + c^2) >= sqrt(2/3) and the rotation stays well
    // conditioned for every direction
    const float ux0 = va.x - vb.x, uy0 = va.y - vb.y, uz0 = va.z - vb.z;
    const float gi = 1.0f / fsqrt(g2);
    const float ux = ux0 * gi, uy = uy0 * gi, uz = uz0 * gi;
    const float mx = fabsf(ux), my = fabsf(uy), mz = fabsf(uz);
    const int k = (my < mx) ? ((mz < my) ? 2 : 1) : ((mz < mx) ? 2 : 0);
    const float ua = k == 0 ? ux : (k == 1 ? uy : uz);
    const float ub = k == 0 ? uy : (k == 1 ? uz : ux);
    const float uc = k == 0 ? uz : (k == 1 ? ux : uy);
    // cos chi = 2 v - 1 and sin chi = 2 sqrt(v (1 - v)), v = u^(1/alpha), in
    // FP64: near-forward deflections (v close to 1) would lose the relative
    // accuracy of 1 - v, and so of sin chi, in FP32
    const double v = pow(u01d(r1.w), I.ainv);
    const float cc = (float)(2.0 * v - 1.0);
    const float sc = (float)(2.0 * sqrt(v * (1.0 - v)));
    const float ep = 6.28318530717958648f * u01f(w8);
    const float se = __sinf(ep), ce = __cosf(ep);
    const float pp = fsqrt(ub * ub + uc * uc);
    const float ip = 1.0f / pp;
    const float na = cc * ua + sc * se * pp;
    const float nb = cc * ub + sc * (ce * uc - ua * ub * se) * ip;
    const float nc = cc * uc - sc * (ce * ub + ua * uc * se) * ip;
    nx = k == 0 ? na : (k == 1 ? nc : nb);
    ny = k == 0 ? nb : (k == 1 ? na : nc);
    nz = k == 0 ? nc : (k == 1 ? nb : na);
  }
  const float cx = 0.5f * (va.x + vb.x), cy = 0.5f * (va.y + vb.y), cz = 0.5f * (va.z + vb.z);
  va.x = cx + hg * nx;
  va.y = cy + hg * ny;
  va.z = cz + hg * nz;
  vb.x = cx - hg * nx;
  vb.y = cy - hg * ny;
  vb.z = cz - hg * nz;
}

// Every cell passed belongs to instance `iu` (wave-uniform index, so the
// parameters come through the scalar cache); a group spanning instances runs
// one call per instance segment.  my_vol: the volume of cell threadIdx.x
// when vol_mine.
//
// Cells with at most seq_max particles run their candidates in order on one
// lane; the Philox words of a chunk of their candidates are drawn beforehand
// by all lanes together.  Larger cells run in parallel rounds.  Both give the
// order of the sequential algorithm exactly.
//
// WINDOW (the oversize-group kernel, whose groups hold many candidates): the
// large cells' candidates run in a window that refills as candidates
// complete; otherwise in fixed chunks of rounds (fewer per-round costs where
// a group holds about one chunk).
// rchunk: candidates of the large cells per chunk of rounds (at most the
// thread count); cw: room for rchunk uint4 + rchunk words (5 rchunk uint32)
// in which they keep the words an accepted collision uses, drawn with the
// pair; null: an accepted candidate draws them in its round.
template <bool EXT, bool WINDOW, class Store>
static __device__ void collide_cells(const StepArgs& a, const CollideShared& S, Store P,
                                     uint32_t* owner, uint32_t omask, int nc, int c_lo,
                                     uint32_t step, int iu, double my_vol, bool vol_mine,
                                     uint4* cw, int rchunk) {
  uint32_t* cphi = (uint32_t*)(cw + rchunk);
  // candidate counts, FP64 Iround as in the oracle; cells cb..cb+per-1 per thread
  // (nc <= group_cells <= 4 * blockDim)
  const int per = (nc + (int)blockDim.x - 1) / (int)blockDim.x;
  const int cb = threadIdx.x * per, ce = min(nc, cb + per);
  // (loops over u with constant bounds keep ks, kg and obs in registers)
  int ks[4] = {0, 0, 0, 0}, kg[4] = {0, 0, 0, 0};
  int tsum_s = 0, tsum_g = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = cb + u;
    if (c >= ce) break;
    const int N = S.start[c + 1] - S.start[c];
    int k = 0;
    if (N >= 2) {
      const InstParam& I = a.params[iu];
      const uint4 r = draw(I, (uint32_t)(c_lo + c - I.cell0), step, TAG_NCAND, 0);
      const double vol = vol_mine && c == (int)threadIdx.x ? my_vol : a.cvol[c_lo + c];
      k = iround(ncand_mean(N, I.weight, (double)S.sgm[c], I.dt, vol), r.x);
    }
    if (N <= a.seq_max) ks[u] = k; else kg[u] = k;
    tsum_s += ks[u];
    tsum_g += kg[u];
  }
  int KS, KG;
  int run_s = block_exscan(tsum_s, S.wsum, &KS);
  int run_g = block_exscan(tsum_g, S.wsum, &KG);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = cb + u;
    if (c >= ce) break;
    S.soff[c] = run_s;
    S.coff[c] = run_g;
    run_s += ks[u];
    run_g += kg[u];
  }
  if (threadIdx.x == 0) {
    S.soff[nc] = KS;
    S.coff[nc] = KG;
  }
  __syncthreads();
  int l_cand = 0, l_acc = 0, l_inel = 0, l_sat = 0;
  // ---- small cells: chunks of candidates in (cell, k) order ----------------
  // In this phase a lane runs one cell's candidates in order; with at least
  // as many threads as cells the cells are dealt round robin over the waves
  // (cell l * waves + w to lane l of wave w) so that every SIMD has chains to
  // run; otherwise each thread keeps its contiguous cells.
  const int nw = (int)blockDim.x >> 6;
  const bool spread = nc <= (int)blockDim.x;
  const int my = lane_id() * nw + ((int)threadIdx.x >> 6);
  const int sb = spread ? my : cb;
  const int se = spread ? (my < nc ? my + 1 : my) : ce;
  float obs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int kb = 0; kb < KS; kb += kCandChunk) {
    const int kc = min(kCandChunk, KS - kb);
    for (int q = threadIdx.x; q < kc; q += blockDim.x) {
      const int k = kb + q;
      const int c = floor_index(S.soff, nc + 1, k);
      const int kk = k - S.soff[c];
      const int N = S.start[c + 1] - S.start[c];
      const InstParam& I = a.params[iu];
      const uint32_t ent = (uint32_t)(c_lo + c - I.cell0);
      const uint4 r0 = draw(I, ent, step, TAG_COLL, 3u * (uint32_t)kk);
      const uint4 r1 = draw(I, ent, step, TAG_COLL, 3u * (uint32_t)kk + 1u);
      const uint4 r2 = draw(I, ent, step, TAG_COLL, 3u * (uint32_t)kk + 2u);
      const uint32_t i = pick(r0.x, (uint32_t)N);
      uint32_t j = pick(r0.y, (uint32_t)(N - 1));
      j += (j >= i);
      uint4* w = S.words + 2 * q;
      w[0] = make_uint4(i | (j << 16), r0.z, r0.w, r2.x);
      w[1] = r1;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = sb + u;
      if (c >= se) break;
      const int k0 = max(S.soff[c], kb), k1 = min(S.soff[c + 1], kb + kc);
      if (k0 >= k1) continue;
      const InstParam& I = a.params[iu];
      const int b = S.start[c];
      const float sgm = S.sgm[c];
      for (int k = k0; k < k1; ++k) {
        const uint4* w = S.words + 2 * (k - kb);
        const uint4 w0 = w[0];
        const int i = b + (int)(w0.x & 0xFFFFu), j = b + (int)(w0.x >> 16);
        float4 va = P.ld(i), vb = P.ld(j);
        float sg, g2;
        const bool acc = vhs_accept(I, sgm, w0.y, va, vb, &sg, &g2);
        obs[u] = fmaxf(obs[u], sg);
        ++l_cand;
        l_sat += sg > sgm;
        if (acc) {
          apply_collision<EXT>(I, g2, w0.z, w[1], w0.w, va, vb, &l_inel,
                               (uint32_t)(c_lo + c - I.cell0), step, (uint32_t)(k - S.soff[c]));
          ++l_acc;
          P.st(i, va);
          P.st(j, vb);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (sb + u < se) atomicMax(&S.obs[sb + u], __float_as_uint(obs[u]));
  if constexpr (WINDOW) {
  // ---- large cells: a window of pending candidates, one per thread,
  // executed in rounds; a candidate runs once it is the earliest pending
  // candidate of both its particles, which reproduces the sequential order.
  // Whenever a thread's candidate has run, the thread takes the next
  // candidate in order (an LDS counter), so every round keeps the window
  // full instead of draining a fixed chunk.  Candidates are numbered within
  // epochs of 65536; ownership keys carry the round, (0xFFFF - r) << 16 |
  // (k - epoch base), so a key of round r is below every key of earlier
  // rounds and stale words need no reset within an epoch (every round runs at
  // least one candidate, so an epoch has fewer than 65536 rounds).  Particle e
  // owns word e & omask: a shared word only delays the later candidate by a
  // round (the earliest pending one always holds both of its words), so a
  // table smaller than the group is safe.  Which thread takes which candidate
  // does not matter: the set of candidates pending in each round is fixed by
  // the sequential order alone ---------------------------------------------
  // cw (room for rchunk uint4 + rchunk words, when the dead source arrays
  // hold a slot per thread): the words an accepted candidate needs, drawn
  // with its pair, so that no round waits on Philox
  if (rchunk < (int)blockDim.x) cw = nullptr;
  const int K = KG;
  const int q = threadIdx.x;
  int* s_next = S.wsum + 15;  // free after the candidate-count scans
  const uint32_t nown = omask == 0xFFFFFFFFu ? (uint32_t)S.start[nc] : omask + 1u;
  for (int eb = 0; eb < K; eb += 65536) {
    const int ee = min(K, eb + 65536);
    for (uint32_t e = threadIdx.x; e < nown; e += blockDim.x) owner[e] = 0xFFFFFFFFu;
    if (threadIdx.x == 0) *s_next = eb + (int)blockDim.x;
    int k = eb + q < ee ? eb + q : -1;
    int ci = 0, cj = 0, cc = 0;
    uint32_t w2 = 0, w3 = 0;
    // pair and acceptance words of candidate k (cell cc, particles ci, cj)
    auto take = [&](int kn) {
      cc = floor_index(S.coff, nc + 1, kn);
      const int kk = kn - S.coff[cc];
      const int N = S.start[cc + 1] - S.start[cc];
      const InstParam& I = a.params[iu];
      const uint4 r = draw(I, (uint32_t)(c_lo + cc - I.cell0), step, TAG_COLL, 3u * (uint32_t)kk);
      const int i = (int)pick(r.x, (uint32_t)N);
      int j = (int)pick(r.y, (uint32_t)(N - 1));
      j += (j >= i);
      ci = S.start[cc] + i;
      cj = S.start[cc] + j;
      w2 = r.z;
      w3 = r.w;
      if (cw) {
        const uint32_t ent = (uint32_t)(c_lo + cc - I.cell0);
        cw[q] = draw(I, ent, step, TAG_COLL, 3u * (uint32_t)kk + 1u);
        cphi[q] = draw(I, ent, step, TAG_COLL, 3u * (uint32_t)kk + 2u).x;
      }
    };
    if (k >= 0) take(k);
    __syncthreads();
    for (uint32_t r = 0;; ++r) {
      const uint32_t key = ((0xFFFFu - r) << 16) | (uint32_t)(k - eb);
      const uint32_t oi = (uint32_t)ci & omask, oj = (uint32_t)cj & omask;
      if (k >= 0) {
        atomicMin(&owner[oi], key);
        atomicMin(&owner[oj], key);
      }
      __syncthreads();
      const bool run = k >= 0 && owner[oi] == key && owner[oj] == key;
      if (run) {
        const InstParam& I = a.params[iu];
        float4 va = P.ld(ci), vb = P.ld(cj);
        float sg, g2;
        const float sgm = S.sgm[cc];
        const bool acc = vhs_accept(I, sgm, w2, va, vb, &sg, &g2);
        atomicMax(&S.obs[cc], __float_as_uint(sg));
        ++l_cand;
        l_sat += sg > sgm;
        if (acc) {
          const uint32_t kk = (uint32_t)(k - S.coff[cc]);
          const uint32_t ent = (uint32_t)(c_lo + cc - I.cell0);
          const uint4 r1 = cw ? cw[q] : draw(I, ent, step, TAG_COLL, 3u * kk + 1u);
          const uint32_t w8 = cw ? cphi[q] : draw(I, ent, step, TAG_COLL, 3u * kk + 2u).x;
          apply_collision<EXT>(I, g2, w3, r1, w8, va, vb, &l_inel, ent, step, kk);
          ++l_acc;
          P.st(ci, va);
          P.st(cj, vb);
        }
      }
      // threads whose candidate ran take the next ones in order (one LDS
      // atomic per wave), if any are left in this epoch
      const unsigned long long m = __ballot(run);
      if (m) {
        const int leader = __ffsll(m) - 1;
        int base = 0;
        if (lane_id() == leader) base = atomicAdd(s_next, __popcll(m));
        base = __shfl(base, leader);
        if (run) {
          k = base + __popcll(m & __lanemask_lt());
          if (k < ee) take(k); else k = -1;
        }
      }
      if (!__syncthreads_or(k >= 0)) break;
    }
  }
  } else {
  // ---- large cells: candidates staged in chunks and executed in rounds; a
  // candidate runs once it is the earliest pending candidate of both its
  // particles.  Ownership keys carry the round, (0xFFFF - r) << 16 | q, so a
  // key of round r is below every key of earlier rounds: the owner words are
  // reset once per chunk (in the staging pass), not before every round.
  // Particle e owns word e & omask: a shared word only delays the later
  // candidate by a round (the earliest pending one always holds both of its
  // words), so a table smaller than the group is safe -------------------------
  // Thread q keeps candidate q of the chunk in registers (both collide
  // kernels run kRoundChunkMax threads).
  const int K = KG;
  const int q = threadIdx.x;
  for (int kb = 0; kb < K; kb += rchunk) {
    const int kc = min(rchunk, K - kb);
    bool pend = q < kc;
    int ci = 0, cj = 0, cc = 0;
    uint32_t w2 = 0, w3 = 0;
    if (pend) {
      const int k = kb + q;
      cc = floor_index(S.coff, nc + 1, k);
      const int kk = k - S.coff[cc];
      const int N = S.start[cc + 1] - S.start[cc];
      const InstParam& I = a.params[iu];
      const uint32_t ent = (uint32_t)(c_lo + cc - I.cell0);
      const uint4 r = draw(I, ent, step, TAG_COLL, 3u * (uint32_t)kk);
      int i = (int)pick(r.x, (uint32_t)N);
      int j = (int)pick(r.y, (uint32_t)(N - 1));
      j += (j >= i);
      ci = S.start[cc] + i;
      cj = S.start[cc] + j;
      owner[(uint32_t)ci & omask] = 0xFFFFFFFFu;
      owner[(uint32_t)cj & omask] = 0xFFFFFFFFu;
      w2 = r.z;
      w3 = r.w;
      if (cw) {
        cw[q] = draw(I, ent, step, TAG_COLL, 3u * (uint32_t)kk + 1u);
        cphi[q] = draw(I, ent, step, TAG_COLL, 3u * (uint32_t)kk + 2u).x;
      }
    }
    __syncthreads();
    for (uint32_t r = 0;; ++r) {
      const uint32_t key = ((0xFFFFu - r) << 16) | (uint32_t)q;  // r < rchunk rounds
      const uint32_t oi = (uint32_t)ci & omask, oj = (uint32_t)cj & omask;
      if (pend) {
        atomicMin(&owner[oi], key);
        atomicMin(&owner[oj], key);
      }
      __syncthreads();
      int more = 0;
      if (pend) {
        if (owner[oi] != key || owner[oj] != key) {
          more = 1;
        } else {
          pend = false;
          const InstParam& I = a.params[iu];
          float4 va = P.ld(ci), vb = P.ld(cj);
          float sg, g2;
          const float sgm = S.sgm[cc];
          const bool acc = vhs_accept(I, sgm, w2, va, vb, &sg, &g2);
          atomicMax(&S.obs[cc], __float_as_uint(sg));
          ++l_cand;
          l_sat += sg > sgm;
          if (acc) {
            uint4 r1;
            uint32_t w8;
            if (cw) {
              r1 = cw[q];
              w8 = cphi[q];
            } else {
              const int kk = kb + q - S.coff[cc];
              const uint32_t ent = (uint32_t)(c_lo + cc - I.cell0);
              r1 = draw(I, ent, step, TAG_COLL, 3u * (uint32_t)kk + 1u);
              w8 = draw(I, ent, step, TAG_COLL, 3u * (uint32_t)kk + 2u).x;
            }
            apply_collision<EXT>(I, g2, w3, r1, w8, va, vb, &l_inel,
                                 (uint32_t)(c_lo + cc - I.cell0), step,
                                 (uint32_t)(kb + q - S.coff[cc]));
            ++l_acc;
            P.st(ci, va);
            P.st(cj, vb);
          }
        }
      }
      if (!__syncthreads_or(more)) break;
    }
  }
  }
  // statistics: wave sums first, one shared-memory atomic per wave and value
  for (int off = 32; off > 0; off >>= 1) {
    l_cand += __shfl_xor(l_cand, off);
    l_acc += __shfl_xor(l_acc, off);
    l_inel += __shfl_xor(l_inel, off);
    l_sat += __shfl_xor(l_sat, off);
  }
  if (lane_id() == 0) {
    if (l_cand) atomicAdd(&S.stat[0], l_cand);
    if (l_acc) atomicAdd(&S.stat[1], l_acc);
    if (l_inel) atomicAdd(&S.stat[2], l_inel);
    if (l_sat) atomicAdd(&S.stat[3], l_sat);
  }
}

// FP64 raw sums of a cell by a subgroup of W lanes (W = 8, or the whole wave
// for cells above kWaveSumMin particles): lane j of the subgroup sums
// particles j, j+W, j+2W, ... in slot order, then a fixed xor butterfly over
// the W lanes.  W is a function of the cell's size alone, so the bits depend
// only on the cell's particle order, never on launch parameters.  All 64
// lanes of the wave must call it.
constexpr int kSub = 8;
constexpr int kWaveSumMin = 256;
template <int W = kSub, class Store>
static __device__ void sub_cell_sums(Store P, int b, int N, double s[17]) {
#pragma unroll
  for (int f = 0; f < 17; ++f) s[f] = 0.0;
  for (int k = lane_id() & (W - 1); k < N; k += W) {
    const float4 v = P.ld(b + k);
    const double x = v.x, y = v.y, z = v.z, e = v.w;
    const double v2 = x * x + y * y + z * z;
    s[0] += 1.0;
    s[1] += x;
    s[2] += y;
    s[3] += z;
    s[4] += x * x;
    s[5] += y * y;
    s[6] += z * z;
    s[7] += x * y;
    s[8] += x * z;
    s[9] += y * z;
    s[10] += x * v2;
    s[11] += y * v2;
    s[12] += z * v2;
    s[13] += e;
    s[14] += x * e;
    s[15] += y * e;
    s[16] += z * e;
  }
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1)
#pragma unroll
    for (int f = 0; f < 17; ++f) s[f] += __shfl_xor(s[f], off);
}

static __device__ __forceinline__ double select17(const double s[17], int f) {
  double r = 0.0;
#pragma unroll
  for (int k = 0; k < 17; ++k) r = (f == k) ? s[k] : r;
  return r;
}

// Sum f of one particle, written as in sub_cell_sums.
static __device__ __forceinline__ double raw_term(int f, double x, double y, double z, double e,
                                                  double v2) {
  switch (f) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * x;
    case 5: return y * y;
    case 6: return z * z;
    case 7: return x * y;
    case 8: return x * z;
    case 9: return y * z;
    case 10: return x * v2;
    case 11: return y * v2;
    case 12: return z * v2;
    case 13: return e;
    case 14: return x * e;
    case 15: return y * e;
    default: return z * e;
  }
}

// Sums F0 .. F0 + NF - 1 of sub_cell_sums, with the same order of additions
// (so the same bits), for fewer live registers.
template <int F0, int NF, int W = kSub, class Store>
static __device__ void sub_cell_sums_part(Store P, int b, int N, double s[NF]) {
#pragma unroll
  for (int f = 0; f < NF; ++f) s[f] = 0.0;
  for (int k = lane_id() & (W - 1); k < N; k += W) {
    const float4 v = P.ld(b + k);
    const double x = v.x, y = v.y, z = v.z, e = v.w;
    double v2 = 0.0;
    if constexpr (F0 <= 12 && F0 + NF > 10) v2 = x * x + y * y + z * z;
#pragma unroll
    for (int f = 0; f < NF; ++f) s[f] += raw_term(F0 + f, x, y, z, e, v2);
  }
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1)
#pragma unroll
    for (int f = 0; f < NF; ++f) s[f] += __shfl_xor(s[f], off);
}

template <int NF>
static __device__ __forceinline__ double select_n(const double s[NF], int f) {
  double r = 0.0;
#pragma unroll
  for (int k = 0; k < NF; ++k) r = (f == k) ? s[k] : r;
  return r;
}

// One workgroup (a single wave) per cell group: gather the group's particles
// from the previous buffer in sorted order (positions and ids straight to the
// destination, velocities and rotational energies into LDS), collide, write
// back, and add the cells' FP64 raw sums to the accumulator.
constexpr int kCollideThreads = 256;
constexpr int kGatherUnroll = 4;
constexpr int kStagePer = 3;   // provisional entries per thread loaded with the cell data
constexpr int kRankMax = 128;  // cells up to this size are ordered by counting ranks
// lown and sord hold 2 * 4 * L bytes, L >= 512
static_assert(2 * sizeof(uint32_t) * 512 >= 2 * sizeof(uint4) * kCandChunk,
              "candidate words must fit the free source arrays");

// Stable order of a group's particles from the provisional scatter (the
// algorithm of k_order, for one cell group inside the collide): runs of the
// provisional segment of a cell (one per reserving wave, increasing sources)
// are ordered by their first source.  st: cell starts relative to the group
// (LDS), raw/ord: provisional and ordered sources (LDS or global).  run_slots
// runs per group (kRunSlots in the small-group collide); more fall back to
// counting ranks.
constexpr int kRunSlots = 256;
template <class Raw, class Ord>
static __device__ __forceinline__ void order_runs(const int* st, int nc, int ng, Raw raw, Ord ord,
                                                  uint32_t* rkey, uint32_t* rre, uint32_t* roff,
                                                  int* s_w, int run_slots) {
  // each thread walks a block of consecutive elements: runs are counted, the
  // counts scanned, then written in element order.  The barrier publishes the
  // caller's writes of st and raw.
  __syncthreads();
  const int per = (ng + (int)blockDim.x - 1) / (int)blockDim.x;
  const int e0 = min(ng, (int)threadIdx.x * per), e1 = min(ng, e0 + per);
  const int c0 = e0 < ng ? floor_index(st, nc + 1, e0) : nc;
  const uint32_t p0 = (e0 > 0 && e0 < ng) ? (uint32_t)raw[e0 - 1] : 0u;
  int cnt = 0;
  {
    int c = c0;
    uint32_t pv = p0;
    for (int e = e0; e < e1; ++e) {
      while (st[c + 1] <= e) ++c;
      const uint32_t sv = (uint32_t)raw[e];
      cnt += (e == st[c]) || ((sv >> 6) != (pv >> 6));
      pv = sv;
    }
  }
  int nr;
  int r = block_exscan(cnt, s_w, &nr);
  if (nr <= run_slots) {
    int c = c0;
    uint32_t pv = p0;
    for (int e = e0; e < e1; ++e) {
      while (st[c + 1] <= e) ++c;
      const uint32_t sv = (uint32_t)raw[e];
      if ((e == st[c]) || ((sv >> 6) != (pv >> 6))) {
        rkey[r] = sv;
        rre[r] = (uint32_t)e;
        ++r;
      }
      pv = sv;
    }
    if (threadIdx.x == 0) rre[nr] = (uint32_t)ng;
    __syncthreads();
    for (int q = threadIdx.x; q < nr; q += blockDim.x) {
      const int c = floor_index(st, nc + 1, (int)rre[q]);
      const int q0 = floor_index(rre, nr + 1, (uint32_t)st[c]);
      const uint32_t key = rkey[q];
      uint32_t off = (uint32_t)st[c];
      for (int t = q0; t < nr && rre[t] < (uint32_t)st[c + 1]; ++t)
        if (rkey[t] < key) off += rre[t + 1] - rre[t];
      roff[q] = off;
    }
    __syncthreads();
    if (e0 < e1) {
      int q = floor_index(rre, nr + 1, (uint32_t)e0);
      for (int e = e0; e < e1; ++e) {
        while (rre[q + 1] <= (uint32_t)e) ++q;
        ord[roff[q] + (uint32_t)e - rre[q]] = raw[e];
      }
    }
  } else {
    for (int e = threadIdx.x; e < ng; e += blockDim.x) {
      const int c = floor_index(st, nc + 1, e);
      const int32_t sv = raw[e];
      int rank = 0;
      for (int q = st[c]; q < st[c + 1]; ++q) rank += (raw[q] < sv);
      ord[st[c] + rank] = sv;
    }
  }
  __syncthreads();
}

// What a collide launch does with a cell group:
//   kModeStaged  every group; the permutation was ordered by k_order.
//   kModeSmall   groups that fit the stage of L particles are ordered here;
//                larger ones are listed for k_collide_big and skipped.
//   kModeBig     a listed group, ordered here in the (larger) stage of L
//                particles or, when it does not fit, in global memory.
enum { kModeStaged = 0, kModeSmall = 1, kModeBig = 2 };

// two_pass: the cells' moment sums in two passes (fewer live registers, for
// the 80-VGPR budget of six waves per SIMD) rather than one.
template <int mode, bool EXT, bool two_pass = false>
static __device__ __forceinline__ void collide_group(const StepArgs& a, int g, int L,
                                                     int run_slots, int do_collide,
                                                     int do_sample) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int c_lo = a.gfirst[g], c_hi = a.gfirst[g + 1];
  if (c_lo >= c_hi) return;
  const int nc = c_hi - c_lo;
  const int Gc = a.group_cells;
  const uint32_t step = (uint32_t)a.ctr->step;
  // shared layout.  Until the gather fills it, the velocity stage sv holds
  // the ordering's run tables and entry -> cell map (16 L bytes >= their
  // 3 (run_slots + 1) words + L bytes, checked on the host).  After the gather
  // the source arrays lown and sord are free: the one-lane cells' pre-drawn
  // words use both (8 L >= 32 kCandChunk bytes for L >= 512) before the
  // round owners of the large cells use lown.
  unsigned char* p = smem;
  float4* sv = (float4*)p;              p += sizeof(float4) * L;
  uint32_t* lown = (uint32_t*)p;        p += sizeof(uint32_t) * L;  // round owners
  int32_t* sord = (int32_t*)p;          p += sizeof(int32_t) * L;   // ordered sources
  uint32_t* rkey = (uint32_t*)sv;
  uint32_t* rre = rkey + (run_slots + 1);
  uint32_t* roff = rre + (run_slots + 1);
  uint8_t* ecell = (uint8_t*)(roff + (run_slots + 1));  // cell of each staged entry
  CollideShared S;
  S.words = (uint4*)lown;
  S.start = (int*)p;                    p += sizeof(int) * (Gc + 1);
  S.coff = (int*)p;                     p += sizeof(int) * (Gc + 1);
  S.soff = (int*)p;                     p += sizeof(int) * (Gc + 1);
  S.sgm = (float*)p;                    p += sizeof(float) * Gc;
  S.obs = (uint32_t*)p;                 p += sizeof(uint32_t) * Gc;
  S.inst = (int*)p;                     p += sizeof(int) * Gc;
  S.stat = (int*)p;                     p += sizeof(int) * 4;
  S.wsum = (int*)p;                     p += sizeof(int) * 16;

  const int e_lo = a.start[c_lo];
  const int ng = a.start[c_hi] - e_lo;
  const bool fast = ng <= L;
  if constexpr (mode == kModeSmall) {
    if (!fast) {
      if (threadIdx.x == 0) a.big_list[atomicAdd(a.big_count, 1u)] = g;
      return;
    }
  }
  if constexpr (mode == kModeBig) {
    if (!fast) {
      // too large even for this stage: ordered in global memory, with the
      // tables in the velocity stage (unused by such a group; 16 L bytes hold
      // them, checked on the host)
      int* t_start = (int*)sv;
      uint32_t* t_key = (uint32_t*)(t_start + Gc + 1);
      uint32_t* t_re = t_key + run_slots;
      uint32_t* t_off = t_re + run_slots + 1;
      int* t_w = (int*)(t_off + run_slots);
      order_group_global(a, g, t_start, t_key, t_re, t_off, t_w, t_w + 16, run_slots);
    }
  }
  const bool stage = mode != kModeStaged && fast;
  // the provisional segment is loaded together with the cell data: the first
  // kStagePer entries of each thread into registers
  int32_t pre[kStagePer];
  if (stage) {
#pragma unroll
    for (int u = 0; u < kStagePer; ++u) {
      const int e = (int)threadIdx.x + u * (int)blockDim.x;
      pre[u] = e < ng ? a.perm_raw[e_lo + e] : 0;
    }
  }
  const double my_vol = (int)threadIdx.x < nc ? a.cvol[c_lo + threadIdx.x] : 0.0;
  for (int c = threadIdx.x; c <= nc; c += blockDim.x) {
    S.start[c] = a.start[c_lo + c] - e_lo;
    if (c < nc) {
      S.sgm[c] = a.sgmax[c_lo + c];
      S.obs[c] = 0u;
      S.inst[c] = a.cell_inst[c_lo + c];
    }
  }
  if (threadIdx.x < 4) S.stat[threadIdx.x] = 0;
  if (stage) {
    // stable order of the group: the provisional segment staged in LDS (in
    // the round-owner array, free until the collisions)
    int32_t* sraw = (int32_t*)lown;
#pragma unroll
    for (int u = 0; u < kStagePer; ++u) {
      const int e = (int)threadIdx.x + u * (int)blockDim.x;
      if (e < ng) sraw[e] = pre[u];
    }
    for (int e = threadIdx.x + kStagePer * blockDim.x; e < ng; e += blockDim.x)
      sraw[e] = a.perm_raw[e_lo + e];
    __syncthreads();
    bool big = false;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
      const int b = S.start[c], n = S.start[c + 1] - b;
      big |= n > kRankMax;
      if (n <= kRankMax)
        for (int e = b; e < b + n; ++e) ecell[e] = (uint8_t)c;
    }
    // the reduction is no memory fence: the fences publish the entry -> cell
    // map to the counting below
    __threadfence_block();
    const bool any_big = __syncthreads_or(big);
    __threadfence_block();
    if (any_big) {
      order_runs(S.start, nc, ng, (const int32_t*)sraw, sord, rkey, rre, roff, S.wsum, run_slots);
    } else {
      // every cell small: an entry's place in its cell is the number of the
      // cell's entries with a smaller source (sources are distinct)
      for (int e = threadIdx.x; e < ng; e += blockDim.x) {
        const int c = ecell[e];
        const int b = S.start[c], n = S.start[c + 1] - b;
        const int32_t key = sraw[e];
        int rank = 0;
#pragma unroll 4
        for (int q = 0; q < n; ++q) rank += sraw[b + q] < key;
        sord[b + rank] = key;
      }
      __syncthreads();
    }
  }
  const bool from_lds = stage;  // ordered sources in LDS, else in perm
  // gather, kGatherUnroll particles per lane in flight
  const bool two = a.dim == 2;
  for (int e0 = threadIdx.x; e0 < ng; e0 += kGatherUnroll * blockDim.x) {
    int src[kGatherUnroll];
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      const int e = e0 + u * blockDim.x;
      src[u] = e < ng ? (from_lds ? sord[e] : a.perm[e_lo + e]) : -1;
    }
    float x[kGatherUnroll], y[kGatherUnroll];
    float4 v[kGatherUnroll];
    uint32_t id[kGatherUnroll];
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      if (src[u] < 0) continue;
      const int q = src[u];
      x[u] = a.A.x[q];
      y[u] = two ? a.A.y[q] : 0.0f;
      id[u] = a.A.id[q];
      v[u] = make_float4(a.A.vx[q], a.A.vy[q], a.A.vz[q], a.A.er[q]);
    }
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      if (src[u] < 0) continue;
      const int e = e0 + u * blockDim.x;
      const int d = e_lo + e;
      a.B.x[d] = x[u];
      if (two) a.B.y[d] = y[u];
      a.B.id[d] = id[u];
      if (fast) sv[e] = v[u];
      else a.vstage[d] = v[u];
    }
  }
  __syncthreads();
  LdsStore ls{sv};
  // a group beyond the stage collides in its records in global memory: a
  // candidate touches two 16-byte records rather than eight words of four
  // arrays, and the records of the groups in flight stay in the caches
  RecordStore gs{a.vstage + e_lo};
  // round owners of a group collided in global memory: the velocity stage,
  // unused by such a group, as a table of the largest power of two words
  const uint32_t gmask = (1u << (31 - __clz(4 * L))) - 1u;
  // the ordered sources are dead after the gather: the large cells' collision
  // words go there when it holds a chunk of them (L >= 5 rchunk) at a 16-byte
  // boundary (sord starts at byte 20 L); chunks of kRoundChunkMax candidates
  // where it holds that many
  const bool al = L % 4 == 0;
  const int rchunk = (al && 5 * kRoundChunkMax <= L) ? kRoundChunkMax : kCandChunk;
  uint4* cw = (al && 5 * rchunk <= L) ? (uint4*)sord : nullptr;
  if (do_collide) {
    // instances are contiguous and increasing in c: one call per instance
    // segment, almost always the whole group
    for (int c0 = 0; c0 < nc;) {
      const int iu = __builtin_amdgcn_readfirstlane(S.inst[c0]);
      const int c1 = __builtin_amdgcn_readfirstlane(floor_index(S.inst, nc, iu) + 1);
      CollideShared Sg = S;
      Sg.start += c0;
      Sg.coff += c0;
      Sg.soff += c0;
      Sg.sgm += c0;
      Sg.obs += c0;
      Sg.inst += c0;
      if (fast)
        collide_cells<EXT, mode == kModeBig>(a, Sg, ls, lown, 0xFFFFFFFFu, c1 - c0, c_lo + c0, step, iu, my_vol,
                      c0 == 0, cw, rchunk);
      else
        collide_cells<EXT, mode == kModeBig>(a, Sg, gs, (uint32_t*)sv, gmask, c1 - c0, c_lo + c0, step, iu,
                           my_vol,
                      c0 == 0, cw, rchunk);
      c0 = c1;
      if (c0 < nc) __syncthreads();  // the next segment reuses the staging arrays
    }
    __syncthreads();
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
      const float o = __uint_as_float(S.obs[c]);
      if (o > S.sgm[c]) a.sgmax[c_lo + c] = o;
    }
    if (threadIdx.x < 4 && S.stat[threadIdx.x])
      atomicAdd(&a.stats[(blockIdx.x % kStatSlots) * ST_N + threadIdx.x],
                (unsigned long long)S.stat[threadIdx.x]);
  }
  // velocities and rotational energies to the destination arrays
  for (int e = threadIdx.x; e < ng; e += blockDim.x) {
    const int d = e_lo + e;
    const float4 v = fast ? sv[e] : a.vstage[d];
    a.B.vx[d] = v.x;
    a.B.vy[d] = v.y;
    a.B.vz[d] = v.z;
    a.B.er[d] = v.w;
  }
  if (do_sample) {
    __syncthreads();
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int sub = lane_id() / kSub, sl = lane_id() & (kSub - 1);
    // cells up to kWaveSumMin particles: eight per wave, an 8-lane subgroup
    // each
    for (int cb = w * (64 / kSub); cb < nc; cb += nw * (64 / kSub)) {
      const int c = cb + sub;
      const int n_c = c < nc ? S.start[c + 1] - S.start[c] : 0;
      const bool ok = c < nc && n_c <= kWaveSumMin;
      const int b = ok ? S.start[c] : 0, N = ok ? n_c : 0;
      // the accumulator is read before the sums, so its latency overlaps
      // them
      double* acc = a.acc + (int64_t)(c_lo + (ok ? c : 0)) * 17;
      if (two_pass && fast) {
        // from LDS in two passes of 9 and 8 sums: lane sl of the subgroup
        // adds sums sl and (sl = 0) 8 of the first, 9 + sl of the second
        const double p0 = ok ? acc[sl] : 0.0;
        const double p8 = ok && sl == 0 ? acc[8] : 0.0;
        const double p9 = ok ? acc[9 + sl] : 0.0;
        {
          double s[9];
          sub_cell_sums_part<0, 9>(ls, b, N, s);
          if (ok) {
            acc[sl] = p0 + select_n<8>(s, sl);
            if (sl == 0) acc[8] = p8 + s[8];
          }
        }
        {
          double s[8];
          sub_cell_sums_part<9, 8>(ls, b, N, s);
          if (ok) acc[9 + sl] = p9 + select_n<8>(s, sl);
        }
      } else {
        // one pass, from LDS or global memory
        double prev[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int f = sl + k * kSub;
          prev[k] = ok && f < 17 ? acc[f] : 0.0;
        }
        double s[17];
        if (fast) sub_cell_sums(ls, b, N, s);
        else sub_cell_sums(gs, b, N, s);
        if (ok) {
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const int f = sl + k * kSub;
            if (f < 17) acc[f] = prev[k] + select17(s, f);
          }
        }
      }
    }
    // larger cells: one wave each, taken in turn by the waves
    const int l = lane_id();
    int j = 0;
    for (int cb = 0; cb < nc; cb += 64) {
      const int c = cb + l;
      unsigned long long m =
          __ballot(c < nc && S.start[c + 1] - S.start[c] > kWaveSumMin);
      for (; m; m &= m - 1, ++j) {
        if (j % nw != w) continue;
        const int cc = cb + __ffsll((long long)m) - 1;
        const int b = S.start[cc], N = S.start[cc + 1] - b;
        double* acc = a.acc + (int64_t)(c_lo + cc) * 17;
        if (two_pass && fast) {
          const double p0 = l < 9 ? acc[l] : 0.0;
          const double p9 = l < 8 ? acc[9 + l] : 0.0;
          {
            double s[9];
            sub_cell_sums_part<0, 9, 64>(ls, b, N, s);
            if (l < 9) acc[l] = p0 + select_n<9>(s, l);
          }
          {
            double s[8];
            sub_cell_sums_part<9, 8, 64>(ls, b, N, s);
            if (l < 8) acc[9 + l] = p9 + select_n<8>(s, l);
          }
        } else {
          const double prev = l < 17 ? acc[l] : 0.0;
          double s[17];
          if (fast) sub_cell_sums<64>(ls, b, N, s);
          else sub_cell_sums<64>(gs, b, N, s);
          if (l < 17) acc[l] = prev + select17(s, l);
        }
      }
    }
  }
}

// Collide + sample of one cell group per workgroup (mode kModeStaged or
// kModeSmall).  With end_step, the last workgroup to take a grid-wide ticket
// closes the step: the sorted count becomes the particle count and the step
// counter advances.  A workgroup takes its ticket after all its threads have
// read the step counter (at their start), so no workgroup can read the
// advanced counter; nothing else the closing workgroup writes is read within
// this kernel.
// MINW: waves per SIMD the register budget must allow.  6 (80 VGPRs) is
// launched where the LDS stage leaves room for 6 workgroups per CU, 1 (no
// constraint) otherwise.  EXT: compiled with the extended collision model,
// VSS scattering and Borgnakke-Larsen fractions for d_r != 2 (instances with
// alpha = 1 and d_r = 2 still take the basic formulas); launched only where
// an instance needs it, so the basic kernels keep their register budget.
template <int MINW, int mode, bool EXT>
__global__ __launch_bounds__(kCollideThreads) __attribute__((amdgpu_waves_per_eu(MINW)))
void k_collide(StepArgs a, int do_collide, int do_sample, int end_step) {
  collide_group<mode, EXT, MINW == 6>(a, xcd_group(blockIdx.x, gridDim.x), a.lds_particles,
                                      kRunSlots, do_collide, do_sample);
  if (!end_step || threadIdx.x != 0) return;
  const uint32_t prev = atomicAdd(a.done, 1u);
  if (prev == gridDim.x - 1) {
    a.ctr->n = a.start[a.ncell];
    a.ctr->step += 1;
    if (do_sample) a.ctr->nsamp += 1;
    atomicExch(a.done, 0u);
  }
}

// The groups k_collide listed as larger than its stage: a persistent grid of
// kBigThreads-thread workgroups (four per CU, as many as its registers allow:
// most listed groups exceed the stage and collide in global memory, where
// more groups in flight pay off), each taking listed groups in turn.  With
// groups listed, every workgroup takes a ticket when done and the last one
// empties the list and, with end_step, closes the step as k_collide does;
// with none (the common case at moderate cell sizes) workgroup 0 closes the
// step alone and the others exit at once.
constexpr int kBigThreads = 256;
constexpr int kBigGrid = 1024;
static_assert(kRoundChunkMax == kCollideThreads && kRoundChunkMax == kBigThreads &&
                  kCandChunk <= kRoundChunkMax,
              "a collision round keeps one candidate per thread");
template <bool EXT>
__global__ __launch_bounds__(kBigThreads) void k_collide_big(StepArgs a, int do_collide,
                                                             int do_sample, int end_step) {
  const int nbig = __builtin_amdgcn_readfirstlane((int)*a.big_count);
  if (nbig == 0) {
    if (end_step && blockIdx.x == 0 && threadIdx.x == 0) {
      a.ctr->n = a.start[a.ncell];
      a.ctr->step += 1;
      if (do_sample) a.ctr->nsamp += 1;
    }
    return;
  }
  for (int i = blockIdx.x; i < nbig; i += gridDim.x) {
    const int g = __builtin_amdgcn_readfirstlane(a.big_list[i]);
    collide_group<kModeBig, EXT>(a, g, a.lds_big, a.big_runs, do_collide, do_sample);
    __syncthreads();  // the next group reuses the shared memory
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const uint32_t prev = atomicAdd(a.done, 1u);
  if (prev == gridDim.x - 1) {
    atomicExch(a.big_count, 0u);
    if (end_step) {
      a.ctr->n = a.start[a.ncell];
      a.ctr->step += 1;
      if (do_sample) a.ctr->nsamp += 1;
    }
    atomicExch(a.done, 0u);
  }
}

// ---------------------------------------------------------------------------
// Freestream inflow at the outer circle of an annulus: every step a reservoir
// shell r_out < r < r_res outside the domain is filled with freestream gas
// (Iround of rho V / N_eff particles per angular sector), appended after the
// current particles and moved with them; those that do not end inside the
// domain are removed by the move.  The shell is thicker than the distance a
// freestream particle travels in one step (|U| + 6 sqrt(T)) dt.
__global__ __launch_bounds__(256) void k_inject_count(StepArgs a) {
  __shared__ int s_w[4];
  __shared__ int s_run;
  const InstParam& I = a.params[0];
  const uint32_t step = (uint32_t)a.ctr->step;
  const int nt = I.nx;
  if (threadIdx.x == 0) s_run = 0;
  __syncthreads();
  for (int f0 = 0; f0 < nt; f0 += 256) {
    const int f = f0 + threadIdx.x;
    int k = 0;
    if (f < nt) {
      const uint4 r = draw(I, (uint32_t)f, step, TAG_INFLOW, 0);
      k = iround(I.res_mean, r.x);
    }
    int incl = k;
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off);
      if (lane_id() >= off) incl += v;
    }
    if (lane_id() == 63) s_w[threadIdx.x >> 6] = incl;
    __syncthreads();
    int pre = s_run;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) pre += s_w[w];
    if (f < nt) a.inj_off[f] = pre + incl - k;
    __syncthreads();
    if (threadIdx.x == 0) s_run += s_w[0] + s_w[1] + s_w[2] + s_w[3];
    __syncthreads();
  }
  // inj_off[nt]: all sectors; inj_off[nt + 1]: the particles that enter.
  // An inflow that would exceed the capacity is not clamped: none of it
  // enters (the state keeps its particles and ids) and the error bit is set.
  if (threadIdx.x == 0) {
    int64_t tot = s_run;
    const int64_t n0 = a.ctr->n;
    a.inj_off[nt] = (int32_t)tot;
    if (n0 + tot > a.capacity) {
      tot = 0;
      atomicOr(&a.ctr->err, (uint32_t)DIG_EBIT_INFLOW);
    }
    a.inj_off[nt + 1] = (int32_t)tot;
  }
}

// One workgroup per angular sector writes that sector's reservoir particles.
__global__ __launch_bounds__(256) void k_inject_fill(StepArgs a) {
  const InstParam& I = a.params[0];
  const int f = blockIdx.x;
  const int nt = I.nx;
  const uint32_t step = (uint32_t)a.ctr->step;
  const int64_t n0 = a.ctr->n;
  const int total = a.inj_off[nt + 1];
  const int o0 = a.inj_off[f], o1 = a.inj_off[f + 1];
  const float T = I.bc_T[1];
  const float sT = sqrtf(T);
  const float ra2 = I.rout2, rb2 = I.res2;
  for (int k = threadIdx.x; k < o1 - o0; k += blockDim.x) {
    const int q = o0 + k;
    if (q >= total) break;
    const uint4 w0 = draw(I, (uint32_t)f, step, TAG_INFLOW, 1u + 2u * (uint32_t)k);
    const uint4 w1 = draw(I, (uint32_t)f, step, TAG_INFLOW, 2u + 2u * (uint32_t)k);
    const float r = sqrtf(ra2 + u01f(w0.x) * (rb2 - ra2));
    const float th = I.dthf * ((float)f + u01f(w0.y));
    float sn, cs;
    sincosf(th, &sn, &cs);
    const float g1 = sqrtf(-2.0f * logf(u01f(w0.z)));
    float s0, c0, s1, c1;
    sincospif(2.0f * u01f(w0.w), &s0, &c0);
    const float g2 = sqrtf(-2.0f * logf(u01f(w1.x)));
    sincospif(2.0f * u01f(w1.y), &s1, &c1);
    const int64_t p = n0 + q;
    a.A.x[p] = r * cs;
    a.A.y[p] = r * sn;
    a.A.vx[p] = I.bc_U[1][0] + sT * (g1 * c0);
    a.A.vy[p] = I.bc_U[1][1] + sT * (g1 * s0);
    a.A.vz[p] = I.bc_U[1][2] + sT * (g2 * c1);
    a.A.er[p] = -T * logf(u01f(w1.z)) +
                (float)rot_extra(I, T, (uint32_t)(a.ctr->next_id + q), step, 0);
    a.A.id[p] = (uint32_t)(a.ctr->next_id + q);
  }
}

// Adopts the inflow: particle count and next id (one thread, after the fill).
__global__ void k_inject_end(StepArgs a) {
  const int total = a.inj_off[a.params[0].nx + 1];
  a.ctr->n += total;
  a.ctr->next_id += total;
  a.stats[ST_INJECTED] += (unsigned long long)total;
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_set_counters(dig_counters* c, int64_t n, int64_t step, int64_t next_id,
                               int reset_all) {
  c->n = n;
  c->step = step;
  c->next_id = next_id;
  if (reset_all) {
    c->nsamp = 0;
    c->candidates = c->accepted = c->inelastic = c->saturated = c->wall_hits = 0;
    c->err = 0;
    c->cur = 0;
  }
}

// ---------------------------------------------------------------------------
// Initialisation from fields [6][C].
__global__ void k_init_count(StepArgs a, const double* fields, int32_t ppc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncell) return;
  if (ppc > 0) {
    a.count[c] = ppc;
    return;
  }
  const InstParam& I = a.params[a.cell_inst[c]];
  const uint4 r = draw(I, (uint32_t)(c - I.cell0), 0, TAG_INIT_N, 0);
  a.count[c] = iround(count_mean(fields[c], a.cvol[c], I.weight), r.x);
}

__global__ void k_init_fill(StepArgs a, const double* fields) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = a.ctr->n;
  if (p >= n) return;
  const int C = a.ncell;
  const int c = floor_index(a.start, C + 1, (int32_t)p);
  const int inst = a.cell_inst[c];
  const InstParam& I = a.params[inst];
  const uint32_t id = (uint32_t)(p - a.inst_pstart[inst]);
  const int lc = c - I.cell0;
  const int ix = lc % I.nx, iy = lc / I.nx;
  const uint4 r0 = draw(I, id, 0, TAG_INIT, 0);
  const uint4 r1 = draw(I, id, 0, TAG_INIT, 1);
  const float st = sqrtf((float)fields[4 * C + c]);
  float s0, c0, s1, c1;
  const float ra = sqrtf(-2.0f * logf(u01f(r0.z)));
  sincospif(2.0f * u01f(r0.w), &s0, &c0);
  const float rb = sqrtf(-2.0f * logf(u01f(r1.x)));
  sincospif(2.0f * u01f(r1.y), &s1, &c1);
  if (I.geom == DIG_GEOM_ANNULUS) {
    // uniform over the cell's area: r^2 uniform between its face radii
    const float ra2 = a.rf2[iy], rb2 = a.rf2[iy + 1];
    const float r = sqrtf(ra2 + u01f(r0.x) * (rb2 - ra2));
    float sn, cs;
    sincosf(I.dthf * ((float)ix + u01f(r0.y)), &sn, &cs);
    a.A.x[p] = r * cs;
    a.A.y[p] = r * sn;
  } else if (I.geom == DIG_GEOM_GRADED) {
    const double* f64 = a.fc64 + I.face0;
    const float* f32 = a.fc32 + I.face0;
    a.A.x[p] = graded_point(f64, f32, ix, u01d(r0.x));
    if (I.dim == 2) a.A.y[p] = graded_point(f64 + I.nx + 1, f32 + I.nx + 1, iy, u01d(r0.y));
  } else {
    a.A.x[p] = keep_inside((float)ix + u01f(r0.x), ix);
    if (I.dim == 2) a.A.y[p] = keep_inside((float)iy + u01f(r0.y), iy);
  }
  a.A.vx[p] = (float)fields[1 * C + c] + st * (ra * c0);
  a.A.vy[p] = (float)fields[2 * C + c] + st * (ra * s0);
  a.A.vz[p] = (float)fields[3 * C + c] + st * (rb * c1);
  a.A.er[p] = -(float)fields[5 * C + c] * logf(u01f(r1.z)) +
              (float)rot_extra(I, fields[5 * C + c], id, 0, 0);
  a.A.id[p] = id;
}

// ---------------------------------------------------------------------------
// Instantaneous sums of the current state: an 8-lane subgroup per cell, or
// the whole wave for a cell above kWaveSumMin particles (the lane counts of
// the collide's sums, so the same bits).
__global__ __launch_bounds__(256) void k_sample_state(StepArgs a) {
  const int subs = (gridDim.x * blockDim.x) / kSub;
  const int s0 = (blockIdx.x * blockDim.x + threadIdx.x) / kSub;
  const int sl = lane_id() & (kSub - 1);
  GlobalStore gs{a.A.vx, a.A.vy, a.A.vz, a.A.er};
  // every lane of a wave runs the same number of iterations
  const int iters = (a.ncell + subs - 1) / subs;
  for (int it = 0; it < iters; ++it) {
    const int c = s0 + it * subs;
    const int n_c = c < a.ncell ? a.start[c + 1] - a.start[c] : 0;
    const bool ok = c < a.ncell && n_c <= kWaveSumMin;
    const int b = ok ? a.start[c] : 0, N = ok ? n_c : 0;
    double s[17];
    sub_cell_sums(gs, b, N, s);
    if (ok)
      for (int f = sl; f < 17; f += kSub) a.sums[(int64_t)c * 17 + f] = select17(s, f);
    // this wave's larger cells, one after another with all 64 lanes
    for (unsigned long long m = __ballot(c < a.ncell && !ok && sl == 0); m; m &= m - 1) {
      const int cc = __shfl(c, __ffsll((long long)m) - 1);
      const int bb = a.start[cc];
      double t[17];
      sub_cell_sums<64>(gs, bb, a.start[cc + 1] - bb, t);
      if (lane_id() < 17) a.sums[(int64_t)cc * 17 + lane_id()] = select17(t, lane_id());
    }
  }
}

// Raw sums -> sampled fields, equation DSMC_macroscopic.
__global__ void k_convert(StepArgs a, const double* sums, int average, double* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int C = a.ncell;
  if (c >= C) return;
  const InstParam& I = a.params[a.cell_inst[c]];
  const double ns = average ? (double)(a.ctr->nsamp > 0 ? a.ctr->nsamp : 1) : 1.0;
  const double* s = sums + (int64_t)c * 17;
  double o[20];
  for (int f = 0; f < 20; ++f) o[f] = 0.0;
  const double N = s[0];
  if (N > 0.0) {
    const double vol = a.cvol[c];
    const double rho = I.weight * N / (vol * ns);
    const double ux = s[1] / N, uy = s[2] / N, uz = s[3] / N;
    const double mxx = s[4] / N, myy = s[5] / N, mzz = s[6] / N;
    const double mxy = s[7] / N, mxz = s[8] / N, myz = s[9] / N;
    const double cxx = mxx - ux * ux, cyy = myy - uy * uy, czz = mzz - uz * uz;
    const double cxy = mxy - ux * uy, cxz = mxz - ux * uz, cyz = myz - uy * uz;
    const double tr = cxx + cyy + czz;
    const double Tt = tr / 3.0;
    const double Tr = 2.0 * (s[13] / N) / I.dr;
    const double rtr = mxx + myy + mzz;
    const double uu = ux * ux + uy * uy + uz * uz;
    const double u[3] = {ux, uy, uz};
    const double r2[3][3] = {{mxx, mxy, mxz}, {mxy, myy, myz}, {mxz, myz, mzz}};
    o[0] = rho;
    o[1] = ux;
    o[2] = uy;
    o[3] = uz;
    o[4] = Tt;
    o[5] = Tr;
    o[6] = rho * (cxx - tr / 3.0);
    o[7] = rho * (cyy - tr / 3.0);
    o[8] = rho * (czz - tr / 3.0);
    o[9] = rho * cxy;
    o[10] = rho * cxz;
    o[11] = rho * cyz;
    for (int i = 0; i < 3; ++i) {
      const double ru = r2[i][0] * ux + r2[i][1] * uy + r2[i][2] * uz;
      const double c3 = s[10 + i] / N - 2.0 * ru - u[i] * rtr + 2.0 * u[i] * uu;
      o[12 + i] = 0.5 * rho * c3;
      o[15 + i] = rho * (s[14 + i] / N - u[i] * (s[13] / N));
    }
    o[18] = (3.0 * Tt + I.dr * Tr) / (3.0 + I.dr);
    o[19] = N / ns;
  }
  for (int f = 0; f < 20; ++f) out[(int64_t)f * C + c] = o[f];
}

// ---------------------------------------------------------------------------
// DIG particle modification.
__global__ void k_adjust_count(StepArgs a, const double* target, uint32_t iter,
                               int32_t* newcount, int32_t* ccount) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int C = a.ncell;
  if (c >= C) return;
  const InstParam& I = a.params[a.cell_inst[c]];
  const double r = target[c], ux = target[C + c], uy = target[2 * C + c],
               uz = target[3 * C + c], tt = target[4 * C + c], trr = target[5 * C + c];
  const bool bad = !isfinite(r) || r < 0.0 || !isfinite(ux) || !isfinite(uy) ||
                   !isfinite(uz) || !isfinite(tt) || !isfinite(trr) ||
                   (r > 0.0 && (tt <= 0.0 || trr < 0.0));
  if (bad) {
    atomicOr(&a.ctr->err, (uint32_t)DIG_EBIT_TARGET);
    newcount[c] = 0;
    ccount[c] = 0;
    return;
  }
  const uint4 w = draw(I, (uint32_t)(c - I.cell0), iter, TAG_DIG_N, 0);
  const int nt = iround(count_mean(r, a.cvol[c], I.weight), w.x);
  const int N = a.start[c + 1] - a.start[c];
  newcount[c] = nt;
  ccount[c] = (N == 0) ? nt : (nt > N ? nt - N : 0);
}

// Exclusive scans of the two per-cell count arrays of a modification (target
// counts and clone counts), both in one pair of launches: blockIdx.y selects
// the array; chunk sums, then per-chunk scans offset by the preceding chunks.
constexpr int kExPer = 8;
constexpr int kExChunk = 256 * kExPer;

__global__ __launch_bounds__(256) void k_exscan_reduce(const int32_t* in0, const int32_t* in1,
                                                       int32_t n, int64_t* csum) {
  __shared__ int s_w[4];
  const int32_t* in = blockIdx.y ? in1 : in0;
  const int c0 = blockIdx.x * kExChunk + threadIdx.x * kExPer;
  int sum = 0;
#pragma unroll
  for (int u = 0; u < kExPer; ++u)
    if (c0 + u < n) sum += in[c0 + u];
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
  if (lane_id() == 0) s_w[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0)
    csum[blockIdx.y * gridDim.x + blockIdx.x] = (int64_t)s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

__global__ __launch_bounds__(256) void k_exscan_apply(const int32_t* in0, int32_t* out0,
                                                      const int32_t* in1, int32_t* out1,
                                                      int32_t n, const int64_t* csum) {
  __shared__ int s_w[4];
  __shared__ int64_t s_o[4];
  const int32_t* in = blockIdx.y ? in1 : in0;
  int32_t* out = blockIdx.y ? out1 : out0;
  const int64_t* cs = csum + blockIdx.y * gridDim.x;
  const int b = blockIdx.x, tid = threadIdx.x;
  int64_t o = 0;
  for (int k = tid; k < b; k += 256) o += cs[k];
  for (int off = 32; off > 0; off >>= 1) o += __shfl_xor(o, off);
  if (lane_id() == 0) s_o[tid >> 6] = o;
  const int c0 = b * kExChunk + tid * kExPer;
  int v[kExPer];
  int sum = 0;
#pragma unroll
  for (int u = 0; u < kExPer; ++u) {
    v[u] = c0 + u < n ? in[c0 + u] : 0;
    sum += v[u];
  }
  int tot;
  const int pre = block_exscan(sum, s_w, &tot);  // its barriers publish s_o
  int64_t run = s_o[0] + s_o[1] + s_o[2] + s_o[3] + pre;
#pragma unroll
  for (int u = 0; u < kExPer; ++u) {
    if (c0 + u < n) out[c0 + u] = (int32_t)run;
    run += v[u];
  }
  if (b == (int)gridDim.x - 1 && tid == 255) out[n] = (int32_t)run;
}

struct Slot {
  float x, y, vx, vy, vz, er;
  uint32_t id;
};

// A point of box cell (ix, iy) from two random words: grid units (ix + u,
// iy + u) in a uniform box, physical units between the faces in a graded one.
static __device__ __forceinline__ void cell_point(const StepArgs& a, const InstParam& I, int ix,
                                                  int iy, uint32_t wx, uint32_t wy, float* x,
                                                  float* y) {
  if (I.geom == DIG_GEOM_GRADED) {
    const double* f64 = a.fc64 + I.face0;
    const float* f32 = a.fc32 + I.face0;
    *x = graded_point(f64, f32, ix, u01d(wx));
    *y = I.dim == 2 ? graded_point(f64 + I.nx + 1, f32 + I.nx + 1, iy, u01d(wy)) : 0.0f;
  } else {
    *x = keep_inside((float)ix + u01f(wx), ix);
    *y = I.dim == 2 ? keep_inside((float)iy + u01f(wy), iy) : 0.0f;
  }
}


// One wave per cell: deletion by partial Fisher-Yates, clones, then the
// FP64 linear transform; writes the cell's new particles into buffer B.
constexpr int kAdjLds = 2048;
__global__ __launch_bounds__(256) void k_adjust_build(StepArgs a, const double* target,
                                                      uint32_t iter, const int32_t* newstart,
                                                      const int32_t* cstart) {
  __shared__ uint32_t s_idx[4][kAdjLds];
  __shared__ uint8_t s_del[4][kAdjLds];
  const int wl = threadIdx.x >> 6;
  const int lane = lane_id();
  const int waves = (gridDim.x * blockDim.x) >> 6;
  const int C = a.ncell;
  const int64_t next_id = a.ctr->next_id;
  for (int c = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; c < C; c += waves) {
    const InstParam& I = a.params[a.cell_inst[c]];
    const int b = a.start[c], N = a.start[c + 1] - b;
    const int ob = newstart[c], Nt = newstart[c + 1] - ob;
    const uint32_t ent = (uint32_t)(c - I.cell0);
    const int lc = c - I.cell0, ix = lc % I.nx, iy = lc / I.nx;
    const bool big = N > kAdjLds;
    uint32_t* idx = big ? (uint32_t*)(a.perm_raw + b) : s_idx[wl];
    uint8_t* del = big ? (uint8_t*)(a.rank + b) : s_del[wl];
    int nsurv = N;
    if (Nt < N) {
      const int D = N - Nt;
      for (int k = lane; k < N; k += 64) {
        idx[k] = (uint32_t)k;
        del[k] = 0;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      if (lane == 0) {
        uint4 w = make_uint4(0, 0, 0, 0);
        for (int k = 0; k < D; ++k) {
          if ((k & 3) == 0) w = draw(I, ent, iter, TAG_DIG_DEL, (uint32_t)(k >> 2));
          const uint32_t r = (k & 3) == 0 ? w.x : (k & 3) == 1 ? w.y : (k & 3) == 2 ? w.z : w.w;
          const int j = k + (int)pick(r, (uint32_t)(N - k));
          const uint32_t t = idx[k];
          idx[k] = idx[j];
          idx[j] = t;
        }
        for (int k = 0; k < D; ++k) del[idx[k]] = 1;
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
      __builtin_amdgcn_wave_barrier();
      // compact survivors in slot order into idx
      int base = 0;
      for (int k0 = 0; k0 < N; k0 += 64) {
        const int k = k0 + lane;
        const bool keep = k < N && !del[k];
        const unsigned long long m = __ballot(keep);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
        if (keep) idx[base + __popcll(m & __lanemask_lt())] = (uint32_t)k;
        base += __popcll(m);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
      }
      nsurv = Nt;
    }
    const double tux = target[C + c], tuy = target[2 * C + c], tuz = target[3 * C + c];
    const double ttt = target[4 * C + c], ttr = target[5 * C + c];
    auto load_slot = [&](int o) -> Slot {
      Slot s;
      if (o < nsurv) {
        const int q = b + (Nt < N ? (int)idx[o] : o);
        s.x = a.A.x[q];
        s.y = I.dim == 2 ? a.A.y[q] : 0.0f;
        s.vx = a.A.vx[q];
        s.vy = a.A.vy[q];
        s.vz = a.A.vz[q];
        s.er = a.A.er[q];
        s.id = a.A.id[q];
      } else if (N > 0) {
        const int k = o - N;
        const uint4 w = draw(I, ent, iter, TAG_DIG_SRC, (uint32_t)k);
        const int q = b + (int)pick(w.x, (uint32_t)N);
        cell_point(a, I, ix, iy, w.y, w.z, &s.x, &s.y);
        s.vx = a.A.vx[q];
        s.vy = a.A.vy[q];
        s.vz = a.A.vz[q];
        s.er = a.A.er[q];
        s.id = (uint32_t)(next_id + cstart[c] + k);
      } else {
        const int k = o;
        const uint4 r0 = draw(I, ent, iter, TAG_DIG_EMPTY, 2u * (uint32_t)k);
        const uint4 r1 = draw(I, ent, iter, TAG_DIG_EMPTY, 2u * (uint32_t)k + 1u);
        const double st = sqrt(ttt);
        const double ra = sqrt(-2.0 * log(u01d(r0.z)));
        const double rb = sqrt(-2.0 * log(u01d(r1.x)));
        const double p0 = 2.0 * M_PI * u01d(r0.w), p1 = 2.0 * M_PI * u01d(r1.y);
        cell_point(a, I, ix, iy, r0.x, r0.y, &s.x, &s.y);
        s.vx = (float)(tux + st * (ra * cos(p0)));
        s.vy = (float)(tuy + st * (ra * sin(p0)));
        s.vz = (float)(tuz + st * (rb * cos(p1)));
        s.id = (uint32_t)(next_id + cstart[c] + k);
        s.er = (float)(-ttr * log(u01d(r1.z)) + rot_extra(I, ttr, s.id, iter, 0));
      }
      return s;
    };
    // temporary moments (two passes, FP64), step iii
    double su[4] = {0, 0, 0, 0};
    for (int o = lane; o < Nt; o += 64) {
      const Slot s = load_slot(o);
      su[0] += s.vx;
      su[1] += s.vy;
      su[2] += s.vz;
      su[3] += s.er;
    }
    for (int off = 32; off > 0; off >>= 1)
      for (int f = 0; f < 4; ++f) su[f] += __shfl_xor(su[f], off);
    const double m = (double)Nt;
    double us[3] = {0, 0, 0}, sc = 0.0;
    if (Nt > 0) {
      us[0] = su[0] / m;
      us[1] = su[1] / m;
      us[2] = su[2] / m;
      for (int o = lane; o < Nt; o += 64) {
        const Slot s = load_slot(o);
        const double dx = s.vx - us[0], dy = s.vy - us[1], dz = s.vz - us[2];
        sc += dx * dx + dy * dy + dz * dz;
      }
      for (int off = 32; off > 0; off >>= 1) sc += __shfl_xor(sc, off);
    }
    const double tts = Nt > 0 ? sc / (3.0 * m) : 0.0;
    const double trs = Nt > 0 ? 2.0 * (su[3] / m) / I.dr : 0.0;
    const double ca = (Nt >= 2 && tts > 0.0) ? sqrt(ttt / tts) : 1.0;
    const double bx = tux - ca * us[0], by = tuy - ca * us[1], bz = tuz - ca * us[2];
    const double cr = trs > 0.0 ? ttr / trs : 1.0;
    // step iv: transform and write
    for (int o = lane; o < Nt; o += 64) {
      const Slot s = load_slot(o);
      const int d = ob + o;
      a.B.x[d] = s.x;
      if (I.dim == 2) a.B.y[d] = s.y;
      a.B.id[d] = s.id;
      a.B.vx[d] = (float)(ca * (double)s.vx + bx);
      a.B.vy[d] = (float)(ca * (double)s.vy + by);
      a.B.vz[d] = (float)(ca * (double)s.vz + bz);
      a.B.er[d] = (float)(cr * (double)s.er);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
  }
}

// ---------------------------------------------------------------------------
// Closure assembly: NSF terms, HoT = DSMC - NSF, Kn_GLL and the adaptive mask.
// Distance between the centres of cells u and v = u + 1 (mod n) along one
// axis: h on a uniform grid; on a graded one from the FP64 faces f (the
// wrapped distance across a periodic seam, L the axis length).
static __device__ __forceinline__ double centre_gap(const double* f, double h, double L, int u,
                                                   int v) {
  if (!f) return h;
  double d = 0.5 * (f[v] + f[v + 1]) - 0.5 * (f[u] + f[u + 1]);
  if (v < u) d += L;
  return d;
}

// Derivative along `axis` at cell (ix, iy): the difference of the two
// neighbours over the distance between their centres, one-sided at walls,
// wrapped across periodic faces (exact for linear fields on any grid).
static __device__ double grad_axis(const StepArgs& a, const InstParam& I, const double* f, int C,
                                   int base, int ix, int iy, int axis) {
  if (axis == 1 && I.dim == 1) return 0.0;
  const int n = axis == 0 ? I.nx : I.ny;
  if (n < 2) return 0.0;
  const double h = axis == 0 ? I.dx : I.dy;
  const double* fc = I.geom == DIG_GEOM_GRADED
                         ? a.fc64 + I.face0 + (axis == 0 ? 0 : I.nx + 1) : nullptr;
  const double L = fc ? fc[n] : 0.0;
  const int i = axis == 0 ? ix : iy;
  auto at = [&](int k) {
    return axis == 0 ? f[base + k + I.nx * iy] : f[base + ix + I.nx * k];
  };
  if (i > 0 && i < n - 1)
    return (at(i + 1) - at(i - 1)) / (centre_gap(fc, h, L, i - 1, i) + centre_gap(fc, h, L, i, i + 1));
  if (I.bc_type[2 * axis] == DIG_BC_PERIODIC) {
    const int ip = (i + 1) % n, im = (i - 1 + n) % n;
    return (at(ip) - at(im)) / (centre_gap(fc, h, L, im, i) + centre_gap(fc, h, L, i, ip));
  }
  if (i == 0) return (at(1) - at(0)) / centre_gap(fc, h, L, 0, 1);
  return (at(n - 1) - at(n - 2)) / centre_gap(fc, h, L, n - 2, n - 1);
}

__global__ void k_closure(StepArgs a, const double* F, double Att, double Atr, double Art,
                          double Arr, double kn_ref, double n_min, double* hot, uint8_t* mask,
                          double* kngll, double* nsf, double* speed) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int C = a.ncell;
  if (c >= C) return;
  const InstParam& I = a.params[a.cell_inst[c]];
  const int lc = c - I.cell0, ix = lc % I.nx, iy = lc / I.nx, base = I.cell0;
  const double rho = F[c], tt = F[4 * C + c], tr = F[5 * C + c];
  double h[12], q[12];
  for (int f = 0; f < 12; ++f) h[f] = q[f] = 0.0;
  double kn = INFINITY;
  const bool ok = rho > 0.0 && tt > 0.0;
  if (ok) {
    const double* ux = F + C;
    const double* uy = F + 2 * C;
    const double* uz = F + 3 * C;
    double d[7][2];
    const double* arr[7] = {ux, uy, uz, F + 4 * C, F + 5 * C, F, speed};
    for (int k = 0; k < 7; ++k)
      for (int ax = 0; ax < 2; ++ax) d[k][ax] = grad_axis(a, I, arr[k], C, base, ix, iy, ax);
    const double mu = I.mu0 * pow(tt, I.omega);
    const double div = d[0][0] + d[1][1];
    q[0] = -mu * (2.0 * d[0][0] - 2.0 / 3.0 * div);
    q[1] = -mu * (2.0 * d[1][1] - 2.0 / 3.0 * div);
    q[2] = -mu * (0.0 - 2.0 / 3.0 * div);
    q[3] = -mu * (d[0][1] + d[1][0]);
    q[4] = -mu * d[2][0];
    q[5] = -mu * d[2][1];
    const double det = Att * Arr - Atr * Art;
    const double kt = 0.5 * mu * (Arr * 5.0 - Atr * I.dr) / det;
    const double kr = 0.5 * mu * (-Art * 5.0 + Att * I.dr) / det;
    q[6] = -kt * d[3][0];
    q[7] = -kt * d[3][1];
    q[9] = -kr * d[4][0];
    q[10] = -kr * d[4][1];
    for (int f = 0; f < 12; ++f) h[f] = F[(int64_t)(6 + f) * C + c] - q[f];
    const double lam = mu / (rho * tt) * sqrt(M_PI * tt / 2.0);
    const double gam = (5.0 + I.dr) / (3.0 + I.dr);
    const double cs = sqrt(gam * tt);
    const double us = speed[c];
    double m = sqrt(d[5][0] * d[5][0] + d[5][1] * d[5][1]) / rho;
    m = fmax(m, sqrt(d[6][0] * d[6][0] + d[6][1] * d[6][1]) / (us > cs ? us : cs));
    m = fmax(m, sqrt(d[3][0] * d[3][0] + d[3][1] * d[3][1]) / tt);
    if (tr > 0.0) m = fmax(m, sqrt(d[4][0] * d[4][0] + d[4][1] * d[4][1]) / tr);
    kn = lam * m;
  }
  // equilibrium: Kn_GLL below kn_ref, or too few particles (mean count, row
  // 19) for the extracted terms to be more than sampling noise
  const uint8_t eq = (kn < kn_ref || F[19 * (int64_t)C + c] < n_min) ? 1 : 0;
  for (int f = 0; f < 12; ++f) {
    hot[(int64_t)f * C + c] = (eq || !ok) ? 0.0 : h[f];
    if (nsf) nsf[(int64_t)f * C + c] = q[f];
  }
  mask[c] = eq;
  kngll[c] = kn;
}

// Inputs and targets of the closure network (Section 3.1 terms, scaled to be
// dimensionless and standardised): features lambda/sqrt(Tt) du_i/dx_j
// (xx, xy, yx, yy), lambda/Tt dTt/dx_j, lambda/Tt dTr/dx_j, Kn_GLL; targets
// HoT sigma_xx/p, sigma_xy/p, sigma_yy/p, HoT q_t,j/(p sqrt(Tt)),
// HoT q_r,j/(p sqrt(Tt)).  Empty cells get zero features and targets.
__global__ void k_learn_features(StepArgs a, const double* F, const double* kn,
                                 const double* hot, MlpScale sc, float* x, float* t) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int C = a.ncell;
  if (c >= C) return;
  const InstParam& I = a.params[a.cell_inst[c]];
  const int lc = c - I.cell0, ix = lc % I.nx, iy = lc / I.nx, base = I.cell0;
  const double rho = F[c], tt = F[4 * C + c];
  double f[9], y[7];
  for (int k = 0; k < 9; ++k) f[k] = 0.0;
  for (int k = 0; k < 7; ++k) y[k] = 0.0;
  if (rho > 0.0 && tt > 0.0 && isfinite(kn[c])) {
    const double mu = I.mu0 * pow(tt, I.omega);
    const double lam = mu / (rho * tt) * sqrt(M_PI * tt / 2.0);
    const double su = lam / sqrt(tt), st = lam / tt;
    f[0] = su * grad_axis(a, I, F + C, C, base, ix, iy, 0);
    f[1] = su * grad_axis(a, I, F + C, C, base, ix, iy, 1);
    f[2] = su * grad_axis(a, I, F + 2 * C, C, base, ix, iy, 0);
    f[3] = su * grad_axis(a, I, F + 2 * C, C, base, ix, iy, 1);
    f[4] = st * grad_axis(a, I, F + 4 * C, C, base, ix, iy, 0);
    f[5] = st * grad_axis(a, I, F + 4 * C, C, base, ix, iy, 1);
    f[6] = st * grad_axis(a, I, F + 5 * C, C, base, ix, iy, 0);
    f[7] = st * grad_axis(a, I, F + 5 * C, C, base, ix, iy, 1);
    f[8] = kn[c];
    if (hot) {
      const double p = rho * tt, pq = p * sqrt(tt);
      const int hk[7] = {0, 3, 1, 6, 7, 9, 10};
      for (int k = 0; k < 7; ++k) y[k] = hot[(int64_t)hk[k] * C + c] / (k < 3 ? p : pq);
    }
    for (int k = 0; k < 9; ++k) f[k] = (f[k] - sc.x_mean[k]) / sc.x_std[k];
    for (int k = 0; k < 7; ++k) y[k] = (y[k] - sc.y_mean[k]) / sc.y_std[k];
  }
  for (int k = 0; k < 9; ++k) x[(int64_t)c * 9 + k] = (float)f[k];
  if (t)
    for (int k = 0; k < 7; ++k) t[(int64_t)c * 7 + k] = (float)y[k];
}

// Adaptive closure with three bands (Section 3.1 and its learned extension):
// Kn_GLL < Kn_ref -> NSF (mask set, HoT already 0); Kn_lo <= Kn_GLL < Kn_hi ->
// the network's prediction, unless it differs from the DSMC-extracted term by
// more than judge_abs + judge_rel |DSMC| in some component (then DSMC);
// otherwise the DSMC-extracted term.  src: 0 NSF, 1 DSMC, 2 network,
// 3 network rejected.
// Judge of the learned closure: standard error of the scaled DSMC-extracted
// term j of a cell from its sampling noise, M = N judge_steps independent
// particle samples (N the cell's mean particle count): the moment sum
// (per-particle standard deviations of an equilibrium cell, the peculiar
// velocity about the cell mean) and the NSF terms subtracted from it, whose
// central differences over 2h carry the noise of the neighbours' mean
// velocity (variance Tt/M), Tt (2 Tt^2/(3M)) and Tr (Tr^2/M).
__device__ void judge_se(const InstParam& I, double hx, double hy, double rho, double tt,
                         double tr, double N, double judge_steps, const JudgeGas& J,
                         double se[7]) {
  const double M = N * judge_steps;
  const double ihx2 = 1.0 / (2.0 * hx * hx);
  const double ihy2 = I.dim == 2 ? 1.0 / (2.0 * hy * hy) : 0.0;
  const double mu = I.mu0 * pow(tt, I.omega);
  const double kt = 0.5 * mu * (J.Arr * 5.0 - J.Atr * I.dr) / J.det;
  const double kr = 0.5 * mu * (-J.Art * 5.0 + J.Att * I.dr) / J.det;
  const double p = rho * tt, pq = p * sqrt(tt);
  const double vu = tt / M, vt = 2.0 * tt * tt / (3.0 * M), vr = tr * tr / M;
  const double nsf[7] = {mu * mu * vu * (16.0 / 9.0 * ihx2 + 4.0 / 9.0 * ihy2) / (p * p),
                         mu * mu * vu * (ihx2 + ihy2) / (p * p),
                         mu * mu * vu * (16.0 / 9.0 * ihy2 + 4.0 / 9.0 * ihx2) / (p * p),
                         kt * kt * vt * ihx2 / (pq * pq), kt * kt * vt * ihy2 / (pq * pq),
                         kr * kr * vr * ihx2 / (pq * pq), kr * kr * vr * ihy2 / (pq * pq)};
  const double d2[7] = {4.0 / 3.0, 1.0, 4.0 / 3.0, 2.5, 2.5, 1.0, 1.0};
  for (int j = 0; j < 7; ++j) se[j] = sqrt(d2[j] / M + nsf[j]);
}

__global__ void k_learn_blend(StepArgs a, const double* F, const double* kn,
                              const uint8_t* mask, const float* yp, MlpScale sc, JudgeGas J,
                              double kn_lo, double kn_hi, double judge_sigma, double judge_rel,
                              double judge_steps, double* hot, uint8_t* src) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int C = a.ncell;
  if (c >= C) return;
  const double rho = F[c], tt = F[4 * C + c];
  const double N = F[19 * (int64_t)C + c];
  uint8_t s = mask[c] ? 0 : 1;
  const double k = kn[c];
  if (!mask[c] && rho > 0.0 && tt > 0.0 && k >= kn_lo && k < kn_hi) {
    const double p = rho * tt, pq = p * sqrt(tt);
    const int hk[7] = {0, 3, 1, 6, 7, 9, 10};
    double se[7];
    if (N > 0.0) {
      const InstParam& I = a.params[a.cell_inst[c]];
      // the cell's own widths (graded box) or the uniform spacing
      double hx = I.dx, hy = I.dy;
      if (I.geom == DIG_GEOM_GRADED) {
        const double* f = a.fc64 + I.face0;
        const int lc = c - I.cell0, ix = lc % I.nx, iy = lc / I.nx;
        hx = f[ix + 1] - f[ix];
        if (I.dim == 2) hy = f[I.nx + 1 + iy + 1] - f[I.nx + 1 + iy];
      }
      judge_se(I, hx, hy, rho, tt, F[5 * C + c], N, judge_steps, J, se);
    } else {
      for (int j = 0; j < 7; ++j) se[j] = INFINITY;
    }
    double pr[7];
    bool ok = true;
    for (int j = 0; j < 7; ++j) {
      const double sc_j = j < 3 ? p : pq;
      pr[j] = ((double)yp[(int64_t)c * 7 + j] * sc.y_std[j] + sc.y_mean[j]) * sc_j;
      const double ds = hot[(int64_t)hk[j] * C + c];
      if (fabs(pr[j] - ds) / sc_j > judge_sigma * se[j] + judge_rel * fabs(ds) / sc_j) ok = false;
    }
    if (ok) {
      hot[0 * (int64_t)C + c] = pr[0];
      hot[1 * (int64_t)C + c] = pr[2];
      hot[2 * (int64_t)C + c] = -(pr[0] + pr[2]);
      hot[3 * (int64_t)C + c] = pr[1];
      hot[4 * (int64_t)C + c] = 0.0;
      hot[5 * (int64_t)C + c] = 0.0;
      hot[6 * (int64_t)C + c] = pr[3];
      hot[7 * (int64_t)C + c] = pr[4];
      hot[8 * (int64_t)C + c] = 0.0;
      hot[9 * (int64_t)C + c] = pr[5];
      hot[10 * (int64_t)C + c] = pr[6];
      hot[11 * (int64_t)C + c] = 0.0;
      s = 2;
    } else {
      s = 3;
    }
  }
  if (src) src[c] = s;
}

__global__ void k_speed(const double* F, int C, double* speed) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const double ux = F[C + c], uy = F[2 * C + c], uz = F[3 * C + c];
  speed[c] = sqrt(ux * ux + uy * uy + uz * uz);
}

// ---------------------------------------------------------------------------
// Launch wrappers.
static inline int blocks_for(int64_t n, int bs) {
  int64_t b = (n + bs - 1) / bs;
  return (int)(b < 1 ? 1 : b);
}

int64_t group_launch(const StepArgs& a) {
  return a.n_upper / a.group_particles + a.ncell / a.group_cells + 2;
}

size_t collide_lds_bytes(int lds_particles, int group_cells) {
  // velocity stage (holding the ordering tables before the gather), round
  // owners and ordered sources per particle (holding the candidate words
  // after it); per-cell offsets and data; statistics and scan slots
  return sizeof(float4) * lds_particles + 2 * sizeof(uint32_t) * lds_particles +
         sizeof(int) * 3 * (group_cells + 1) +
         (sizeof(float) + 2 * sizeof(int)) * group_cells + sizeof(int) * 20 + 16;
}

int big_run_slots(int lds_big, int group_cells) {
  // runs that fit the stage next to the entry -> cell map (in-LDS ordering)
  // and next to the cell starts (global-memory ordering), at most kRunMax
  const int64_t st = (int64_t)sizeof(float4) * lds_big;
  const int64_t a = (st - lds_big) / (3 * (int64_t)sizeof(uint32_t)) - 1;
  const int64_t b = (st - (int64_t)sizeof(int) * (group_cells + 1 + 17) - 4) /
                    (3 * (int64_t)sizeof(uint32_t));
  return (int)std::min<int64_t>(kRunMax, std::min(a, b));
}

bool big_stage_fits(int lds_big, int group_cells, size_t budget) {
  return lds_big >= 512 && big_run_slots(lds_big, group_cells) >= kRunSlots &&
         collide_lds_bytes(lds_big, group_cells) <= budget;
}

hipError_t collide_setup() {
  const hipError_t e = hipFuncSetAttribute((const void*)k_collide_big<false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)kBigLdsMax);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_collide_big<true>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBigLdsMax);
}

hipError_t launch_move(const StepArgs& a, hipStream_t s) {
  if (a.dr_any)
    hipLaunchKernelGGL(k_move<true>, dim3(blocks_for(a.n_upper, 256)), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_move<false>, dim3(blocks_for(a.n_upper, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

int scan_blocks(int ncell) { return (ncell + kScanChunk - 1) / kScanChunk; }

hipError_t launch_scan(const StepArgs& a, int32_t* counts, bool set_n, hipStream_t s) {
  const int nb = scan_blocks(a.ncell);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(256), 0, s, a, counts);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(256), 0, s, a, counts,
                     (int32_t)group_launch(a), set_n ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_place(const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_place, dim3(blocks_for(a.n_upper, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_order(const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_order, dim3((int)group_launch(a)), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <bool EXT>
static hipError_t launch_collide_t(const StepArgs& a, bool collide, bool sample, bool end_step,
                                   bool fused, hipStream_t s) {
  const size_t lds = collide_lds_bytes(a.lds_particles, a.group_cells);
  const dim3 grid((int)group_launch(a)), block(kCollideThreads);
  const int f0 = collide ? 1 : 0, f1 = sample ? 1 : 0;
  // fused: small groups here, the listed larger ones in k_collide_big, which
  // then closes the step
  const int f2 = (end_step && !fused) ? 1 : 0;
  // 160 KiB of LDS per CU; 1 KiB per workgroup kept for static LDS and
  // allocation granularity
  const bool six = 6 * (lds + 1024) <= 160 * 1024;
  if (fused) {
    if (six)
      hipLaunchKernelGGL((k_collide<6, kModeSmall, EXT>), grid, block, lds, s, a, f0, f1, f2);
    else
      hipLaunchKernelGGL((k_collide<1, kModeSmall, EXT>), grid, block, lds, s, a, f0, f1, f2);
  } else {
    if (six)
      hipLaunchKernelGGL((k_collide<6, kModeStaged, EXT>), grid, block, lds, s, a, f0, f1, f2);
    else
      hipLaunchKernelGGL((k_collide<1, kModeStaged, EXT>), grid, block, lds, s, a, f0, f1, f2);
  }
  if (fused) {
    if (!big_stage_fits(a.lds_big, a.group_cells, kBigLdsMax)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_collide_big<EXT>, dim3(kBigGrid), dim3(kBigThreads),
                       collide_lds_bytes(a.lds_big, a.group_cells), s, a, f0, f1,
                       end_step ? 1 : 0);
  }
  return hipGetLastError();
}

hipError_t launch_collide(const StepArgs& a, bool collide, bool sample, bool end_step,
                          bool fused, hipStream_t s) {
  return a.ext_any ? launch_collide_t<true>(a, collide, sample, end_step, fused, s)
                   : launch_collide_t<false>(a, collide, sample, end_step, fused, s);
}

hipError_t launch_inject(const StepArgs& a, hipStream_t s) {
  const int nt = a.inj_sectors;
  if (nt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_inject_count, dim3(1), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_inject_fill, dim3(nt), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_inject_end, dim3(1), dim3(1), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(min(blocks_for(n, 256), 4096)), dim3(256), 0, s, p,
                     n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<float>, dim3(min(blocks_for(n, 256), 4096)), dim3(256), 0, s, p, n,
                     v);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<double>, dim3(min(blocks_for(n, 256), 4096)), dim3(256), 0, s, p,
                     n, v);
  return hipGetLastError();
}

hipError_t launch_set_counters(dig_counters* c, int64_t n, int64_t step, int64_t next_id,
                               bool reset_all, hipStream_t s) {
  hipLaunchKernelGGL(k_set_counters, dim3(1), dim3(1), 0, s, c, n, step, next_id,
                     reset_all ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_init(const StepArgs& a, const double* fields, int32_t ppc, hipStream_t s,
                       int phase) {
  if (phase == 0)
    hipLaunchKernelGGL(k_init_count, dim3(blocks_for(a.ncell, 256)), dim3(256), 0, s, a, fields,
                       ppc);
  else
    hipLaunchKernelGGL(k_init_fill, dim3(blocks_for(a.n_upper, 256)), dim3(256), 0, s, a,
                       fields);
  return hipGetLastError();
}

hipError_t launch_sample_state(const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_sample_state, dim3(min(blocks_for((int64_t)a.ncell * kSub, 256), 8192)),
                     dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_convert(const StepArgs& a, const double* sums, bool average, double* out,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_convert, dim3(blocks_for(a.ncell, 128)), dim3(128), 0, s, a, sums,
                     average ? 1 : 0, out);
  return hipGetLastError();
}

hipError_t launch_adjust_count(const StepArgs& a, const double* target, uint32_t iter,
                               int32_t* newcount, int32_t* ccount, hipStream_t s) {
  hipLaunchKernelGGL(k_adjust_count, dim3(blocks_for(a.ncell, 256)), dim3(256), 0, s, a, target,
                     iter, newcount, ccount);
  return hipGetLastError();
}

int exscan_chunks(int n) { return (n + kExChunk - 1) / kExChunk; }

hipError_t launch_exscan2(const int32_t* in0, int32_t* out0, const int32_t* in1,
                          int32_t* out1, int32_t n, int64_t* csum, hipStream_t s) {
  const dim3 grid(std::max(1, exscan_chunks(n)), 2);
  hipLaunchKernelGGL(k_exscan_reduce, grid, dim3(256), 0, s, in0, in1, n, csum);
  hipLaunchKernelGGL(k_exscan_apply, grid, dim3(256), 0, s, in0, out0, in1, out1, n,
                     (const int64_t*)csum);
  return hipGetLastError();
}

hipError_t launch_adjust_build(const StepArgs& a, const double* target, uint32_t iter,
                               const int32_t* newstart, const int32_t* cstart, hipStream_t s) {
  hipLaunchKernelGGL(k_adjust_build, dim3(min(blocks_for((int64_t)a.ncell * 64, 256), 4096)),
                     dim3(256), 0, s, a, target, iter, newstart, cstart);
  return hipGetLastError();
}

// Empty cells of a time average take the fallback state (see fields_fill_empty).
__global__ void k_fill_empty(StepArgs a, double* F, const double* fb) {
#pragma clang fp contract(off)
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int C = a.ncell;
  if (c >= C) return;
  const double rho = F[c], tt = F[4 * C + c], tr = F[5 * C + c], n = F[19 * (int64_t)C + c];
  bool usable = n > 0.0 && rho > 0.0 && tt > 0.0 && tr >= 0.0;
  for (int k = 0; k < 6; ++k) usable = usable && isfinite(F[(int64_t)k * C + c]);
  if (usable) return;
  const int dr = a.params[a.cell_inst[c]].dr;
  for (int k = 0; k < 6; ++k) F[(int64_t)k * C + c] = fb[(int64_t)k * C + c];
  for (int k = 6; k < 18; ++k) F[(int64_t)k * C + c] = 0.0;
  F[18 * (int64_t)C + c] = (3.0 * fb[4 * C + c] + dr * fb[5 * C + c]) / (3.0 + dr);
  F[19 * (int64_t)C + c] = 0.0;
}

hipError_t launch_fill_empty(const StepArgs& a, double* fields, const double* fallback,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_fill_empty, dim3(blocks_for(a.ncell, 256)), dim3(256), 0, s, a, fields,
                     fallback);
  return hipGetLastError();
}

hipError_t launch_closure(const StepArgs& a, const double* fields, double Att, double Atr,
                          double Art, double Arr, double kn_ref, double n_min, double* hot,
                          uint8_t* mask, double* kngll, double* nsf, hipStream_t s) {
  // speed of each cell, staged in the sums scratch (C doubles)
  hipLaunchKernelGGL(k_speed, dim3(blocks_for(a.ncell, 256)), dim3(256), 0, s, fields, a.ncell,
                     a.sums);
  hipLaunchKernelGGL(k_closure, dim3(blocks_for(a.ncell, 128)), dim3(128), 0, s, a, fields, Att,
                     Atr, Art, Arr, kn_ref, n_min, hot, mask, kngll, nsf, a.sums);
  return hipGetLastError();
}

hipError_t launch_learn_features(const StepArgs& a, const double* F, const double* kn,
                                 const double* hot, const MlpScale& sc, float* x, float* t,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_learn_features, dim3(blocks_for(a.ncell, 256)), dim3(256), 0, s, a, F, kn,
                     hot, sc, x, t);
  return hipGetLastError();
}

hipError_t launch_learn_blend(const StepArgs& a, const double* F, const double* kn,
                              const uint8_t* mask, const float* y, const MlpScale& sc,
                              const JudgeGas& J, double kn_lo, double kn_hi,
                              double judge_sigma, double judge_rel, double judge_steps,
                              double* hot, uint8_t* src, hipStream_t s) {
  hipLaunchKernelGGL(k_learn_blend, dim3(blocks_for(a.ncell, 256)), dim3(256), 0, s, a, F, kn,
                     mask, y, sc, J, kn_lo, kn_hi, judge_sigma, judge_rel, judge_steps, hot,
                     src);
  return hipGetLastError();
}

}  // namespace dig
