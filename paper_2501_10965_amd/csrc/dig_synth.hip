// Synthetic-equation solve on the GPU (DIG step 3, Section 3), FP64.
//
// Steady conservation of mass, momentum and total energy plus the rotational
// relaxation equation (equation macroscopic_equation), closed by NSF terms
// plus the DSMC higher-order terms, which are zeroed where the adaptive mask
// is set (equations full_constitutive, ns_constitutive, kappa_A; Section 3.1).
// The paper defers the numerics to other work; this library uses finite
// volumes on the uniform or graded box grid (cell widths, centre gaps) with
// HLLC inviscid fluxes, central viscous and heat fluxes and Dirichlet wall
// faces (wall values or the DSMC slip and jump of the wall-adjacent cell).
// Two pseudo-time schemes march the same residual: explicit steps that are
// the same in every cell (the total mass is conserved exactly), and LU-SGS
// (the implicit scheme Section 4 names) in matrix-free form with a two-colour
// cell order, each iteration's state scaled back to the initial mass.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <mutex>
#include <vector>
#include <string>

#include "dig_internal.h"

namespace dig {

struct SynthGrid {
  int nx, ny, dim, dr;
  double hx, hy, mu0, omega, zrot, gam, cv, cfl;
  double Att, Atr, Art, Arr;
  int bc_periodic[2];  // axis periodic?
  // cell widths wx [nx], wy [ny] and, for every face, the distance between
  // the centres on either side of it, gx [nx + 1], gy [ny + 1] (half a cell
  // at a wall, the wrapped distance at a periodic seam); uniform grids: h
  const double *wx, *wy, *gx, *gy;
};

struct SynthArrays {
  const double* W;   // [6][C] current state
  double* Wn;        // [6][C] next state
  double* Fx;        // [6][ny][nx+1]
  double* Fy;        // [6][ny+1][nx]
  const double* H;   // [12][C] masked HoT (zeros when none)
  double* P;         // [6][C] primitives (rho, ux, uy, uz, Tt, Tr) of W: written by the kernel
                     // that produces a state, read by the next iteration's kernels
  const double* wall;  // [4 faces][5][max(nx,ny)]: ux uy uz tt tr of each wall face
  unsigned long long* red;  // [2][2]: dtau (min), change (max), by iteration parity
};

// T^omega of the viscosity law as exp(omega ln T): within a few ulps of pow
// (T is positive), with a shorter chain of dependent FP64 operations.
__device__ __forceinline__ double visc_pow(const SynthGrid& g, double T) {
  return exp(g.omega * log(T));
}

struct Prim {
  double rho, u[3], tt, tr;
};

// Stored primitives of cell c.
__device__ __forceinline__ Prim prim_at(const double* P, int C, int c) {
  Prim p;
  p.rho = P[c];
  for (int k = 0; k < 3; ++k) p.u[k] = P[(1 + k) * C + c];
  p.tt = P[4 * C + c];
  p.tr = P[5 * C + c];
  return p;
}

__device__ __forceinline__ void store_prim(double* P, int C, int c, const Prim& p) {
  P[c] = p.rho;
  for (int k = 0; k < 3; ++k) P[(1 + k) * C + c] = p.u[k];
  P[4 * C + c] = p.tt;
  P[5 * C + c] = p.tr;
}

__device__ __forceinline__ Prim prim_of(const double* W, int C, int c, int dr) {
  Prim p;
  p.rho = W[c];
  for (int k = 0; k < 3; ++k) p.u[k] = W[(1 + k) * C + c] / p.rho;
  p.tr = 2.0 * W[5 * C + c] / (dr * p.rho);
  const double uu = p.u[0] * p.u[0] + p.u[1] * p.u[1] + p.u[2] * p.u[2];
  p.tt = (W[4 * C + c] / p.rho - 0.5 * uu - 0.5 * dr * p.tr) * 2.0 / 3.0;
  return p;
}

__device__ __forceinline__ void conductivities(const SynthGrid& g, double mu, double* kt,
                                               double* kr) {
  const double det = g.Att * g.Arr - g.Atr * g.Art;
  *kt = 0.5 * mu * (g.Arr * 5.0 - g.Atr * g.dr) / det;
  *kr = 0.5 * mu * (-g.Art * 5.0 + g.Att * g.dr) / det;
}

// central derivative of velocity component k along axis at cell (ix, iy):
// the two neighbours (one-sided at a wall) over the distance between their
// centres.  The neighbours are chosen first and then loaded without a branch,
// so the loads of all calls issue together.
__device__ double dcen_u(const SynthGrid& g, const double* P, int C, int ix, int iy, int k,
                         int axis) {
  if (axis == 1 && g.dim == 1) return 0.0;
  const int n = axis == 0 ? g.nx : g.ny;
  const double* gap = axis == 0 ? g.gx : g.gy;
  const int i = axis == 0 ? ix : iy;
  const bool per = g.bc_periodic[axis] != 0;
  const bool inner = per || (i > 0 && i < n - 1);
  int jp, jm;
  if (n < 2) {
    jp = jm = i;
  } else if (per) {
    jp = (i + 1) % n;
    jm = (i - 1 + n) % n;
  } else {
    jp = i == 0 ? 1 : (i == n - 1 ? n - 1 : i + 1);
    jm = i == 0 ? 0 : (i == n - 1 ? n - 2 : i - 1);
  }
  // centre distance: gap[i] + gap[i + 1] inside, gap[1] or gap[n - 1] at a wall
  const int ga = inner ? i : (i == 0 ? 1 : n - 1);
  const double g0 = gap[ga];
  const double g1 = gap[i + 1];
  const int cp = axis == 0 ? jp + g.nx * iy : ix + g.nx * jp;
  const int cm = axis == 0 ? jm + g.nx * iy : ix + g.nx * jm;
  const double up = P[(1 + k) * C + cp];
  const double um = P[(1 + k) * C + cm];
  if (!per && n < 2) return 0.0;
  return (up - um) / (inner ? g0 + g1 : g0);
}

// NSF + HoT stress and heat flux through a face normal to `axis`.
template <int axis>
__device__ __forceinline__ void visc_flux(const SynthGrid& g, double tf, const double uf[3],
                                          const double dn[3], const double dt[3], double dTt,
                                          double dTr, const double Hf[12], double V[6]) {
  const double mu = g.mu0 * visc_pow(g, tf);
  double kt, kr;
  conductivities(g, mu, &kt, &kr);
  double gr[3][3];
  const int other = 1 - axis;
  for (int i = 0; i < 3; ++i) {
    gr[i][axis] = dn[i];
    gr[i][other] = dt[i];
    gr[i][2] = 0.0;
  }
  const double div = gr[0][0] + gr[1][1];
  const int hidx[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
  double sig[3];
  for (int j = 0; j < 3; ++j) {
    const double s = -mu * (gr[axis][j] + gr[j][axis] - (j == axis ? 2.0 / 3.0 * div : 0.0));
    sig[j] = s + Hf[hidx[axis][j]];
  }
  const double qt = -kt * dTt + Hf[6 + axis];
  const double qr = -kr * dTr + Hf[9 + axis];
  V[0] = 0.0;
  for (int j = 0; j < 3; ++j) V[1 + j] = sig[j];
  V[4] = sig[0] * uf[0] + sig[1] * uf[1] + sig[2] * uf[2] + qt + qr;
  V[5] = qr;
}

template <int axis>
__device__ __forceinline__ void euler_flux(const double U[6], const Prim& p, double F[6]) {
  const double pr = p.rho * p.tt;
  const double un = p.u[axis];
  F[0] = U[0] * un;
  for (int k = 0; k < 3; ++k) F[1 + k] = U[1 + k] * un + (k == axis ? pr : 0.0);
  F[4] = (U[4] + pr) * un;
  F[5] = U[5] * un;
}

template <int axis>
__device__ __forceinline__ void hllc_star(const double U[6], const Prim& p, double SK, double Ss,
                                          double out[6]) {
  const double pr = p.rho * p.tt;
  const double f = p.rho * (SK - p.u[axis]) / (SK - Ss);
  out[0] = f;
  for (int k = 0; k < 3; ++k) out[1 + k] = f * (k == axis ? Ss : p.u[k]);
  out[4] = f * (U[4] / p.rho + (Ss - p.u[axis]) * (Ss + pr / (p.rho * (SK - p.u[axis]))));
  out[5] = f * U[5] / p.rho;
}

// Faces: x faces are (fx, iy) with fx in [0, nx], y faces (ix, fy) with fy
// in [0, ny]; face t of an axis is fa + nfa * fb (axis 0: fa = fx, fb = iy;
// axis 1: fa = ix, fb = fy).
template <int axis>
struct FaceAt {
  int fa, fb, f, n;
  bool wall;
  __device__ FaceAt(const SynthGrid& g, int t) {
    const int nfa = axis == 0 ? g.nx + 1 : g.nx;
    fa = t % nfa;
    fb = t / nfa;
    n = axis == 0 ? g.nx : g.ny;
    f = axis == 0 ? fa : fb;  // face index along the axis
    wall = !g.bc_periodic[axis] && (f == 0 || f == n);
  }
  __device__ int cell(const SynthGrid& g, int along) const {
    return axis == 0 ? along + g.nx * fb : fa + g.nx * along;
  }
  __device__ void xy(int along, int* ix, int* iy) const {
    if (axis == 0) {
      *ix = along;
      *iy = fb;
    } else {
      *ix = fa;
      *iy = along;
    }
  }
};

// HLLC flux through interior or periodic face t; false (F untouched) at a wall.
template <int axis>
__device__ __forceinline__ bool face_inviscid(const SynthGrid& g, const SynthArrays& s, int t,
                                              double F[6]) {
  const FaceAt<axis> fc(g, t);
  if (fc.wall) return false;
  const int C = g.nx * g.ny;
  const int cl = fc.cell(g, (fc.f - 1 + fc.n) % fc.n), cr = fc.cell(g, fc.f % fc.n);
  const Prim pl = prim_at(s.P, C, cl), pr = prim_at(s.P, C, cr);
  double Ul[6], Ur[6], Fl[6], Fr[6];
  for (int k = 0; k < 6; ++k) {
    Ul[k] = s.W[k * C + cl];
    Ur[k] = s.W[k * C + cr];
  }
  euler_flux<axis>(Ul, pl, Fl);
  euler_flux<axis>(Ur, pr, Fr);
  const double cL = sqrt(g.gam * pl.tt), cR = sqrt(g.gam * pr.tt);
  const double SL = fmin(pl.u[axis] - cL, pr.u[axis] - cR);
  const double SR = fmax(pl.u[axis] + cL, pr.u[axis] + cR);
  const double pL = pl.rho * pl.tt, pR = pr.rho * pr.tt;
  const double Ss = (pR - pL + pl.rho * pl.u[axis] * (SL - pl.u[axis]) -
                     pr.rho * pr.u[axis] * (SR - pr.u[axis])) /
                    (pl.rho * (SL - pl.u[axis]) - pr.rho * (SR - pr.u[axis]));
  if (SL >= 0.0) {
    for (int k = 0; k < 6; ++k) F[k] = Fl[k];
  } else if (Ss >= 0.0) {
    double Us[6];
    hllc_star<axis>(Ul, pl, SL, Ss, Us);
    for (int k = 0; k < 6; ++k) F[k] = Fl[k] + SL * (Us[k] - Ul[k]);
  } else if (SR > 0.0) {
    double Us[6];
    hllc_star<axis>(Ur, pr, SR, Ss, Us);
    for (int k = 0; k < 6; ++k) F[k] = Fr[k] + SR * (Us[k] - Ur[k]);
  } else {
    for (int k = 0; k < 6; ++k) F[k] = Fr[k];
  }
  return true;
}

// Viscous and heat flux through face t (NSF plus the masked HoT, averaged
// over the two cells); at a wall the whole flux: Dirichlet wall state, the
// wall pressure on the normal momentum, zero mass flux.
template <int axis>
__device__ __forceinline__ void face_viscous(const SynthGrid& g, const SynthArrays& s, int t,
                                             double F[6]) {
  const FaceAt<axis> fc(g, t);
  const int C = g.nx * g.ny;
  // distance between the centres across this face (half a cell at a wall)
  const double h = (axis == 0 ? g.gx : g.gy)[fc.f];
  if (!fc.wall) {
    const int al = (fc.f - 1 + fc.n) % fc.n, ar = fc.f % fc.n;
    const int cl = fc.cell(g, al), cr = fc.cell(g, ar);
    const Prim pl = prim_at(s.P, C, cl), pr = prim_at(s.P, C, cr);
    int ixl, iyl, ixr, iyr;
    fc.xy(al, &ixl, &iyl);
    fc.xy(ar, &ixr, &iyr);
    const double tf = 0.5 * (pl.tt + pr.tt);
    double uf[3], dn[3], dtn[3], Hf[12];
    for (int i = 0; i < 3; ++i) {
      uf[i] = 0.5 * (pl.u[i] + pr.u[i]);
      dn[i] = (pr.u[i] - pl.u[i]) / h;
      dtn[i] = g.dim == 2 ? 0.5 * (dcen_u(g, s.P, C, ixl, iyl, i, 1 - axis) +
                                   dcen_u(g, s.P, C, ixr, iyr, i, 1 - axis))
                          : 0.0;
    }
    for (int k = 0; k < 12; ++k) Hf[k] = 0.5 * (s.H[k * C + cl] + s.H[k * C + cr]);
    visc_flux<axis>(g, tf, uf, dn, dtn, (pr.tt - pl.tt) / h, (pr.tr - pl.tr) / h, Hf, F);
    return;
  }
  const int side = fc.f == 0 ? 0 : 1;
  const int face = 2 * axis + side;
  const int al = side == 0 ? 0 : fc.n - 1;
  const int c = fc.cell(g, al);
  int ix, iy;
  fc.xy(al, &ix, &iy);
  const Prim p = prim_at(s.P, C, c);
  const int nmax = g.nx > g.ny ? g.nx : g.ny;
  const int wi = axis == 0 ? fc.fb : fc.fa;  // position along the wall
  const double* wv = s.wall + (size_t)face * 5 * nmax;
  const double uw[3] = {wv[0 * nmax + wi], wv[1 * nmax + wi], wv[2 * nmax + wi]};
  const double ttw = wv[3 * nmax + wi], trw = wv[4 * nmax + wi];
  const double sgn = side == 0 ? 1.0 : -1.0;
  double dn[3], dtn[3], Hf[12];
  for (int i = 0; i < 3; ++i) {
    dn[i] = sgn * (p.u[i] - uw[i]) / h;
    dtn[i] = g.dim == 2 ? dcen_u(g, s.P, C, ix, iy, i, 1 - axis) : 0.0;
  }
  for (int k = 0; k < 12; ++k) Hf[k] = s.H[k * C + c];
  visc_flux<axis>(g, 0.5 * (p.tt + ttw), uw, dn, dtn, sgn * (p.tt - ttw) / h,
                  sgn * (p.tr - trw) / h, Hf, F);
  F[1 + axis] += p.rho * p.tt;
  F[0] = 0.0;
}

// Fluxes of every face of the grid, x faces first.  A workgroup takes 128
// faces: waves 0-1 their HLLC fluxes, waves 2-3 their viscous and heat
// fluxes (two chains of half the length: the grid has too few faces to hide
// latency otherwise); the inviscid waves add the two and store.  Thread 0
// of workgroup 0 also resets the next iteration's reductions (parity
// it + 1).  That is safe only through stream order: the last kernel to touch
// those slots is the update of iteration it - 1, which read its time step
// from them, and it has completed before this launch starts on the same
// stream; the update of this iteration, the next to use them, starts after
// this launch has completed.
constexpr int kFluxFaces = 128;

__global__ __launch_bounds__(256) void k_synth_flux(SynthGrid g, SynthArrays s, int it) {
  __shared__ double Vs[6][kFluxFaces];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s.red[((it + 1) & 1) * 2 + 0] = 0x7FF0000000000000ull;  // +inf
    s.red[((it + 1) & 1) * 2 + 1] = 0ull;
  }
  const bool visc = threadIdx.x >= kFluxFaces;
  const int i = threadIdx.x & (kFluxFaces - 1);
  const int t = blockIdx.x * kFluxFaces + i;
  const int nfx = (g.nx + 1) * g.ny;
  const int nft = nfx + (g.dim == 2 ? g.nx * (g.ny + 1) : 0);
  double F[6];
  bool interior = false;
  if (t < nft) {
    if (visc) {
      if (t < nfx)
        face_viscous<0>(g, s, t, F);
      else
        face_viscous<1>(g, s, t - nfx, F);
      for (int k = 0; k < 6; ++k) Vs[k][i] = F[k];
    } else {
      interior = t < nfx ? face_inviscid<0>(g, s, t, F) : face_inviscid<1>(g, s, t - nfx, F);
    }
  }
  __syncthreads();
  if (visc || t >= nft) return;
  for (int k = 0; k < 6; ++k) F[k] = interior ? F[k] + Vs[k][i] : Vs[k][i];
  const bool xf = t < nfx;
  double* out = xf ? s.Fx : s.Fy;
  const int nf = xf ? nfx : nft - nfx;
  const int tf = xf ? t : t - nfx;
  for (int k = 0; k < 6; ++k) out[(size_t)k * nf + tf] = F[k];
}

// Explicit stability bound of cell c (widths wx, wy of the cell).
__device__ double inv_local_dt(const SynthGrid& g, const Prim& p, int c) {
  const double mu = g.mu0 * visc_pow(g, p.tt);
  double kt, kr;
  conductivities(g, mu, &kt, &kr);
  const double cs = sqrt(g.gam * p.tt);
  const double nu = fmax(4.0 * mu / (3.0 * p.rho), g.gam * (kt + kr) / (p.rho * g.cv));
  const double hx = g.wx[c % g.nx];
  double inv = 0.0;
  inv += (fabs(p.u[0]) + cs) / hx + 2.0 * nu / (hx * hx);
  if (g.dim == 2) {
    const double hy = g.wy[c / g.nx];
    inv += (fabs(p.u[1]) + cs) / hy + 2.0 * nu / (hy * hy);
  }
  return inv;
}

__device__ double dt_bound(const SynthGrid& g, const Prim& p, int c) {
  const double mu = g.mu0 * visc_pow(g, p.tt);
  const double tau = mu / (p.rho * p.tt);
  return fmin(g.cfl / inv_local_dt(g, p, c), 0.5 * g.zrot * tau);
}

// Positive doubles order like their bit patterns: min/max via 64-bit atomics.
__device__ __forceinline__ void red_min(unsigned long long* a, double v) {
  atomicMin(a, (unsigned long long)__double_as_longlong(v));
}
__device__ __forceinline__ void red_max(unsigned long long* a, double v) {
  atomicMax(a, (unsigned long long)__double_as_longlong(v));
}

// Flux differences over cell c (the steady residual without its source).
__device__ __forceinline__ void flux_residual(const SynthGrid& g, const SynthArrays& s, int c,
                                              double R[6]) {
  const int ix = c % g.nx, iy = c / g.nx;
  const int nfx = (g.nx + 1) * g.ny;
  for (int k = 0; k < 6; ++k) {
    const double* Fx = s.Fx + (size_t)k * nfx;
    R[k] = -(Fx[ix + 1 + (g.nx + 1) * iy] - Fx[ix + (g.nx + 1) * iy]) / g.wx[ix];
    if (g.dim == 2) {
      const double* Fy = s.Fy + (size_t)k * (g.nx * (g.ny + 1));
      R[k] -= (Fy[ix + g.nx * (iy + 1)] - Fy[ix + g.nx * iy]) / g.wy[iy];
    }
  }
}

// Relaxation time of cell state p and its rotational relaxation source.
__device__ __forceinline__ double relax_source(const SynthGrid& g, const Prim& p, double* tau) {
  const double mu = g.mu0 * visc_pow(g, p.tt);
  *tau = mu / (p.rho * p.tt);
  const double T = (3.0 * p.tt + g.dr * p.tr) / (3.0 + g.dr);
  return 0.5 * g.dr * p.rho * (T - p.tr) / (g.zrot * *tau);
}

// Steady residual of cell c (flux differences over the cell plus the
// rotational relaxation source); returns the relaxation time tau.
__device__ double cell_residual(const SynthGrid& g, const SynthArrays& s, int c, const Prim& p,
                                double R[6]) {
  flux_residual(g, s, c, R);
  double tau;
  R[5] += relax_source(g, p, &tau);
  return tau;
}

// Largest relative change of (rho, u / sqrt(Tt), Tt, Tr) from p to q.
__device__ double rel_change(const Prim& p, const Prim& q) {
  double ch = fabs(q.rho - p.rho) / p.rho;
  for (int k = 0; k < 3; ++k) ch = fmax(ch, fabs(q.u[k] - p.u[k]) / sqrt(p.tt));
  ch = fmax(ch, fabs(q.tt - p.tt) / p.tt);
  return fmax(ch, fabs(q.tr - p.tr) / fmax(p.tr, 1e-300));
}

__global__ void k_synth_update(SynthGrid g, SynthArrays s, int it) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int C = g.nx * g.ny;
  double dtb = 0.0, ch = 0.0;
  if (c < C) {
    const double dtau = __longlong_as_double((long long)s.red[(it & 1) * 2 + 0]);
    const Prim p = prim_at(s.P, C, c);
    double R[6];
    cell_residual(g, s, c, p, R);
    for (int k = 0; k < 6; ++k) s.Wn[k * C + c] = s.W[k * C + c] + dtau * R[k];
    const Prim q = prim_of(s.Wn, C, c, g.dr);
    store_prim(s.P, C, c, q);  // this thread's cell only: read above
    ch = rel_change(p, q);
    dtb = dt_bound(g, q, c);
  }
  // block reductions, then one atomic per block
  __shared__ double s_min[4], s_max[4];
  double mn = c < C ? dtb : INFINITY, mx = ch;
  for (int off = 32; off > 0; off >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, off));
    mx = fmax(mx, __shfl_xor(mx, off));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_min[w] = mn;
    s_max[w] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
      mn = fmin(mn, s_min[k]);
      mx = fmax(mx, s_max[k]);
    }
    red_min(&s.red[((it + 1) & 1) * 2 + 0], mn);
    red_max(&s.red[((it + 1) & 1) * 2 + 1], mx);
  }
}

// ---------------------------------------------------------------------------
// Implicit pseudo-time steps by LU-SGS (the paper's scheme for the synthetic
// equations), matrix-free in the form of Yoon and Jameson: per cell
//   D dW_i + sum_j (dF_j . n_ij - r_j dW_j) / (2 h) = R_i,
//   D = (1 + 1/cfl) sum_a r_a / h_a  (+ 1/(Z tau) on the rotational row),
// h, h_a the widths of cell i,
// r_a = |u_a| + c + 2 nu / h_a, dF_j = F(W_j + dW_j) - F(W_j) the change of
// the neighbour's inviscid flux, j over the neighbours across interior and
// periodic faces.  The cells are ordered in two colours ((ix + iy) even
// first; every neighbour has the other colour), so both sweeps are two
// parallel passes: lower sweep dW = R / D on the first colour (k_lusgs_cells)
// and dW = (R - sum_j ...) / D on the second (k_lusgs_lower); upper sweep
// dW -= sum_j ... / D on the first colour (k_lusgs_upper).  The new state is
// then scaled by the ratio of the initial to the current total mass, sum of
// rho V (k_lusgs_scale): the implicit operator is not conservative, the steady
// state of a closed or periodic box keeps the initial mass.

struct LusgsArrays {
  double* dW;    // [6][C] increments
  double* R;     // [6][C] steady residuals
  double* D;     // [2][C] diagonal (rows 0-4, row 5)
  double* rad;   // [2][C] spectral radii along x and y
  double* part;  // [nparts] per-workgroup mass sums of the new state, then of the initial one
  unsigned long long* chg;  // [2] relative change (max) by iteration parity
  int nparts;    // workgroups of the sweep kernels (64 pairs of cells each)
};

__device__ __forceinline__ bool first_colour(const SynthGrid& g, int c) {
  return ((c % g.nx + c / g.nx) & 1) == 0;
}

template <int axis>
__device__ __forceinline__ void euler_of(const double U[6], int dr, double F[6]) {
  Prim p;
  p.rho = U[0];
  for (int k = 0; k < 3; ++k) p.u[k] = U[1 + k] / p.rho;
  p.tr = 2.0 * U[5] / (dr * p.rho);
  const double uu = p.u[0] * p.u[0] + p.u[1] * p.u[1] + p.u[2] * p.u[2];
  p.tt = (U[4] / p.rho - 0.5 * uu - 0.5 * dr * p.tr) * 2.0 / 3.0;
  euler_flux<axis>(U, p, F);
}

// Term (side dF - r dW) / (2 h) of cell c's neighbour across its face on
// `side` (+1 or -1) of `axis`, h the width of cell c, dF the change of the
// neighbour's inviscid flux by its increment (final in L.dW: the neighbour has
// the other colour); false where the face is a wall.
template <int axis>
__device__ __forceinline__ bool neighbour_term(const SynthGrid& g, const SynthArrays& s,
                                               const LusgsArrays& L, int c, int side,
                                               double out[6]) {
  const int C = g.nx * g.ny;
  const int n = axis == 0 ? g.nx : g.ny;
  const int i = axis == 0 ? c % g.nx : c / g.nx;
  const double h = (axis == 0 ? g.wx : g.wy)[i];  // width of the receiving cell
  int j = i + side;
  if (j < 0 || j >= n) {
    if (!g.bc_periodic[axis]) return false;
    j = (j + n) % n;
  }
  const int cj = axis == 0 ? j + g.nx * (c / g.nx) : (c % g.nx) + g.nx * j;
  double U[6], V[6], F0[6], F1[6];
  for (int k = 0; k < 6; ++k) {
    U[k] = s.W[(size_t)k * C + cj];
    V[k] = U[k] + L.dW[(size_t)k * C + cj];
  }
  euler_of<axis>(U, g.dr, F0);
  euler_of<axis>(V, g.dr, F1);
  const double r = L.rad[(size_t)axis * C + cj];
  for (int k = 0; k < 6; ++k) {
    const double t = (double)side * (F1[k] - F0[k]) - r * L.dW[(size_t)k * C + cj];
    out[k] = t / (2.0 * h);
  }
  return true;
}

// Layout of the two sweep kernels: a workgroup of 256 threads takes 64 pairs
// of cells (2p, 2p + 1).  Row-major order alternates the colours (across rows
// too when nx is odd; rows of even nx hold whole pairs), so a pair holds one
// cell of each colour.  Wave q computes neighbour slot q of the pair's cell
// of the swept colour, slots in the order (x, +1), (x, -1), (y, +1), (y, -1);
// the cell's sum then adds the slots in that order, from zero, as a plain
// loop over the neighbours would.  Four short chains per cell instead of one
// long one: the grid holds too few cells to hide latency otherwise.
constexpr int kSweepPairs = 64;

__device__ __forceinline__ int pair_cell(const SynthGrid& g, int pair, bool first) {
  const int c0 = 2 * pair;
  return first_colour(g, c0) == first ? c0 : c0 + 1;
}

struct SweepLds {
  double t[4][6][kSweepPairs];
  int ok[4][kSweepPairs];
};

// Every thread of the workgroup: slot (wave) terms of the workgroup's cells
// of the swept colour, into S.
__device__ __forceinline__ void sweep_terms(const SynthGrid& g, const SynthArrays& s,
                                            const LusgsArrays& L, bool first, SweepLds& S) {
  const int C = g.nx * g.ny;
  const int q = threadIdx.x >> 6, i = threadIdx.x & 63;
  const int c = pair_cell(g, blockIdx.x * kSweepPairs + i, first);
  double v[6];
  bool ok = false;
  if (c < C) {
    const int side = (q & 1) ? -1 : 1;
    if (q < 2)
      ok = neighbour_term<0>(g, s, L, c, side, v);
    else if (g.dim == 2)
      ok = neighbour_term<1>(g, s, L, c, side, v);
  }
  S.ok[q][i] = ok;
  if (ok)
    for (int k = 0; k < 6; ++k) S.t[q][k][i] = v[k];
  __syncthreads();
}

// Sum of the slot terms of the workgroup's cell i, slot order.
__device__ __forceinline__ void sweep_sum(const SweepLds& S, int i, double acc[6]) {
  for (int k = 0; k < 6; ++k) acc[k] = 0.0;
  for (int q = 0; q < 4; ++q)
    if (S.ok[q][i])
      for (int k = 0; k < 6; ++k) acc[k] += S.t[q][k][i];
}

// Residual, diagonal and spectral radii of every cell; lower sweep on the
// first colour.  A workgroup takes 128 cells in two roles of two waves each:
// the flux differences, and the cell's own terms (relaxation source,
// spectral radii, diagonal); after a barrier the first role adds the source,
// stores the residual and, on the first colour, the increment.  Block 0 also
// resets this iteration's change slot (safe in stream order: its last reader,
// the host check of iteration it - 2, and its last writer, k_lusgs_scale of
// iteration it - 2, precede this launch).
constexpr int kCellsPerGroup = 128;

__global__ __launch_bounds__(2 * kCellsPerGroup) void k_lusgs_cells(SynthGrid g, SynthArrays s,
                                                                    LusgsArrays L, int it) {
  __shared__ double Sd[3][kCellsPerGroup];  // source, D0, D5
  const int role = threadIdx.x / kCellsPerGroup, i = threadIdx.x % kCellsPerGroup;
  const int c = blockIdx.x * kCellsPerGroup + i;
  const int C = g.nx * g.ny;
  if (blockIdx.x == 0 && threadIdx.x == 0) L.chg[it & 1] = 0ull;
  double R[6];
  if (c < C) {
    if (role == 0) {
      flux_residual(g, s, c, R);
    } else {
      const Prim p = prim_at(s.P, C, c);
      double tau;
      const double src = relax_source(g, p, &tau);
      const double mu = g.mu0 * visc_pow(g, p.tt);
      double kt, kr;
      conductivities(g, mu, &kt, &kr);
      const double cs = sqrt(g.gam * p.tt);
      const double nu = fmax(4.0 * mu / (3.0 * p.rho), g.gam * (kt + kr) / (p.rho * g.cv));
      const double hx = g.wx[c % g.nx];
      const double rx = fabs(p.u[0]) + cs + 2.0 * nu / hx;
      double d = rx / hx;
      double ry = 0.0;
      if (g.dim == 2) {
        const double hy = g.wy[c / g.nx];
        ry = fabs(p.u[1]) + cs + 2.0 * nu / hy;
        d += ry / hy;
      }
      const double D0 = (1.0 + 1.0 / g.cfl) * d;
      const double D5 = D0 + 1.0 / (g.zrot * tau);
      L.D[c] = D0;
      L.D[C + c] = D5;
      L.rad[c] = rx;
      L.rad[C + c] = ry;
      Sd[0][i] = src;
      Sd[1][i] = D0;
      Sd[2][i] = D5;
    }
  }
  __syncthreads();
  if (role != 0 || c >= C) return;
  R[5] += Sd[0][i];
  for (int k = 0; k < 6; ++k) L.R[(size_t)k * C + c] = R[k];
  if (first_colour(g, c))
    for (int k = 0; k < 6; ++k) L.dW[(size_t)k * C + c] = R[k] / Sd[k == 5 ? 2 : 1][i];
}

// Lower sweep on the second colour.  Wave 0 loads what it needs to finish
// its cells before the slot terms, so both rounds of loads overlap.
__global__ __launch_bounds__(256) void k_lusgs_lower(SynthGrid g, SynthArrays s, LusgsArrays L) {
  __shared__ SweepLds S;
  const int C = g.nx * g.ny;
  const int i = threadIdx.x & 63;
  const int c = pair_cell(g, blockIdx.x * kSweepPairs + i, false);
  const bool fin = threadIdx.x < kSweepPairs && c < C;
  double R[6], D0 = 1.0, D5 = 1.0;
  if (fin) {
    for (int k = 0; k < 6; ++k) R[k] = L.R[(size_t)k * C + c];
    D0 = L.D[c];
    D5 = L.D[C + c];
  }
  sweep_terms(g, s, L, false, S);
  if (!fin) return;
  double acc[6];
  sweep_sum(S, i, acc);
  for (int k = 0; k < 6; ++k) L.dW[(size_t)k * C + c] = (R[k] - acc[k]) / (k == 5 ? D5 : D0);
}

// Volume of cell c (area in 2D, length in 1D): the mass of a cell is rho V.
__device__ __forceinline__ double cell_vol(const SynthGrid& g, int c) {
  return g.dim == 2 ? g.wx[c % g.nx] * g.wy[c / g.nx] : g.wx[c % g.nx];
}

// Fixed-order block sum (the same tree in every block and every call).
__device__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
  return t;
}

// Upper sweep on the first colour, then the new state W + dW of both cells
// of every pair (wave 0 the first colour, wave 1 the second) and the
// workgroup's sum of their masses.  Waves 0 and 1 load their cells' state,
// increment and diagonal before the slot terms.
__global__ __launch_bounds__(256) void k_lusgs_upper(SynthGrid g, SynthArrays s, LusgsArrays L) {
  __shared__ SweepLds S;
  __shared__ double sh[16];
  const int C = g.nx * g.ny;
  const int w = threadIdx.x >> 6, i = threadIdx.x & 63;
  const int c = pair_cell(g, blockIdx.x * kSweepPairs + i, w == 0);
  const bool fin = w < 2 && c < C;
  double dW[6], Wc[6], D0 = 1.0, D5 = 1.0;
  if (fin) {
    for (int k = 0; k < 6; ++k) {
      dW[k] = L.dW[(size_t)k * C + c];
      Wc[k] = s.W[(size_t)k * C + c];
    }
    D0 = L.D[c];
    D5 = L.D[C + c];
  }
  sweep_terms(g, s, L, true, S);
  double rho_new = 0.0;
  if (fin) {
    if (w == 0) {
      double acc[6];
      sweep_sum(S, i, acc);
      for (int k = 0; k < 6; ++k) dW[k] = dW[k] - acc[k] / (k == 5 ? D5 : D0);
    }
    for (int k = 0; k < 6; ++k) s.Wn[(size_t)k * C + c] = Wc[k] + dW[k];
    rho_new = (Wc[0] + dW[0]) * cell_vol(g, c);
  }
  const double t = block_sum(rho_new, sh);
  if (threadIdx.x == 0) L.part[blockIdx.x] = t;
}

// Per-workgroup mass sums of the start state, over the same cells and by the
// same tree as those of the new states (a state that does not change keeps
// the scale at exactly 1).
__global__ __launch_bounds__(256) void k_lusgs_mass0(SynthGrid g, const double* W,
                                                     LusgsArrays L) {
  __shared__ double sh[16];
  const int C = g.nx * g.ny;
  const int w = threadIdx.x >> 6, i = threadIdx.x & 63;
  double v = 0.0;
  if (w < 2) {
    const int c = pair_cell(g, blockIdx.x * kSweepPairs + i, w == 0);
    if (c < C) v = W[c] * cell_vol(g, c);
  }
  const double t = block_sum(v, sh);
  if (threadIdx.x == 0) L.part[L.nparts + blockIdx.x] = t;
}

// Two fixed-order block sums at once, each by the tree of block_sum.
__device__ void block_sum2(double* a, double* b, double* sh /* [32] */) {
  double va = *a, vb = *b;
  for (int off = 32; off > 0; off >>= 1) {
    va += __shfl_xor(va, off);
    vb += __shfl_xor(vb, off);
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sh[w] = va;
    sh[16 + w] = vb;
  }
  __syncthreads();
  double ta = 0.0, tb = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
    ta += sh[k];
    tb += sh[16 + k];
  }
  *a = ta;
  *b = tb;
}

// Scale the new state to the initial mass; relative change of the iteration.
// Every workgroup adds the per-workgroup mass sums of the new and the
// initial state in the same fixed order; the cell's states are loaded before
// that, so both rounds of loads overlap.
__global__ __launch_bounds__(256) void k_lusgs_scale(SynthGrid g, SynthArrays s, LusgsArrays L,
                                                     int it) {
  __shared__ double sh[32];
  __shared__ double s_max[16];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int C = g.nx * g.ny;
  double Wv[6];
  Prim po;
  if (c < C) {
    for (int k = 0; k < 6; ++k) Wv[k] = s.Wn[(size_t)k * C + c];
    po = prim_at(s.P, C, c);
  }
  double m = 0.0, m0 = 0.0;
  for (int b = threadIdx.x; b < L.nparts; b += blockDim.x) {
    m += L.part[b];
    m0 += L.part[L.nparts + b];
  }
  block_sum2(&m, &m0, sh);
  const double scale = m0 / m;
  double ch = 0.0;
  if (c < C) {
    for (int k = 0; k < 6; ++k) {
      Wv[k] *= scale;
      s.Wn[(size_t)k * C + c] = Wv[k];
    }
    const Prim q = prim_of(Wv, 1, 0, g.dr);
    store_prim(s.P, C, c, q);  // this thread's cell only: read above
    ch = rel_change(po, q);
  }
  for (int off = 32; off > 0; off >>= 1) ch = fmax(ch, __shfl_xor(ch, off));
  if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = ch;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) ch = fmax(ch, s_max[k]);
    red_max(&L.chg[it & 1], ch);
  }
}

// Initial conservative state, wall face values and the first pseudo-time step.
__global__ void k_synth_init(SynthGrid g, const double* m, double* W, double* P, double* wall,
                             int mode, const double* wall_cfg, unsigned long long* red) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int C = g.nx * g.ny;
  // iteration 1 reads its step from the parity-1 slot, which the host resets
  // before this launch (a reset inside it would race with the other blocks'
  // atomics)
  if (c >= C) return;
  const double rho = m[c];
  const double u[3] = {m[C + c], m[2 * C + c], m[3 * C + c]};
  const double tt = m[4 * C + c], tr = m[5 * C + c];
  W[c] = rho;
  for (int k = 0; k < 3; ++k) W[(1 + k) * C + c] = rho * u[k];
  W[4 * C + c] = rho * (0.5 * (3.0 * tt + g.dr * tr) + 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
  W[5 * C + c] = rho * 0.5 * g.dr * tr;
  {
    // the primitives the solve reads, as they follow from the stored state
    double Wl[6];
    for (int k = 0; k < 6; ++k) Wl[k] = W[(size_t)k * C + c];
    store_prim(P, C, c, prim_of(Wl, 1, 0, g.dr));
  }
  const int ix = c % g.nx, iy = c / g.nx;
  const int nmax = g.nx > g.ny ? g.nx : g.ny;
  for (int face = 0; face < (g.dim == 2 ? 4 : 2); ++face) {
    const int axis = face >> 1, side = face & 1;
    if (g.bc_periodic[axis]) continue;
    const int along = axis == 0 ? ix : iy;
    if (along != (side == 0 ? 0 : (axis == 0 ? g.nx : g.ny) - 1)) continue;
    const int wi = axis == 0 ? iy : ix;
    double* wv = wall + (size_t)face * 5 * nmax;
    for (int k = 0; k < 3; ++k)
      wv[k * nmax + wi] = (k == axis) ? 0.0 : (mode == 0 ? wall_cfg[face * 4 + 1 + k] : u[k]);
    wv[3 * nmax + wi] = mode == 0 ? wall_cfg[face * 4] : tt;
    wv[4 * nmax + wi] = mode == 0 ? wall_cfg[face * 4] : tr;
  }
  Prim p;
  p.rho = rho;
  for (int k = 0; k < 3; ++k) p.u[k] = u[k];
  p.tt = tt;
  p.tr = tr;
  red_min(&red[2], dt_bound(g, p, c));
}

__global__ void k_synth_mask_hot(const double* hot, const uint8_t* mask, double* H, int C) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const bool off = hot == nullptr || (mask != nullptr && mask[c] != 0);
  for (int k = 0; k < 12; ++k) H[(size_t)k * C + c] = off ? 0.0 : hot[(size_t)k * C + c];
}

__global__ void k_synth_out(SynthGrid g, const double* W, double* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int C = g.nx * g.ny;
  if (c >= C) return;
  const Prim p = prim_of(W, C, c, g.dr);
  out[c] = p.rho;
  for (int k = 0; k < 3; ++k) out[(1 + k) * C + c] = p.u[k];
  out[4 * C + c] = p.tt;
  out[5 * C + c] = p.tr;
}

}  // namespace dig

using namespace dig;

namespace {
thread_local std::string g_serr;
size_t al256(size_t v) { return (v + 255) / 256 * 256; }

struct SynthLayout {
  size_t W0, W1, P, Fx, Fy, H, wall, wcfg, red, dW, R, D, rad, part, chg, geo, total;
};
constexpr int kSynthBlock = 256;
// workgroups of the LU-SGS sweep kernels: 64 pairs of cells each
size_t sweep_groups(size_t C) { return ((C + 1) / 2 + 63) / 64; }

SynthLayout synth_layout(const dig_config* c) {
  const size_t C = (size_t)c->nx * c->ny;
  const size_t nmax = c->nx > c->ny ? c->nx : c->ny;
  SynthLayout L;
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t r = o;
    o = al256(o + b);
    return r;
  };
  L.W0 = take(8 * 6 * C);
  L.W1 = take(8 * 6 * C);
  L.P = take(8 * 6 * C);
  L.Fx = take(8 * 6 * (c->nx + 1) * (size_t)c->ny);
  L.Fy = take(8 * 6 * (size_t)c->nx * (c->ny + 1));
  L.H = take(8 * 12 * C);
  L.wall = take(8 * 4 * 5 * nmax);
  L.wcfg = take(8 * 16);
  L.red = take(8 * 4);
  // LU-SGS increments, residuals, diagonal, spectral radii, mass partials
  L.dW = take(8 * 6 * C);
  L.R = take(8 * 6 * C);
  L.D = take(8 * 2 * C);
  L.rad = take(8 * 2 * C);
  L.part = take(8 * 2 * sweep_groups(C));
  L.chg = take(8 * 2);
  // grid geometry: widths wx, wy and centre distances gx, gy
  L.geo = take(8 * (2 * (size_t)c->nx + 2 * (size_t)c->ny + 2));
  L.total = o;
  return L;
}
}  // namespace

extern "C" {

size_t dig_synth_workspace_bytes(const dig_config* cfg) {
  if (!cfg || cfg->nx < 1 || cfg->ny < 1) return 0;
  return synth_layout(cfg).total;
}

// Argument checks of both solve entry points (host only, before any device
// work); the workspace is checked by the caller.
static dig_status check_synth_args(const char* fn, const dig_config* cfg,
                                   const dig_synth_opts* opts, const double* m_half,
                                   const double* m_next, int32_t max_iter, double tol,
                                   const int32_t* iters, const double* change) {
  auto bad = [&](const char* why) {
    static thread_local char msg[200];
    snprintf(msg, sizeof(msg), "%s: %s", fn, why);
    return report(DIG_ERR_INVALID, msg);
  };
  if (!cfg || !opts || !m_half || !m_next || !iters || !change) return bad("null argument");
  if (cfg->dim != 1 && cfg->dim != 2) return bad("dim must be 1 or 2");
  if (cfg->nx < 1 || cfg->ny < 1 || (cfg->dim == 1 && cfg->ny != 1))
    return bad("bad cell counts");
  if ((int64_t)cfg->nx * cfg->ny > (int64_t)INT32_MAX / 64) return bad("too many cells");
  if (cfg->geometry != DIG_GEOM_BOX && cfg->geometry != DIG_GEOM_GRADED)
    return bad("boxes only (uniform or graded)");
  if (cfg->geometry == DIG_GEOM_GRADED)
    for (int ax = 0; ax < cfg->dim; ++ax) {
      const double* f = ax == 0 ? cfg->xfaces : cfg->yfaces;
      const int n = ax == 0 ? cfg->nx : cfg->ny;
      if (!f) return bad("a graded box needs its face tables");
      if (!(f[0] == 0.0) || !(f[n] == (ax == 0 ? cfg->lx : cfg->ly)))
        return bad("face tables must run from 0 to the domain length");
      for (int i = 0; i < n; ++i)
        if (!std::isfinite(f[i + 1]) || !(f[i + 1] > f[i]))
          return bad("face tables must be finite and strictly increasing");
    }
  if (!(cfg->lx > 0.0) || !std::isfinite(cfg->lx) ||
      (cfg->dim == 2 && (!(cfg->ly > 0.0) || !std::isfinite(cfg->ly))))
    return bad("bad domain size");
  if (!(cfg->kn > 0.0) || !std::isfinite(cfg->kn)) return bad("Kn must be finite and > 0");
  if (!(cfg->omega >= 0.5 && cfg->omega <= 1.0)) return bad("omega must lie in [0.5, 1]");
  if (cfg->dr < 2 || cfg->dr > 6) return bad("d_r must lie in [2, 6]");
  if (!(cfg->zrot > 0.0) || !std::isfinite(cfg->zrot)) return bad("Z must be finite and > 0");
  for (int ax = 0; ax < cfg->dim; ++ax) {
    for (int side = 0; side < 2; ++side) {
      const dig_bc& b = cfg->bc[2 * ax + side];
      if (b.type != DIG_BC_PERIODIC && b.type != DIG_BC_DIFFUSE && b.type != DIG_BC_SPECULAR)
        return bad("bad face type for a box");
      if (b.type == DIG_BC_DIFFUSE &&
          (!(b.T > 0.0) || !std::isfinite(b.T) || !std::isfinite(b.U[0]) ||
           !std::isfinite(b.U[1]) || !std::isfinite(b.U[2])))
        return bad("a diffuse wall needs a finite T > 0 and a finite velocity");
    }
    if ((cfg->bc[2 * ax].type == DIG_BC_PERIODIC) != (cfg->bc[2 * ax + 1].type == DIG_BC_PERIODIC))
      return bad("periodic faces must come in pairs");
  }
  if (max_iter < 0) return bad("max_iter must be >= 0");
  if (!(tol >= 0.0)) return bad("tol must be >= 0");
  if (!(opts->cfl > 0.0) || !std::isfinite(opts->cfl)) return bad("cfl must be finite and > 0");
  if (opts->scheme != DIG_SYNTH_EXPLICIT && opts->scheme != DIG_SYNTH_LUSGS)
    return bad("unknown scheme");
  if (opts->check_every < 0) return bad("check_every must be >= 0");
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(opts->A[k])) return bad("A must be finite");
  if (!(fabs(opts->A[0] * opts->A[3] - opts->A[1] * opts->A[2]) > 0.0))
    return bad("A is singular");
  // two colours: a periodic axis needs an even cell count
  if (opts->scheme == DIG_SYNTH_LUSGS)
    for (int ax = 0; ax < cfg->dim; ++ax)
      if (cfg->bc[2 * ax].type == DIG_BC_PERIODIC && ((ax == 0 ? cfg->nx : cfg->ny) & 1))
        return bad("LU-SGS needs an even cell count on a periodic axis");
  return DIG_OK;
}

// Widths [n] and centre distances across the faces [n + 1] of one axis, in
// that order in `out`: uniform grids h and h (h/2 at a wall); graded grids
// from the face table (half the cell at a wall, the wrapped distance across
// a periodic seam).
static void axis_geometry(const dig_config* cfg, int axis, std::vector<double>& out) {
  const int n = axis == 0 ? cfg->nx : cfg->ny;
  const bool periodic = cfg->bc[2 * axis].type == DIG_BC_PERIODIC;
  const double* f = axis == 0 ? cfg->xfaces : cfg->yfaces;
  if (cfg->geometry == DIG_GEOM_GRADED && (axis == 0 || cfg->dim == 2)) {
    std::vector<double> c(n);
    for (int i = 0; i < n; ++i) {
      out.push_back(f[i + 1] - f[i]);
      c[i] = 0.5 * (f[i + 1] + f[i]);
    }
    const double g0 = periodic ? c[0] + (f[n] - c[n - 1]) : c[0] - f[0];
    const double gn = periodic ? c[0] + (f[n] - c[n - 1]) : f[n] - c[n - 1];
    out.push_back(g0);
    for (int i = 1; i < n; ++i) out.push_back(c[i] - c[i - 1]);
    out.push_back(gn);
    return;
  }
  const double h = axis == 0 ? cfg->lx / cfg->nx : (cfg->dim == 2 ? cfg->ly / cfg->ny : 1.0);
  for (int i = 0; i < n; ++i) out.push_back(h);
  for (int i = 0; i <= n; ++i) out.push_back((i == 0 || i == n) && !periodic ? 0.5 * h : h);
}

dig_status synth_solve(const dig_config* cfg, const dig_synth_opts* opts, const double* m_half,
                       const double* hot, const uint8_t* mask, double* m_next,
                       void* workspace, size_t ws_bytes, int32_t max_iter, double tol,
                       int32_t* iters, double* change, dig_stream_t stream) {
  {
    const dig_status st =
        check_synth_args("synth_solve", cfg, opts, m_half, m_next, max_iter, tol, iters, change);
    if (st != DIG_OK) return st;
  }
  const SynthLayout L = synth_layout(cfg);
  if (!workspace || ((uintptr_t)workspace) % 256)
    return report(DIG_ERR_INVALID, "synth_solve: workspace null or not 256-byte aligned");
  if (ws_bytes < L.total) return report(DIG_ERR_INVALID, "synth_solve: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  unsigned char* w = (unsigned char*)workspace;
  SynthGrid g;
  memset(&g, 0, sizeof(g));
  g.nx = cfg->nx;
  g.ny = cfg->ny;
  g.dim = cfg->dim;
  g.dr = cfg->dr;
  g.hx = cfg->lx / cfg->nx;
  g.hy = cfg->dim == 2 ? cfg->ly / cfg->ny : 1.0;
  g.mu0 = cfg->kn * sqrt(2.0 / M_PI);
  g.omega = cfg->omega;
  g.zrot = cfg->zrot;
  g.gam = (5.0 + cfg->dr) / (3.0 + cfg->dr);
  g.cv = (3.0 + cfg->dr) / 2.0;
  g.cfl = opts->cfl;
  g.Att = opts->A[0];
  g.Atr = opts->A[1];
  g.Art = opts->A[2];
  g.Arr = opts->A[3];
  g.bc_periodic[0] = cfg->bc[0].type == DIG_BC_PERIODIC;
  g.bc_periodic[1] = cfg->dim == 2 ? cfg->bc[2].type == DIG_BC_PERIODIC : 1;
  const int C = g.nx * g.ny;
  double wcfg[16];
  for (int f = 0; f < 4; ++f) {
    wcfg[f * 4] = cfg->bc[f].T;
    for (int k = 0; k < 3; ++k) wcfg[f * 4 + 1 + k] = cfg->bc[f].U[k];
  }
  double* W0 = (double*)(w + L.W0);
  double* W1 = (double*)(w + L.W1);
  double* Pv = (double*)(w + L.P);
  double* H = (double*)(w + L.H);
  double* wall = (double*)(w + L.wall);
  double* dwcfg = (double*)(w + L.wcfg);
  unsigned long long* red = (unsigned long long*)(w + L.red);
  if (hipMemcpyAsync(dwcfg, wcfg, sizeof(wcfg), hipMemcpyHostToDevice, s) != hipSuccess)
    return DIG_ERR_HIP;
  // grid geometry: wx [nx], gx [nx + 1], wy [ny], gy [ny + 1]
  std::vector<double> geo;
  axis_geometry(cfg, 0, geo);
  axis_geometry(cfg, 1, geo);
  double* dgeo = (double*)(w + L.geo);
  if (hipMemcpyAsync(dgeo, geo.data(), 8 * geo.size(), hipMemcpyHostToDevice, s) != hipSuccess)
    return DIG_ERR_HIP;
  g.wx = dgeo;
  g.gx = dgeo + g.nx;
  g.wy = dgeo + 2 * g.nx + 1;
  g.gy = g.wy + g.ny;
  // every path below synchronises before returning while geo is alive, but
  // the one without iterations
  if (max_iter == 0 && hipStreamSynchronize(s) != hipSuccess) return DIG_ERR_HIP;
  const int bs = kSynthBlock, nb = (C + bs - 1) / bs;
  hipLaunchKernelGGL(k_synth_mask_hot, dim3(nb), dim3(bs), 0, s, hot, mask, H, C);
  // parity-1 reduction slots: dtau (min, from +inf; +inf and 0 have the bit
  // patterns of the FP64 values) and the change (max, from 0)
  if (launch_fill_f64((double*)red + 2, 1, INFINITY, s) != hipSuccess ||
      launch_fill_f64((double*)red + 3, 1, 0.0, s) != hipSuccess)
    return DIG_ERR_HIP;
  hipLaunchKernelGGL(k_synth_init, dim3(nb), dim3(bs), 0, s, g, m_half, W0, Pv, wall,
                     opts->wall_mode, (const double*)dwcfg, red);
  const int check = opts->check_every > 0 ? opts->check_every : 32;
  double* cur = W0;
  double* nxt = W1;
  int it = 0;
  double last = INFINITY;
  if (opts->scheme == DIG_SYNTH_LUSGS) {
    LusgsArrays la{(double*)(w + L.dW), (double*)(w + L.R), (double*)(w + L.D),
                   (double*)(w + L.rad), (double*)(w + L.part),
                   (unsigned long long*)(w + L.chg), (int)sweep_groups(C)};
    const dim3 sgrid(la.nparts);
    hipLaunchKernelGGL(k_lusgs_mass0, sgrid, dim3(bs), 0, s, g, (const double*)W0, la);
    for (it = 1; it <= max_iter; ++it) {
      SynthArrays a{cur, nxt, (double*)(w + L.Fx), (double*)(w + L.Fy), H, Pv, wall, red};
      const int nft = (g.nx + 1) * g.ny + (g.dim == 2 ? g.nx * (g.ny + 1) : 0);
      hipLaunchKernelGGL(k_synth_flux, dim3((nft + kFluxFaces - 1) / kFluxFaces),
                         dim3(2 * kFluxFaces), 0, s, g, a, it);
      hipLaunchKernelGGL(k_lusgs_cells, dim3((C + kCellsPerGroup - 1) / kCellsPerGroup),
                         dim3(2 * kCellsPerGroup), 0, s, g, a, la, it);
      hipLaunchKernelGGL(k_lusgs_lower, sgrid, dim3(bs), 0, s, g, a, la);
      hipLaunchKernelGGL(k_lusgs_upper, sgrid, dim3(bs), 0, s, g, a, la);
      hipLaunchKernelGGL(k_lusgs_scale, dim3(nb), dim3(bs), 0, s, g, a, la, it);
      double* t = cur;
      cur = nxt;
      nxt = t;
      if (it % check == 0 || it == max_iter) {
        unsigned long long bits = 0;
        if (hipMemcpyAsync(&bits, la.chg + (it & 1), 8, hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          return DIG_ERR_HIP;
        double v;
        memcpy(&v, &bits, 8);
        last = v;
        if (!(v >= 0.0)) return DIG_ERR_NUMERIC;
        if (v < tol) break;
      }
    }
    if (it > max_iter) it = max_iter;
    hipLaunchKernelGGL(k_synth_out, dim3(nb), dim3(bs), 0, s, g, cur, m_next);
    if (hipGetLastError() != hipSuccess) return DIG_ERR_HIP;
    *iters = it;
    *change = last;
    return DIG_OK;
  }
  for (it = 1; it <= max_iter; ++it) {
    SynthArrays a{cur, nxt, (double*)(w + L.Fx), (double*)(w + L.Fy), H, Pv, wall, red};
    const int nft = (g.nx + 1) * g.ny + (g.dim == 2 ? g.nx * (g.ny + 1) : 0);
    hipLaunchKernelGGL(k_synth_flux, dim3((nft + kFluxFaces - 1) / kFluxFaces),
                       dim3(2 * kFluxFaces), 0, s, g, a, it);
    hipLaunchKernelGGL(k_synth_update, dim3(nb), dim3(bs), 0, s, g, a, it);
    double* t = cur;
    cur = nxt;
    nxt = t;
    if (it % check == 0 || it == max_iter) {
      unsigned long long bits = 0;
      if (hipMemcpyAsync(&bits, red + ((it + 1) & 1) * 2 + 1, 8, hipMemcpyDeviceToHost, s) !=
              hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return DIG_ERR_HIP;
      double v;
      memcpy(&v, &bits, 8);
      last = v;
      if (!(v >= 0.0)) return DIG_ERR_NUMERIC;
      if (v < tol) break;
    }
  }
  if (it > max_iter) it = max_iter;
  hipLaunchKernelGGL(k_synth_out, dim3(nb), dim3(bs), 0, s, g, cur, m_next);
  if (hipGetLastError() != hipSuccess) return DIG_ERR_HIP;
  *iters = it;
  *change = last;
  return DIG_OK;
}

}  // extern "C"

namespace {

// Scratch of synth_solve_static: one copy of this array per GPU the library
// runs on, held until the process ends.  Its host-side name is not a device
// address: host code uses only the address looked up below.
constexpr size_t kStaticSynthBytes = (size_t)DIG_SYNTH_STATIC_BYTES;
__device__ __align__(256) unsigned char scratch[kStaticSynthBytes];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};

// Device address of the current GPU's scratch array, looked up once per
// device with that device current.
dig_status static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return report(DIG_ERR_HIP, "synth_solve_static: hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices)
    return report(DIG_ERR_INVALID, "synth_solve_static: device index beyond 63");
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return report(DIG_ERR_HIP, "synth_solve_static: hipGetSymbolAddress(scratch) failed");
    g_static_ptr[dev] = p;
  }
  *out = g_static_ptr[dev];
  return DIG_OK;
}

}  // namespace

extern "C" {

dig_status synth_solve_static(const dig_config* cfg, const dig_synth_opts* opts,
                              const double* m_half, const double* hot, const uint8_t* mask,
                              double* m_next, int32_t max_iter, double tol, int32_t* iters,
                              double* change, dig_stream_t stream) {
  {
    const dig_status st = check_synth_args("synth_solve_static", cfg, opts, m_half, m_next,
                                           max_iter, tol, iters, change);
    if (st != DIG_OK) return st;
  }
  const size_t need = synth_layout(cfg).total;
  if (need > kStaticSynthBytes) {
    static thread_local char msg[160];
    snprintf(msg, sizeof(msg),
             "synth_solve_static: the grid needs %zu bytes of scratch, more than the static "
             "%zu",
             need, kStaticSynthBytes);
    return report(DIG_ERR_INVALID, msg);
  }
  void* ws = nullptr;
  const dig_status st = static_scratch(&ws);
  if (st != DIG_OK) return st;
  return synth_solve(cfg, opts, m_half, hot, mask, m_next, ws, kStaticSynthBytes, max_iter, tol,
                     iters, change, stream);
}

}  // extern "C"
