// common.h -- device-side building blocks of the gfx950 library: grid geometry and
// boundary index maps, the van der Waals thermodynamics, the logarithmic mean, the
// multi-resolution WENO reconstruction and wavefront reductions.  FP64 throughout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/esvdw.h"

#define MAXD 3
#define MAXNV 5
#define GH 3 /* ghost layers of node data (the stencils reach i-3 .. i+3) */

struct Geo {
  int dim, nv;
  int n[3];    // interior nodes (1 in unused directions)
  int g[3];    // ghost layers of the node buffer (GH in active directions)
  int P[3];    // node-buffer extents; P[0] is the row stride, n0 + 2 g0 rounded up to 16 doubles
  int E0;      // nodes per node-buffer row that hold data: n0 + 2 g0
  long N, PN;  // interior / padded node counts
  double lo[3], hi[3], dxi[3], idxi[3], period[3];
  int bc[3];
  int walls;  // ESVDW_WALL_* bits
  double R, cv, a, b, delta, iR;
  double wl0, wl1, wl2, weps, iwl0;
  int diss;
  double lmc[8];  // log-mean series coefficients 1/15, 1/13, ..., 1/3, 1/17 (see inv_logmean_rn)
  int s0, s1;     // 2D backward-facing step: nodes i0 < s0, i1 < s1 are solid (s0 = 0: none)
  int inflow;     // 1: the lo face of direction 0 holds the fixed state qin
  double qin[4];  // inflow rho, v_1, v_2, T
};

// sixth-order central / high-order flux coefficients alpha_{3,m}: sum m a = 1, sum m^3 a = sum m^5 a = 0
#define AL1 1.5
#define AL2 (-0.3)
#define AL3 (1.0 / 30.0)

// 1/x for the flux kernels: the hardware reciprocal estimate refined by two Newton-Raphson
// steps for 1/x (r <- r + r (1 - x r), each doubling the correct bits), within about one unit
// in the last place for normal, finite x (the kernels' denominators are products of positive
// thermodynamic quantities or of MR-WENO weights, far from zero, overflow and denormals).
// Cheaper than the correctly rounded division sequence, which also handles those edge cases.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// sqrt(x) for the flux kernels, x > 0 normal and finite: the hardware estimate y of 1/sqrt(x)
// refined by the coupled Newton iteration for g = sqrt(x) and h = 1/(2 sqrt(x)) (Markstein's
// method: r = 1/2 - g h, g += g r, h += h r), then two corrections g += (x - g^2) h.  The
// library square root adds range scaling and special cases that the kernels' positive
// thermodynamic and metric magnitudes do not need.
__device__ __forceinline__ double sqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
}

__device__ __forceinline__ int floordiv(int i, int n) { return i >= 0 ? i / n : -((-i + n - 1) / n); }

// interior source of a (possibly ghost) state index along direction k: periodic wrap, mirror
// at a wall face, else the nearest node
__device__ __forceinline__ int state_src(int i, int n, int bc, int walls, int k) {
  if (i >= 0 && i < n) return i;
  if (bc == ESVDW_BC_PERIODIC) return i - floordiv(i, n) * n;
  if (i < 0) return (walls & ESVDW_WALL_LO(k)) ? -1 - i : 0;
  return (walls & ESVDW_WALL_HI(k)) ? 2 * n - 1 - i : n - 1;
}

// ---- the backward-facing step (2D): a solid block of nodes whose two faces are walls ----------
__device__ __forceinline__ bool step_solid(const Geo &G, int i0, int i1) {
  return G.s0 > 0 && i0 < G.s0 && i1 < G.s1;
}
// Seen along direction K, a solid node within 3 nodes of the step's face normal to K is the
// mirror image of a fluid node across that face: true, with the source's index along K in src.
__device__ __forceinline__ bool step_image(const Geo &G, int K, int i0, int i1, int &src) {
  if (!step_solid(G, i0, i1)) return false;
  if (K == 0 && i0 >= G.s0 - 3) {
    src = 2 * G.s0 - 1 - i0;
    return true;
  }
  if (K == 1 && i1 >= G.s1 - 3) {
    src = 2 * G.s1 - 1 - i1;
    return true;
  }
  return false;
}
__device__ __forceinline__ long lin(const Geo &G, int i0, int i1, int i2) {
  return ((long)i2 * G.n[1] + i1) * G.n[0] + i0;
}

__device__ __forceinline__ long state_index(const Geo &G, int i0, int i1, int i2) {
  if ((unsigned)i0 < (unsigned)G.n[0] && (unsigned)i1 < (unsigned)G.n[1] && (unsigned)i2 < (unsigned)G.n[2])
    return lin(G, i0, i1, i2);
  return lin(G, state_src(i0, G.n[0], G.bc[0], G.walls, 0), state_src(i1, G.n[1], G.bc[1], G.walls, 1),
             state_src(i2, G.n[2], G.bc[2], G.walls, 2));
}

// Mesh coordinate j at any index within the ghost reach: periodic directions wrap with a
// shift of one period per wrap (only for the coordinate along that direction); outflow
// directions mirror about the boundary face (the coordinate along the direction is odd,
// the others even).  vel != 0: a mesh velocity component (no shift, same parity).
__device__ __forceinline__ double mesh_at(const Geo &G, const double *__restrict__ x, int j, int i0, int i1,
                                          int i2, int vel) {
  if ((unsigned)i0 < (unsigned)G.n[0] && (unsigned)i1 < (unsigned)G.n[1] && (unsigned)i2 < (unsigned)G.n[2])
    return x[(long)j * G.N + lin(G, i0, i1, i2)];
  int ii[3] = {i0, i1, i2};
  double sg = 1.0, off = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k >= G.dim) break;
    int i = ii[k], n = G.n[k];
    if (i >= 0 && i < n) continue;
    if (G.bc[k] == ESVDW_BC_PERIODIC) {
      int q = floordiv(i, n);
      ii[k] = i - q * n;
      if (k == j && !vel) off = q * G.period[k];
    } else {
      ii[k] = i < 0 ? -1 - i : 2 * n - 1 - i;
      if (k == j) {
        sg = -1.0;
        if (!vel) off = 2.0 * (i < 0 ? G.lo[k] : G.hi[k]);
      }
    }
  }
  return sg * x[(long)j * G.N + lin(G, ii[0], ii[1], ii[2])] + off;
}

// ---------------------------------------------------------------------------------
// discrete metrics (eq. SCLCoeff) on a stage mesh
// ---------------------------------------------------------------------------------
// stage-mesh coordinate: x_n + cdt * xdot, both ghost-extended by the mesh maps
__device__ __forceinline__ double stage_x(const Geo &G, const double *__restrict__ xn, const double *__restrict__ xd,
                                          double cdt, int j, int i0, int i1, int i2) {
  double v = mesh_at(G, xn, j, i0, i1, i2, 0);
  if (xd && cdt != 0.0) v += cdt * mesh_at(G, xd, j, i0, i1, i2, 1);
  return v;
}

// The stage mesh xn + cdt xd (cdt = c_s dt) at any index within the ghost reach, formed at the
// interior source node with the arithmetic of the update kernels' next-stage mesh and then mapped
// as mesh_at maps a coordinate: the same bits as that materialised mesh read through mesh_at.
__device__ __forceinline__ double stage_x_src(const Geo &G, const double *__restrict__ xn,
                                              const double *__restrict__ xd, double cs, double dt, int j, int i0,
                                              int i1, int i2) {
  int ii[3] = {i0, i1, i2};
  double sg = 1.0, off = 0.0;
  bool ghost = false;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k >= G.dim) break;
    int i = ii[k], n = G.n[k];
    if (i >= 0 && i < n) continue;
    ghost = true;
    if (G.bc[k] == ESVDW_BC_PERIODIC) {
      int q = floordiv(i, n);
      ii[k] = i - q * n;
      if (k == j) off = q * G.period[k];
    } else {
      ii[k] = i < 0 ? -1 - i : 2 * n - 1 - i;
      if (k == j) {
        sg = -1.0;
        off = 2.0 * (i < 0 ? G.lo[k] : G.hi[k]);
      }
    }
  }
  const long q = (long)j * G.N + lin(G, ii[0], ii[1], ii[2]);
  const double v = fma(cs * dt, xd[q], xn[q]);
  return ghost ? sg * v + off : v;
}

// delta_k[x_j] at (i0, i1, i2): (1/2) sum_m alpha_m (x_{i+m e_k} - x_{i-m e_k})
__device__ __forceinline__ double delta_x(const Geo &G, const double *xn, const double *xd, double cdt, int k, int j,
                                          int i0, int i1, int i2) {
  int e0 = k == 0, e1 = k == 1, e2 = k == 2;
  double s = 0.0;
  const double al[3] = {AL1, AL2, AL3};
#pragma unroll
  for (int m = 1; m <= 3; ++m)
    s += al[m - 1] * (stage_x(G, xn, xd, cdt, j, i0 + m * e0, i1 + m * e1, i2 + m * e2) -
                      stage_x(G, xn, xd, cdt, j, i0 - m * e0, i1 - m * e1, i2 - m * e2));
  return 0.5 * s;
}

__device__ __forceinline__ long dp_index(const Geo &G, int i0, int i1, int i2) {
  int P0 = G.n[0] + 12, P1 = G.n[1] + 12;
  return ((long)(i2 + 6) * P1 + (i1 + 6)) * P0 + (i0 + 6);
}

// metric J dxi_k/dx_j at (i0, i1, i2) from the stage mesh (2D directly, 3D from dprod)
template <int D>
__device__ __forceinline__ double metric_at(const Geo &G, const double *xn, const double *xd, double cdt,
                                            const double *dp, long dpN, int k, int j, int i0, int i1, int i2) {
  if (D == 1) return 1.0;
  if (D == 2) {
    // J dxi_1/dx_1 = x_2,xi2 ; J dxi_1/dx_2 = -x_1,xi2 ; J dxi_2/dx_1 = -x_2,xi1 ; J dxi_2/dx_2 = x_1,xi1
    int kk = 1 - k, jj = 1 - j;
    double sg = (k == j) ? 1.0 : -1.0;
    return sg * delta_x(G, xn, xd, cdt, kk, jj, i0, i1, i2) * G.idxi[kk];
  }
  // D == 3: (delta_{k2}[delta_{k1}[x_{j1}] x_{j2}] - delta_{k1}[delta_{k2}[x_{j1}] x_{j2}]) / (dxi_{k1} dxi_{k2})
  int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
  const double al[3] = {AL1, AL2, AL3};
  // dp holds delta_in[x_{j+1}] x_{j+2} at every padded node; the stencil is the node's own
  // index plus or minus m strides along `out`
  const long c = dp_index(G, i0, i1, i2);
  const long stride[3] = {1, (long)(G.n[0] + 12), (long)(G.n[0] + 12) * (G.n[1] + 12)};
  double s = 0.0;
  for (int term = 0; term < 2; ++term) {
    int in = term == 0 ? k1 : k2, out = term == 0 ? k2 : k1;
    const double *f = dp + (long)(in * 3 + j) * dpN + c;
    const long st = stride[out];
    double acc = 0.0;
#pragma unroll
    for (int m = 1; m <= 3; ++m) {
      double fa = f[m * st];
      double fb = f[-m * st];
      acc += al[m - 1] * (fa - fb);
    }
    s += (term == 0 ? 0.5 : -0.5) * acc;
  }
  return s * G.idxi[k1] * G.idxi[k2];
}

// 2D metrics m[k][j] = J dxi_k/dx_j at (i0, i1) on the stage mesh x_n + cdt xdot.  Nodes whose
// whole stencil (3 nodes each way) is interior read the mesh directly, in the same arithmetic
// order as delta_x; the others go through the boundary maps of mesh_at.  Keeping the common
// case free of the boundary logic keeps the node kernels' code small.
__device__ __forceinline__ void metrics2(const Geo &G, const double *__restrict__ xn, const double *__restrict__ xd,
                                         double cdt, int i0, int i1, double m[2][2]) {
  if (i0 >= 3 && i0 + 3 < G.n[0] && i1 >= 3 && i1 + 3 < G.n[1]) {
    const double al[3] = {AL1, AL2, AL3};
    const long t = (long)i1 * G.n[0] + i0, s1 = G.n[0];
    const bool mv = xd && cdt != 0.0;
    double d[2][2];  // d[q][r] = delta_q[x_r]
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const long e = q == 0 ? 1 : s1;
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const double *xr = xn + (long)r * G.N, *vr = mv ? xd + (long)r * G.N : nullptr;
        double acc = 0.0;
#pragma unroll
        for (int k = 1; k <= 3; ++k) {
          double p = xr[t + k * e], n = xr[t - k * e];
          if (mv) {
            p += cdt * vr[t + k * e];
            n += cdt * vr[t - k * e];
          }
          acc += al[k - 1] * (p - n);
        }
        d[q][r] = 0.5 * acc;
      }
    }
    // J dxi_1/dx_1 = x_2,xi2 ; J dxi_1/dx_2 = -x_1,xi2 ; J dxi_2/dx_1 = -x_2,xi1 ; J dxi_2/dx_2 = x_1,xi1
    m[0][0] = d[1][1] * G.idxi[1];
    m[0][1] = -d[1][0] * G.idxi[1];
    m[1][0] = -d[0][1] * G.idxi[0];
    m[1][1] = d[0][0] * G.idxi[0];
    return;
  }
  // boundary nodes: one rolled loop over (q, r, k) keeps this rare path compact; the sums run
  // over k = 1, 2, 3 in order, as in delta_x
  double d00 = 0.0, d01 = 0.0, d10 = 0.0, d11 = 0.0;
#pragma unroll 1
  for (int it = 0; it < 12; ++it) {
    const int q = it / 6, r = (it / 3) & 1, k = it % 3 + 1;
    const int e0 = q == 0 ? k : 0, e1 = q == 1 ? k : 0;
    const double c = (k == 1 ? AL1 : (k == 2 ? AL2 : AL3)) *
                     (stage_x(G, xn, xd, cdt, r, i0 + e0, i1 + e1, 0) - stage_x(G, xn, xd, cdt, r, i0 - e0, i1 - e1, 0));
    if (q == 0) {
      if (r == 0) d00 += c;
      else d01 += c;
    } else {
      if (r == 0) d10 += c;
      else d11 += c;
    }
  }
  m[0][0] = (0.5 * d11) * G.idxi[1];
  m[0][1] = -(0.5 * d10) * G.idxi[1];
  m[1][0] = -(0.5 * d01) * G.idxi[0];
  m[1][1] = (0.5 * d00) * G.idxi[0];
}

// 2D metric stencils from LDS: a tile of TX x TY nodes whose first node has interior index
// (c0, c1), with the stage mesh x_n + cdt xdot of the tile and a 3-node halo staged once per
// block (each mesh value is then read from memory about (TX+6)(TY+6)/(TX TY) times instead of
// 12 or 24 times per node).  Values and sums are those of metrics2.
template <int TX, int TY> struct MeshTile2 {
  double x[2][TY + 6][TX + 6];
};

template <int TX, int TY>
__device__ __forceinline__ void mesh_tile_fill(const Geo &G, const double *__restrict__ xn, const double *__restrict__ xd,
                                               double cdt, int c0, int c1, MeshTile2<TX, TY> &T, int tid, int nth) {
  constexpr int W = TX + 6, NS = W * (TY + 6);
  for (int idx = tid; idx < NS; idx += nth) {
    const int a = idx % W, b = idx / W;
    const int i0 = c0 - 3 + a, i1 = c1 - 3 + b;
    // the stencils of the padded grid (3 ghost layers) reach 6 nodes beyond the interior
    const bool in = i0 >= -6 && i0 < G.n[0] + 6 && i1 >= -6 && i1 < G.n[1] + 6;
    T.x[0][b][a] = in ? stage_x(G, xn, xd, cdt, 0, i0, i1, 0) : 0.0;
    T.x[1][b][a] = in ? stage_x(G, xn, xd, cdt, 1, i0, i1, 0) : 0.0;
  }
}

// the same tile of the stage mesh xn + cs dt xd formed at the source nodes (stage_x_src)
template <int TX, int TY>
__device__ __forceinline__ void mesh_tile_fill_stage(const Geo &G, const double *__restrict__ xn,
                                                     const double *__restrict__ xd, double cs, double dt, int c0,
                                                     int c1, MeshTile2<TX, TY> &T, int tid, int nth) {
  constexpr int W = TX + 6, NS = W * (TY + 6);
  for (int idx = tid; idx < NS; idx += nth) {
    const int a = idx % W, b = idx / W;
    const int i0 = c0 - 3 + a, i1 = c1 - 3 + b;
    const bool in = i0 >= -6 && i0 < G.n[0] + 6 && i1 >= -6 && i1 < G.n[1] + 6;
    T.x[0][b][a] = in ? stage_x_src(G, xn, xd, cs, dt, 0, i0, i1, 0) : 0.0;
    T.x[1][b][a] = in ? stage_x_src(G, xn, xd, cs, dt, 1, i0, i1, 0) : 0.0;
  }
}

// m[k][j] = J dxi_k/dx_j of the node at tile coordinates (u, v)
template <int TX, int TY>
__device__ __forceinline__ void mesh_tile_metrics(const Geo &G, const MeshTile2<TX, TY> &T, int u, int v,
                                                  double m[2][2]) {
  const double al[3] = {AL1, AL2, AL3};
  const int a = u + 3, b = v + 3;
  double d[2][2];  // d[q][r] = delta_q[x_r]
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int k = 1; k <= 3; ++k) {
        const double p = q == 0 ? T.x[r][b][a + k] : T.x[r][b + k][a];
        const double n = q == 0 ? T.x[r][b][a - k] : T.x[r][b - k][a];
        acc += al[k - 1] * (p - n);
      }
      d[q][r] = 0.5 * acc;
    }
  m[0][0] = d[1][1] * G.idxi[1];
  m[0][1] = -d[1][0] * G.idxi[1];
  m[1][0] = -d[0][1] * G.idxi[0];
  m[1][1] = d[0][0] * G.idxi[0];
}

// ---------------------------------------------------------------------------------
// thermodynamics (eq. vdWEOS and the closed forms of Section 2, general units)
// ---------------------------------------------------------------------------------
__device__ __forceinline__ double eos_p(const Geo &G, double rho, double T) {
  return rho * G.R * T / (1.0 - G.b * rho) - G.a * rho * rho;
}
__device__ __forceinline__ double eos_T_rho_e(const Geo &G, double rho, double e) { return (e + G.a * rho) / G.cv; }
__device__ __forceinline__ double eos_T_rho_p(const Geo &G, double rho, double p) {
  return (p + G.a * rho * rho) * (1.0 - G.b * rho) / (G.R * rho);
}
__device__ __forceinline__ double eos_c2(const Geo &G, double rho, double T) {
  double ob = 1.0 - G.b * rho;
  return (1.0 + G.delta) * G.R * T / (ob * ob) - 2.0 * G.a * rho;
}
__device__ __forceinline__ double eos_G(const Geo &G, double rho, double T) {
  double ob = 1.0 - G.b * rho;
  return ((1.0 + G.delta) * (2.0 + G.delta) * G.R * T / (ob * ob * ob) - 6.0 * G.a * rho) / (2.0 * eos_c2(G, rho, T));
}
// 1/J, rho, v and T of interior node t (the monitor's rho and G come from the same values)
template <int D>
__device__ __forceinline__ void node_prim(const Geo &G, const double *__restrict__ JU, const double *__restrict__ J,
                                          long t, double &iJ, double &rho, double (&v)[D], double &T) {
  iJ = 1.0 / J[t];
  rho = JU[t] * iJ;
  double v2 = 0.0;
#pragma unroll
  for (int m = 0; m < D; ++m) {
    v[m] = JU[(long)(1 + m) * G.N + t] * iJ / rho;
    v2 += v[m] * v[m];
  }
  T = eos_T_rho_e(G, rho, JU[(long)(D + 1) * G.N + t] * iJ / rho - 0.5 * v2);
}

// eq. coefflimit / eq. Tlimit
__device__ __forceinline__ bool admissible(const Geo &G, double rho, double T) {
  double ob = 1.0 - G.b * rho;
  bool ok = rho > 0.0 && ob > 0.0;
  ok = ok && (G.b > 0.0 ? T * 4.0 * G.R * G.b > G.a : T > 0.0);
  return ok && (G.R * T - 2.0 * G.a * rho * ob * ob > 0.0);
}

// 1/L(a_l, a_r) for the logarithmic mean L = (a_r - a_l)/(ln a_r - ln a_l), given the node
// logarithms.  Close arguments (|a_r - a_l| < 0.1 (a_l + a_r), i.e. f = (a_r - a_l)/(a_r + a_l)
// with f^2 < 0.01) use 1/L = 2 (atanh(f)/f)/(a_l + a_r) with the Taylor series of atanh(f)/f to
// u^8, u = f^2 (truncation < 1e-17); otherwise the logarithms.  The reciprocal of the
// denominator is supplied, so that several log means can share one division:
// den = logmean_den(al, ar) is the sum (series) or the difference (logarithms).
__device__ __forceinline__ double logmean_den(double al, double ar) {
  double d = ar - al, s = al + ar;
  return fabs(d) < 0.1 * s ? s : d;
}

// N values 1/L(al_j, ar_j) with la_j = ln al_j, lb_j = ln ar_j and iden_j = 1/logmean_den,
// the N series evaluated side by side.  cf: 1/15, 1/13, ..., 1/3 and 1/17 (Geo::lmc: passed as
// uniform values, so that the FMAs read them from scalar registers; a 64-bit literal cannot be
// an FMA operand and would be rebuilt in vector registers at every use).
template <int N>
__device__ __forceinline__ void inv_logmean_rn(const double *cf, const double (&al)[N], const double (&ar)[N],
                                               const double (&la)[N], const double (&lb)[N], const double (&iden)[N],
                                               double (&out)[N]) {
  double u[N], h[N];
  bool ser[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const double d = ar[j] - al[j], s = al[j] + ar[j], f = d * iden[j];
    ser[j] = fabs(d) < 0.1 * s;
    u[j] = f * f;
    h[j] = cf[7];
  }
#pragma unroll
  for (int k = 0; k < 7; ++k) {
#pragma unroll
    for (int j = 0; j < N; ++j) h[j] = fma(u[j], h[j], cf[k]);
  }
#pragma unroll
  for (int j = 0; j < N; ++j) h[j] = fma(u[j], h[j], 1.0);
#pragma unroll
  for (int j = 0; j < N; ++j) out[j] = ser[j] ? 2.0 * h[j] * iden[j] : (lb[j] - la[j]) * iden[j];
}

// Multi-resolution WENO, fifth order: left limit at the right face of the centre cell of
// (a, b, c, d, e) = w_{i-2..i+2}.  Hierarchy of central levels: 1 point (w_i), 3 points
// (quadratic), 5 points (quartic) with linear weights wl2, wl1, wl0.
__device__ __forceinline__ double mrweno5(const Geo &G, double a, double b, double c, double d, double e) {
  double q5 = (2.0 * a - 13.0 * b + 47.0 * c + 27.0 * d - 3.0 * e) * (1.0 / 60.0);
  double q3 = (-b + 5.0 * c + 2.0 * d) * (1.0 / 6.0);
  double dl = c - b, dr = d - c;
  double s1 = fmin(dl * dl, dr * dr);
  double t1 = b - 2.0 * c + d, t2 = d - b;
  double s3 = (13.0 / 12.0) * t1 * t1 + 0.25 * t2 * t2;
  // the Jiang-Shu functional of the quartic depends only on its derivatives, so it is evaluated
  // on the data relative to the centre value c: the same quadratic form without cancellation
  // between terms of the size of the data's square (entropy-variable data carry c_v ln T offsets)
  const double am = a - c, bm = b - c, dp = d - c, ep = e - c;
  double s5 = (104963.0 * (bm * bm + dp * dp) - 51001.0 * (am * bm + dp * ep) + 179098.0 * bm * dp -
               38947.0 * (bm * ep + am * dp) + 6908.0 * (am * am + ep * ep) + 8209.0 * am * ep) *
              (1.0 / 5040.0);
  double tt = 0.5 * (fabs(s5 - s1) + fabs(s5 - s3));
  double tau = tt * tt;
  // w_l = wl_l (1 + tau/(s_l + eps)), normalised; multiplied through by the product of the
  // (s_l + eps) so that one division remains
  double e5 = s5 + G.weps, e3 = s3 + G.weps, e1 = s1 + G.weps;
  double w5 = G.wl0 * (e3 * e1) * (e5 + tau);
  double w3 = G.wl1 * (e5 * e1) * (e3 + tau);
  double w1 = G.wl2 * (e5 * e3) * (e1 + tau);
  double top = (q5 - G.wl1 * q3 - G.wl2 * c) * G.iwl0;
  return (w5 * top + w3 * q3 + w1 * c) / (w5 + w3 + w1);
}

// mrweno5 relative to the centre value, as a fraction: mrweno5(a, b, c, d, e) = c + num / den
// with den > 0 (the caller divides, possibly sharing the division).  Every level is formed
// from the differences to c (the levels' coefficients sum to one, and the 1-point level is c
// itself), which also removes the cancellation of c in the weighted sum.  The weights are
// those of mrweno5 multiplied through by (s5 + eps)(s3 + eps)(s1 + eps): with e_l = s_l + eps
// and P = e5 e3 e1, w_l = wl_l (P + tau P / e_l); the linear weights then cancel from the
// quartic level's numerator, w5 (q5 - wl1 q3 - wl2 c)/wl0 = (P + tau e3 e1)(q5 - wl1 q3 - wl2 c).
__device__ __forceinline__ void mrweno5_cfrac(const Geo &G, double a, double b, double c, double d, double e,
                                              double &num, double &den) {
  const double am = a - c, bm = b - c, dp = d - c, ep = e - c;
  const double q5 = (2.0 / 60.0) * am - (13.0 / 60.0) * bm + (27.0 / 60.0) * dp - (3.0 / 60.0) * ep;
  const double q3 = (1.0 / 3.0) * dp - (1.0 / 6.0) * bm;
  const double b2 = bm * bm, d2 = dp * dp, t0 = b2 + d2;
  const double s1 = fmin(b2, d2);
  // (13/12)(bm + dp)^2 + (1/4)(dp - bm)^2
  const double s3 = fma((5.0 / 3.0) * bm, dp, (4.0 / 3.0) * t0);
  // the Jiang-Shu functional of the quartic (see mrweno5), grouped by the first factor:
  // c1 (bm^2 + dp^2) + bm (-c2 am + c3 dp - c4 ep) - dp (c2 ep + c4 am) + am (c5 am + c6 ep) + c5 ep^2
  const double X = fma(179098.0 / 5040.0, dp, fma(-38947.0 / 5040.0, ep, (-51001.0 / 5040.0) * am));
  const double Y = fma(-51001.0 / 5040.0, ep, (-38947.0 / 5040.0) * am);
  const double Z = fma(8209.0 / 5040.0, ep, (6908.0 / 5040.0) * am);
  double s5 = fma(bm, X, (104963.0 / 5040.0) * t0);
  s5 = fma(dp, Y, s5);
  s5 = fma(am, Z, s5);
  s5 = fma(ep, (6908.0 / 5040.0) * ep, s5);
  const double tt = 0.5 * (fabs(s5 - s1) + fabs(s5 - s3));
  const double tau = tt * tt;
  const double e5 = s5 + G.weps, e3 = s3 + G.weps, e1 = s1 + G.weps;
  const double e31 = e3 * e1, P = e5 * e31;
  const double A5 = fma(e31, tau, P), A3 = fma(e5 * e1, tau, P), A1 = fma(e5 * e3, tau, P);
  const double wq3 = G.wl1 * q3;
  num = fma(A5, q5 - wq3, A3 * wq3);
  den = fma(G.wl0, A5, fma(G.wl1, A3, G.wl2 * A1));
}

// ---------------------------------------------------------------------------------
// reductions: wavefront (64 lanes) by shuffles, then across the block through LDS; each
// block writes one partial, and a one-block kernel reduces the partials (no atomics on a
// single address)
// ---------------------------------------------------------------------------------
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int flat_tid() { return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z); }
__device__ __forceinline__ int flat_bid() { return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z); }
__device__ __forceinline__ int block_threads() { return blockDim.x * blockDim.y * blockDim.z; }

// block-wide max / min (any block size up to 1024); the result is valid in thread 0
__device__ __forceinline__ double block_max(double v) {
  __shared__ double part[16];
  v = wave_max(v);
  int ft = flat_tid(), lane = ft & 63, w = ft >> 6;
  if (lane == 0) part[w] = v;
  __syncthreads();
  double m = part[0];
  if (ft == 0) {
    int nw = (block_threads() + 63) >> 6;
    for (int i = 1; i < nw; ++i) m = fmax(m, part[i]);
  }
  __syncthreads();
  return m;
}
__device__ __forceinline__ double block_min(double v) {
  __shared__ double part[16];
  v = wave_min(v);
  int ft = flat_tid(), lane = ft & 63, w = ft >> 6;
  if (lane == 0) part[w] = v;
  __syncthreads();
  double m = part[0];
  if (ft == 0) {
    int nw = (block_threads() + 63) >> 6;
    for (int i = 1; i < nw; ++i) m = fmin(m, part[i]);
  }
  __syncthreads();
  return m;
}

__device__ __forceinline__ void raise_flag(unsigned *flags, unsigned f) { atomicOr(flags, f); }

// Node-wise kernels run on a 3D grid: blockDim (64, 4, 1) (or (256, 1, 1) in 1D), one grid
// z-slice per z index, so node coordinates need no integer division.
#define NODE_COORDS(n0, n1)                                                                                  \
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x, i1 = blockIdx.y * blockDim.y + threadIdx.y,        \
            i2 = blockIdx.z;                                                                               \
  const bool inside = i0 < (n0) && i1 < (n1)

static inline void node_grid(int n0, int n1, int n2, dim3 &g, dim3 &b) {
  if (n1 == 1 && n2 == 1) {
    b = dim3(256, 1, 1);
    g = dim3((n0 + 255) / 256, 1, 1);
  } else {
    b = dim3(64, 4, 1);
    g = dim3((n0 + 63) / 64, (n1 + 3) / 4, n2);
  }
}

// device scalar slots of a context
enum { SC_CFL = 0, SC_MON = 1, SC_GAMMA = 4, SC_RESID = 5, SC_DT = 6, SC_N = 8 };

// ---------------------------------------------------------------------------------
// host-side context
// ---------------------------------------------------------------------------------
struct esvdw_ctx {
  esvdw_params p;
  Geo G;
  int dev;
  int NF;            // node-buffer fields
  double *node;      // NF * PN padded node data (rows start so that node g0 is 128-byte aligned)
  double *node_mem;  // the allocation behind node
  double *flux[3];   // per direction: (nv + 1) * interfaces
  long nif[3];       // interfaces per direction
  double *dprod;     // 3D: 9 fields of delta_q[x_{j+1}] x_{j+2} on a 6-ghost padded grid
  long dpN;          // padded node count of dprod
  double *met;       // dim*dim + dim fields (interior), scratch for cfl/jacobian
  double *stA, *stB; // RK stage buffers, (nv + 1) * N each
  double *xdot, *xmu, *xtmp;  // dim * N each
  double *omega, *omega2, *mterm;  // N, N, 3N
  double *rhoG;      // 2N
  double *scal;      // SC_N doubles
  double *part;      // per-block partial reductions (4 * max blocks)
  long npart;        // capacity of part per slot
  unsigned *flags;
};

// node-buffer field offsets for dimension D: primitives, 1/T, 1/(1 - b rho), the logarithms
// of rho, 1 - b rho, T, p, the first entropy variable V_1 (the others are v/T and -1/T), the
// metrics J dxi_k/dx_j and J dxi_k/dt
template <int D> struct NF_ {
  static constexpr int RHO = 0, V = 1, T = D + 1, P = D + 2, IT = D + 3, IOB = D + 4, LNR = D + 5, LNB = D + 6,
                       LNT = D + 7, LNP = D + 8, V1 = D + 9, MS = D + 10, XS = MS + D * D, COUNT = XS + D;
};
