// meshdev.h -- per-node building blocks of the adaptive moving mesh (Section 4), shared by the
// single-problem kernels (mesh.hip) and the batched ones (batch.hip): density and fundamental
// derivative, monitor terms, monitor omega, one low-pass filter pass, one Jacobi sweep of the
// discretised Winslow equations, the movement-limiter bound.
#pragma once
#include "common.h"

// (rho, G) at interior node t
template <int D>
__device__ __forceinline__ void rhoG_vals(const Geo &G, const double *__restrict__ JU, const double *__restrict__ J,
                                          long t, double &rho, double &g) {
  double iJ, v[D], T;
  node_prim<D>(G, JU, J, t, iJ, rho, v, T);
  g = eos_G(G, rho, T);
}
template <int D>
__device__ __forceinline__ void rhoG_point(const Geo &G, const double *__restrict__ JU, const double *__restrict__ J,
                                           double *__restrict__ rg, long t) {
  double rho, g;
  rhoG_vals<D>(G, JU, J, t, rho, g);
  rg[t] = rho;
  rg[G.N + t] = g;
}

// which field term q of the monitor differentiates (0: rho, 1: G) and whether by the Laplacian
// (second differences) instead of the gradient
__device__ __forceinline__ void mon_term_kind(int kind, int kappa, int var0, int var1, int q, int &field,
                                              bool &second) {
  if (kind == ESVDW_MON_VDW) {
    if (q < kappa) {
      field = (q == 0 ? var0 : var1) == ESVDW_VAR_G ? 1 : 0;
      second = false;
    } else {
      field = 1;
      second = true;
    }
  } else {
    field = 0;
    second = q == 1;
  }
}

// one direction's contribution to a monitor term from the centre value f0 and the neighbours fp, fm
__device__ __forceinline__ double mon_term_part(double fp, double f0, double fm, double idxi, bool second) {
  const double g = second ? (fp - 2.0 * f0 + fm) * idxi * idxi : (fp - fm) * 0.5 * idxi;
  return g * g;
}

// the monitor terms at node (i0, i1, i2) into term[q N + t] and val[q]; returns the term count
template <int D>
__device__ __forceinline__ int mon_terms_point(const Geo &G, int kind, int kappa, int var0, int var1,
                                               const double *__restrict__ rg, double *__restrict__ term, int i0,
                                               int i1, int i2, double val[3]) {
  const long t = lin(G, i0, i1, i2);
  int nterm = kind == ESVDW_MON_VDW ? kappa + 1 : 2;
  for (int q = 0; q < nterm; ++q) {
    int field;
    bool second;
    mon_term_kind(kind, kappa, var0, var1, q, field, second);
    const double *f = rg + (long)field * G.N;
    double f0 = f[t], s2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      int e0 = k == 0, e1 = k == 1, e2 = k == 2;
      double fp = f[state_index(G, i0 + e0, i1 + e1, i2 + e2)];
      double fm = f[state_index(G, i0 - e0, i1 - e1, i2 - e2)];
      s2 += mon_term_part(fp, f0, fm, G.idxi[k], second);
    }
    val[q] = kind == ESVDW_MON_VDW ? s2 : sqrt(s2);
    term[(long)q * G.N + t] = val[q];
  }
  return nterm;
}

// omega = (1 + sum_q alpha_q term_q / max_q)^(1/2) at node t (a term with zero maximum drops)
__device__ __forceinline__ double mon_omega_point(const Geo &G, int nterm, const double al[3],
                                                  const double *__restrict__ term, const double *__restrict__ mx,
                                                  long t) {
  double s = 1.0;
  for (int q = 0; q < nterm; ++q) {
    double m = mx[q];
    if (m > 0.0) s += al[q] * term[(long)q * G.N + t] / m;
  }
  return sqrt(s);
}

// one filter pass at node (i0, i1, i2): sum_{j in {-1,0,1}^d} 2^-(|j|_1 + d) in_{i+j}, replicated /
// wrapped at the boundary
template <int D>
__device__ __forceinline__ double filter_point(const Geo &G, const double *__restrict__ in, int i0, int i1, int i2) {
  double s = 0.0;
  const int r1 = D > 1, r2 = D > 2;
  for (int j2 = -r2; j2 <= r2; ++j2)
    for (int j1 = -r1; j1 <= r1; ++j1)
#pragma unroll
      for (int j0 = -1; j0 <= 1; ++j0) {
        int l1 = (j0 != 0) + (j1 != 0) + (j2 != 0) + D;
        s += ldexp(1.0, -l1) * in[state_index(G, i0 + j0, i1 + j1, i2 + j2)];
      }
  return s;
}

// one Jacobi update of the mesh at node (i0, i1, i2) with face-averaged omega; returns the
// largest coordinate change
template <int D>
__device__ __forceinline__ double jacobi_point(const Geo &G, const double *__restrict__ omega,
                                              const double *__restrict__ xin, double *__restrict__ xout, int i0,
                                              int i1, int i2) {
  // no contraction here: k_jacobi_multi2 repeats this arithmetic and must give the same bits
#pragma clang fp contract(off)
  const long t = lin(G, i0, i1, i2);
  double w0 = omega[t];
  double den = 0.0, num[D];
#pragma unroll
  for (int j = 0; j < D; ++j) num[j] = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    int e0 = k == 0, e1 = k == 1, e2 = k == 2;
    double h2 = G.idxi[k] * G.idxi[k];
    double wp = 0.5 * (w0 + omega[state_index(G, i0 + e0, i1 + e1, i2 + e2)]) * h2;
    double wm = 0.5 * (w0 + omega[state_index(G, i0 - e0, i1 - e1, i2 - e2)]) * h2;
    den += wp + wm;
#pragma unroll
    for (int j = 0; j < D; ++j)
      num[j] += fma(wp, mesh_at(G, xin, j, i0 + e0, i1 + e1, i2 + e2, 0),
                    wm * mesh_at(G, xin, j, i0 - e0, i1 - e1, i2 - e2, 0));
  }
  double iden = 1.0 / den, r = 0.0;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    double v = num[j] * iden;
    r = fmax(r, fabs(v - xin[(long)j * G.N + t]));
    xout[(long)j * G.N + t] = v;
  }
  return r;
}

// movement-limiter bound at node (i0, i1, i2) for the move x_n -> x_mu (1 if the node does not move)
template <int D>
__device__ __forceinline__ double limiter_point(const Geo &G, const double *__restrict__ xn,
                                               const double *__restrict__ xmu, int i0, int i1, int i2) {
  const long t = lin(G, i0, i1, i2);
  double g = 1.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    int e0 = k == 0, e1 = k == 1, e2 = k == 2;
    double x0 = xn[(long)k * G.N + t];
    double dx = xmu[(long)k * G.N + t] - x0;
    if (dx < 0.0) g = fmin(g, -(x0 - mesh_at(G, xn, k, i0 - e0, i1 - e1, i2 - e2, 0)) / (2.0 * dx));
    else if (dx > 0.0) g = fmin(g, (mesh_at(G, xn, k, i0 + e0, i1 + e1, i2 + e2, 0) - x0) / (2.0 * dx));
  }
  return g;
}
