// rhs.hip -- metrics, node thermodynamics, interface fluxes and the RK-stage update of the
// entropy-stable moving-mesh scheme (Sections 3.1-3.3).  One launch pipeline per RHS:
//   k_dprod (3D only)  delta_q[x_r] x_s products on the stage mesh
//   k_nodes            per padded node: primitives, 1/T, g, entropy variables, metrics
//   k_flux<K>          per interface along K: sixth-order EC flux + MR-WENO dissipation
//   k_update           flux differences, optional SSP-RK3 combination
#include "common.h"
#include "kernels.h"
#include "scheme.h"

// =============================== metrics ========================================

// 3D: dprod[q*3 + j] = delta_q[x_{j+1}] x_{j+2} (indices mod 3), the inner products of the
// nested metric form, on a grid padded by 6 in every direction (valid where the q index is
// within 3 of the interior, which is where it is used)
__global__ void k_dprod(Geo G, const double *__restrict__ xn, const double *__restrict__ xd, double cdt,
                        double *__restrict__ dp, long dpN) {
  const int P0 = G.n[0] + 12, P1 = G.n[1] + 12;
  NODE_COORDS(P0, P1);
  if (!inside) return;
  const long t = ((long)i2 * P1 + i1) * P0 + i0;
  {
  const int i0 = (int)(blockIdx.x * blockDim.x + threadIdx.x) - 6,
            i1 = (int)(blockIdx.y * blockDim.y + threadIdx.y) - 6, i2 = (int)blockIdx.z - 6;
  int ii[3] = {i0, i1, i2};
  const double xs[3] = {stage_x(G, xn, xd, cdt, 0, i0, i1, i2), stage_x(G, xn, xd, cdt, 1, i0, i1, i2),
                        stage_x(G, xn, xd, cdt, 2, i0, i1, i2)};
  for (int q = 0; q < 3; ++q) {
    bool ok = ii[q] >= -3 && ii[q] < G.n[q] + 3;
    for (int j = 0; j < 3; ++j)
      dp[(long)(q * 3 + j) * dpN + t] =
          ok ? delta_x(G, xn, xd, cdt, q, (j + 1) % 3, i0, i1, i2) * xs[(j + 2) % 3] : 0.0;
  }
  }
}

// interior metrics (compute_metrics) and, optionally, the Jacobian (init_mesh)
template <int D>
__global__ void k_metrics(Geo G, const double *__restrict__ xn, const double *__restrict__ xd,
                          const double *__restrict__ dp, long dpN, double *__restrict__ met,
                          double *__restrict__ xit, double *__restrict__ J) {
  NODE_COORDS(G.n[0], G.n[1]);
  if (!inside) return;
  const long t = lin(G, i0, i1, i2);
  double m[D][D];
  for (int k = 0; k < D; ++k)
    for (int j = 0; j < D; ++j) m[k][j] = metric_at<D>(G, xn, nullptr, 0.0, dp, dpN, k, j, i0, i1, i2);
  if (met)
    for (int k = 0; k < D; ++k)
      for (int j = 0; j < D; ++j) met[(long)(k * D + j) * G.N + t] = m[k][j];
  if (xit) {
    for (int k = 0; k < D; ++k) {
      double s = 0.0;
      if (xd)
        for (int j = 0; j < D; ++j) s -= xd[(long)j * G.N + t] * m[k][j];
      xit[(long)k * G.N + t] = s;
    }
  }
  if (J) {
    double v;
    if (D == 1) {
      v = delta_x(G, xn, nullptr, 0.0, 0, 0, i0, i1, i2) * G.idxi[0];
    } else if (D == 2) {
      v = (delta_x(G, xn, nullptr, 0.0, 0, 0, i0, i1, i2) * delta_x(G, xn, nullptr, 0.0, 1, 1, i0, i1, i2) -
           delta_x(G, xn, nullptr, 0.0, 1, 0, i0, i1, i2) * delta_x(G, xn, nullptr, 0.0, 0, 1, i0, i1, i2)) *
          G.idxi[0] * G.idxi[1];
    } else {
      v = 0.0;
      for (int j = 0; j < D; ++j) v += delta_x(G, xn, nullptr, 0.0, 0, j, i0, i1, i2) * G.idxi[0] * m[0][j];
    }
    J[t] = v;
  }
}

// =============================== node data =======================================

template <int D>
__global__ void k_nodes(Geo G, const double *__restrict__ JU, const double *__restrict__ J,
                        const double *__restrict__ met_in, const double *__restrict__ xit_in,
                        const double *__restrict__ xn, const double *__restrict__ xd, double cdt,
                        const double *__restrict__ dp, long dpN, double *__restrict__ nd, unsigned *flags) {
  const int p0 = blockIdx.x * blockDim.x + threadIdx.x, p1 = blockIdx.y * blockDim.y + threadIdx.y, p2 = blockIdx.z;
  if (p0 >= G.E0 || p1 >= G.P[1]) return;
  node_point<D>(G, JU, J, met_in, xit_in, xn, xd, cdt, dp, dpN, nd, flags, p0, p1, p2);
}

// =============================== interface fluxes ================================

template <int D, int K>
__global__ void __launch_bounds__(256, 3) k_flux(Geo G, const double *__restrict__ nd, double *__restrict__ Fo, long nif,
                                              unsigned *flags) {
  using TL = Tile<D, K>;
  __shared__ double sP[FluxLds<D, K, TL::X, TL::Y, TL::Z>::SIZE];
  flux_tile<D, K, TL::X, TL::Y, TL::Z>(G, nd, Fo, nif, flags, blockIdx.x * TL::X, blockIdx.y * TL::Y,
                                       blockIdx.z * TL::Z, sP);
}

// =============================== update ==========================================

template <int D>
__global__ void k_update(Geo G, const double *__restrict__ F0, const double *__restrict__ F1,
                         const double *__restrict__ F2, long nif0, long nif1, long nif2, int mode, int s,
                         const double *__restrict__ dtp, const double *__restrict__ base_JU,
                         const double *__restrict__ base_J, const double *__restrict__ in_JU,
                         const double *__restrict__ in_J, double *__restrict__ out_JU, double *__restrict__ out_J,
                         unsigned *flags, const double *mx, const double *mxd, double mf, double *mout) {
  NODE_COORDS(G.n[0], G.n[1]);
  if (!inside) return;
  update_point<D>(G, F0, F1, F2, nif0, nif1, nif2, mode, s, dtp, base_JU, base_J, in_JU, in_J, out_JU, out_J, flags,
                  i0, i1, i2);
  if (mout) {
    // the next stage's mesh x_n + f dt xdot at this node (k_axpy_mesh's arithmetic; mout may be mx)
    const long t = lin(G, i0, i1, i2);
#pragma unroll
    for (int j = 0; j < D; ++j) mout[(long)j * G.N + t] = mx[(long)j * G.N + t] + mf * (*dtp) * mxd[(long)j * G.N + t];
  }
}

// =============================== small kernels ===================================

__global__ void k_uniform_mesh(Geo G, double *__restrict__ x) {
  NODE_COORDS(G.n[0], G.n[1]);
  if (!inside) return;
  const long t = lin(G, i0, i1, i2);
  int ii[3] = {i0, i1, i2};
  for (int j = 0; j < G.dim; ++j) x[(long)j * G.N + t] = G.lo[j] + (ii[j] + 0.5) * G.dxi[j];
}

template <int D>
__global__ void k_init_state(Geo G, const double *__restrict__ prim, const double *__restrict__ J,
                             double *__restrict__ JU) {
  NODE_COORDS(G.n[0], G.n[1]);
  if (!inside) return;
  const long t = lin(G, i0, i1, i2);
  double rho = prim[t], p = prim[(long)(D + 1) * G.N + t];
  double T = eos_T_rho_p(G, rho, p);
  double jj = J[t], v2 = 0.0;
  JU[t] = jj * rho;
  for (int m = 0; m < D; ++m) {
    double v = prim[(long)(1 + m) * G.N + t];
    v2 += v * v;
    JU[(long)(1 + m) * G.N + t] = jj * rho * v;
  }
  JU[(long)(D + 1) * G.N + t] = jj * (rho * (G.cv * T - G.a * rho) + 0.5 * rho * v2);
}

__global__ void k_axpy_mesh(long n, const double *__restrict__ x, const double *__restrict__ xd,
                            const double *__restrict__ dtp, double f, double *out) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  out[t] = x[t] + f * (*dtp) * xd[t];
}

// =============================== launchers =======================================

static inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

int launch_dprod(esvdw_ctx *c, const double *xn, const double *xd, double cdt, hipStream_t st) {
  if (c->G.dim != 3) return 0;
  dim3 g, b;
  node_grid(c->G.n[0] + 12, c->G.n[1] + 12, c->G.n[2] + 12, g, b);
  hipLaunchKernelGGL(k_dprod, g, b, 0, st, c->G, xn, xd, cdt, c->dprod, c->dpN);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_metrics(esvdw_ctx *c, const double *x, const double *xd, double *met, double *xit, double *J,
                   hipStream_t st) {
  const Geo &G = c->G;
  if (launch_dprod(c, x, nullptr, 0.0, st)) return -1;
  dim3 b, g;
  node_grid(G.n[0], G.n[1], G.n[2], g, b);
  if (G.dim == 1) hipLaunchKernelGGL(k_metrics<1>, g, b, 0, st, G, x, xd, c->dprod, c->dpN, met, xit, J);
  else if (G.dim == 2) hipLaunchKernelGGL(k_metrics<2>, g, b, 0, st, G, x, xd, c->dprod, c->dpN, met, xit, J);
  else hipLaunchKernelGGL(k_metrics<3>, g, b, 0, st, G, x, xd, c->dprod, c->dpN, met, xit, J);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int D, int K> static void launch_flux_dk(esvdw_ctx *c, hipStream_t st) {
  using TL = Tile<D, K>;
  const Geo &G = c->G;
  int e0 = G.n[0] + (K == 0), e1 = G.n[1] + (K == 1), e2 = G.n[2] + (K == 2);
  dim3 grid((e0 + TL::X - 1) / TL::X, (e1 + TL::Y - 1) / TL::Y, (e2 + TL::Z - 1) / TL::Z);
  hipLaunchKernelGGL((k_flux<D, K>), grid, dim3(256), 0, st, G, c->node, c->flux[K], c->nif[K], c->flags);
}

template <int D> static void launch_flux_d(esvdw_ctx *c, int K, hipStream_t st) {
  if (K == 0) launch_flux_dk<D, 0>(c, st);
  if constexpr (D > 1)
    if (K == 1) launch_flux_dk<D, 1>(c, st);
  if constexpr (D > 2)
    if (K == 2) launch_flux_dk<D, 2>(c, st);
}

template <int D>
static int rhs_pipeline_d(esvdw_ctx *c, const double *JU, const double *J, const double *met, const double *xit,
                          const double *xn, const double *xd, double cdt, int mode, int s, const double *dtp,
                          const double *bJU, const double *bJ, double *oJU, double *oJ, const double *mx,
                          const double *mxd, double mf, double *mout, hipStream_t st) {
  const Geo &G = c->G;
  if (!met && D == 3)
    if (launch_dprod(c, xn, xd, cdt, st)) return -1;
  dim3 gn, bn, gu, bu;
  node_grid(G.E0, G.P[1], G.P[2], gn, bn);
  node_grid(G.n[0], G.n[1], G.n[2], gu, bu);
  hipLaunchKernelGGL(k_nodes<D>, gn, bn, 0, st, G, JU, J, met, xit, xn, xd, cdt, c->dprod, c->dpN, c->node, c->flags);
  launch_flux_d<D>(c, 0, st);
  if (D > 1) launch_flux_d<D>(c, 1, st);
  if (D > 2) launch_flux_d<D>(c, 2, st);
  hipLaunchKernelGGL(k_update<D>, gu, bu, 0, st, G, c->flux[0], c->flux[1], c->flux[2],
                     c->nif[0], c->nif[1], c->nif[2], mode, s, dtp, bJU, bJ, JU, J, oJU, oJ, c->flags, mx, mxd, mf,
                     mout);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_rhs_mesh(esvdw_ctx *c, const double *JU, const double *J, const double *met, const double *xit,
                    const double *xn, const double *xd, double cdt, int mode, int s, const double *dtp,
                    const double *bJU, const double *bJ, double *oJU, double *oJ, const double *mx, const double *mxd,
                    double mf, double *mout, hipStream_t st) {
  switch (c->G.dim) {
    case 1: return rhs_pipeline_d<1>(c, JU, J, met, xit, xn, xd, cdt, mode, s, dtp, bJU, bJ, oJU, oJ, mx, mxd, mf, mout, st);
    case 2: return rhs_pipeline_d<2>(c, JU, J, met, xit, xn, xd, cdt, mode, s, dtp, bJU, bJ, oJU, oJ, mx, mxd, mf, mout, st);
    default: return rhs_pipeline_d<3>(c, JU, J, met, xit, xn, xd, cdt, mode, s, dtp, bJU, bJ, oJU, oJ, mx, mxd, mf, mout, st);
  }
}

int launch_rhs(esvdw_ctx *c, const double *JU, const double *J, const double *met, const double *xit,
               const double *xn, const double *xd, double cdt, int mode, int s, const double *dtp,
               const double *bJU, const double *bJ, double *oJU, double *oJ, hipStream_t st) {
  return launch_rhs_mesh(c, JU, J, met, xit, xn, xd, cdt, mode, s, dtp, bJU, bJ, oJU, oJ, nullptr, nullptr, 0.0,
                         nullptr, st);
}

int launch_uniform_mesh(esvdw_ctx *c, double *x, hipStream_t st) {
  dim3 g, b;
  node_grid(c->G.n[0], c->G.n[1], c->G.n[2], g, b);
  hipLaunchKernelGGL(k_uniform_mesh, g, b, 0, st, c->G, x);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_init_state(esvdw_ctx *c, const double *prim, const double *J, double *JU, hipStream_t st) {
  dim3 g, b;
  node_grid(c->G.n[0], c->G.n[1], c->G.n[2], g, b);
  if (c->G.dim == 1) hipLaunchKernelGGL(k_init_state<1>, g, b, 0, st, c->G, prim, J, JU);
  else if (c->G.dim == 2) hipLaunchKernelGGL(k_init_state<2>, g, b, 0, st, c->G, prim, J, JU);
  else hipLaunchKernelGGL(k_init_state<3>, g, b, 0, st, c->G, prim, J, JU);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_axpy_mesh(esvdw_ctx *c, const double *x, const double *xd, const double *dtp, double f, double *out,
                     hipStream_t st) {
  long n = (long)c->G.dim * c->G.N;
  hipLaunchKernelGGL(k_axpy_mesh, dim3(nblk(n, 256)), dim3(256), 0, st, n, x, xd, dtp, f, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_flux_only(esvdw_ctx *c, int K, hipStream_t st) {
  if (K < 0 || K >= c->G.dim) return -1;
  if (c->G.dim == 1) launch_flux_d<1>(c, K, st);
  else if (c->G.dim == 2) launch_flux_d<2>(c, K, st);
  else launch_flux_d<3>(c, K, st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
