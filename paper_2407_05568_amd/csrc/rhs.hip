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
// within 3 of the interior, which is where it is used; zero elsewhere).
//
// A block covers DP_TX x DP_TY padded columns (i0, i1) and marches along i2 through DP_TZ
// output planes.  Each plane of the stage mesh is staged in LDS with a 3-node halo in i0 and
// i1, from which delta_0 and delta_1 are taken; each thread keeps the last seven planes of its
// own column in registers for delta_2.  A stage-mesh value is thus read from memory about 1.6
// times per padded node (halo and the six warm-up planes of a chunk) instead of 54 times.
// The values and the order of every sum are those of delta_x and stage_x.
#define DP_TX 32
#define DP_TY 16
#define DP_TZ 24

__device__ __forceinline__ double delta_of(double p1, double m1, double p2, double m2, double p3, double m3) {
  double s = 0.0;
  s += AL1 * (p1 - m1);
  s += AL2 * (p2 - m2);
  s += AL3 * (p3 - m3);
  return 0.5 * s;
}

__global__ void __launch_bounds__(DP_TX * DP_TY) k_dprod(Geo G, const double *__restrict__ xn,
                                                        const double *__restrict__ xd, double cdt,
                                                        double *__restrict__ dp, long dpN) {
  __shared__ double sx[3][DP_TY + 6][DP_TX + 6];
  const int n0 = G.n[0], n1 = G.n[1], n2 = G.n[2];
  const int P0 = n0 + 12, P1 = n1 + 12;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * DP_TX + tx;
  const int b0 = (int)blockIdx.x * DP_TX - 6, b1 = (int)blockIdx.y * DP_TY - 6;  // first column of the tile
  const int i0 = b0 + tx, i1 = b1 + ty;
  const bool col = i0 < n0 + 6 && i1 < n1 + 6;
  const bool ok0 = i0 >= -3 && i0 < n0 + 3, ok1 = i1 >= -3 && i1 < n1 + 3;
  const int z0 = (int)blockIdx.z * DP_TZ - 6, z1 = min(z0 + DP_TZ, n2 + 6);  // output planes [z0, z1)
  const int pa = max(z0 - 3, -6), pe = z1 + 3;
  double ring[3][7];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int r = 0; r < 7; ++r) ring[j][r] = 0.0;
  const long tcol = (long)(i1 + 6) * P0 + (i0 + 6);
  for (int p = pa; p < pe; ++p) {
    const bool have = p < n2 + 6;  // planes beyond the padded grid feed only zero outputs
    if (have) {  // all loads of the plane are issued before the first LDS store
      constexpr int NS = (DP_TX + 6) * (DP_TY + 6), NIT = (NS + DP_TX * DP_TY - 1) / (DP_TX * DP_TY);
      double v[NIT][3];
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int idx = tid + it * DP_TX * DP_TY;
        const int a = idx % (DP_TX + 6), b = idx / (DP_TX + 6);
        const int g0 = b0 - 3 + a, g1 = b1 - 3 + b;
        const bool in = idx < NS && g0 >= -6 && g0 < n0 + 6 && g1 >= -6 && g1 < n1 + 6;
#pragma unroll
        for (int j = 0; j < 3; ++j) v[it][j] = in ? stage_x(G, xn, xd, cdt, j, g0, g1, p) : 0.0;
      }
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int idx = tid + it * DP_TX * DP_TY;
        if (idx < NS) {
          const int a = idx % (DP_TX + 6), b = idx / (DP_TX + 6);
#pragma unroll
          for (int j = 0; j < 3; ++j) sx[j][b][a] = v[it][j];
        }
      }
    }
    __syncthreads();
    double xc[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      xc[j] = have ? sx[j][ty + 3][tx + 3] : 0.0;
#pragma unroll
      for (int r = 0; r < 6; ++r) ring[j][r] = ring[j][r + 1];
      ring[j][6] = xc[j];
    }
    if (col && p >= z0 && p < z1) {
      const long t = (long)(p + 6) * P1 * P0 + tcol;
      double d[3];
#pragma unroll
      for (int j = 0; j < 3; ++j)
        d[j] = delta_of(sx[j][ty + 3][tx + 4], sx[j][ty + 3][tx + 2], sx[j][ty + 3][tx + 5], sx[j][ty + 3][tx + 1],
                        sx[j][ty + 3][tx + 6], sx[j][ty + 3][tx]);
#pragma unroll
      for (int j = 0; j < 3; ++j) dp[(long)j * dpN + t] = ok0 ? d[(j + 1) % 3] * xc[(j + 2) % 3] : 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j)
        d[j] = delta_of(sx[j][ty + 4][tx + 3], sx[j][ty + 2][tx + 3], sx[j][ty + 5][tx + 3], sx[j][ty + 1][tx + 3],
                        sx[j][ty + 6][tx + 3], sx[j][ty][tx + 3]);
#pragma unroll
      for (int j = 0; j < 3; ++j) dp[(long)(3 + j) * dpN + t] = ok1 ? d[(j + 1) % 3] * xc[(j + 2) % 3] : 0.0;
    }
    const int z = p - 3;  // the plane whose delta_2 the ring now spans
    if (col && z >= z0 && z < z1) {
      const long t = (long)(z + 6) * P1 * P0 + tcol;
      const bool ok2 = z >= -3 && z < n2 + 3;
      double d[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) d[j] = delta_of(ring[j][4], ring[j][2], ring[j][5], ring[j][1], ring[j][6], ring[j][0]);
#pragma unroll
      for (int j = 0; j < 3; ++j) dp[(long)(6 + j) * dpN + t] = ok2 ? d[(j + 1) % 3] * ring[(j + 2) % 3][3] : 0.0;
    }
    __syncthreads();
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

// 2D node data with the stage mesh staged in LDS (mesh_tile_*): a block of 64 x 4 threads
// covers 64 x 8 padded nodes, two rows per thread, the two unrolled so that both rows' loads
// are in flight together (measured: 64 x 16 with the row loop rolled took 10 us more per launch).
#define ND_TX 64
#define ND_TY 8
// cs != 0 (with xd and dtp): the stage mesh is xn + cs dt xd, formed here at the source nodes
// with the arithmetic of the update kernels' next-stage mesh (the same bits as that mesh)
__global__ void __launch_bounds__(256) k_nodes_t2(Geo G, const double *__restrict__ JU, const double *__restrict__ J,
                                                  const double *__restrict__ xn, const double *__restrict__ xd,
                                                  double cdt, const double *__restrict__ dtp, double cs,
                                                  double *__restrict__ nd, unsigned *flags) {
  __shared__ MeshTile2<ND_TX, ND_TY> T;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int b0 = blockIdx.x * ND_TX, b1 = blockIdx.y * ND_TY;  // first padded node of the tile
  if (cs != 0.0 && xd && dtp) {
    mesh_tile_fill_stage<ND_TX, ND_TY>(G, xn, xd, cs, *dtp, b0 - G.g[0], b1 - G.g[1], T, ty * 64 + tx, 256);
  } else {
    const double *xv_src = (xd && cdt != 0.0) ? xd : nullptr;
    mesh_tile_fill<ND_TX, ND_TY>(G, xn, xv_src, cdt, b0 - G.g[0], b1 - G.g[1], T, ty * 64 + tx, 256);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ND_TY / 4; ++r) {
    const int u = tx, v = ty + 4 * r;
    const int p0 = b0 + u, p1 = b1 + v;
    if (p0 >= G.E0 || p1 >= G.P[1]) continue;
    const int i0 = p0 - G.g[0], i1 = p1 - G.g[1];
    const long t = (long)p1 * G.P[0] + p0;
    node_state<2>(G, JU, J, nd, flags, t, i0, i1, 0);
    double m[2][2];
    mesh_tile_metrics<ND_TX, ND_TY>(G, T, u, v, m);
    double xv[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) xv[j] = xd ? mesh_at(G, xd, j, i0, i1, 0, 1) : 0.0;
    node_metrics_store<2>(G, nd, t, m, xv);
  }
}

// =============================== interface fluxes ================================

// ST: the 2D backward-facing step (solid nodes next to its faces stand for mirror images)
template <int D, int K, bool ST = false>
__global__ void __launch_bounds__(256, 3) k_flux(Geo G, const double *__restrict__ nd, double *__restrict__ Fo, long nif,
                                              unsigned *flags) {
  using TL = Tile<D, K>;
  __shared__ double sP[FluxLds<D, K, TL::X, TL::Y, TL::Z>::SIZE];
  flux_tile<D, K, TL::X, TL::Y, TL::Z, TL::PX, TL::PY, ST>(G, nd, Fo, nif, flags, blockIdx.x * TL::X,
                                                           blockIdx.y * TL::Y, blockIdx.z * TL::Z, sP);
}

// =============================== update ==========================================

// 2D: the direction-0 interface fluxes and the stage update in one kernel (flux_upd2_tile), one
// 62 x 4 tile per block, tiles stepping by 61 nodes along x.
// ST: the 2D backward-facing step
template <bool ST>
__global__ void __launch_bounds__(256, 3)
    k_flux_upd2(Geo G, const double *__restrict__ nd, const double *__restrict__ F1, long nif1, int mode, int s,
                const double *__restrict__ dtp, const double *__restrict__ base_JU, const double *__restrict__ base_J,
                const double *__restrict__ in_JU, const double *__restrict__ in_J, double *__restrict__ out_JU,
                double *__restrict__ out_J, unsigned *flags, const double *mx, const double *mxd, double mf,
                double *mout) {
  __shared__ double sP[FluxLds<2, 0, FU_TX, FU_TY, 1>::SIZE];
  flux_upd2_tile<ST>(G, nd, F1, nif1, mode, s, dtp, base_JU, base_J, in_JU, in_J, out_JU, out_J, flags, mx, mxd, mf,
                     mout, blockIdx.x * (FU_TX - 1), blockIdx.y * FU_TY, sP);
}

// 3D: the direction-0 interface fluxes of a 62 x 4 x 1 tile and the update of the 61 x 4 nodes
// between them, as k_flux_upd2 does in 2D; the direction-1 and direction-2 fluxes are read from
// their buffers.  The node's sums are those of update_point (direction 0, then 1, then 2).
__global__ void __launch_bounds__(256, 3)
    k_flux_upd3(Geo G, const double *__restrict__ nd, const double *__restrict__ F1, long nif1,
                const double *__restrict__ F2, long nif2, int mode, int s, const double *__restrict__ dtp,
                const double *__restrict__ base_JU, const double *__restrict__ base_J,
                const double *__restrict__ in_JU, const double *__restrict__ in_J, double *__restrict__ out_JU,
                double *__restrict__ out_J, unsigned *flags, const double *mx, const double *mxd, double mf,
                double *mout) {
  constexpr int NV = 5;
  __shared__ double sP[FluxLds<3, 0, FU_TX, FU_TY, 1>::SIZE];
  static_assert(FluxLds<3, 0, FU_TX, FU_TY, 1>::SIZE >= (NV + 1) * 256, "the interface fluxes reuse the pair-flux LDS");
  const int bx0 = blockIdx.x * (FU_TX - 1), by0 = blockIdx.y * FU_TY, i2 = blockIdx.z;
  double Fl[NV + 1];
  int a0, a1, a2;
  const bool ok =
      flux_tile_eval<3, 0, FU_TX, FU_TY, 1, FU_PX, FU_TY, false>(G, nd, flags, bx0, by0, i2, sP, Fl, a0, a1, a2);
  const int tid = threadIdx.x, tx = tid % FU_PX, ty = tid / FU_PX;
  const int i0 = bx0 + tx, i1 = by0 + ty;
  const bool upd = tx < FU_TX - 1 && i0 < G.n[0] && i1 < G.n[1];
  const long t = lin(G, i0, i1, i2);
  // the update's operands are loaded before the two barriers below (as in k_flux_upd2)
  double f1l[NV + 1], f1h[NV + 1], f2l[NV + 1], f2h[NV + 1], mxv[3], mxdv[3];
  const double dtm = mout ? *dtp : 0.0;
  UpdIn<3> u;
  u.dt = mode == 1 ? *dtp : 0.0;
  if (upd) {
    const long r1 = ((long)i2 * (G.n[1] + 1) + i1) * G.n[0] + i0;
    const long r2 = ((long)i2 * G.n[1] + i1) * G.n[0] + i0, st = (long)G.n[0] * G.n[1];
#pragma unroll
    for (int c = 0; c <= NV; ++c) {
      f1l[c] = F1[(long)c * nif1 + r1];
      f1h[c] = F1[(long)c * nif1 + r1 + G.n[0]];
      f2l[c] = F2[(long)c * nif2 + r2];
      f2h[c] = F2[(long)c * nif2 + r2 + st];
    }
    update_load<3>(G, t, mode, s, base_JU, base_J, in_JU, in_J, u);
    if (mout) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        mxv[j] = mx[(long)j * G.N + t];
        mxdv[j] = mxd[(long)j * G.N + t];
      }
    }
  }
  __syncthreads();  // every thread has read its pair fluxes
  if (ok) {
#pragma unroll
    for (int c = 0; c <= NV; ++c) sP[c * 256 + tid] = Fl[c];
  }
  __syncthreads();
  if (!upd) return;
  if (mout) {
#pragma unroll
    for (int j = 0; j < 3; ++j) mout[(long)j * G.N + t] = fma(mf * dtm, mxdv[j], mxv[j]);
  }
  double L[NV + 1];
#pragma unroll
  for (int c = 0; c <= NV; ++c) L[c] = 0.0;
#pragma unroll
  for (int c = 0; c <= NV; ++c) L[c] += (sP[c * 256 + tid] - sP[c * 256 + tid + 1]) * G.idxi[0];
#pragma unroll
  for (int c = 0; c <= NV; ++c) L[c] += (f1l[c] - f1h[c]) * G.idxi[1];
#pragma unroll
  for (int c = 0; c <= NV; ++c) L[c] += (f2l[c] - f2h[c]) * G.idxi[2];
  update_store<3>(G, L, u, t, mode, s, out_JU, out_J, flags);
}

// backward-facing step: the state at the solid nodes next to the step becomes the image of its
// fluid source (normal momentum reversed, J copied); the corner block takes the image across
// the vertical face.  One thread per node of the solid block; sources are fluid nodes.
__global__ void k_step_fill_state(Geo G, double *__restrict__ JU, double *__restrict__ J) {
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x, i1 = blockIdx.y;
  if (i0 >= G.s0 || i1 >= G.s1) return;
  int src, k;
  if (step_image(G, 0, i0, i1, src)) k = 0;
  else if (step_image(G, 1, i0, i1, src)) k = 1;
  else return;
  const long t = lin(G, i0, i1, 0), ts = k == 0 ? lin(G, src, i1, 0) : lin(G, i0, src, 0);
#pragma unroll
  for (int c = 0; c < 4; ++c) JU[(long)c * G.N + t] = (c == 1 + k ? -1.0 : 1.0) * JU[(long)c * G.N + ts];
  J[t] = J[ts];
}

int launch_step_fill_state(const Geo &G, double *JU, double *J, hipStream_t st) {
  if (G.s0 <= 0) return 0;
  hipLaunchKernelGGL(k_step_fill_state, dim3((G.s0 + 63) / 64, G.s1), dim3(64), 0, st, G, JU, J);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}



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
    for (int j = 0; j < D; ++j) mout[(long)j * G.N + t] = fma(mf * (*dtp), mxd[(long)j * G.N + t], mx[(long)j * G.N + t]);
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
  out[t] = fma(f * (*dtp), xd[t], x[t]);
}

// =============================== launchers =======================================

static inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

int launch_dprod(esvdw_ctx *c, const double *xn, const double *xd, double cdt, hipStream_t st) {
  if (c->G.dim != 3) return 0;
  const int P0 = c->G.n[0] + 12, P1 = c->G.n[1] + 12, P2 = c->G.n[2] + 12;
  dim3 g((P0 + DP_TX - 1) / DP_TX, (P1 + DP_TY - 1) / DP_TY, (P2 + DP_TZ - 1) / DP_TZ), b(DP_TX, DP_TY);
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
  if constexpr (D == 2) {
    if (G.s0 > 0) {
      hipLaunchKernelGGL((k_flux<2, K, true>), grid, dim3(256), 0, st, G, c->node, c->flux[K], c->nif[K], c->flags);
      return;
    }
  }
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
                          const double *xn, const double *xd, double cdt, double cs, int mode, int s,
                          const double *dtp, const double *bJU, const double *bJ, double *oJU, double *oJ,
                          const double *mx, const double *mxd, double mf, double *mout, hipStream_t st) {
  const Geo &G = c->G;
  if (!met && D == 3)
    if (launch_dprod(c, xn, xd, cdt, st)) return -1;
  dim3 gn, bn, gu, bu;
  node_grid(G.E0, G.P[1], G.P[2], gn, bn);
  node_grid(G.n[0], G.n[1], G.n[2], gu, bu);
  if (D == 2 && !met) {
    dim3 gt((G.E0 + ND_TX - 1) / ND_TX, (G.P[1] + ND_TY - 1) / ND_TY, 1);
    hipLaunchKernelGGL(k_nodes_t2, gt, dim3(64, 4, 1), 0, st, G, JU, J, xn, xd, cdt, dtp, cs, c->node, c->flags);
  } else {
    hipLaunchKernelGGL(k_nodes<D>, gn, bn, 0, st, G, JU, J, met, xit, xn, xd, cdt, c->dprod, c->dpN, c->node,
                       c->flags);
  }
  if (D == 2) {
    // direction 1 first; the direction-0 flux kernel then also forms the update
    launch_flux_d<D>(c, 1, st);
    dim3 gf((G.n[0] + FU_TX - 2) / (FU_TX - 1), (G.n[1] + FU_TY - 1) / FU_TY, 1);
    if (G.s0 > 0) {
      hipLaunchKernelGGL(k_flux_upd2<true>, gf, dim3(256), 0, st, G, c->node, c->flux[1], c->nif[1], mode, s, dtp,
                         bJU, bJ, JU, J, oJU, oJ, c->flags, mx, mxd, mf, mout);
      if (mode == 1 && launch_step_fill_state(G, oJU, oJ, st)) return -1;
    } else {
      hipLaunchKernelGGL(k_flux_upd2<false>, gf, dim3(256), 0, st, G, c->node, c->flux[1], c->nif[1], mode, s, dtp,
                         bJU, bJ, JU, J, oJU, oJ, c->flags, mx, mxd, mf, mout);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  if (D == 3) {
    // directions 1 and 2 first; the direction-0 flux kernel then also forms the update
    launch_flux_d<D>(c, 1, st);
    launch_flux_d<D>(c, 2, st);
    dim3 gf((G.n[0] + FU_TX - 2) / (FU_TX - 1), (G.n[1] + FU_TY - 1) / FU_TY, G.n[2]);
    hipLaunchKernelGGL(k_flux_upd3, gf, dim3(256), 0, st, G, c->node, c->flux[1], c->nif[1], c->flux[2], c->nif[2],
                       mode, s, dtp, bJU, bJ, JU, J, oJU, oJ, c->flags, mx, mxd, mf, mout);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  launch_flux_d<D>(c, 0, st);
  if (D > 1) launch_flux_d<D>(c, 1, st);
  hipLaunchKernelGGL(k_update<D>, gu, bu, 0, st, G, c->flux[0], c->flux[1], c->flux[2],
                     c->nif[0], c->nif[1], c->nif[2], mode, s, dtp, bJU, bJ, JU, J, oJU, oJ, c->flags, mx, mxd, mf,
                     mout);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_rhs_mesh(esvdw_ctx *c, const double *JU, const double *J, const double *met, const double *xit,
                    const double *xn, const double *xd, double cdt, double cs, int mode, int s, const double *dtp,
                    const double *bJU, const double *bJ, double *oJU, double *oJ, const double *mx, const double *mxd,
                    double mf, double *mout, hipStream_t st) {
  switch (c->G.dim) {
    case 1:
      return rhs_pipeline_d<1>(c, JU, J, met, xit, xn, xd, cdt, cs, mode, s, dtp, bJU, bJ, oJU, oJ, mx, mxd, mf, mout, st);
    case 2:
      return rhs_pipeline_d<2>(c, JU, J, met, xit, xn, xd, cdt, cs, mode, s, dtp, bJU, bJ, oJU, oJ, mx, mxd, mf, mout, st);
    default:
      return rhs_pipeline_d<3>(c, JU, J, met, xit, xn, xd, cdt, cs, mode, s, dtp, bJU, bJ, oJU, oJ, mx, mxd, mf, mout, st);
  }
}

int launch_rhs(esvdw_ctx *c, const double *JU, const double *J, const double *met, const double *xit,
               const double *xn, const double *xd, double cdt, int mode, int s, const double *dtp,
               const double *bJU, const double *bJ, double *oJU, double *oJ, hipStream_t st) {
  return launch_rhs_mesh(c, JU, J, met, xit, xn, xd, cdt, 0.0, mode, s, dtp, bJU, bJ, oJU, oJ, nullptr, nullptr, 0.0,
                         nullptr, st);
}

int launch_uniform_mesh(esvdw_ctx *c, double *x, hipStream_t st) {
  dim3 g, b;
  node_grid(c->G.n[0], c->G.n[1], c->G.n[2], g, b);
  hipLaunchKernelGGL(k_uniform_mesh, g, b, 0, st, c->G, x);
  if (launch_step_fill_mesh(c->G, x, st)) return -1;
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
