// mesh.hip -- adaptive moving mesh (Section 4): monitor, low-pass filter, Jacobi sweeps
// of the discretised Winslow equations, movement limiter, CFL time step (eq. cfl) and the
// mesh velocity.  Global reductions: per-block partials (wavefront shuffles, then LDS), reduced
// by a one-block kernel into a device scalar of the context.
#include <mutex>

#include "common.h"
#include "kernels.h"
#include "meshdev.h"
#include "scheme.h"

static inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

__global__ void k_set_scalars(double *s) {
  if (threadIdx.x == 0) {
    s[SC_CFL] = 0.0;
    s[SC_MON] = s[SC_MON + 1] = s[SC_MON + 2] = 0.0;
    s[SC_GAMMA] = 1.0;
    s[SC_RESID] = 0.0;
  }
}

__global__ void k_set1(double *p, double v) {
  if (threadIdx.x == 0) *p = v;
}

__global__ void k_set_int(int *p, int v) {
  if (threadIdx.x == 0) *p = v;
}

__global__ void k_copy(const double *__restrict__ a, double *__restrict__ b, long n) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t < n) b[t] = a[t];
}

__global__ void k_add(const double *__restrict__ a, const double *__restrict__ b, double *__restrict__ c, long n) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t < n) c[t] = a[t] + b[t];
}

// reduce nb per-block partials into *dst (mode 0: max, 1: min); one block of 1024 threads
__global__ void k_final(const double *__restrict__ part, long nb, double *dst, int mode) {
  double v = mode == 0 ? 0.0 : 1.0;
  for (long i = threadIdx.x; i < nb; i += blockDim.x) v = mode == 0 ? fmax(v, part[i]) : fmin(v, part[i]);
  v = mode == 0 ? block_max(v) : block_min(v);
  if (threadIdx.x == 0) *dst = v;
}

// ---- the backward-facing step: values at the solid nodes ---------------------------------
// A solid node within 3 of one face of the step holds the image of its fluid source across
// that face; within 3 of both (the corner block) the image across the vertical face
// (i0 = s0).  Scalars (the monitor) copy the source.  One thread per node of the solid block.
__global__ void k_step_fill_scalar(Geo G, double *__restrict__ w) {
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x, i1 = blockIdx.y;
  if (i0 >= G.s0 || i1 >= G.s1) return;
  int src;
  if (step_image(G, 0, i0, i1, src)) w[lin(G, i0, i1, 0)] = w[lin(G, src, i1, 0)];
  else if (step_image(G, 1, i0, i1, src)) w[lin(G, i0, i1, 0)] = w[lin(G, i0, src, 0)];
}

// The mesh.  The 6 x 6 block of nodes within 3 of the corner along both directions is a lattice
// mirror-symmetric about both faces (x_1 = face_1 +- a_m on the columns s0 + m and s0 - 1 - m,
// x_2 = face_2 +- b_m on the rows s1 + m and s1 - 1 - m), so that a solid corner node, the image
// of one fluid node across each face, is the same point in both roles and the discrete metric
// identities hold at the corner; a_m is the mean distance to the vertical face of the 9 fluid
// nodes of the block on the two columns of index m, b_m likewise for the rows.  A solid node
// within 3 of one face only holds the image of its fluid source (normal coordinate 2 face - x,
// the other unchanged); the other solid nodes their uniform positions.
// Grid: rows 0 .. s1 - 1 of the solid block, one thread per node outside the corner block
// (their sources are fluid nodes outside the corner block); the extra row s1, workgroup 0: the
// corner block, all its reads before a barrier and its writes after it.
__global__ void k_step_fill_mesh(Geo G, double *__restrict__ x) {
  const int s0 = G.s0, s1 = G.s1;
  const double face[2] = {G.lo[0] + s0 * G.dxi[0], G.lo[1] + s1 * G.dxi[1]};
  if (blockIdx.y == (unsigned)s1) {
    if (blockIdx.x != 0) return;
    __shared__ double off[6];  // a_0..a_2, b_0..b_2
    const int t = threadIdx.x;
    if (t < 6) {
      const int m = t % 3, j = t / 3;
      double sum = 0.0;
      if (j == 0) {
        for (int k = -3; k < 3; ++k) sum += x[lin(G, s0 + m, s1 + k, 0)] - face[0];
        for (int k = 0; k < 3; ++k) sum += face[0] - x[lin(G, s0 - 1 - m, s1 + k, 0)];
      } else {
        for (int k = -3; k < 3; ++k) sum += x[G.N + lin(G, s0 + k, s1 + m, 0)] - face[1];
        for (int k = 0; k < 3; ++k) sum += face[1] - x[G.N + lin(G, s0 + k, s1 - 1 - m, 0)];
      }
      off[t] = sum / 9.0;
    }
    __syncthreads();
    if (t < 36) {
      const int i0 = s0 - 3 + t % 6, i1 = s1 - 3 + t / 6;
      const long q = lin(G, i0, i1, 0);
      x[q] = i0 >= s0 ? face[0] + off[i0 - s0] : face[0] - off[s0 - 1 - i0];
      x[G.N + q] = i1 >= s1 ? face[1] + off[3 + i1 - s1] : face[1] - off[3 + s1 - 1 - i1];
    }
    return;
  }
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x, i1 = blockIdx.y;
  if (i0 >= s0 || i1 >= s1 || (i0 >= s0 - 3 && i1 >= s1 - 3)) return;
  const long t = lin(G, i0, i1, 0);
  int s;
  const bool row = step_image(G, 0, i0, i1, s), col = step_image(G, 1, i0, i1, s);
  if (row != col) {
    const int k = row ? 0 : 1;
    int src;
    step_image(G, k, i0, i1, src);
    const long ts = k == 0 ? lin(G, src, i1, 0) : lin(G, i0, src, 0);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      x[(long)j * G.N + t] = j == k ? 2.0 * face[k] - x[(long)j * G.N + ts] : x[(long)j * G.N + ts];
  } else {
    x[t] = G.lo[0] + (i0 + 0.5) * G.dxi[0];
    x[G.N + t] = G.lo[1] + (i1 + 0.5) * G.dxi[1];
  }
}

int launch_step_fill_scalar(const Geo &G, double *w, hipStream_t st) {
  if (G.s0 <= 0) return 0;
  hipLaunchKernelGGL(k_step_fill_scalar, dim3(nblk(G.s0, 64), G.s1), dim3(64), 0, st, G, w);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_step_fill_mesh(const Geo &G, double *x, hipStream_t st) {
  if (G.s0 <= 0) return 0;
  hipLaunchKernelGGL(k_step_fill_mesh, dim3(nblk(G.s0, 64), G.s1 + 1), dim3(64), 0, st, G, x);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---- monitor -------------------------------------------------------------------
template <int D>
__global__ void k_rho_G(Geo G, const double *__restrict__ JU, const double *__restrict__ J, double *__restrict__ rg) {
  NODE_COORDS(G.n[0], G.n[1]);
  if (!inside) return;
  rhoG_point<D>(G, JU, J, rg, lin(G, i0, i1, i2));
}

// term t of the monitor at each node; maxima into scal[SC_MON + t]
template <int D>
__global__ void k_mon_terms(Geo G, int kind, int kappa, int var0, int var1, const double *__restrict__ rg,
                            double *__restrict__ term, double *part, long npart) {
  NODE_COORDS(G.n[0], G.n[1]);
  double val[3] = {0.0, 0.0, 0.0};
  int nterm = kind == ESVDW_MON_VDW ? kappa + 1 : 2;
  if (inside) {
    mon_terms_point<D>(G, kind, kappa, var0, var1, rg, term, i0, i1, i2, val);
    if (step_solid(G, i0, i1)) val[0] = val[1] = val[2] = 0.0;  // maxima over the fluid nodes
  }
  for (int q = 0; q < 3; ++q) {
    if (q >= nterm) break;
    double mq = block_max(val[q]);
    if (flat_tid() == 0) part[q * npart + flat_bid()] = mq;
  }
}

__global__ void k_mon_omega(Geo G, int nterm, double a0, double a1, double a2, const double *__restrict__ term,
                            const double *__restrict__ scal, double *__restrict__ omega) {
  NODE_COORDS(G.n[0], G.n[1]);
  if (!inside) return;
  const long t = lin(G, i0, i1, i2);
  const double al[3] = {a0, a1, a2};
  omega[t] = mon_omega_point(G, nterm, al, term, scal + SC_MON, t);
}

// omega <- sum_{j in {-1,0,1}^d} 2^-(|j|_1 + d) omega_{i+j}; replicate / wrap at the boundary
template <int D>
__global__ void k_filter(Geo G, const double *__restrict__ in, double *__restrict__ out) {
  NODE_COORDS(G.n[0], G.n[1]);
  if (!inside) return;
  out[lin(G, i0, i1, i2)] = filter_point<D>(G, in, i0, i1, i2);
}

// ---- Jacobi sweep -----------------------------------------------------------------
template <int D>
__global__ void k_jacobi(Geo G, const double *__restrict__ omega, const double *__restrict__ xin,
                         double *__restrict__ xout, double *part) {
  NODE_COORDS(G.n[0], G.n[1]);
  const double r = inside ? jacobi_point<D>(G, omega, xin, xout, i0, i1, i2) : 0.0;
  if (part) {
    double mr = block_max(r);
    if (flat_tid() == 0) part[flat_bid()] = mr;
  }
}

// ---- several Jacobi sweeps per launch (2D, outflow walls) ---------------------------------
// A 64 x 4 block owns a JT_X x JT_Y tile and loads it with a halo of nsw (<= JT_H) nodes into
// LDS (one extended row per 64-lane row of threads); sweep s updates the extended region shrunk
// by s, so the owned tile is exact after nsw sweeps.  Nodes outside the domain are never
// updated: the first ghost layer (the only one a 5-point update reads) is refreshed after every
// sweep as the mirror image of the wall node (normal coordinate 2 wall - x, tangential x),
// exactly as mesh_at forms it; omega ghosts are static.  The per-node arithmetic is
// jacobi_point's, term for term (both with contraction off and their fused multiply-adds
// written out), so the mesh equals nsw launches of k_jacobi bit for bit.
// Periodic directions are not handled (the launcher falls back to k_jacobi).
constexpr int JT_X = 54, JT_Y = 10, JT_H = 5;
constexpr int JT_EX = JT_X + 2 * JT_H, JT_EY = JT_Y + 2 * JT_H, JT_NE = JT_EX * JT_EY;
static_assert(JT_EX <= 64, "one extended row per 64-lane row of threads");

__global__ void __launch_bounds__(256) k_jacobi_multi2(Geo G, const double *__restrict__ omega,
                                                       const double *__restrict__ xin, double *__restrict__ xout,
                                                       int nsw, double *part) {
#pragma clang fp contract(off)
  __shared__ double sw[JT_NE], sx[2][2][JT_NE];
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 64 + tx;
  const int exn = JT_X + 2 * nsw, eyn = JT_Y + 2 * nsw;
  const int gx0 = blockIdx.x * JT_X - nsw, gy0 = blockIdx.y * JT_Y - nsw;
  const int n0 = G.n[0], n1 = G.n[1];
  const int gx = gx0 + tx;
  const bool inner = gx0 >= 0 && gx0 + exn <= n0 && gy0 >= 0 && gy0 + eyn <= n1;  // no ghost in the region
  if (tx < exn) {
    if (inner) {
      for (int ey = ty; ey < eyn; ey += 4) {
        const int e = ey * exn + tx;
        const long t = lin(G, gx, gy0 + ey, 0);
        sw[e] = omega[t];
        sx[0][0][e] = xin[t];
        sx[0][1][e] = xin[G.N + t];
      }
    } else {
      for (int ey = ty; ey < eyn; ey += 4) {
        const int gy = gy0 + ey, e = ey * exn + tx;
        double w = 0.0, a0 = 0.0, a1 = 0.0;
        if (gx >= -1 && gx <= n0 && gy >= -1 && gy <= n1) {
          w = omega[state_index(G, gx, gy, 0)];
          a0 = mesh_at(G, xin, 0, gx, gy, 0, 0);
          a1 = mesh_at(G, xin, 1, gx, gy, 0, 0);
        }
        sw[e] = w;
        sx[0][0][e] = a0;
        sx[0][1][e] = a1;
      }
    }
  }
  __syncthreads();
  const double h2x = G.idxi[0] * G.idxi[0], h2y = G.idxi[1] * G.idxi[1];
  const bool inx = gx >= 0 && gx < n0;
  // columns / rows of the first ghost layer inside the extended region (-1 if absent)
  const int cl = gx0 < 0 ? -1 - gx0 : -1, cr = n0 - gx0 < exn ? n0 - gx0 : -1;
  const int rb = gy0 < 0 ? -1 - gy0 : -1, rt = n1 - gy0 < eyn ? n1 - gy0 : -1;
  const bool wall = cl >= 0 || cr >= 0 || rb >= 0 || rt >= 0;
  double r = 0.0;
  int cur = 0;
  // omega does not change between sweeps: the face weights and 1/den of the thread's rows
  // (ey = ty + 4 j) are formed once, with jacobi_point's arithmetic
  constexpr int NR = (JT_EY + 3) / 4;
  double wx[NR][2], wy[NR][2], iden[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    const int ey = ty + 4 * j;
    wx[j][0] = wx[j][1] = wy[j][0] = wy[j][1] = iden[j] = 0.0;
    if (tx >= 1 && tx < exn - 1 && ey >= 1 && ey < eyn - 1) {
      const int e = ey * exn + tx;
      const double w0 = sw[e];
      double den = 0.0;
      wx[j][0] = 0.5 * (w0 + sw[e + 1]) * h2x;
      wx[j][1] = 0.5 * (w0 + sw[e - 1]) * h2x;
      den += wx[j][0] + wx[j][1];
      wy[j][0] = 0.5 * (w0 + sw[e + exn]) * h2y;
      wy[j][1] = 0.5 * (w0 + sw[e - exn]) * h2y;
      den += wy[j][0] + wy[j][1];
      iden[j] = 1.0 / den;
    }
  }
  for (int s = 1; s <= nsw; ++s) {
    const double *A0 = sx[cur][0], *A1 = sx[cur][1];
    double *B0 = sx[cur ^ 1][0], *B1 = sx[cur ^ 1][1];
    if (tx >= s && tx < exn - s && inx)
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        const int ey = ty + 4 * j;
        if (ey < s || ey >= eyn - s) continue;
        const int gy = gy0 + ey;
        if (gy < 0 || gy >= n1) continue;
        const int e = ey * exn + tx;
        double num0 = 0.0, num1 = 0.0;
        {  // direction 0, as jacobi_point with k = 0
          const double wp = wx[j][0], wm = wx[j][1];
          num0 += fma(wp, A0[e + 1], wm * A0[e - 1]);
          num1 += fma(wp, A1[e + 1], wm * A1[e - 1]);
        }
        {  // direction 1
          const double wp = wy[j][0], wm = wy[j][1];
          num0 += fma(wp, A0[e + exn], wm * A0[e - exn]);
          num1 += fma(wp, A1[e + exn], wm * A1[e - exn]);
        }
        const double v0 = num0 * iden[j], v1 = num1 * iden[j];
        if (s == nsw) r = fmax(r, fmax(fabs(v0 - A0[e]), fabs(v1 - A1[e])));
        B0[e] = v0;
        B1[e] = v1;
      }
    __syncthreads();
    if (s < nsw && wall) {
      // ghost columns: for rows of the region inside the domain
      for (int ey = s + tid; ey < eyn - s; ey += 256) {
        const int gy = gy0 + ey;
        if (gy < 0 || gy >= n1) continue;
        if (cl >= s && cl < exn - s) {
          const int e = ey * exn + cl;
          B0[e] = -1.0 * B0[e + 1] + 2.0 * G.lo[0];
          B1[e] = B1[e + 1];
        }
        if (cr >= s && cr < exn - s) {
          const int e = ey * exn + cr;
          B0[e] = -1.0 * B0[e - 1] + 2.0 * G.hi[0];
          B1[e] = B1[e - 1];
        }
      }
      // ghost rows: for columns of the region inside the domain
      for (int ex = s + tid; ex < exn - s; ex += 256) {
        const int gxx = gx0 + ex;
        if (gxx < 0 || gxx >= n0) continue;
        if (rb >= s && rb < eyn - s) {
          const int e = rb * exn + ex;
          B0[e] = B0[e + exn];
          B1[e] = -1.0 * B1[e + exn] + 2.0 * G.lo[1];
        }
        if (rt >= s && rt < eyn - s) {
          const int e = rt * exn + ex;
          B0[e] = B0[e - exn];
          B1[e] = -1.0 * B1[e - exn] + 2.0 * G.hi[1];
        }
      }
      __syncthreads();
    }
    cur ^= 1;
  }
  if (tx < JT_X) {
    const int ex = nsw + tx, gxo = gx0 + ex;
    if (gxo < n0)
      for (int ey = nsw + ty; ey < nsw + JT_Y; ey += 4) {
        const int gy = gy0 + ey;
        if (gy >= n1) continue;
        const long t = lin(G, gxo, gy, 0);
        const int e = ey * exn + ex;
        xout[t] = sx[cur][0][e];
        xout[G.N + t] = sx[cur][1][e];
      }
  }
  if (part) {
    double mr = block_max(r);
    if (flat_tid() == 0) part[flat_bid()] = mr;
  }
}

// ---- several low-pass filter passes per launch (2D, outflow walls) ---------------------------
// The tile scheme of k_jacobi_multi2 for the 9-point filter: pass s updates the extended region
// shrunk by s; the first ghost layer (corners included) is refreshed after every pass with the
// replicated nearest node, as state_index forms it.  filter_point's arithmetic, term for term.
__global__ void __launch_bounds__(256) k_filter_multi2(Geo G, const double *__restrict__ in, double *__restrict__ out,
                                                       int npass) {
  __shared__ double sa[2][JT_NE];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int exn = JT_X + 2 * npass, eyn = JT_Y + 2 * npass;
  const int gx0 = blockIdx.x * JT_X - npass, gy0 = blockIdx.y * JT_Y - npass;
  const int n0 = G.n[0], n1 = G.n[1];
  const int gx = gx0 + tx;
  if (tx < exn)
    for (int ey = ty; ey < eyn; ey += 4) {
      const int gy = gy0 + ey;
      sa[0][ey * exn + tx] = gx >= -1 && gx <= n0 && gy >= -1 && gy <= n1 ? in[state_index(G, gx, gy, 0)] : 0.0;
    }
  __syncthreads();
  const bool inx = gx >= 0 && gx < n0;
  const bool wall = gx0 < 0 || gy0 < 0 || gx0 + exn > n0 || gy0 + eyn > n1;
  int cur = 0;
  for (int s = 1; s <= npass; ++s) {
    const double *A = sa[cur];
    double *B = sa[cur ^ 1];
    if (tx >= s && tx < exn - s && inx)
      for (int ey = s + ty; ey < eyn - s; ey += 4) {
        const int gy = gy0 + ey;
        if (gy < 0 || gy >= n1) continue;
        const int e = ey * exn + tx;
        double v = 0.0;
#pragma unroll
        for (int j1 = -1; j1 <= 1; ++j1)
#pragma unroll
          for (int j0 = -1; j0 <= 1; ++j0) {
            int l1 = (j0 != 0) + (j1 != 0) + 2;
            v += ldexp(1.0, -l1) * A[e + j1 * exn + j0];
          }
        B[e] = v;
      }
    __syncthreads();
    if (s < npass && wall) {
      // first ghost layer inside the region: the nearest node's value
      if (tx >= s && tx < exn - s)
        for (int ey = s + ty; ey < eyn - s; ey += 4) {
          const int gy = gy0 + ey;
          const bool iny = gy >= 0 && gy < n1;
          if (inx && iny) continue;
          if (gx < -1 || gx > n0 || gy < -1 || gy > n1) continue;
          const int sx = gx < 0 ? 0 : (gx >= n0 ? n0 - 1 : gx), sy = gy < 0 ? 0 : (gy >= n1 ? n1 - 1 : gy);
          B[ey * exn + tx] = B[(sy - gy0) * exn + (sx - gx0)];
        }
      __syncthreads();
    }
    cur ^= 1;
  }
  if (tx < JT_X) {
    const int ex = npass + tx, gxo = gx0 + ex;
    if (gxo < n0)
      for (int ey = npass + ty; ey < npass + JT_Y; ey += 4) {
        const int gy = gy0 + ey;
        if (gy < n1) out[lin(G, gxo, gy, 0)] = sa[cur][ey * exn + ex];
      }
  }
}

// ---- red-black SOR half-sweep ---------------------------------------------------------
// Nodes of one colour (i0 + i1 + i2 = colour mod 2), in place.  Thread t of a row takes
// i0 = 2 t + ((i1 + i2 + colour) & 1).  Each node solves its own equation with the other colour
// fixed: a neighbour across an outflow wall is the node's own mirror image (normal coordinate
// 2 wall - x, tangential x), whose term moves to the left-hand side; every other neighbour
// (including a periodic wrap, which needs even node counts so that it joins opposite colours)
// is read as in the Jacobi sweep.  x <- x + relax (v - x); partial maxima of |v - x|.
template <int D>
__global__ void k_sor(Geo G, const double *__restrict__ omega, double *__restrict__ x, int colour, double relax,
                      double *part) {
  // no contraction: k_sor_multi2 repeats this arithmetic and must give the same bits
#pragma clang fp contract(off)
  const int t = blockIdx.x * blockDim.x + threadIdx.x, i1 = blockIdx.y * blockDim.y + threadIdx.y,
            i2 = blockIdx.z;
  const int i0 = 2 * t + ((i1 + i2 + colour) & 1);
  double r = 0.0;
  if (i0 < G.n[0] && i1 < G.n[1]) {
    const long q = lin(G, i0, i1, i2);
    const double w0 = omega[q];
    const int ii[3] = {i0, i1, i2};
    double den[D], num[D];
#pragma unroll
    for (int j = 0; j < D; ++j) den[j] = num[j] = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const int e0 = k == 0, e1 = k == 1, e2 = k == 2;
      const double h2 = G.idxi[k] * G.idxi[k];
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int sg = side ? 1 : -1;
        const int n0 = i0 + sg * e0, n1 = i1 + sg * e1, n2 = i2 + sg * e2;
        const double wf = 0.5 * (w0 + omega[state_index(G, n0, n1, n2)]) * h2;
        const int ik = ii[k] + sg;
        const bool self = G.bc[k] != ESVDW_BC_PERIODIC && (ik < 0 || ik >= G.n[k]);
#pragma unroll
        for (int j = 0; j < D; ++j) {
          if (!self) {
            den[j] += wf;
            num[j] += wf * mesh_at(G, x, j, n0, n1, n2, 0);
          } else if (j == k) {
            den[j] += 2.0 * wf;
            num[j] += wf * 2.0 * (side ? G.hi[k] : G.lo[k]);
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double old = x[(long)j * G.N + q];
      const double v = num[j] / den[j];
      r = fmax(r, fabs(v - old));
      x[(long)j * G.N + q] = old + relax * (v - old);
    }
  }
  if (part) {
    double mr = block_max(r);
    if (flat_tid() == 0) part[flat_bid()] = mr;
  }
}

// ---- several red-black SOR sweeps per launch (2D, outflow in both directions) ----------------
// A block of 32 x 8 threads owns a JS_X x JS_Y tile and loads it with omega and a halo of
// h = 2 nsw nodes into LDS (nsw <= JS_S sweeps).  Half-sweep q (colour q mod 2, colour 0 first as
// in k_sor) updates its colour in place over the extended region shrunk by q, reading the other
// colour, so the owned tile is exact after the 2 nsw half-sweeps; a thread takes the two columns
// 2 tx and 2 tx + 1 of its rows and updates the one of the current colour, so every lane works in
// every half-sweep.  A node next to a wall takes the self terms of k_sor instead of a ghost, so no
// ghost values are needed; the per-node arithmetic is k_sor's, term for term and with contraction
// off in both, so nsw sweeps here equal nsw sweeps of k_sor bit for bit.  part != nullptr: the
// partial maxima of |v - x| over the last sweep's two half-sweeps.  The global arrays alternate
// (xin is never written): other blocks read xin's values around their tiles.
constexpr int JS_X = 56, JS_Y = 12, JS_S = 2;
constexpr int JS_EX = JS_X + 4 * JS_S, JS_EY = JS_Y + 4 * JS_S, JS_NE = JS_EX * JS_EY;
static_assert(JS_EX <= 64, "two extended columns per thread of a 32-thread row");

__global__ void __launch_bounds__(256) k_sor_multi2(Geo G, const double *__restrict__ omega,
                                                    const double *__restrict__ xin, double *__restrict__ xout,
                                                    int nsw, double relax, double *part) {
#pragma clang fp contract(off)
  __shared__ double sw[JS_NE], sx[2][JS_NE];
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 32 + tx;
  const int hw = 2 * nsw, exn = JS_X + 2 * hw, eyn = JS_Y + 2 * hw, nex = exn * eyn;
  const int gx0 = blockIdx.x * JS_X - hw, gy0 = blockIdx.y * JS_Y - hw;
  const int n0 = G.n[0], n1 = G.n[1];
  for (int e = tid; e < nex; e += 256) {
    const int gx = gx0 + e % exn, gy = gy0 + e / exn;
    const bool in = gx >= 0 && gx < n0 && gy >= 0 && gy < n1;
    const long t = in ? lin(G, gx, gy, 0) : 0;
    sw[e] = in ? omega[t] : 0.0;
    sx[0][e] = in ? xin[t] : 0.0;
    sx[1][e] = in ? xin[G.N + t] : 0.0;
  }
  __syncthreads();
  const double h2x = G.idxi[0] * G.idxi[0], h2y = G.idxi[1] * G.idxi[1];
  const double wall[2][2] = {{G.lo[0], G.hi[0]}, {G.lo[1], G.hi[1]}};
  double r = 0.0;
  for (int q = 1; q <= hw; ++q) {
    const int colour = (q - 1) & 1;
    for (int ey = ty; ey < eyn; ey += 8) {
      const int gy = gy0 + ey;
      const int ex = 2 * tx + ((gx0 + 2 * tx + gy + colour) & 1);  // the column of this colour
      const int gx = gx0 + ex;
      if (ey < q || ey >= eyn - q || ex < q || ex >= exn - q || gx < 0 || gx >= n0 || gy < 0 || gy >= n1) continue;
      const int e = ey * exn + ex;
      const double w0 = sw[e];
      double den[2] = {0.0, 0.0}, num[2] = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const double h2 = k == 0 ? h2x : h2y;
        const int step = k == 0 ? 1 : exn, ik = k == 0 ? gx : gy, nk = k == 0 ? n0 : n1;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          const int sg = side ? 1 : -1, en = e + sg * step;
          const bool self = ik + sg < 0 || ik + sg >= nk;
          const double wf = 0.5 * (w0 + (self ? w0 : sw[en])) * h2;
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            if (!self) {
              den[j] += wf;
              num[j] += wf * sx[j][en];
            } else if (j == k) {
              den[j] += 2.0 * wf;
              num[j] += wf * 2.0 * wall[k][side];
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const double old = sx[j][e];
        const double v = num[j] / den[j];
        if (q > hw - 2) r = fmax(r, fabs(v - old));
        sx[j][e] = old + relax * (v - old);
      }
    }
    __syncthreads();
  }
  for (int o = tid; o < JS_X * JS_Y; o += 256) {
    const int ex = hw + o % JS_X, ey = hw + o / JS_X, gx = gx0 + ex, gy = gy0 + ey;
    if (gx >= n0 || gy >= n1) continue;
    const long t = lin(G, gx, gy, 0);
    const int e = ey * exn + ex;
    xout[t] = sx[0][e];
    xout[G.N + t] = sx[1][e];
  }
  if (part) {
    double mr = block_max(r);
    if (flat_tid() == 0) part[flat_bid()] = mr;
  }
}

// ---- limiter ----------------------------------------------------------------------
template <int D>
__global__ void k_limiter(Geo G, const double *__restrict__ xn, const double *__restrict__ xmu, double *part) {
  NODE_COORDS(G.n[0], G.n[1]);
  const double g = (inside && !step_solid(G, i0, i1)) ? limiter_point<D>(G, xn, xmu, i0, i1, i2) : 1.0;
  double mg = block_min(g);
  if (flat_tid() == 0) part[flat_bid()] = mg;
}

// ---- CFL ----------------------------------------------------------------------------
// CFL spectral-radius sum per node (cfl_rate); per-block maxima into part
template <int D>
__global__ void k_cfl(Geo G, const double *__restrict__ JU, const double *__restrict__ J,
                      const double *__restrict__ x, const double *__restrict__ met, double *part) {
  NODE_COORDS(G.n[0], G.n[1]);
  double s = (inside && !step_solid(G, i0, i1)) ? cfl_rate<D>(G, JU, J, x, met, i0, i1, i2) : 0.0;
  double ms = block_max(s);
  if (flat_tid() == 0) part[flat_bid()] = ms;
}

// 2D CFL maxima with the mesh staged in LDS (mesh_tile_*): a block of 64 x 4 threads covers
// 64 x 16 nodes, four rows per thread; the same per-node values as k_cfl<2>, so the maximum
// (exact in any order) is the same
#define CF_TX 64
#define CF_TY 16
__global__ void __launch_bounds__(256) k_cfl_t2(Geo G, const double *__restrict__ JU, const double *__restrict__ J,
                                                const double *__restrict__ x, double *part) {
  __shared__ MeshTile2<CF_TX, CF_TY> T;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int b0 = blockIdx.x * CF_TX, b1 = blockIdx.y * CF_TY;
  mesh_tile_fill<CF_TX, CF_TY>(G, x, nullptr, 0.0, b0, b1, T, ty * 64 + tx, 256);
  __syncthreads();
  double mx = 0.0;
#pragma unroll 1
  for (int r = 0; r < CF_TY / 4; ++r) {
    const int u = tx, v = ty + 4 * r;
    const int i0 = b0 + u, i1 = b1 + v;
    if (i0 >= G.n[0] || i1 >= G.n[1] || step_solid(G, i0, i1)) continue;  // fluid nodes only
    double m[2][2];
    mesh_tile_metrics<CF_TX, CF_TY>(G, T, u, v, m);
    mx = fmax(mx, cfl_rate_m<2>(G, JU, J, (long)i1 * G.n[0] + i0, m));
  }
  const double bm = block_max(mx);
  if (flat_tid() == 0) part[flat_bid()] = bm;
}

// 2D without a step: the monitor terms of U^n (k_rho_G + k_mon_terms) and the CFL maxima on x^n
// (k_cfl_t2) in one pass over the state.  The mesh of the tile with a 3-node halo is staged in
// LDS first; then each node of the tile and its 1-node halo gets its primitive values once, which
// give rho and G (staged in LDS for the monitor's differences) and, at the tile's own nodes, the
// CFL sum.  A block of 64 x 4 threads covers 64 x 8 nodes.  The per-node values are those of
// rhoG_point, mon_terms_point and cfl_rate_m, so the terms, their maxima and the CFL maximum
// equal the separate kernels'.
#define MC_TX 64
#define MC_TY 8
__global__ void __launch_bounds__(256) k_mon_cfl_t2(Geo G, int kind, int kappa, int var0, int var1,
                                                    const double *__restrict__ JU, const double *__restrict__ J,
                                                    const double *__restrict__ x, double *__restrict__ term,
                                                    double *part, long npart, double *pc) {
  constexpr int RW = MC_TX + 2, RS = RW * (MC_TY + 2);
  __shared__ MeshTile2<MC_TX, MC_TY> T;
  __shared__ double sRG[2][RS];
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 64 + tx;
  const int b0 = blockIdx.x * MC_TX, b1 = blockIdx.y * MC_TY;
  const long bid = (long)blockIdx.y * gridDim.x + blockIdx.x;
  mesh_tile_fill<MC_TX, MC_TY>(G, x, nullptr, 0.0, b0, b1, T, tid, 256);
  __syncthreads();
  double mc = 0.0;
  for (int idx = tid; idx < RS; idx += 256) {
    const int a = idx % RW, b = idx / RW, i0 = b0 - 1 + a, i1 = b1 - 1 + b;
    double rho = 0.0, g = 0.0;
    // a neighbour outside the grid is the node state_index maps it to, as in mon_terms_point
    if (i0 >= -1 && i0 <= G.n[0] && i1 >= -1 && i1 <= G.n[1]) {
      double iJ, v[2], Tn;
      node_prim<2>(G, JU, J, state_index(G, i0, i1, 0), iJ, rho, v, Tn);
      g = eos_G(G, rho, Tn);
      if (a >= 1 && a <= MC_TX && b >= 1 && b <= MC_TY && i0 < G.n[0] && i1 < G.n[1]) {  // a node of the tile
        double m[2][2];
        mesh_tile_metrics<MC_TX, MC_TY>(G, T, a - 1, b - 1, m);
        mc = fmax(mc, cfl_rate_prim<2>(G, iJ, rho, v, Tn, m));
      }
    }
    sRG[0][idx] = rho;
    sRG[1][idx] = g;
  }
  __syncthreads();
  const int nterm = kind == ESVDW_MON_VDW ? kappa + 1 : 2;
  double mx[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < MC_TY / 4; ++r) {
    const int u = tx, v = ty + 4 * r;
    const int i0 = b0 + u, i1 = b1 + v;
    if (i0 >= G.n[0] || i1 >= G.n[1]) continue;
    const long t = (long)i1 * G.n[0] + i0;
    const int e = (v + 1) * RW + u + 1;
    for (int q = 0; q < nterm; ++q) {
      int field;
      bool second;
      mon_term_kind(kind, kappa, var0, var1, q, field, second);
      const double *f = sRG[field];
      double s2 = 0.0;
      s2 += mon_term_part(f[e + 1], f[e], f[e - 1], G.idxi[0], second);
      s2 += mon_term_part(f[e + RW], f[e], f[e - RW], G.idxi[1], second);
      const double val = kind == ESVDW_MON_VDW ? s2 : sqrt(s2);
      term[(long)q * G.N + t] = val;
      mx[q] = fmax(mx[q], val);
    }
  }
  for (int q = 0; q < 3; ++q) {
    if (q >= nterm) break;
    const double bm = block_max(mx[q]);
    if (tid == 0) part[q * npart + bid] = bm;
  }
  const double bc = block_max(mc);
  if (tid == 0) pc[bid] = bc;
}

static inline void cfl_launch(esvdw_ctx *c, const double *JU, const double *J, const double *x, double *part,
                              long &nb, hipStream_t st) {
  const Geo &G = c->G;
  if (G.dim == 2) {
    dim3 g((G.n[0] + CF_TX - 1) / CF_TX, (G.n[1] + CF_TY - 1) / CF_TY, 1);
    nb = (long)g.x * g.y;
    hipLaunchKernelGGL(k_cfl_t2, g, dim3(64, 4, 1), 0, st, G, JU, J, x, part);
    return;
  }
  dim3 b, g;
  node_grid(G.n[0], G.n[1], G.n[2], g, b);
  nb = (long)g.x * g.y * g.z;
  if (G.dim == 1) hipLaunchKernelGGL(k_cfl<1>, g, b, 0, st, G, JU, J, x, c->met, part);
  else hipLaunchKernelGGL(k_cfl<3>, g, b, 0, st, G, JU, J, x, c->met, part);
}

// k_final (maxima) for several partial arrays at once: block q reduces part + q * stride into dst[q]
__global__ void k_final_many(const double *__restrict__ part, long stride, long nb, double *dst) {
  const double *pq = part + blockIdx.x * stride;
  double v = 0.0;
  for (long i = threadIdx.x; i < nb; i += blockDim.x) v = fmax(v, pq[i]);
  v = block_max(v);
  if (threadIdx.x == 0) dst[blockIdx.x] = v;
}

// k_final for the CFL maxima followed by k_dt's dt = cfl / max, in one launch
__global__ void k_final_dt(const double *__restrict__ part, long nb, double cfl, double *scal, double *dt_out) {
  double v = 0.0;
  for (long i = threadIdx.x; i < nb; i += blockDim.x) v = fmax(v, part[i]);
  v = block_max(v);
  if (threadIdx.x == 0) {
    scal[SC_CFL] = v;
    double dt = cfl / scal[SC_CFL];
    scal[SC_DT] = dt;
    if (dt_out) *dt_out = dt;
  }
}

// k_final's movement-limiter minimum and k_final_dt's CFL maximum and dt in one launch (the
// same reductions in the same order)
__global__ void k_final_gamma_dt(const double *__restrict__ pl, long nbl, const double *__restrict__ pc, long nbc,
                                 double cfl, double *scal, double *dt_out) {
  double g = 1.0;
  for (long i = threadIdx.x; i < nbl; i += blockDim.x) g = fmin(g, pl[i]);
  g = block_min(g);
  double v = 0.0;
  for (long i = threadIdx.x; i < nbc; i += blockDim.x) v = fmax(v, pc[i]);
  v = block_max(v);
  if (threadIdx.x == 0) {
    scal[SC_GAMMA] = g;
    scal[SC_CFL] = v;
    double dt = cfl / scal[SC_CFL];
    scal[SC_DT] = dt;
    if (dt_out) *dt_out = dt;
  }
}

__global__ void k_dt(double cfl, double dt_fixed, double *scal, double *dt_out) {
  if (threadIdx.x == 0) {
    double dt = dt_fixed > 0.0 ? dt_fixed : cfl / scal[SC_CFL];
    scal[SC_DT] = dt;
    if (dt_out) *dt_out = dt;
  }
}

__global__ void k_xdot(long n, const double *__restrict__ xn, const double *__restrict__ xmu,
                       const double *__restrict__ gam, const double *__restrict__ dtp, double *__restrict__ xd) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t < n) xd[t] = (*gam) * (xmu[t] - xn[t]) / (*dtp);
}

// ---- launchers ----------------------------------------------------------------------
#define CHK() (hipGetLastError() == hipSuccess ? 0 : -1)

int launch_set_scalars(esvdw_ctx *c, hipStream_t st) {
  hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, st, c->scal);
  return CHK();
}

int launch_set_int(int *p, int v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, p, v);
  return CHK();
}

int launch_copy(const double *src, double *dst, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3(nblk(n, 256)), dim3(256), 0, st, src, dst, n);
  return CHK();
}

int launch_add(const double *a, const double *b, double *dst, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_add, dim3(nblk(n, 256)), dim3(256), 0, st, a, b, dst, n);
  return CHK();
}

// xn != nullptr (2D without a step): the CFL partial maxima of (JU, J) on xn are formed in the same
// pass (k_mon_cfl_t2) into part + 3 npart, their block count into *nbc; otherwise *nbc = 0
template <int D>
static int monitor_d(esvdw_ctx *c, const double *JU, const double *J, const double *xn, double *omega, long *nbc,
                     hipStream_t st) {
  const Geo &G = c->G;
  const esvdw_params &p = c->p;
  dim3 b, g;
  node_grid(G.n[0], G.n[1], G.n[2], g, b);
  long nb = (long)g.x * g.y * g.z;
  int nterm = p.monitor_kind == ESVDW_MON_VDW ? p.kappa + 1 : 2;
  if (nbc) *nbc = 0;
  if (D == 2 && xn && nbc && G.s0 == 0) {
    const dim3 gt((G.n[0] + MC_TX - 1) / MC_TX, (G.n[1] + MC_TY - 1) / MC_TY, 1);
    nb = (long)gt.x * gt.y;  // <= npart
    hipLaunchKernelGGL(k_mon_cfl_t2, gt, dim3(64, 4, 1), 0, st, G, p.monitor_kind, p.kappa, p.mon_var[0],
                       p.mon_var[1], JU, J, xn, c->mterm, c->part, c->npart, c->part + 3 * c->npart);
    *nbc = nb;
  } else {
    hipLaunchKernelGGL(k_rho_G<D>, g, b, 0, st, G, JU, J, c->rhoG);
    hipLaunchKernelGGL(k_mon_terms<D>, g, b, 0, st, G, p.monitor_kind, p.kappa, p.mon_var[0], p.mon_var[1], c->rhoG,
                       c->mterm, c->part, c->npart);
  }
  hipLaunchKernelGGL(k_final_many, dim3(nterm), dim3(1024), 0, st, c->part, c->npart, nb, c->scal + SC_MON);
  // 2D outflow grids run up to JT_H passes per launch; the filtered result must end in `omega`:
  // start in omega2 when the launch count is odd
  // (with the step every pass is its own launch, followed by the images at the solid nodes)
  const bool multi = D == 2 && G.bc[0] != ESVDW_BC_PERIODIC && G.bc[1] != ESVDW_BC_PERIODIC && p.n_filter >= 2 &&
                     G.s0 == 0;
  const int nlaunch = multi ? (p.n_filter + JT_H - 1) / JT_H : p.n_filter;
  double *cur = (nlaunch % 2) ? c->omega2 : omega;
  double *oth = (nlaunch % 2) ? omega : c->omega2;
  hipLaunchKernelGGL(k_mon_omega, g, b, 0, st, G, nterm, p.alpha[0], p.alpha[1], p.alpha[2], c->mterm, c->scal, cur);
  if (launch_step_fill_scalar(G, cur, st)) return -1;
  const dim3 gm((G.n[0] + JT_X - 1) / JT_X, (G.n[1] + JT_Y - 1) / JT_Y, 1);
  for (int done = 0; done < p.n_filter;) {
    const int k = multi ? (p.n_filter - done < JT_H ? p.n_filter - done : JT_H) : 1;
    if (multi) hipLaunchKernelGGL(k_filter_multi2, gm, dim3(64, 4), 0, st, G, cur, oth, k);
    else hipLaunchKernelGGL(k_filter<D>, g, b, 0, st, G, cur, oth);
    double *tmp = cur;
    cur = oth;
    oth = tmp;
    done += k;
    if (launch_step_fill_scalar(G, cur, st)) return -1;
  }
  return CHK();
}

int launch_monitor(esvdw_ctx *c, const double *JU, const double *J, double *omega, hipStream_t st) {
  switch (c->G.dim) {
    case 1: return monitor_d<1>(c, JU, J, nullptr, omega, nullptr, st);
    case 2: return monitor_d<2>(c, JU, J, nullptr, omega, nullptr, st);
    default: return monitor_d<3>(c, JU, J, nullptr, omega, nullptr, st);
  }
}

int launch_monitor_cfl(esvdw_ctx *c, const double *JU, const double *J, const double *xn, double *omega, long *nbc,
                       hipStream_t st) {
  switch (c->G.dim) {
    case 1: return monitor_d<1>(c, JU, J, xn, omega, nbc, st);
    case 2: return monitor_d<2>(c, JU, J, xn, omega, nbc, st);
    default: return monitor_d<3>(c, JU, J, xn, omega, nbc, st);
  }
}

template <int D>
static int jacobi_d(esvdw_ctx *c, const double *omega, const double *x0, double *x, int nsweep, double *resid_dev,
                    hipStream_t st) {
  const Geo &G = c->G;
  dim3 b, g;
  node_grid(G.n[0], G.n[1], G.n[2], g, b);
  const long nb = (long)g.x * g.y * g.z;
  // the first launch reads x0 (when given) and writes the scratch iterate; later ones alternate
  // between x and the scratch, so x0 is never written
  const double *a0 = x0 ? x0 : x;
  double *a = x, *o = c->xtmp;
  const bool multi = D == 2 && G.bc[0] != ESVDW_BC_PERIODIC && G.bc[1] != ESVDW_BC_PERIODIC && nsweep >= 2 &&
                     G.s0 == 0;
  if (multi) {
    const dim3 gm((G.n[0] + JT_X - 1) / JT_X, (G.n[1] + JT_Y - 1) / JT_Y, 1);
    const long nbm = (long)gm.x * gm.y;  // <= 4 npart
    for (int done = 0; done < nsweep;) {
      const int k = nsweep - done < JT_H ? nsweep - done : JT_H;
      const bool last = done + k == nsweep && resid_dev;  // the residual only when asked for
      hipLaunchKernelGGL(k_jacobi_multi2, gm, dim3(64, 4), 0, st, G, omega, done == 0 ? a0 : a, o, k,
                         last ? c->part : nullptr);
      if (last) hipLaunchKernelGGL(k_final, dim3(1), dim3(1024), 0, st, c->part, nbm, c->scal + SC_RESID, 0);
      double *tmp = a;
      a = o;
      o = tmp;
      done += k;
    }
  }
  for (int it = 0; !multi && it < nsweep; ++it) {
    bool last = it == nsweep - 1 && resid_dev;
    hipLaunchKernelGGL(k_jacobi<D>, g, b, 0, st, G, omega, it == 0 ? a0 : a, o, last ? c->part : nullptr);
    if (last) hipLaunchKernelGGL(k_final, dim3(1), dim3(1024), 0, st, c->part, nb, c->scal + SC_RESID, 0);
    if (launch_step_fill_mesh(G, o, st)) return -1;  // the images and the corner lattice after each sweep
    double *tmp = a;
    a = o;
    o = tmp;
  }
  if (a != x) launch_copy(a, x, (long)D * G.N, st);
  else if (nsweep == 0 && x0 && x0 != x) launch_copy(x0, x, (long)D * G.N, st);
  if (resid_dev) launch_copy(c->scal + SC_RESID, resid_dev, 1, st);
  return CHK();
}

template <int D>
static int sor_d(esvdw_ctx *c, const double *omega, double *x, int nsweep, double relax, double *resid_dev,
                 hipStream_t st) {
  const Geo &G = c->G;
  if (D == 2 && G.bc[0] != ESVDW_BC_PERIODIC && G.bc[1] != ESVDW_BC_PERIODIC && G.s0 == 0 && nsweep > 0) {
    const dim3 gm((G.n[0] + JS_X - 1) / JS_X, (G.n[1] + JS_Y - 1) / JS_Y, 1);
    const long nbm = (long)gm.x * gm.y;  // <= npart
    const double *a = x;
    double *o = c->xtmp;
    for (int done = 0; done < nsweep;) {
      const int k = nsweep - done < JS_S ? nsweep - done : JS_S;
      const bool last = done + k == nsweep;
      hipLaunchKernelGGL(k_sor_multi2, gm, dim3(32, 8), 0, st, G, omega, a, o, k, relax, last ? c->part : nullptr);
      a = o;
      o = (o == c->xtmp) ? x : c->xtmp;
      done += k;
    }
    hipLaunchKernelGGL(k_final, dim3(1), dim3(1024), 0, st, c->part, nbm, c->scal + SC_RESID, 0);
    if (a != x) launch_copy(a, x, 2L * G.N, st);
    if (resid_dev) launch_copy(c->scal + SC_RESID, resid_dev, 1, st);
    return CHK();
  }
  dim3 b, g;
  node_grid((G.n[0] + 1) / 2, G.n[1], G.n[2], g, b);
  const long nb = (long)g.x * g.y * g.z;  // 2 nb <= 4 npart: both halves' partial maxima fit
  for (int it = 0; it < nsweep; ++it) {
    bool last = it == nsweep - 1;
    for (int colour = 0; colour < 2; ++colour)
      hipLaunchKernelGGL(k_sor<D>, g, b, 0, st, G, omega, x, colour, relax, last ? c->part + colour * nb : nullptr);
    if (last) hipLaunchKernelGGL(k_final, dim3(1), dim3(1024), 0, st, c->part, 2 * nb, c->scal + SC_RESID, 0);
  }
  if (resid_dev && nsweep > 0) launch_copy(c->scal + SC_RESID, resid_dev, 1, st);
  return CHK();
}

int launch_sor(esvdw_ctx *c, const double *omega, double *x, int nsweep, double relax, double *resid_dev,
               hipStream_t st) {
  switch (c->G.dim) {
    case 1: return sor_d<1>(c, omega, x, nsweep, relax, resid_dev, st);
    case 2: return sor_d<2>(c, omega, x, nsweep, relax, resid_dev, st);
    default: return sor_d<3>(c, omega, x, nsweep, relax, resid_dev, st);
  }
}

int launch_jacobi_from(esvdw_ctx *c, const double *omega, const double *x0, double *x, int nsweep, double *resid_dev,
                       hipStream_t st) {
  switch (c->G.dim) {
    case 1: return jacobi_d<1>(c, omega, x0, x, nsweep, resid_dev, st);
    case 2: return jacobi_d<2>(c, omega, x0, x, nsweep, resid_dev, st);
    default: return jacobi_d<3>(c, omega, x0, x, nsweep, resid_dev, st);
  }
}

int launch_jacobi(esvdw_ctx *c, const double *omega, double *x, int nsweep, double *resid_dev, hipStream_t st) {
  return launch_jacobi_from(c, omega, nullptr, x, nsweep, resid_dev, st);
}

int launch_limiter(esvdw_ctx *c, const double *xn, const double *xmu, double *gamma_dev, hipStream_t st) {
  const Geo &G = c->G;
  dim3 b, g;
  node_grid(G.n[0], G.n[1], G.n[2], g, b);
  const long nb = (long)g.x * g.y * g.z;
  if (G.dim == 1) hipLaunchKernelGGL(k_limiter<1>, g, b, 0, st, G, xn, xmu, c->part);
  else if (G.dim == 2) hipLaunchKernelGGL(k_limiter<2>, g, b, 0, st, G, xn, xmu, c->part);
  else hipLaunchKernelGGL(k_limiter<3>, g, b, 0, st, G, xn, xmu, c->part);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(1024), 0, st, c->part, nb, c->scal + SC_GAMMA, 1);
  if (gamma_dev) launch_copy(c->scal + SC_GAMMA, gamma_dev, 1, st);
  return CHK();
}

int launch_cfl(esvdw_ctx *c, const double *JU, const double *J, const double *x, double *dt_dev, hipStream_t st) {
  const Geo &G = c->G;
  if (c->p.dt_fixed <= 0.0) {
    if (G.dim == 3 && launch_metrics(c, x, nullptr, c->met, nullptr, nullptr, st)) return -1;
    long nb = 0;
    cfl_launch(c, JU, J, x, c->part, nb, st);
    hipLaunchKernelGGL(k_final_dt, dim3(1), dim3(1024), 0, st, c->part, nb, c->p.cfl, c->scal, dt_dev);
  } else {
    hipLaunchKernelGGL(k_dt, dim3(1), dim3(64), 0, st, c->p.cfl, c->p.dt_fixed, c->scal, dt_dev);
  }
  return CHK();
}

// ---- CFL time step without allocation (cfl_dt_noalloc) ------------------------------------
// The per-block maxima and the two result slots live in a file-scope device array: each GPU
// holds its own copy for the life of the process.  Its address differs per device and the
// array's name is not a device address in host code, so it is looked up once per device with
// hipGetSymbolAddress and only that pointer is passed to kernels.
#define NOALLOC_PARTS 65536                     // per-block partial maxima (256 nodes in 1D, 1024 in 2D)
#define NOALLOC_DOUBLES (NOALLOC_PARTS + SC_N)  // + the scalar slots k_final_dt writes
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

#define NOALLOC_MAXDEV 64
static double *g_scratch_ptr[NOALLOC_MAXDEV];
static std::mutex g_scratch_mu;

static double *noalloc_scratch(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAXDEV) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = (double *)ptr;
  }
  return g_scratch_ptr[dev];
}

int launch_cfl_noalloc(const Geo &G, double cfl, double dt_fixed, const double *JU, const double *J,
                       const double *x, double *dt_dev, hipStream_t st) {
  // the kernels of launch_cfl: 1D one node per thread, 2D the LDS-tiled kernel
  dim3 b, g;
  if (G.dim == 2) {
    g = dim3((G.n[0] + CF_TX - 1) / CF_TX, (G.n[1] + CF_TY - 1) / CF_TY, 1);
    b = dim3(64, 4, 1);
  } else {
    node_grid(G.n[0], G.n[1], G.n[2], g, b);
  }
  const long nb = (long)g.x * g.y * g.z;
  if (nb > NOALLOC_PARTS) return ESVDW_ESCRATCH;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return ESVDW_EHIP;
  double *ptr = noalloc_scratch(dev);  // set-up on this device's first call
  if (!ptr) return ESVDW_EHIP;
  double *scal = ptr + NOALLOC_PARTS;
  if (dt_fixed > 0.0) {
    hipLaunchKernelGGL(k_dt, dim3(1), dim3(64), 0, st, cfl, dt_fixed, scal, dt_dev);
  } else {
    // every block writes its partial, so nothing needs clearing between calls
    if (G.dim == 1) hipLaunchKernelGGL(k_cfl<1>, g, b, 0, st, G, JU, J, x, nullptr, ptr);
    else hipLaunchKernelGGL(k_cfl_t2, g, b, 0, st, G, JU, J, x, ptr);
    hipLaunchKernelGGL(k_final_dt, dim3(1), dim3(1024), 0, st, ptr, nb, cfl, scal, dt_dev);
  }
  return CHK() ? ESVDW_EHIP : ESVDW_OK;
}

int launch_limiter_cfl(esvdw_ctx *c, const double *xn, const double *xmu, const double *JU, const double *J,
                       double *dt_dev, long nbc_ready, hipStream_t st) {
  const Geo &G = c->G;
  if (c->p.dt_fixed > 0.0) {
    if (launch_limiter(c, xn, xmu, nullptr, st)) return -1;
    return launch_cfl(c, JU, J, xn, dt_dev, st);
  }
  dim3 b, g;
  node_grid(G.n[0], G.n[1], G.n[2], g, b);
  const long nb = (long)g.x * g.y * g.z;
  double *pc = c->part + 3 * c->npart;  // the CFL partials beside the limiter's
  if (G.dim == 1) hipLaunchKernelGGL(k_limiter<1>, g, b, 0, st, G, xn, xmu, c->part);
  else if (G.dim == 2) hipLaunchKernelGGL(k_limiter<2>, g, b, 0, st, G, xn, xmu, c->part);
  else hipLaunchKernelGGL(k_limiter<3>, g, b, 0, st, G, xn, xmu, c->part);
  if (G.dim == 3 && launch_metrics(c, xn, nullptr, c->met, nullptr, nullptr, st)) return -1;
  long nbc = nbc_ready;  // > 0: the CFL partials of (JU, J) on xn are already in pc (launch_monitor_cfl)
  if (nbc == 0) cfl_launch(c, JU, J, xn, pc, nbc, st);
  hipLaunchKernelGGL(k_final_gamma_dt, dim3(1), dim3(1024), 0, st, c->part, nb, pc, nbc, c->p.cfl, c->scal, dt_dev);
  return CHK();
}

int launch_xdot(esvdw_ctx *c, const double *xn, const double *xmu, const double *gam, const double *dtp, double *xdot,
                hipStream_t st) {
  long n = (long)c->G.dim * c->G.N;
  hipLaunchKernelGGL(k_xdot, dim3(nblk(n, 256)), dim3(256), 0, st, n, xn, xmu, gam, dtp, xdot);
  return CHK();
}

// ---- |grad_xi rho|^2 per node and its global max (features of the learned warm start) -------
template <int D> static int grad_rho_d(esvdw_ctx *c, const double *JU, const double *J, hipStream_t st) {
  const Geo &G = c->G;
  dim3 b, g;
  node_grid(G.n[0], G.n[1], G.n[2], g, b);
  const long nb = (long)g.x * g.y * g.z;
  hipLaunchKernelGGL(k_rho_G<D>, g, b, 0, st, G, JU, J, c->rhoG);
  // vdW form with one gradient term of rho: term 0 = |grad rho|^2 (term 1 = |Delta G|^2, unused)
  hipLaunchKernelGGL(k_mon_terms<D>, g, b, 0, st, G, (int)ESVDW_MON_VDW, 1, (int)ESVDW_VAR_RHO, 0, c->rhoG, c->mterm,
                     c->part, c->npart);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(1024), 0, st, c->part, nb, c->scal + SC_MON, 0);
  return CHK();
}

int launch_grad_rho_terms(esvdw_ctx *c, const double *JU, const double *J, hipStream_t st) {
  switch (c->G.dim) {
    case 1: return grad_rho_d<1>(c, JU, J, st);
    case 2: return grad_rho_d<2>(c, JU, J, st);
    default: return grad_rho_d<3>(c, JU, J, st);
  }
}
