// batch.hip -- many independent 2D problems (each with its own grid size, EOS constants and
// boundary conditions) advanced together: one launch of a persistent kernel per SSP-RK3
// stage covers every instance.  Inside a stage, grid-wide barriers separate the phases
//   [stage 0]  CFL spectral radius per node chunk -> per-chunk maxima, then dt per instance
//   node data of every padded node of every instance
//   interface fluxes of every instance, both directions
//   flux differences and the RK combination (+ x^{n+1} = x^n + dt xdot at stage 2)
// The same phases also run as separate launches (the phased kernels, in which the direction-0
// fluxes of 62 x 4 tiles are formed together with the update of their nodes), and the mesh
// redistribution of Section 4 (monitor with per-instance maxima, filter, Jacobi, limiter,
// mesh velocity) runs batched over the same work lists.  The work items of a phase
// (interface tiles, or chunks of 256 nodes) are listed instance by instance.  Workgroups are
// handed to the 8 XCDs round-robin, so the blocks with equal blockIdx % 8 share one XCD; each
// such group walks one contiguous eighth of the list, and neighbouring tiles (which read the
// same node data) share that XCD's L2.
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "common.h"
#include "kernels.h"
#include "meshdev.h"
#include "scheme.h"

#define HIPOK(x) ((x) == hipSuccess)

struct BInst {
  Geo G;
  long off;         // first node of the instance in the pooled arrays
  double *nd;       // node buffer (NF_<2>::COUNT * PN)
  double *F0, *F1;  // interface fluxes per direction ((nv + 1) * nif)
  long nif0, nif1;
  double cfl, dt_fixed;
  int u0, u1;       // the instance's chunks in the update list
  int mkind, kappa, var0, var1, nterm;  // monitor of the mesh redistribution
  double alpha[3];
};

// a work item: a flux tile (first interface (x0, y0), direction k) or a chunk of 256
// consecutive nodes starting at x0 (node data over the padded grid, CFL and update over the
// interior); y0 unused for chunks
struct BItem {
  int inst, x0, y0, k;
};

// tile variants of the flux phase (direction 0 tile X0 x Y0, direction 1 tile X1 x Y1) and
// blocks per CU requested from the compiler
template <int V> struct BVar;
template <> struct BVar<0> { static constexpr int X0 = 64, Y0 = 4, X1 = 16, Y1 = 16, OCC = 2; };
template <> struct BVar<1> { static constexpr int X0 = 32, Y0 = 8, X1 = 16, Y1 = 16, OCC = 2; };
template <> struct BVar<2> { static constexpr int X0 = 64, Y0 = 4, X1 = 32, Y1 = 8, OCC = 2; };
template <> struct BVar<3> { static constexpr int X0 = 32, Y0 = 8, X1 = 8, Y1 = 32, OCC = 2; };
template <> struct BVar<4> { static constexpr int X0 = 64, Y0 = 4, X1 = 16, Y1 = 16, OCC = 3; };
#define BATCH_NTILE 5
// variants 0 .. BATCH_NTILE - 1: the persistent kernel with tile set v; BATCH_NTILE .. 2 BATCH_NTILE - 1:
// the phased kernels with tile set v - BATCH_NTILE
#define BATCH_NVAR (2 * BATCH_NTILE)

struct esvdw_batch {
  int ninst, variant, dev;
  int nblocks[BATCH_NTILE];
  std::vector<Geo> geo;
  std::vector<long> off;  // ninst + 1
  std::vector<BInst> inst;
  BInst *dI;
  BItem *dNode, *dFlux, *dUpd, *dFU;  // dFU: direction-0 flux + update tiles of the phased mode
  int nNode, nFlux, nUpd, nFU;
  double *nd_pool, *f_pool, *sAU, *sAJ, *sBU, *sBJ, *cpart;
  unsigned *bar, *flags;
  // mesh redistribution (fixed sweep count, shared by all instances)
  int redist_ok, n_filter, mu;
  double *rg, *term, *omA, *omB, *xa, *xb, *part3, *monmax, *gam;
};

// ---- grid-wide barrier with a bounded wait ---------------------------------------------------
// bar[0] counts arrivals, bar[1] is the generation.  Every thread fences its stores at device
// scope before the block arrives and again after the release, so data written in one phase is
// seen by every block (on every XCD) in the next.  A wait longer than about a second (the grid
// was not co-resident) raises ESVDW_F_BARRIER and proceeds, so the kernel always terminates.
#define BATCH_SPIN_LIMIT (1u << 24)

__device__ __forceinline__ void grid_barrier(unsigned *bar, unsigned nblocks, unsigned *flags) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned gen = __hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned arrived = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(bar + 1, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > BATCH_SPIN_LIMIT) {
          atomicOr(flags, ESVDW_F_BARRIER);
          break;
        }
      }
    }
  }
  __syncthreads();
  __threadfence();
}

// this block's share of n items: XCD x = blockIdx % 8 owns [x c, (x + 1) c), c = ceil(n / 8),
// walked with stride gridDim / 8 (gridDim is a multiple of 8)
#define XCD_WALK(n, it)                                                                              \
  for (int it = (int)(blockIdx.x & 7u) * (((n) + 7) >> 3) + (int)(blockIdx.x >> 3),                  \
           it##_end = min((n), ((int)(blockIdx.x & 7u) + 1) * (((n) + 7) >> 3));                      \
       it < it##_end; it += (int)(gridDim.x >> 3))

// ---- work items (shared by the persistent kernel and the phased kernels) -------------------

// CFL rate of this thread's node of a 256-node chunk of the update list; block maximum to *out
__device__ __forceinline__ void cfl_chunk(const BInst &B, int x0, const double *__restrict__ bU,
                                          const double *__restrict__ bJ, const double *__restrict__ x, double *out) {
  const int t = x0 + (int)threadIdx.x;
  double r = 0.0;
  if (t < B.G.N) {
    const int i1 = t / B.G.n[0], i0 = t - i1 * B.G.n[0];
    r = cfl_rate<2>(B.G, bU + 4 * B.off, bJ + B.off, x + 2 * B.off, nullptr, i0, i1, 0);
  }
  double m = block_max(r);
  if (threadIdx.x == 0) *out = m;
}

// dt of one instance from its chunks' maxima (block-wide)
__device__ __forceinline__ void dt_instance(const BInst &B, const double *__restrict__ cpart, double *dti) {
  double m = 0.0;
  for (int u = B.u0 + (int)threadIdx.x; u < B.u1; u += 256) m = fmax(m, cpart[u]);
  m = block_max(m);
  if (threadIdx.x == 0) *dti = B.dt_fixed > 0.0 ? B.dt_fixed : B.cfl / m;
}

// node data of this thread's padded node of a 256-node chunk, on the stage mesh x^n + c_s dt xdot
__device__ __forceinline__ void node_chunk(const BInst &B, int inst, int x0, int s, const double *__restrict__ inU,
                                           const double *__restrict__ inJ, const double *__restrict__ x,
                                           const double *__restrict__ xd, const double *__restrict__ dt,
                                           unsigned *flags) {
  // chunks run over the E0 x P1 nodes that hold data
  const int t = x0 + (int)threadIdx.x;
  if (t < B.G.E0 * B.G.P[1]) {
    const int p1 = t / B.G.E0, p0 = t - p1 * B.G.E0;
    const double cdt = (xd && s > 0) ? (s == 1 ? 1.0 : 0.5) * dt[inst] : 0.0;
    node_point<2>(B.G, inU + 4 * B.off, inJ + B.off, nullptr, nullptr, x + 2 * B.off, xd ? xd + 2 * B.off : nullptr,
                  cdt, nullptr, 0, B.nd, flags, p0, p1, 0);
  }
}

template <int X0, int Y0, int X1, int Y1>
__device__ __forceinline__ void flux_item(const BInst &B, const BItem &w, unsigned *flags, double *sP) {
  if (w.k == 0) flux_tile<2, 0, X0, Y0, 1>(B.G, B.nd, B.F0, B.nif0, flags, w.x0, w.y0, 0, sP);
  else flux_tile<2, 1, X1, Y1, 1>(B.G, B.nd, B.F1, B.nif1, flags, w.x0, w.y0, 0, sP);
}

// flux differences and the RK combination at this thread's node of a chunk; at stage 2 with a
// mesh velocity also x^{n+1} = x^n + dt xdot
__device__ __forceinline__ void update_chunk(const BInst &B, int inst, int x0, int s, const double *__restrict__ bU,
                                             const double *__restrict__ bJ, const double *__restrict__ inU,
                                             const double *__restrict__ inJ, double *outU, double *outJ, double *x,
                                             const double *__restrict__ xd, const double *__restrict__ dt,
                                             unsigned *flags) {
  const int t = x0 + (int)threadIdx.x;
  if (t < B.G.N) {
    const int i1 = t / B.G.n[0], i0 = t - i1 * B.G.n[0];
    update_point<2>(B.G, B.F0, B.F1, nullptr, B.nif0, B.nif1, 0, 1, s, dt + inst, bU + 4 * B.off, bJ + B.off,
                    inU + 4 * B.off, inJ + B.off, outU + 4 * B.off, outJ + B.off, flags, i0, i1, 0);
    if (s == 2 && xd) {
      const double d = dt[inst];
      for (int j = 0; j < 2; ++j) {
        const long q = 2 * B.off + (long)j * B.G.N + t;
        x[q] = x[q] + d * xd[q];
      }
    }
  }
}

// ---- the persistent stage kernel: one launch per RK stage -----------------------------------

template <int X0, int Y0, int X1, int Y1, int OCC>
__global__ void __launch_bounds__(256, OCC)
    k_batch_stage(const BInst *__restrict__ I, int ninst, const BItem *__restrict__ inode, int nnode,
                  const BItem *__restrict__ iflux, int nflux, const BItem *__restrict__ iupd, int nupd, int s,
                  const double *__restrict__ bU, const double *__restrict__ bJ, const double *__restrict__ inU,
                  const double *__restrict__ inJ, double *outU, double *outJ, double *x,
                  const double *__restrict__ xd, double *dt, double *cpart, unsigned *bar, unsigned *flags) {
  constexpr int L0 = FluxLds<2, 0, X0, Y0, 1>::SIZE, L1 = FluxLds<2, 1, X1, Y1, 1>::SIZE;
  __shared__ double sP[L0 > L1 ? L0 : L1];
  const unsigned nb = gridDim.x;
  if (s == 0) {
    XCD_WALK(nupd, it) {
      const BItem w = iupd[it];
      cfl_chunk(I[w.inst], w.x0, bU, bJ, x, cpart + it);
    }
    grid_barrier(bar, nb, flags);
    for (int i = blockIdx.x; i < ninst; i += nb) dt_instance(I[i], cpart, dt + i);
  }
  XCD_WALK(nnode, it) {
    const BItem w = inode[it];
    node_chunk(I[w.inst], w.inst, w.x0, s, inU, inJ, x, xd, dt, flags);
  }
  grid_barrier(bar, nb, flags);
  XCD_WALK(nflux, it) {
    const BItem w = iflux[it];
    flux_item<X0, Y0, X1, Y1>(I[w.inst], w, flags, sP);
    __syncthreads();  // sP is reused by the next tile
  }
  grid_barrier(bar, nb, flags);
  XCD_WALK(nupd, it) {
    const BItem w = iupd[it];
    update_chunk(I[w.inst], w.inst, w.x0, s, bU, bJ, inU, inJ, outU, outJ, x, xd, dt, flags);
  }
}

// ---- the phased kernels: the same items, one launch per phase --------------------------------
// Each launch gives each phase its own occupancy.  Grid = 8 ceil(n / 8) blocks; block b takes
// item (b % 8) ceil(n / 8) + b / 8, so each XCD takes a contiguous eighth of the list.
__device__ __forceinline__ int xcd_item(int n) {
  const int c = (n + 7) >> 3, j = (int)(blockIdx.x >> 3), it = (int)(blockIdx.x & 7u) * c + j;
  return (j < c && it < n) ? it : -1;
}

__global__ void __launch_bounds__(256) k_bph_cfl(const BInst *__restrict__ I, const BItem *__restrict__ iupd, int nupd,
                                                 const double *__restrict__ bU, const double *__restrict__ bJ,
                                                 const double *__restrict__ x, double *cpart) {
  const int it = xcd_item(nupd);
  if (it < 0) return;
  const BItem w = iupd[it];
  cfl_chunk(I[w.inst], w.x0, bU, bJ, x, cpart + it);
}

__global__ void __launch_bounds__(256) k_bph_dt(const BInst *__restrict__ I, const double *__restrict__ cpart,
                                                double *dt) {
  dt_instance(I[blockIdx.x], cpart, dt + blockIdx.x);
}

__global__ void __launch_bounds__(256) k_bph_nodes(const BInst *__restrict__ I, const BItem *__restrict__ inode,
                                                   int nnode, int s, const double *__restrict__ inU,
                                                   const double *__restrict__ inJ, const double *__restrict__ x,
                                                   const double *__restrict__ xd, const double *__restrict__ dt,
                                                   unsigned *flags) {
  const int it = xcd_item(nnode);
  if (it < 0) return;
  const BItem w = inode[it];
  node_chunk(I[w.inst], w.inst, w.x0, s, inU, inJ, x, xd, dt, flags);
}

template <int X0, int Y0, int X1, int Y1, int OCC>
__global__ void __launch_bounds__(256, OCC) k_bph_flux(const BInst *__restrict__ I, const BItem *__restrict__ iflux,
                                                       int nflux, unsigned *flags) {
  constexpr int L0 = FluxLds<2, 0, X0, Y0, 1>::SIZE, L1 = FluxLds<2, 1, X1, Y1, 1>::SIZE;
  __shared__ double sP[L0 > L1 ? L0 : L1];
  const int it = xcd_item(nflux);
  if (it < 0) return;
  const BItem w = iflux[it];
  flux_item<X0, Y0, X1, Y1>(I[w.inst], w, flags, sP);
}

// the direction-0 fluxes of a 62 x 4 tile and the stage update of its 61 x 4 nodes (as the
// single-problem k_flux_upd2), with x^{n+1} = x^n + dt xdot at stage 2 with a mesh velocity
__global__ void __launch_bounds__(256, 3) k_bph_fupd(const BInst *__restrict__ I, const BItem *__restrict__ ifu,
                                                     int nfu, int s, const double *__restrict__ bU,
                                                     const double *__restrict__ bJ, const double *__restrict__ inU,
                                                     const double *__restrict__ inJ, double *outU, double *outJ,
                                                     double *x, const double *__restrict__ xd,
                                                     const double *__restrict__ dt, unsigned *flags) {
  __shared__ double sP[FluxLds<2, 0, FU_TX, FU_TY, 1>::SIZE];
  const int it = xcd_item(nfu);
  if (it < 0) return;
  const BItem w = ifu[it];
  const BInst &B = I[w.inst];
  double *mx = (s == 2 && xd) ? x + 2 * B.off : nullptr;
  flux_upd2_tile<false>(B.G, B.nd, B.F1, B.nif1, 1, s, dt + w.inst, bU + 4 * B.off, bJ + B.off, inU + 4 * B.off,
                        inJ + B.off, outU + 4 * B.off, outJ + B.off, flags, mx, mx ? xd + 2 * B.off : nullptr, 1.0,
                        mx, w.x0, w.y0, sP);
}

__global__ void __launch_bounds__(256) k_bph_update(const BInst *__restrict__ I, const BItem *__restrict__ iupd,
                                                    int nupd, int s, const double *__restrict__ bU,
                                                    const double *__restrict__ bJ, const double *__restrict__ inU,
                                                    const double *__restrict__ inJ, double *outU, double *outJ,
                                                    double *x, const double *__restrict__ xd,
                                                    const double *__restrict__ dt, unsigned *flags) {
  const int it = xcd_item(nupd);
  if (it < 0) return;
  const BItem w = iupd[it];
  update_chunk(I[w.inst], w.inst, w.x0, s, bU, bJ, inU, inJ, outU, outJ, x, xd, dt, flags);
}

// ---- batched mesh redistribution (Section 4): the same per-node building blocks over the
// update list's 256-node chunks; per-instance maxima / minima through chunk partials ----------

// interior node (i0, i1) of this thread in a chunk; false past the instance's last node
__device__ __forceinline__ bool chunk_node(const BInst &B, int x0, int &i0, int &i1, long &t) {
  const int tt = x0 + (int)threadIdx.x;
  if (tt >= B.G.N) return false;
  i1 = tt / B.G.n[0];
  i0 = tt - i1 * B.G.n[0];
  t = tt;
  return true;
}

__global__ void __launch_bounds__(256) k_bm_rhoG(const BInst *__restrict__ I, const BItem *__restrict__ iupd, int nupd,
                                                 const double *__restrict__ JU, const double *__restrict__ J,
                                                 double *rg) {
  const int it = xcd_item(nupd);
  if (it < 0) return;
  const BItem w = iupd[it];
  const BInst &B = I[w.inst];
  int i0, i1;
  long t;
  if (chunk_node(B, w.x0, i0, i1, t)) rhoG_point<2>(B.G, JU + 4 * B.off, J + B.off, rg + 2 * B.off, t);
}

__global__ void __launch_bounds__(256) k_bm_terms(const BInst *__restrict__ I, const BItem *__restrict__ iupd, int nupd,
                                                  const double *__restrict__ rg, double *term, double *part3) {
  const int it = xcd_item(nupd);
  if (it < 0) return;
  const BItem w = iupd[it];
  const BInst &B = I[w.inst];
  int i0, i1;
  long t;
  double val[3] = {0.0, 0.0, 0.0};
  if (chunk_node(B, w.x0, i0, i1, t))
    mon_terms_point<2>(B.G, B.mkind, B.kappa, B.var0, B.var1, rg + 2 * B.off, term + 3 * B.off, i0, i1, 0, val);
  for (int q = 0; q < 3; ++q) {
    double m = block_max(val[q]);
    if (threadIdx.x == 0) part3[(long)q * nupd + it] = m;
  }
}

// per-instance reductions of chunk partials: maxima of the 3 monitor terms, or the limiter minimum
__global__ void __launch_bounds__(256) k_bm_max3(const BInst *__restrict__ I, const double *__restrict__ part3,
                                                 int nupd, double *monmax) {
  const BInst &B = I[blockIdx.x];
  for (int q = 0; q < 3; ++q) {
    double m = 0.0;
    for (int u = B.u0 + (int)threadIdx.x; u < B.u1; u += 256) m = fmax(m, part3[(long)q * nupd + u]);
    m = block_max(m);
    if (threadIdx.x == 0) monmax[3 * blockIdx.x + q] = m;
  }
}

__global__ void __launch_bounds__(256) k_bm_min(const BInst *__restrict__ I, const double *__restrict__ part,
                                                double *gam) {
  const BInst &B = I[blockIdx.x];
  double m = 1.0;
  for (int u = B.u0 + (int)threadIdx.x; u < B.u1; u += 256) m = fmin(m, part[u]);
  m = block_min(m);
  if (threadIdx.x == 0) gam[blockIdx.x] = m;
}

__global__ void __launch_bounds__(256) k_bm_omega(const BInst *__restrict__ I, const BItem *__restrict__ iupd, int nupd,
                                                  const double *__restrict__ term, const double *__restrict__ monmax,
                                                  double *om) {
  const int it = xcd_item(nupd);
  if (it < 0) return;
  const BItem w = iupd[it];
  const BInst &B = I[w.inst];
  int i0, i1;
  long t;
  if (chunk_node(B, w.x0, i0, i1, t))
    om[B.off + t] = mon_omega_point(B.G, B.nterm, B.alpha, term + 3 * B.off, monmax + 3 * w.inst, t);
}

__global__ void __launch_bounds__(256) k_bm_filter(const BInst *__restrict__ I, const BItem *__restrict__ iupd,
                                                   int nupd, const double *__restrict__ in, double *out) {
  const int it = xcd_item(nupd);
  if (it < 0) return;
  const BItem w = iupd[it];
  const BInst &B = I[w.inst];
  int i0, i1;
  long t;
  if (chunk_node(B, w.x0, i0, i1, t)) out[B.off + t] = filter_point<2>(B.G, in + B.off, i0, i1, 0);
}

__global__ void __launch_bounds__(256) k_bm_jacobi(const BInst *__restrict__ I, const BItem *__restrict__ iupd,
                                                   int nupd, const double *__restrict__ om,
                                                   const double *__restrict__ xin, double *xout) {
  const int it = xcd_item(nupd);
  if (it < 0) return;
  const BItem w = iupd[it];
  const BInst &B = I[w.inst];
  int i0, i1;
  long t;
  if (chunk_node(B, w.x0, i0, i1, t)) jacobi_point<2>(B.G, om + B.off, xin + 2 * B.off, xout + 2 * B.off, i0, i1, 0);
}

__global__ void __launch_bounds__(256) k_bm_limiter(const BInst *__restrict__ I, const BItem *__restrict__ iupd,
                                                    int nupd, const double *__restrict__ xn,
                                                    const double *__restrict__ xmu, double *part) {
  const int it = xcd_item(nupd);
  if (it < 0) return;
  const BItem w = iupd[it];
  const BInst &B = I[w.inst];
  int i0, i1;
  long t;
  double g = 1.0;
  if (chunk_node(B, w.x0, i0, i1, t)) g = limiter_point<2>(B.G, xn + 2 * B.off, xmu + 2 * B.off, i0, i1, 0);
  g = block_min(g);
  if (threadIdx.x == 0) part[it] = g;
}

// xdot = Delta_gamma (x^[mu] - x^n) / dt per instance
__global__ void __launch_bounds__(256) k_bm_xdot(const BInst *__restrict__ I, const BItem *__restrict__ iupd, int nupd,
                                                 const double *__restrict__ xn, const double *__restrict__ xmu,
                                                 const double *__restrict__ gam, const double *__restrict__ dt,
                                                 double *xdot) {
  const int it = xcd_item(nupd);
  if (it < 0) return;
  const BItem w = iupd[it];
  const BInst &B = I[w.inst];
  int i0, i1;
  long t;
  if (!chunk_node(B, w.x0, i0, i1, t)) return;
  const double g = gam[w.inst], d = dt[w.inst];
  for (int j = 0; j < 2; ++j) {
    const long q = 2 * B.off + (long)j * B.G.N + t;
    xdot[q] = g * (xmu[q] - xn[q]) / d;
  }
}

// ---- host side ---------------------------------------------------------------------------------

template <int V> static int stage_blocks(int ncu) {
  using C = BVar<V>;
  int occ = 0;
  if (!HIPOK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch_stage<C::X0, C::Y0, C::X1, C::Y1, C::OCC>,
                                                          256, 0)))
    return 0;
  int nb = ncu * occ;
  return nb - nb % 8;
}

template <int V>
static int launch_stage_v(esvdw_batch *b, int s, const double *bU, const double *bJ, const double *inU,
                          const double *inJ, double *outU, double *outJ, double *x, const double *xd, double *dt,
                          hipStream_t st) {
  using C = BVar<V>;
  hipLaunchKernelGGL((k_batch_stage<C::X0, C::Y0, C::X1, C::Y1, C::OCC>), dim3(b->nblocks[V]), dim3(256), 0, st,
                     b->dI, b->ninst, b->dNode, b->nNode, b->dFlux, b->nFlux, b->dUpd, b->nUpd, s, bU, bJ, inU, inJ,
                     outU, outJ, x, xd, dt, b->cpart, b->bar, b->flags);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

static inline unsigned xcd_grid(int n) { return 8u * (unsigned)((n + 7) / 8); }

template <int V>
static int launch_phased_v(esvdw_batch *b, int s, const double *bU, const double *bJ, const double *inU,
                           const double *inJ, double *outU, double *outJ, double *x, const double *xd, double *dt,
                           hipStream_t st) {
  using C = BVar<V>;
  if (s == 0) {
    hipLaunchKernelGGL(k_bph_cfl, dim3(xcd_grid(b->nUpd)), dim3(256), 0, st, b->dI, b->dUpd, b->nUpd, bU, bJ, x,
                       b->cpart);
    hipLaunchKernelGGL(k_bph_dt, dim3(b->ninst), dim3(256), 0, st, b->dI, b->cpart, dt);
  }
  hipLaunchKernelGGL(k_bph_nodes, dim3(xcd_grid(b->nNode)), dim3(256), 0, st, b->dI, b->dNode, b->nNode, s, inU, inJ,
                     x, xd, dt, b->flags);
  // the flux list holds the direction-1 tiles; the direction-0 tiles form the update
  hipLaunchKernelGGL((k_bph_flux<C::X0, C::Y0, C::X1, C::Y1, C::OCC>), dim3(xcd_grid(b->nFlux)), dim3(256), 0, st,
                     b->dI, b->dFlux, b->nFlux, b->flags);
  hipLaunchKernelGGL(k_bph_fupd, dim3(xcd_grid(b->nFU)), dim3(256), 0, st, b->dI, b->dFU, b->nFU, s, bU, bJ, inU, inJ,
                     outU, outJ, x, xd, dt, b->flags);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

static int launch_stage(esvdw_batch *b, int s, const double *bU, const double *bJ, const double *inU,
                        const double *inJ, double *outU, double *outJ, double *x, const double *xd, double *dt,
                        hipStream_t st) {
  switch (b->variant) {
    case 0: return launch_stage_v<0>(b, s, bU, bJ, inU, inJ, outU, outJ, x, xd, dt, st);
    case 1: return launch_stage_v<1>(b, s, bU, bJ, inU, inJ, outU, outJ, x, xd, dt, st);
    case 2: return launch_stage_v<2>(b, s, bU, bJ, inU, inJ, outU, outJ, x, xd, dt, st);
    case 3: return launch_stage_v<3>(b, s, bU, bJ, inU, inJ, outU, outJ, x, xd, dt, st);
    case 4: return launch_stage_v<4>(b, s, bU, bJ, inU, inJ, outU, outJ, x, xd, dt, st);
    case 5: return launch_phased_v<0>(b, s, bU, bJ, inU, inJ, outU, outJ, x, xd, dt, st);
    case 6: return launch_phased_v<1>(b, s, bU, bJ, inU, inJ, outU, outJ, x, xd, dt, st);
    case 7: return launch_phased_v<2>(b, s, bU, bJ, inU, inJ, outU, outJ, x, xd, dt, st);
    case 8: return launch_phased_v<3>(b, s, bU, bJ, inU, inJ, outU, outJ, x, xd, dt, st);
    default: return launch_phased_v<4>(b, s, bU, bJ, inU, inJ, outU, outJ, x, xd, dt, st);
  }
}

// flux tiles of tile set V: both directions, or (dir0 false) direction 1 only
template <int V> static void flux_items(const esvdw_batch *b, std::vector<BItem> &v, bool dir0) {
  using C = BVar<V>;
  v.clear();
  for (int i = 0; i < b->ninst; ++i) {
    const Geo &G = b->geo[i];
    if (dir0)
      for (int y = 0; y < G.n[1]; y += C::Y0)
        for (int x = 0; x < G.n[0] + 1; x += C::X0) v.push_back({i, x, y, 0});
    for (int y = 0; y < G.n[1] + 1; y += C::Y1)
      for (int x = 0; x < G.n[0]; x += C::X1) v.push_back({i, x, y, 1});
  }
}

// a device copy of a work list (replacing *d)
static int upload_items(BItem **d, int *n, const std::vector<BItem> &items) {
  if (*d) (void)hipFree(*d);
  *d = nullptr;
  *n = 0;
  if (items.empty()) return 1;
  if (!HIPOK(hipMalloc((void **)d, items.size() * sizeof(BItem)))) return 0;
  if (!HIPOK(hipMemcpy(*d, items.data(), items.size() * sizeof(BItem), hipMemcpyHostToDevice))) return 0;
  *n = (int)items.size();
  return 1;
}

static int set_flux_items(esvdw_batch *b, int v) {
  std::vector<BItem> items, fu;
  const bool phased = v >= BATCH_NTILE;  // the phased mode fuses the direction-0 fluxes into the update
  switch (v % BATCH_NTILE) {
    case 0: flux_items<0>(b, items, !phased); break;
    case 1: flux_items<1>(b, items, !phased); break;
    case 2: flux_items<2>(b, items, !phased); break;
    case 3: flux_items<3>(b, items, !phased); break;
    default: flux_items<4>(b, items, !phased); break;
  }
  if (phased)
    for (int i = 0; i < b->ninst; ++i) {  // tiles of FU_TX interfaces stepping by FU_TX - 1 nodes
      const Geo &G = b->geo[i];
      for (int y = 0; y < G.n[1]; y += FU_TY)
        for (int x = 0; x < G.n[0]; x += FU_TX - 1) fu.push_back({i, x, y, 0});
    }
  if (!upload_items(&b->dFlux, &b->nFlux, items) || !upload_items(&b->dFU, &b->nFU, fu)) return 0;
  b->variant = v;
  return 1;
}

template <typename T> static int balloc(T **p, size_t n) {
  *p = nullptr;
  return n == 0 ? 1 : HIPOK(hipMalloc((void **)p, n * sizeof(T)));
}

extern "C" {

void esvdw_batch_destroy(esvdw_batch *b) {
  if (!b) return;
  void *bufs[] = {b->dI,  b->dNode, b->dFlux, b->dUpd, b->dFU, b->nd_pool, b->f_pool, b->sAU,  b->sAJ,
                  b->sBU, b->sBJ,   b->cpart, b->bar,  b->flags,   b->rg,     b->term, b->omA,
                  b->omB, b->xa,    b->xb,    b->part3, b->monmax, b->gam};
  for (void *p : bufs)
    if (p) (void)hipFree(p);
  delete b;
}

int esvdw_batch_create(int ninst, const esvdw_params *params, esvdw_batch **out) {
  if (!out) return ESVDW_EINVAL;
  *out = nullptr;
  if (ninst < 1 || !params) return ESVDW_EINVAL;
  for (int i = 0; i < ninst; ++i)
    if (!params_valid(&params[i]) || params[i].dim != 2 || params[i].walls != 0 || params[i].step[0] != 0 ||
        params[i].step[1] != 0 || params[i].inflow != 0)
      return ESVDW_EINVAL;
  esvdw_batch *b = new esvdw_batch();
  b->ninst = ninst;
  (void)hipGetDevice(&b->dev);
  b->geo.resize(ninst);
  b->off.assign(ninst + 1, 0);
  b->inst.resize(ninst);
  long nd_total = 0, f_total = 0;
  std::vector<BItem> node_items, upd_items;
  for (int i = 0; i < ninst; ++i) {
    Geo &G = b->geo[i];
    make_geo(&params[i], &G);
    b->off[i + 1] = b->off[i] + G.N;
    BInst &B = b->inst[i];
    memset(&B, 0, sizeof(B));
    B.G = G;
    B.off = b->off[i];
    B.nif0 = (long)(G.n[0] + 1) * G.n[1];
    B.nif1 = (long)G.n[0] * (G.n[1] + 1);
    B.cfl = params[i].cfl;
    B.dt_fixed = params[i].dt_fixed;
    B.mkind = params[i].monitor_kind;
    B.kappa = params[i].kappa;
    B.var0 = params[i].mon_var[0];
    B.var1 = params[i].mon_var[1];
    B.nterm = B.mkind == ESVDW_MON_VDW ? B.kappa + 1 : 2;
    for (int q = 0; q < 3; ++q) B.alpha[q] = params[i].alpha[q];
    nd_total += (long)NF_<2>::COUNT * G.PN;
    f_total += 5 * (B.nif0 + B.nif1);
    for (long t = 0; t < (long)G.E0 * G.P[1]; t += 256) node_items.push_back({i, (int)t, 0, 0});
    B.u0 = (int)upd_items.size();
    for (long t = 0; t < G.N; t += 256) upd_items.push_back({i, (int)t, 0, 0});
    B.u1 = (int)upd_items.size();
  }
  const long total = b->off[ninst];
  bool ok = balloc(&b->nd_pool, nd_total + 16) && balloc(&b->f_pool, f_total) && balloc(&b->sAU, 4 * total) &&
            balloc(&b->sAJ, total) && balloc(&b->sBU, 4 * total) && balloc(&b->sBJ, total) &&
            balloc(&b->cpart, upd_items.size()) && balloc(&b->bar, 2) && balloc(&b->flags, 1) &&
            balloc(&b->dI, ninst) && balloc(&b->dNode, node_items.size()) && balloc(&b->dUpd, upd_items.size()) &&
            balloc(&b->rg, 2 * total) && balloc(&b->term, 3 * total) && balloc(&b->omA, total) &&
            balloc(&b->omB, total) && balloc(&b->xa, 2 * total) && balloc(&b->xb, 2 * total) &&
            balloc(&b->part3, 3 * upd_items.size()) && balloc(&b->monmax, 3 * (size_t)ninst) &&
            balloc(&b->gam, ninst);
  // the batched redistribution runs a fixed number of filter passes and Jacobi sweeps for all
  // instances: it is available when they agree on both
  b->n_filter = params[0].n_filter;
  b->mu = params[0].mu;
  b->redist_ok = 1;
  for (int i = 0; i < ninst; ++i)
    if (params[i].n_filter != b->n_filter || params[i].mu != b->mu || !params[i].fixed_mu) b->redist_ok = 0;
  if (ok) {
    // each instance's node buffer: PN is a multiple of 16 doubles, so starting the first at
    // 16 - g0 puts node g0 of every row of every instance at the start of a 128-byte line
    long nd_off = (16 - GH) % 16, f_off = 0;
    for (int i = 0; i < ninst; ++i) {
      BInst &B = b->inst[i];
      B.nd = b->nd_pool + nd_off;
      nd_off += (long)NF_<2>::COUNT * B.G.PN;
      B.F0 = b->f_pool + f_off;
      B.F1 = B.F0 + 5 * B.nif0;
      f_off += 5 * (B.nif0 + B.nif1);
    }
    b->nNode = (int)node_items.size();
    b->nUpd = (int)upd_items.size();
    ok = HIPOK(hipMemcpy(b->dI, b->inst.data(), ninst * sizeof(BInst), hipMemcpyHostToDevice)) &&
         HIPOK(hipMemcpy(b->dNode, node_items.data(), node_items.size() * sizeof(BItem), hipMemcpyHostToDevice)) &&
         HIPOK(hipMemcpy(b->dUpd, upd_items.data(), upd_items.size() * sizeof(BItem), hipMemcpyHostToDevice)) &&
         HIPOK(hipMemset(b->bar, 0, 2 * sizeof(unsigned))) && HIPOK(hipMemset(b->flags, 0, sizeof(unsigned)));
  }
  if (ok) {
    int ncu = 0;
    ok = HIPOK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->dev)) && ncu > 0;
    if (ok) {
      b->nblocks[0] = stage_blocks<0>(ncu);
      b->nblocks[1] = stage_blocks<1>(ncu);
      b->nblocks[2] = stage_blocks<2>(ncu);
      b->nblocks[3] = stage_blocks<3>(ncu);
      b->nblocks[4] = stage_blocks<4>(ncu);
      for (int v = 0; v < BATCH_NTILE; ++v) ok = ok && b->nblocks[v] >= 8;
    }
  }
  ok = ok && set_flux_items(b, 0) && HIPOK(hipDeviceSynchronize());
  if (!ok) {
    esvdw_batch_destroy(b);
    return ESVDW_EHIP;
  }
  *out = b;
  return ESVDW_OK;
}

long esvdw_batch_offsets(const esvdw_batch *b, long *off) {
  if (!b) return -1;
  if (off)
    for (int i = 0; i <= b->ninst; ++i) off[i] = b->off[i];
  return b->off[b->ninst];
}

int esvdw_batch_variants(void) { return BATCH_NVAR; }

int esvdw_batch_set_variant(esvdw_batch *b, int v) {
  if (!b || v < 0 || v >= BATCH_NVAR) return ESVDW_EINVAL;
  if (v == b->variant) return ESVDW_OK;
  if (!HIPOK(hipDeviceSynchronize())) return ESVDW_EHIP;
  return set_flux_items(b, v) ? ESVDW_OK : ESVDW_EHIP;
}

int esvdw_batch_get_status(esvdw_batch *b, unsigned *flags_host) {
  if (!b || !flags_host) return ESVDW_EINVAL;
  if (!HIPOK(hipDeviceSynchronize())) return ESVDW_EHIP;
  if (!HIPOK(hipMemcpy(flags_host, b->flags, sizeof(unsigned), hipMemcpyDeviceToHost))) return ESVDW_EHIP;
  return HIPOK(hipMemset(b->flags, 0, sizeof(unsigned))) ? ESVDW_OK : ESVDW_EHIP;
}

int esvdw_batch_init_mesh(esvdw_batch *b, double *x, double *J, hipStream_t st) {
  if (!b || !x || !J) return ESVDW_EINVAL;
  for (int i = 0; i < b->ninst; ++i) {
    esvdw_ctx c;
    memset(&c, 0, sizeof(c));
    c.G = b->geo[i];
    if (launch_uniform_mesh(&c, x + 2 * b->off[i], st)) return ESVDW_EHIP;
    if (launch_metrics(&c, x + 2 * b->off[i], nullptr, nullptr, nullptr, J + b->off[i], st)) return ESVDW_EHIP;
  }
  return ESVDW_OK;
}

int esvdw_batch_init_state(esvdw_batch *b, const double *prim, const double *J, double *JU, hipStream_t st) {
  if (!b || !prim || !J || !JU) return ESVDW_EINVAL;
  for (int i = 0; i < b->ninst; ++i) {
    esvdw_ctx c;
    memset(&c, 0, sizeof(c));
    c.G = b->geo[i];
    if (launch_init_state(&c, prim + 4 * b->off[i], J + b->off[i], JU + 4 * b->off[i], st)) return ESVDW_EHIP;
  }
  return ESVDW_OK;
}

int esvdw_batch_stage(esvdw_batch *b, int s, const double *JU0, const double *J0, const double *JUs,
                      const double *Js, double *JUout, double *Jout, double *x, const double *xdot, double *dt,
                      hipStream_t st) {
  if (!b || s < 0 || s > 2 || !JU0 || !J0 || !JUs || !Js || !JUout || !Jout || !x || !dt) return ESVDW_EINVAL;
  if (JUout == JUs || Jout == Js) return ESVDW_EINVAL;
  return launch_stage(b, s, JU0, J0, JUs, Js, JUout, Jout, x, xdot, dt, st) ? ESVDW_EHIP : ESVDW_OK;
}

int esvdw_batch_redistribute(esvdw_batch *b, const double *JU, const double *J, const double *x, double *xdot,
                             double *dt, hipStream_t st) {
  if (!b || !JU || !J || !x || !xdot || !dt) return ESVDW_EINVAL;
  if (!b->redist_ok) return ESVDW_EINVAL;
  const unsigned gu = xcd_grid(b->nUpd);
  const int ni = b->ninst, nu = b->nUpd;
  hipLaunchKernelGGL(k_bm_rhoG, dim3(gu), dim3(256), 0, st, b->dI, b->dUpd, nu, JU, J, b->rg);
  hipLaunchKernelGGL(k_bm_terms, dim3(gu), dim3(256), 0, st, b->dI, b->dUpd, nu, b->rg, b->term, b->part3);
  hipLaunchKernelGGL(k_bm_max3, dim3(ni), dim3(256), 0, st, b->dI, b->part3, nu, b->monmax);
  double *cur = b->omA, *oth = b->omB;
  hipLaunchKernelGGL(k_bm_omega, dim3(gu), dim3(256), 0, st, b->dI, b->dUpd, nu, b->term, b->monmax, cur);
  for (int i = 0; i < b->n_filter; ++i) {
    hipLaunchKernelGGL(k_bm_filter, dim3(gu), dim3(256), 0, st, b->dI, b->dUpd, nu, cur, oth);
    double *tmp = cur;
    cur = oth;
    oth = tmp;
  }
  // Jacobi from x^[0] = x^n, ping-pong between the batch's two mesh buffers
  const double *xin = x;
  double *xo = b->xa;
  for (int k = 0; k < b->mu; ++k) {
    hipLaunchKernelGGL(k_bm_jacobi, dim3(gu), dim3(256), 0, st, b->dI, b->dUpd, nu, cur, xin, xo);
    xin = xo;
    xo = xo == b->xa ? b->xb : b->xa;
  }
  hipLaunchKernelGGL(k_bm_limiter, dim3(gu), dim3(256), 0, st, b->dI, b->dUpd, nu, x, xin, b->part3);
  hipLaunchKernelGGL(k_bm_min, dim3(ni), dim3(256), 0, st, b->dI, b->part3, b->gam);
  hipLaunchKernelGGL(k_bph_cfl, dim3(gu), dim3(256), 0, st, b->dI, b->dUpd, nu, JU, J, x, b->cpart);
  hipLaunchKernelGGL(k_bph_dt, dim3(ni), dim3(256), 0, st, b->dI, b->cpart, dt);
  hipLaunchKernelGGL(k_bm_xdot, dim3(gu), dim3(256), 0, st, b->dI, b->dUpd, nu, x, xin, b->gam, dt, xdot);
  return hipGetLastError() == hipSuccess ? ESVDW_OK : ESVDW_EHIP;
}

int esvdw_batch_step(esvdw_batch *b, double *JU, double *J, double *x, const double *xdot, double *dt,
                     hipStream_t st) {
  if (!b || !JU || !J || !x || !dt) return ESVDW_EINVAL;
  if (launch_stage(b, 0, JU, J, JU, J, b->sAU, b->sAJ, x, xdot, dt, st)) return ESVDW_EHIP;
  if (launch_stage(b, 1, JU, J, b->sAU, b->sAJ, b->sBU, b->sBJ, x, xdot, dt, st)) return ESVDW_EHIP;
  if (launch_stage(b, 2, JU, J, b->sBU, b->sBJ, JU, J, x, xdot, dt, st)) return ESVDW_EHIP;
  return ESVDW_OK;
}

}  // extern "C"
