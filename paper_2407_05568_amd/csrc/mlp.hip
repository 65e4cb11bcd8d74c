// mlp.hip -- learned warm start for the mesh equations: a 50 -> 64 -> 64 -> 2 ReLU MLP on
// the 5x5 stencil of two node features (normalised |grad_xi rho|^2 and tanh G) proposes the
// displacement x* - x^n of the converged mesh (in units of dxi).  BF16 operands, FP32
// accumulation on the matrix cores (v_mfma_f32_16x16x16_bf16); inference and training
// (forward, backward, Adam) are hand-written here.
#include "common.h"
#include "kernels.h"

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// packed parameters (floats): W[k][j] maps input k to output j; paddings stay zero
#define MLP_IN 50
#define MLP_H 64
#define MLP_OUT 2
#define OFF_W1 0      // 64 x 64 (rows >= 50 unused)
#define OFF_B1 4096   // 64
#define OFF_W2 4160   // 64 x 64
#define OFF_B2 8256   // 64
#define OFF_W3 8320   // 64 x 16 (columns >= 2 unused)
#define OFF_B3 9344   // 16
#define MLP_NP 9360

__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

// A operand: element (r, k) = base[r * rs + k * cs], r = lane % 16, k = k0 + 4 (lane / 16) + q
__device__ __forceinline__ bf4 frag_a(const unsigned short *base, int rs, int cs, int k0, int lane) {
  int r = lane & 15, k = k0 + ((lane >> 4) << 2);
  bf4 v;
  v.x = (short)base[r * rs + k * cs];
  v.y = (short)base[r * rs + (k + 1) * cs];
  v.z = (short)base[r * rs + (k + 2) * cs];
  v.w = (short)base[r * rs + (k + 3) * cs];
  return v;
}
// B operand: element (k, n) = base[k * rs + n * cs], n = n0 + lane % 16, k = k0 + 4 (lane / 16) + q
__device__ __forceinline__ bf4 frag_b(const unsigned short *base, int rs, int cs, int k0, int n0, int lane) {
  int n = n0 + (lane & 15), k = k0 + ((lane >> 4) << 2);
  bf4 v;
  v.x = (short)base[k * rs + n * cs];
  v.y = (short)base[(k + 1) * rs + n * cs];
  v.z = (short)base[(k + 2) * rs + n * cs];
  v.w = (short)base[(k + 3) * rs + n * cs];
  return v;
}
// LDS hand-off between lanes of one wave (every wave runs its own trip count, so block-wide
// barriers cannot be used here)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// D fragment element r sits at row 4 (lane / 16) + r, column n0 + lane % 16
__device__ __forceinline__ f4 mfma16(bf4 a, bf4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }

struct MlpLds {
  unsigned short W1[64 * 64], W2[64 * 64], W3[64 * 16];
  float b1[64], b2[64], b3[16];
};

__device__ __forceinline__ void load_weights(MlpLds &s, const float *__restrict__ P, int tid, int nt) {
  for (int i = tid; i < 64 * 64; i += nt) {
    s.W1[i] = f2bf(P[OFF_W1 + i]);
    s.W2[i] = f2bf(P[OFF_W2 + i]);
  }
  for (int i = tid; i < 64 * 16; i += nt) s.W3[i] = f2bf(P[OFF_W3 + i]);
  for (int i = tid; i < 64; i += nt) {
    s.b1[i] = P[OFF_B1 + i];
    s.b2[i] = P[OFF_B2 + i];
  }
  for (int i = tid; i < 16; i += nt) s.b3[i] = P[OFF_B3 + i];
}

// feature k of node (i0, i1): (dy, dx) = (k / 10 - 2, (k % 10) / 2 - 2), channel k % 2, boundary
// values replicated; feat = [f1 field | f2 field] for one frame
__device__ __forceinline__ float feature(const Geo &G, const float *__restrict__ feat, int i0, int i1, int k) {
  int dy = k / 10 - 2, dx = (k % 10) / 2 - 2, ch = k & 1;
  long s = state_index(G, i0 + dx, i1 + dy, 0);
  return feat[ch * G.N + s];
}

// forward pass of one group of 16 samples (rows) held by one wave: X (16 x 64) -> H1 -> H2 ->
// y (16 x 16, columns 0..1 meaningful).  Returns this lane's 4 output elements (rows
// 4 (lane/16) + r, column lane % 16).
__device__ __forceinline__ f4 forward16(const MlpLds &s, const unsigned short *sX, unsigned short *sH1,
                                        unsigned short *sH2, int lane) {
  const int rb = (lane >> 4) << 2, col = lane & 15;
  for (int nt = 0; nt < 4; ++nt) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < 4; ++kt) acc = mfma16(frag_a(sX, 64, 1, kt * 16, lane), frag_b(s.W1, 64, 1, kt * 16, nt * 16, lane), acc);
    for (int r = 0; r < 4; ++r) sH1[(rb + r) * 64 + nt * 16 + col] = f2bf(fmaxf(acc[r] + s.b1[nt * 16 + col], 0.f));
  }
  wave_sync();
  for (int nt = 0; nt < 4; ++nt) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < 4; ++kt) acc = mfma16(frag_a(sH1, 64, 1, kt * 16, lane), frag_b(s.W2, 64, 1, kt * 16, nt * 16, lane), acc);
    for (int r = 0; r < 4; ++r) sH2[(rb + r) * 64 + nt * 16 + col] = f2bf(fmaxf(acc[r] + s.b2[nt * 16 + col], 0.f));
  }
  wave_sync();
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int kt = 0; kt < 4; ++kt) acc = mfma16(frag_a(sH2, 64, 1, kt * 16, lane), frag_b(s.W3, 16, 1, kt * 16, 0, lane), acc);
  for (int r = 0; r < 4; ++r) acc[r] += s.b3[col];
  return acc;
}

// ---- per-node features: f1 = |grad_xi rho|^2 / max, f2 = tanh G --------------------------
__global__ void k_mlp_feat(Geo G, const double *__restrict__ rg, const double *__restrict__ term,
                           const double *__restrict__ scal, float *__restrict__ feat) {
  NODE_COORDS(G.n[0], G.n[1]);
  if (!inside) return;
  const long t = lin(G, i0, i1, i2);
  double m = scal[SC_MON];
  feat[t] = (float)(m > 0.0 ? term[t] / m : 0.0);
  feat[G.N + t] = (float)tanh(rg[G.N + t]);
}

// ---- inference: warm_dx = dxi * y, clipped to +-64 dxi ------------------------------------
__global__ void __launch_bounds__(256) k_mlp_infer(Geo G, const float *__restrict__ feat, const float *__restrict__ P,
                                                   double *__restrict__ warm) {
  __shared__ MlpLds s;
  __shared__ unsigned short sX[4][16 * 64], sH1[4][16 * 64], sH2[4][16 * 64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  load_weights(s, P, tid, 256);
  __syncthreads();
  const long ngroups = (G.N + 15) / 16;
  for (long g = (long)blockIdx.x * 4 + w; g < ngroups; g += (long)gridDim.x * 4) {
    // gather the 16 x 64 feature tile (zero padding beyond 50 features and past the last node)
    for (int e = lane; e < 16 * 64; e += 64) {
      int r = e >> 6, k = e & 63;
      long node = g * 16 + r;
      float v = 0.f;
      if (k < MLP_IN && node < G.N) {
        int a0 = (int)(node % G.n[0]), a1 = (int)(node / G.n[0]);
        v = feature(G, feat, a0, a1, k);
      }
      sX[w][e] = f2bf(v);
    }
    wave_sync();
    f4 y = forward16(s, sX[w], sH1[w], sH2[w], lane);
    const int rb = (lane >> 4) << 2, col = lane & 15;
    if (col < MLP_OUT) {
      for (int r = 0; r < 4; ++r) {
        long node = g * 16 + rb + r;
        if (node < G.N) {
          double d = G.dxi[col] * (double)y[r];
          d = fmin(fmax(d, -64.0 * G.dxi[col]), 64.0 * G.dxi[col]);
          warm[(long)col * G.N + node] = d;
        }
      }
    }
    wave_sync();
  }
}

// ---- training: forward + backward over a sample list, gradients into grad -------------------
// samples[2 s] = frame, samples[2 s + 1] = node; feats: frame-major [f][2][N]; tgt: [f][2][N]
__global__ void __launch_bounds__(256) k_mlp_grad(Geo G, const float *__restrict__ feats, const float *__restrict__ tgt,
                                                  const int *__restrict__ samples, long nsamp, float scale,
                                                  const float *__restrict__ P, float *grad, float *loss) {
  __shared__ MlpLds s;
  __shared__ float sG[MLP_NP];
  __shared__ unsigned short sX[4][16 * 64], sH1[4][16 * 64], sH2[4][16 * 64], sD1[4][16 * 64], sD2[4][16 * 64],
      sD3[4][16 * 16];
  __shared__ float sLoss;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  load_weights(s, P, tid, 256);
  for (int i = tid; i < MLP_NP; i += 256) sG[i] = 0.f;
  if (tid == 0) sLoss = 0.f;
  __syncthreads();
  const int rb = (lane >> 4) << 2, col = lane & 15;
  const long ngroups = (nsamp + 15) / 16;
  float myloss = 0.f;
  for (long g = (long)blockIdx.x * 4 + w; g < ngroups; g += (long)gridDim.x * 4) {
    for (int e = lane; e < 16 * 64; e += 64) {
      int r = e >> 6, k = e & 63;
      long sidx = g * 16 + r;
      float v = 0.f;
      if (k < MLP_IN && sidx < nsamp) {
        int f = samples[2 * sidx], node = samples[2 * sidx + 1];
        int a0 = node % G.n[0], a1 = node / G.n[0];
        v = feature(G, feats + (long)f * 2 * G.N, a0, a1, k);
      }
      sX[w][e] = f2bf(v);
    }
    wave_sync();
    f4 y = forward16(s, sX[w], sH1[w], sH2[w], lane);
    // dL/dy for L = scale * sum (y - t)^2 over the two outputs
    for (int r = 0; r < 4; ++r) {
      long sidx = g * 16 + rb + r;
      float d = 0.f;
      if (col < MLP_OUT && sidx < nsamp) {
        int f = samples[2 * sidx], node = samples[2 * sidx + 1];
        float e = y[r] - tgt[((long)f * 2 + col) * G.N + node];
        myloss += scale * e * e;
        d = 2.f * scale * e;
      }
      sD3[w][(rb + r) * 16 + col] = f2bf(d);
    }
    wave_sync();
    // dW3 (64 x 16) += H2^T dY ;  db3 += column sums of dY
    for (int mt = 0; mt < 4; ++mt) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma16(frag_a(sH2[w] + mt * 16, 1, 64, 0, lane), frag_b(sD3[w], 16, 1, 0, 0, lane), acc);
      for (int r = 0; r < 4; ++r) atomicAdd(&sG[OFF_W3 + (mt * 16 + rb + r) * 16 + col], acc[r]);
    }
    if (lane < 16) {
      float a = 0.f;
      for (int r = 0; r < 16; ++r) a += bf2f(sD3[w][r * 16 + lane]);
      atomicAdd(&sG[OFF_B3 + lane], a);
    }
    // dH2 = dY W3^T, masked by H2 > 0
    for (int nt = 0; nt < 4; ++nt) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma16(frag_a(sD3[w], 16, 1, 0, lane), frag_b(s.W3, 1, 16, 0, nt * 16, lane), acc);
      for (int r = 0; r < 4; ++r) {
        int e = (rb + r) * 64 + nt * 16 + col;
        sD2[w][e] = f2bf(sH2[w][e] != 0 ? acc[r] : 0.f);
      }
    }
    wave_sync();
    // dW2 += H1^T dH2 ; db2
    for (int mt = 0; mt < 4; ++mt)
      for (int nt = 0; nt < 4; ++nt) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma16(frag_a(sH1[w] + mt * 16, 1, 64, 0, lane), frag_b(sD2[w], 64, 1, 0, nt * 16, lane), acc);
        for (int r = 0; r < 4; ++r) atomicAdd(&sG[OFF_W2 + (mt * 16 + rb + r) * 64 + nt * 16 + col], acc[r]);
      }
    {
      float a = 0.f;
      for (int r = 0; r < 16; ++r) a += bf2f(sD2[w][r * 64 + lane]);
      atomicAdd(&sG[OFF_B2 + lane], a);
    }
    // dH1 = dH2 W2^T, masked by H1 > 0
    for (int nt = 0; nt < 4; ++nt) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int kt = 0; kt < 4; ++kt)
        acc = mfma16(frag_a(sD2[w], 64, 1, kt * 16, lane), frag_b(s.W2, 1, 64, kt * 16, nt * 16, lane), acc);
      for (int r = 0; r < 4; ++r) {
        int e = (rb + r) * 64 + nt * 16 + col;
        sD1[w][e] = f2bf(sH1[w][e] != 0 ? acc[r] : 0.f);
      }
    }
    wave_sync();
    // dW1 += X^T dH1 ; db1
    for (int mt = 0; mt < 4; ++mt)
      for (int nt = 0; nt < 4; ++nt) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma16(frag_a(sX[w] + mt * 16, 1, 64, 0, lane), frag_b(sD1[w], 64, 1, 0, nt * 16, lane), acc);
        for (int r = 0; r < 4; ++r) atomicAdd(&sG[OFF_W1 + (mt * 16 + rb + r) * 64 + nt * 16 + col], acc[r]);
      }
    {
      float a = 0.f;
      for (int r = 0; r < 16; ++r) a += bf2f(sD1[w][r * 64 + lane]);
      atomicAdd(&sG[OFF_B1 + lane], a);
    }
    wave_sync();
  }
  atomicAdd(&sLoss, myloss);
  __syncthreads();
  for (int i = tid; i < MLP_NP; i += 256)
    if (sG[i] != 0.f) atomicAdd(&grad[i], sG[i]);
  if (tid == 0) atomicAdd(loss, sLoss);
}

__global__ void k_fill_f(float *p, long n, float v) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

// Adam (FP32 master weights); padded entries keep zero gradients and stay zero
__global__ void k_mlp_adam(float *__restrict__ P, const float *__restrict__ grad, float *__restrict__ m,
                           float *__restrict__ v, int step, float lr, float b1, float b2, float eps) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MLP_NP) return;
  float g = grad[i];
  float mi = b1 * m[i] + (1.f - b1) * g, vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  float mh = mi / (1.f - powf(b1, (float)step)), vh = vi / (1.f - powf(b2, (float)step));
  P[i] -= lr * mh / (sqrtf(vh) + eps);
}

// ---- launchers -------------------------------------------------------------------------------
int launch_mlp_infer(esvdw_ctx *c, const float *feat, const float *P, double *warm, hipStream_t st) {
  if (c->G.dim != 2) return -1;
  long ngroups = (c->G.N + 15) / 16;
  unsigned nb = (unsigned)((ngroups + 3) / 4);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_mlp_infer, dim3(nb), dim3(256), 0, st, c->G, feat, P, warm);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_mlp_grad(esvdw_ctx *c, const float *feats, const float *tgt, const int *samples, long nsamp, float scale,
                    const float *P, float *grad, float *loss, hipStream_t st) {
  if (c->G.dim != 2) return -1;
  hipLaunchKernelGGL(k_fill_f, dim3((MLP_NP + 255) / 256), dim3(256), 0, st, grad, (long)MLP_NP, 0.f);
  hipLaunchKernelGGL(k_fill_f, dim3(1), dim3(64), 0, st, loss, 1L, 0.f);
  long ngroups = (nsamp + 15) / 16;
  unsigned nb = (unsigned)((ngroups + 3) / 4);
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(256), 0, st, c->G, feats, tgt, samples, nsamp, scale, P, grad, loss);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_mlp_adam(float *P, const float *grad, float *m, float *v, int step, float lr, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NP + 255) / 256), dim3(256), 0, st, P, grad, m, v, step, lr, 0.9f, 0.999f,
                     1e-8f);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_mlp_feat(esvdw_ctx *c, const double *JU, const double *J, float *feat, hipStream_t st) {
  if (launch_grad_rho_terms(c, JU, J, st)) return -1;
  dim3 b, g;
  node_grid(c->G.n[0], c->G.n[1], c->G.n[2], g, b);
  hipLaunchKernelGGL(k_mlp_feat, g, b, 0, st, c->G, c->rhoG, c->mterm, c->scal, feat);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
