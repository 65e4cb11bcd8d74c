// scheme.h -- device-level building blocks of the entropy-stable moving-mesh scheme
// (Sections 3.1-3.3 and the CFL condition of Section 5), shared by the single-problem
// kernels and the batched persistent stage kernel:
//   node_point    per padded node: primitives, 1/T, logarithms, entropy variable, metrics
//   flux_tile     one 256-thread tile of interfaces: sixth-order EC flux + MR-WENO dissipation
//   update_point  flux differences and the SSP-RK3 stage combination at one node
//   cfl_rate      sum over directions of the spectral radius over J dxi at one node
#pragma once
#include "common.h"

// =============================== node data =======================================

// Metrics given at interior nodes only (es_rhs): ghost values by the boundary symmetry.
// Outflow mirror normal to q flips J dxi_k/dx_j iff exactly one of k, j is q, and J dxi_k/dt iff k = q.
__device__ __forceinline__ long ghost_metric_src(const Geo &G, int i0, int i1, int i2, unsigned &mirror) {
  int ii[3] = {i0, i1, i2};
  mirror = 0;
  for (int q = 0; q < G.dim; ++q) {
    int i = ii[q], n = G.n[q];
    if (i >= 0 && i < n) continue;
    if (G.bc[q] == ESVDW_BC_PERIODIC) {
      ii[q] = i - floordiv(i, n) * n;
    } else {
      ii[q] = i < 0 ? -1 - i : 2 * n - 1 - i;
      mirror |= 1u << q;
    }
  }
  return lin(G, ii[0], ii[1], ii[2]);
}

// thermodynamic node data (everything but the metrics) of node (i0, i1, i2) into slot t of
// the node buffer nd
template <int D>
__device__ __forceinline__ void node_state(const Geo &G, const double *__restrict__ JU, const double *__restrict__ J,
                                           double *__restrict__ nd, unsigned *flags, long t, int i0, int i1, int i2) {
  using F = NF_<D>;
  long s = state_index(G, i0, i1, i2);
  double iJ = 1.0 / J[s];
  double rho = JU[s] * iJ;
  double irho = 1.0 / rho;
  double v[D], v2 = 0.0;
#pragma unroll
  for (int m = 0; m < D; ++m) {
    v[m] = JU[(long)(1 + m) * G.N + s] * iJ * irho;
    v2 += v[m] * v[m];
  }
  if (G.walls) {  // a ghost beyond a wall face carries the mirrored velocity
    const int ii[3] = {i0, i1, i2};
#pragma unroll
    for (int q = 0; q < D; ++q)
      if ((ii[q] < 0 && (G.walls & ESVDW_WALL_LO(q))) || (ii[q] >= G.n[q] && (G.walls & ESVDW_WALL_HI(q))))
        v[q] = -v[q];
  }
  double e = JU[(long)(D + 1) * G.N + s] * iJ * irho - 0.5 * v2;
  if (G.inflow && i0 < 0) {  // the inflow face's ghost layers hold the fixed inflow state
    rho = G.qin[0];
    irho = 1.0 / rho;
    v2 = 0.0;
#pragma unroll
    for (int m = 0; m < D; ++m) {
      v[m] = G.qin[1 + m];
      v2 += v[m] * v[m];
    }
    e = G.cv * G.qin[3] - G.a * rho;
  }
  double T = (e + G.a * rho) / G.cv;
  double iT = 1.0 / T;
  double ob = 1.0 - G.b * rho;
  double iob = 1.0 / ob;
  double p = rho * G.R * T * iob - G.a * rho * rho;
  bool interior = (i0 >= 0 && i0 < G.n[0]) && (i1 >= 0 && i1 < G.n[1]) && (i2 >= 0 && i2 < G.n[2]);
  if (interior && !admissible(G, rho, T)) raise_flag(flags, ESVDW_F_INADMISSIBLE);
  double lnr = log(rho), lnb = log(ob), lnt = log(T), lnp = log(p);
  nd[F::RHO * G.PN + t] = rho;
#pragma unroll
  for (int m = 0; m < D; ++m) nd[(long)(F::V + m) * G.PN + t] = v[m];
  nd[F::T * G.PN + t] = T;
  nd[F::P * G.PN + t] = p;
  nd[F::IT * G.PN + t] = iT;
  nd[F::IOB * G.PN + t] = iob;
  nd[F::LNR * G.PN + t] = lnr;
  nd[F::LNB * G.PN + t] = lnb;
  nd[F::LNT * G.PN + t] = lnt;
  nd[F::LNP * G.PN + t] = lnp;
  // entropy variables: V = (-s + (e + p/rho - |v|^2/2)/T, v/T, -1/T), s = c_v ln T + R ln(1/rho - b)
  double sent = G.cv * lnt + G.R * (lnb - lnr);
  nd[(long)F::V1 * G.PN + t] = -sent + (e + p * irho - 0.5 * v2) * iT;
}

// metrics of slot t of the node buffer: m[k][j] = J dxi_k/dx_j, and J dxi_k/dt = -xv . m[k]
template <int D>
__device__ __forceinline__ void node_metrics_store(const Geo &G, double *__restrict__ nd, long t, const double (&m)[D][D],
                                                   const double (&xv)[D]) {
  using F = NF_<D>;
#pragma unroll
  for (int k = 0; k < D; ++k)
#pragma unroll
    for (int j = 0; j < D; ++j) nd[(long)(F::MS + k * D + j) * G.PN + t] = m[k][j];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    double s2 = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) s2 -= xv[j] * m[k][j];
    nd[(long)(F::XS + k) * G.PN + t] = s2;
  }
}

// node data of padded node (p0, p1, p2) into the node buffer nd
template <int D>
__device__ __forceinline__ void node_point(const Geo &G, const double *__restrict__ JU, const double *__restrict__ J,
                                           const double *__restrict__ met_in, const double *__restrict__ xit_in,
                                           const double *__restrict__ xn, const double *__restrict__ xd, double cdt,
                                           const double *__restrict__ dp, long dpN, double *__restrict__ nd,
                                           unsigned *flags, int p0, int p1, int p2) {
  using F = NF_<D>;
  const long t = ((long)p2 * G.P[1] + p1) * G.P[0] + p0;
  const int i0 = p0 - G.g[0], i1 = p1 - G.g[1], i2 = p2 - G.g[2];
  node_state<D>(G, JU, J, nd, flags, t, i0, i1, i2);
  // metrics
  if (met_in) {
    unsigned mir;
    long ms = ghost_metric_src(G, i0, i1, i2, mir);
#pragma unroll
    for (int k = 0; k < D; ++k) {
#pragma unroll
      for (int j = 0; j < D; ++j) {
        double sg = 1.0;
        for (int q = 0; q < D; ++q)
          if ((mir >> q) & 1u)
            if ((k == q) != (j == q)) sg = -sg;
        nd[(long)(F::MS + k * D + j) * G.PN + t] = sg * met_in[(long)(k * D + j) * G.N + ms];
      }
      double xv = 0.0;
      if (xit_in) {
        double sg = ((mir >> k) & 1u) ? -1.0 : 1.0;
        xv = sg * xit_in[(long)k * G.N + ms];
      }
      nd[(long)(F::XS + k) * G.PN + t] = xv;
    }
  } else {
    // the mesh velocity first: with its loads after the nine 3D metrics the compiler kept
    // twice the registers and spilled 436 bytes per lane
    double xv[D];
#pragma unroll
    for (int j = 0; j < D; ++j) xv[j] = xd ? mesh_at(G, xd, j, i0, i1, i2, 1) : 0.0;
    double m[D][D];
    if constexpr (D == 2) {
      metrics2(G, xn, xd, cdt, i0, i1, m);
    } else {
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int j = 0; j < D; ++j) m[k][j] = metric_at<D>(G, xn, xd, cdt, dp, dpN, k, j, i0, i1, i2);
    }
    node_metrics_store<D>(G, nd, t, m, xv);
  }
}


// =============================== interface fluxes ================================
//
// One block owns a tile of interfaces normal to direction K.  Phase 1: every node that
// owns a pair flux used by the tile (the tile's nodes along K plus two more on the low
// side) computes its three two-point fluxes F(i, i+m), m = 1, 2, 3, into LDS.  Phase 2:
// each thread combines the six pair fluxes of its interface with alpha_m (eq.
// ECFlux_curv_2p) and subtracts the dissipation of eq. HOstable.

// Tile<D, K>: X x Y x Z interfaces per 256-thread block, threads in rows of PX (PX >= X; lanes
// tx >= X of a row have no interface).  The x tiles compute 62 interfaces per row of 64
// threads so that the pair-flux items (X + 2 per row) are exactly one per thread.
template <int D, int K> struct Tile;
template <> struct Tile<1, 0> { static constexpr int X = 256, Y = 1, Z = 1, PX = X, PY = Y; };
template <> struct Tile<2, 0> { static constexpr int X = 62, Y = 4, Z = 1, PX = 64, PY = Y; };
template <> struct Tile<2, 1> { static constexpr int X = 16, Y = 16, Z = 1, PX = X, PY = Y; };
template <> struct Tile<3, 0> { static constexpr int X = 62, Y = 4, Z = 1, PX = 64, PY = Y; };
template <> struct Tile<3, 1> { static constexpr int X = 16, Y = 16, Z = 1, PX = X, PY = Y; };
template <> struct Tile<3, 2> { static constexpr int X = 16, Y = 4, Z = 4, PX = X, PY = Y; };

// node data used by a pair flux (direction K)
template <int D> struct Pq {
  double rho, v[D], T, iT, g, iob, lr, lb, lt, m[D], mt;
};

// Field f of the node buffer at the byte offset ob of a node.  The field's base address is the
// same for every lane and the lane's offset is 32 bits wide, so the load takes the form with a
// scalar base and a 32-bit vector offset: no 64-bit address arithmetic per lane and field.
// Needs 8 PN < 2^32, which esvdw_create checks.
__device__ __forceinline__ double ndf(const Geo &G, const double *__restrict__ nd, int f, unsigned ob) {
  const char *base = reinterpret_cast<const char *>(nd + (long)f * G.PN);
  return *reinterpret_cast<const double *>(base + ob);
}

template <int D, int K>
__device__ __forceinline__ void load_pq(const Geo &G, const double *__restrict__ nd, unsigned ob, Pq<D> &q) {
  using F = NF_<D>;
  q.rho = ndf(G, nd, F::RHO, ob);
#pragma unroll
  for (int m = 0; m < D; ++m) q.v[m] = ndf(G, nd, F::V + m, ob);
  q.T = ndf(G, nd, F::T, ob);
  q.iT = ndf(G, nd, F::IT, ob);
  q.iob = ndf(G, nd, F::IOB, ob);
  q.g = G.R * q.iob - G.a * q.rho * q.iT;  // g = R/(1 - b rho) - a rho/T
  q.lr = ndf(G, nd, F::LNR, ob);
  q.lb = ndf(G, nd, F::LNB, ob);
  q.lt = ndf(G, nd, F::LNT, ob);
#pragma unroll
  for (int j = 0; j < D; ++j) q.m[j] = ndf(G, nd, F::MS + K * D + j, ob);
  q.mt = ndf(G, nd, F::XS + K, ob);
}

// node data of the mirror image across a face normal to K: the velocity component and the
// metrics J dxi_K/dx_j (j != K) and J dxi_K/dt change sign
template <int D, int K>
__device__ __forceinline__ void pq_mirror(Pq<D> &q) {
  q.v[K] = -q.v[K];
#pragma unroll
  for (int j = 0; j < D; ++j)
    if (j != K) q.m[j] = -q.m[j];
  q.mt = -q.mt;
}

// Two-point EC flux (eq. ECfluxMM with the closed-form U~, F~_j of Section 3.1), written in
// contracted form: with the pair-averaged metrics mb, mbt and u = mbt + mb.v per node,
//   F_rho = ({rho u} A + {g}{u})/D,  F_v = {v} F_rho + mb {rho}{T}{g},
//   F_E = ({v/T}.F_v - K F_rho + a {rho u}{rho/T})/{1/T},
// D = R/L(rho) + R b/L(1 - b rho) + R b/Pi - 2a/{T}, A = R b/Pi - a/{T},
// K = {|v|^2/T}/2 - c_v {T}/L(T) + 2a{rho/T}; out[nv] receives {J dxi/dt}.
// The means are carried as sums (S x = x_l + x_r = 2{x}, with ul2 = 2u per node) and the
// factors 1/2 collected into a few constants: F_rho = (S(rho u2) A + S g S u2 / 2) / (4D),
// F_v = (S v F_rho + S m pt) / 2 with pt = S rho S T S g / 8, and with K4 = 4K,
// F_E = (S(v/T).F_v - K4 F_rho / 2 + a S(rho u2) S(rho/T) / 4) / S(1/T) (one shared division by
// D S(1/T) gives both 1/D and 1/{1/T}).
template <int D>
__device__ __forceinline__ void ec_pair(const Geo &G, const Pq<D> &l, const Pq<D> &r, double *out, unsigned &bad) {
  double Sm[D];
#pragma unroll
  for (int j = 0; j < D; ++j) Sm[j] = l.m[j] + r.m[j];
  const double Smt = l.mt + r.mt;
  double ul2 = Smt, ur2 = Smt;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    ul2 = fma(Sm[j], l.v[j], ul2);
    ur2 = fma(Sm[j], r.v[j], ur2);
  }
  const double SiT = l.iT + r.iT, SrT = fma(l.rho, l.iT, r.rho * r.iT), Sg = l.g + r.g, Sr = l.rho + r.rho;
  const double Sru = fma(l.rho, ul2, r.rho * ur2), Su = ul2 + ur2;
  const double Rb_Pi = G.R * G.b * l.iob * r.iob;
  // the denominators of 1/L(rho), 1/L(1 - b rho), 1/L(T) and of the mean 1/{T} share one division
  const double obl = 1.0 - G.b * l.rho, obr = 1.0 - G.b * r.rho;
  const double dR = logmean_den(l.rho, r.rho), dB = logmean_den(obl, obr), dT = logmean_den(l.T, r.T);
  const double sT = l.T + r.T;
  const double t1 = dR * dB, t2 = dT * sT, rq = rcp_nr(t1 * t2), r1 = rq * t2, r2 = rq * t1;
  const double iTmean = 2.0 * (r2 * dT);
  // 1/L(rho), 1/L(1 - b rho), 1/L(T) (the second is multiplied by b = 0 without a covolume)
  double il[3];
  inv_logmean_rn<3>(G.lmc, {l.rho, obl, l.T}, {r.rho, obr, r.T}, {l.lr, l.lb, l.lt}, {r.lr, r.lb, r.lt},
                    {r1 * dB, r1 * dR, r2 * sT}, il);
  const double Dd = G.R * il[0] + Rb_Pi - 2.0 * G.a * iTmean + G.R * G.b * il[1];
  const double A = Rb_Pi - G.a * iTmean;
  double vTl[D], vTr[D], Sv2T = 0.0;
#pragma unroll
  for (int m = 0; m < D; ++m) {
    vTl[m] = l.v[m] * l.iT;
    vTr[m] = r.v[m] * r.iT;
    Sv2T = fma(l.v[m], vTl[m], fma(r.v[m], vTr[m], Sv2T));
  }
  const double K4 = Sv2T - 2.0 * G.cv * sT * il[2] + 4.0 * G.a * SrT;
  if (!(Dd > 0.0)) bad = 1u;
  const double rd = rcp_nr(Dd * SiT);
  const double Fr = 0.25 * fma(Sru, A, 0.5 * (Sg * Su)) * (rd * SiT);
  const double Fh = 0.5 * Fr, ph = 0.0625 * (Sr * sT * Sg);
  double sumS = 0.0;
#pragma unroll
  for (int m = 0; m < D; ++m) {
    const double Fv = fma(l.v[m] + r.v[m], Fh, Sm[m] * ph);
    out[1 + m] = Fv;
    sumS = fma(vTl[m] + vTr[m], Fv, sumS);
  }
  out[0] = Fr;
  out[D + 1] = (fma(-K4, Fh, sumS) + 0.25 * G.a * Sru * SrT) * (rd * Dd);
  out[D + 2] = 0.5 * Smt;
}

// interface eigen-system in the rotated frame
template <int D> struct Eig {
  double n[D], tg[D - 1 > 0 ? D - 1 : 1][D];  // normal and tangent rows of the rotation
  double un, ut[D > 1 ? D - 1 : 1], H, c, c2G, s0, s1, st;
};

// scaled entropy variables W = R^T T V at one node
template <int D>
__device__ __forceinline__ void w_of(const Eig<D> &E, const double *V, double *W) {
  double vn = 0.0;
#pragma unroll
  for (int j = 0; j < D; ++j) vn += E.n[j] * V[1 + j];
  double vt[D > 1 ? D - 1 : 1];
#pragma unroll
  for (int t = 0; t < D - 1; ++t) {
    vt[t] = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) vt[t] += E.tg[t][j] * V[1 + j];
  }
  double VE = V[D + 1];
  double base = V[0] + E.un * vn + E.H * VE;
#pragma unroll
  for (int t = 0; t < D - 1; ++t) base += E.ut[t] * vt[t];
  double ac = E.c * (vn + E.un * VE);
  W[0] = E.s0 * (base - ac);
  W[1] = E.s1 * (base - E.c2G * VE);
#pragma unroll
  for (int t = 0; t < D - 1; ++t) W[2 + t] = E.st * (vt[t] + E.ut[t] * VE);
  W[D + 1] = E.s0 * (base + ac);
}

// magnitudes |R|^T |T V| of the terms summed into each W component (rounding scale of W)
template <int D>
__device__ __forceinline__ void wmag_of(const Eig<D> &E, const double *V, double *A) {
  double vn = 0.0;
#pragma unroll
  for (int j = 0; j < D; ++j) vn += E.n[j] * V[1 + j];
  double avt = 0.0, vt[D > 1 ? D - 1 : 1];
#pragma unroll
  for (int t = 0; t < D - 1; ++t) {
    vt[t] = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) vt[t] += E.tg[t][j] * V[1 + j];
    avt += fabs(E.ut[t]) * fabs(vt[t]);
  }
  double a0 = fabs(V[0]), an = fabs(vn), aE = fabs(V[D + 1]);
  A[0] = E.s0 * (a0 + fabs(E.un - E.c) * an + avt + fabs(E.H - E.un * E.c) * aE);
  A[1] = E.s1 * (a0 + fabs(E.un) * an + avt + fabs(E.H - E.c2G) * aE);
#pragma unroll
  for (int t = 0; t < D - 1; ++t) A[2 + t] = E.st * (fabs(vt[t]) + fabs(E.ut[t]) * aE);
  A[D + 1] = E.s0 * (a0 + fabs(E.un + E.c) * an + avt + fabs(E.H + E.un * E.c) * aE);
}

// LDS doubles used by flux_tile for a TX x TY x TZ tile of interfaces normal to K
template <int X_, int Y_, int Z_> struct TileShape { static constexpr int X = X_, Y = Y_, Z = Z_; };

// (pair fluxes of the nodes owning pairs, then the entropy-variable inputs V_1, v, 1/T of the
// dissipation stencils: the tile's nodes along K with 3 more on the low side and 2 on the high)
template <int D, int K, int TX, int TY, int TZ> struct FluxLds {
  static constexpr int QX = TX + 2 * (K == 0), QY = TY + 2 * (K == 1), QZ = TZ + 2 * (K == 2);
  static constexpr int Q = QX * QY * QZ;
  static constexpr int WX = TX + 5 * (K == 0), WY = TY + 5 * (K == 1), WZ = TZ + 5 * (K == 2);
  static constexpr int W = WX * WY * WZ;
  static constexpr int SIZE = (D + 3) * 3 * Q + (D + 2) * W;
};

// One 256-thread block computes the interface fluxes of the tile whose first interface is
// (bx0, by0, bz0): this thread's interface (a0, a1, a2) into Fl (nv + 1 values: the ES flux and
// the GCL flux of J dxi_K/dt); false if the thread has no interface.  The threads form a
// PX x PY x TZ block, PX >= TX, PY >= TY (threads outside TX x TY x TZ have no interface).
// sP: FluxLds<...>::SIZE doubles of LDS.
// Every thread reaches the internal barrier.
template <int D, int K, int TX, int TY, int TZ, int PX = TX, int PY = TY, bool ST = false>
__device__ __forceinline__ bool flux_tile_eval(const Geo &G, const double *__restrict__ nd, unsigned *flags, int bx0,
                                               int by0, int bz0, double *__restrict__ sP, double (&Fl)[D + 3],
                                               int &a0, int &a1, int &a2) {
  using F = NF_<D>;
  static_assert(PX >= TX && PY >= TY && PX * PY * TZ == 256, "flux tiles map at most one interface to each of 256 threads");
  using TL = TileShape<PX, PY, TZ>;
  constexpr int NV = D + 2, NC = NV + 1;
  using LQ = FluxLds<D, K, TX, TY, TZ>;
  constexpr int QX = LQ::QX, QY = LQ::QY;
  constexpr int Q = LQ::Q;
  constexpr int WX = LQ::WX, WY = LQ::WY, QW = LQ::W;
  double *__restrict__ sV = sP + NC * 3 * Q;  // [V_1, v_1..v_D, 1/T][QW]
  const int tid = threadIdx.x;
  const long sK = K == 0 ? 1 : (K == 1 ? (long)G.P[0] : (long)G.P[0] * G.P[1]);
  unsigned bad = 0;

  // ---- phase 1: pair fluxes of the nodes owning pairs of this tile ----
  // byte offset of node (i0, i1, i2) in the node buffer; with the step (ST), a solid node next
  // to the face normal to K stands for the mirror image of its fluid source (mir set)
  auto node_off = [&](int i0, int i1, int i2, bool &mir) -> unsigned {
    mir = false;
    if constexpr (ST) {
      int src;
      if (step_image(G, K, i0, i1, src)) {
        mir = true;
        if (K == 0) i0 = src;
        else i1 = src;
      }
    }
    return 8u * (unsigned)(((i2 + G.g[2]) * G.P[1] + (i1 + G.g[1])) * G.P[0] + (i0 + G.g[0]));
  };
  // item q (local coordinates qx, qy, qz); along K the first item is the node two below the
  // tile's first left node.  Returns false for items whose node lies beyond the grid.
  auto item_node = [&](int q, int (&ii)[3]) -> bool {
    const int qx = q % QX, qy = (q / QX) % QY, qz = q / (QX * QY);
    ii[0] = bx0 + qx - (K == 0 ? 3 : 0);
    ii[1] = by0 + qy - (K == 1 ? 3 : 0);
    ii[2] = bz0 + qz - (K == 2 ? 3 : 0);
    const int ik = ii[K];
    return ik <= G.n[K] - 1 && (K == 0 || ii[0] < G.n[0]) && (K == 1 || ii[1] < G.n[1]) && (K == 2 || ii[2] < G.n[2]);
  };
  // node data of item node ii (mirrored if it stands for an image)
  auto load_item = [&](const int (&ii)[3], unsigned &ob, Pq<D> &a) {
    bool mir;
    ob = node_off(ii[0], ii[1], ii[2], mir);
    load_pq<D, K>(G, nd, ob, a);
    if (mir) pq_mirror<D, K>(a);
  };
  // the pair F(node ii of item q, node m further along K) into its LDS slots
  auto pair_to_lds = [&](int q, const int (&ii)[3], unsigned ob, const Pq<D> &a, int m) {
    Pq<D> b;
    unsigned bp = 0;
    if constexpr (ST) {
      bool mir;
      const int j0 = ii[0] + (K == 0 ? m : 0), j1 = ii[1] + (K == 1 ? m : 0);
      load_pq<D, K>(G, nd, node_off(j0, j1, ii[2], mir), b);
      if (mir) pq_mirror<D, K>(b);
      double o[NC];
      ec_pair<D>(G, a, b, o, bp);
      // only pairs ending at a fluid node enter a flux of the fluid
      if (!step_solid(G, j0, j1)) bad |= bp;
#pragma unroll
      for (int c = 0; c < NC; ++c) sP[(c * 3 + (m - 1)) * Q + q] = o[c];
    } else {
      load_pq<D, K>(G, nd, ob + 8u * (unsigned)(m * sK), b);
      double o[NC];
      ec_pair<D>(G, a, b, o, bad);
#pragma unroll
      for (int c = 0; c < NC; ++c) sP[(c * 3 + (m - 1)) * Q + q] = o[c];
    }
    (void)bp;
  };
  constexpr int QK = K == 0 ? QX : (K == 1 ? QY : LQ::QZ);  // items per line along K
  constexpr int NL = Q / QK;                                // lines along K
  if constexpr (Q <= 256 || NL * (QK - 2) != 256) {
    // every item with all three of its pairs, one item per thread and round
    for (int q = tid; q < Q; q += 256) {
      int ii[3];
      if (!item_node(q, ii)) continue;
      unsigned ob;
      Pq<D> a;
      load_item(ii, ob, a);
#pragma unroll
      for (int m = 1; m <= 3; ++m) pair_to_lds(q, ii, ob, a, m);
    }
  } else {
    // 256 inner items (k-index >= 2 along K), one per thread with its three pairs; then the
    // pairs the combination uses from the two low halo items, F(0, 3), F(1, 3) and F(1, 2),
    // one per thread (the halo items' other pairs are not needed)
    // (consecutive threads take consecutive nodes along x, for coalesced loads)
    {
      int q;
      if constexpr (K == 0) {
        q = (tid / (QX - 2)) * QX + 2 + tid % (QX - 2);
      } else if constexpr (K == 1) {
        const int r = tid / QX;
        q = ((r / (QY - 2)) * QY + 2 + r % (QY - 2)) * QX + tid % QX;
      } else {
        const int r = tid / QX;
        q = ((2 + r / QY) * QY + r % QY) * QX + tid % QX;
      }
      int ii[3];
      if (item_node(q, ii)) {
        unsigned ob;
        Pq<D> a;
        load_item(ii, ob, a);
#pragma unroll
        for (int m = 1; m <= 3; ++m) pair_to_lds(q, ii, ob, a, m);
      }
    }
    for (int u = tid; u < 3 * NL; u += 256) {
      // unit u: halo item k (0 or 1) of its line along K and the pair m it supplies
      int q, r;
      if constexpr (K == 0) {
        r = u % 3;
        q = (u / 3) * QX + (r == 0 ? 0 : 1);
      } else if constexpr (K == 1) {
        const int w = u / QX;
        r = w % 3;
        q = ((w / 3) * QY + (r == 0 ? 0 : 1)) * QX + u % QX;
      } else {
        const int w = u / QX;
        r = w / QY;
        q = ((r == 0 ? 0 : 1) * QY + w % QY) * QX + u % QX;
      }
      const int m = r == 1 ? 2 : 3;
      int ii[3];
      if (!item_node(q, ii)) continue;
      unsigned ob;
      Pq<D> a;
      load_item(ii, ob, a);
      pair_to_lds(q, ii, ob, a, m);
    }
  }
  if (G.diss) {
    for (int q = tid; q < QW; q += 256) {
      int qx = q % WX, qy = (q / WX) % WY, qz = q / (WX * WY);
      int i0 = bx0 + qx - (K == 0 ? 3 : 0), i1 = by0 + qy - (K == 1 ? 3 : 0), i2 = bz0 + qz - (K == 2 ? 3 : 0);
      int ik = K == 0 ? i0 : (K == 1 ? i1 : i2);
      // the node buffer holds 3 ghost layers: node indices -3 .. n_K + 2 along K
      bool ok = ik <= G.n[K] + 2 && (K == 0 || i0 < G.n[0]) && (K == 1 || i1 < G.n[1]) && (K == 2 || i2 < G.n[2]);
      if (!ok) continue;
      bool mir;
      const unsigned ob = node_off(i0, i1, i2, mir);
      sV[q] = ndf(G, nd, F::V1, ob);
#pragma unroll
      for (int m = 0; m < D; ++m) sV[(1 + m) * QW + q] = (mir && m == K) ? -ndf(G, nd, F::V + m, ob) : ndf(G, nd, F::V + m, ob);
      sV[(D + 1) * QW + q] = ndf(G, nd, F::IT, ob);
    }
  }
  __syncthreads();

  // ---- phase 2: this thread's interface ----
  const int tx = tid % TL::X, ty = (tid / TL::X) % TL::Y, tz = tid / (TL::X * TL::Y);
  a0 = bx0 + tx;  // interface index (along K: 0..n_K)
  a1 = by0 + ty;
  a2 = bz0 + tz;
  const int e0 = G.n[0] + (K == 0), e1 = G.n[1] + (K == 1), e2 = G.n[2] + (K == 2);
  // with the step, a face carries a flux only if its right node (a0, a1) is fluid
  if (tx >= TX || ty >= TY || a0 >= e0 || a1 >= e1 || a2 >= e2 || (ST && step_solid(G, a0, a1))) {
    if (bad) raise_flag(flags, ESVDW_F_MEANCONSTRAINT);
    return false;
  }
  const int i0 = a0 - (K == 0), i1 = a1 - (K == 1), i2 = a2 - (K == 2);  // left node i
  // LDS item of node i (local coordinates shifted by 2 along K)
  const int qi = ((tz + 2 * (K == 2)) * QY + (ty + 2 * (K == 1))) * QX + (tx + 2 * (K == 0));
  const int qs = K == 0 ? 1 : (K == 1 ? QX : QX * QY);
  // dissipation first (its projection dd, scaled by h, is subtracted from the EC flux at the
  // end), so that the EC combination is not held in registers across it
  double dd[NV], h = 0.0;
#pragma unroll
  for (int c = 0; c < NV; ++c) dd[c] = 0.0;
  if (G.diss) {
    // the left node may stand for an image (ST); the right node is fluid
    bool mirl;
    const unsigned pc = node_off(i0, i1, i2, mirl);
    const unsigned pr = ST ? 8u * (unsigned)(((i2 + (K == 2) + G.g[2]) * G.P[1] + (i1 + (K == 1) + G.g[1])) * G.P[0] +
                                             (i0 + (K == 0) + G.g[0]))
                           : pc + 8u * (unsigned)sK;
    const double sl = mirl ? -1.0 : 1.0;  // sign of the left node's normal components
    // (the divisions of the averaged state are grouped so that each group shares one)
    double rl = ndf(G, nd, F::RHO, pc), rr = ndf(G, nd, F::RHO, pr);
    double pl = ndf(G, nd, F::P, pc), pq = ndf(G, nd, F::P, pr);
    // rho/p at the two nodes and its logarithm
    const double rpp = rcp_nr(pl * pq);
    double zl = rl * (pq * rpp), zr = rr * (pl * rpp);
    const double dR = logmean_den(rl, rr), dZ = logmean_den(zl, zr), rRZ = rcp_nr(dR * dZ);
    const double lrl = ndf(G, nd, F::LNR, pc), lrr = ndf(G, nd, F::LNR, pr);
    double il2[2];
    inv_logmean_rn<2>(G.lmc, {rl, zl}, {rr, zr}, {lrl, lrl - ndf(G, nd, F::LNP, pc)}, {lrr, lrr - ndf(G, nd, F::LNP, pr)},
                      {rRZ * dZ, rRZ * dR}, il2);
    const double ilr = il2[0], ilz = il2[1];
    double vb[D];
#pragma unroll
    for (int m = 0; m < D; ++m)
      vb[m] = 0.5 * ((m == K ? sl : 1.0) * ndf(G, nd, F::V + m, pc) + ndf(G, nd, F::V + m, pr));
    double mm[D], L2 = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      mm[j] = 0.5 * ((j != K ? sl : 1.0) * ndf(G, nd, F::MS + K * D + j, pc) + ndf(G, nd, F::MS + K * D + j, pr));
      L2 += mm[j] * mm[j];
    }
    double mtb = 0.5 * (sl * ndf(G, nd, F::XS + K, pc) + ndf(G, nd, F::XS + K, pr));
    double L = sqrt_nr(L2);
    // L(rho) = 1/ilr and 1/L share a division
    const double rLL = rcp_nr(ilr * L);
    double rb = rLL * L;       // L(rho)
    double iL = rLL * ilr;
    double pb = rb * ilz;      // L(rho)/L(rho/p)
    double ob = 1.0 - G.b * rb;
    double Tb = (pb + G.a * rb * rb) * ob * ilr * G.iR;
    // c^2 (1 - b rho)^2 and the S_2 factor R T - 2 a rho (1 - b rho)^2; 1/(1 - b rho), 1/c^2 and
    // 1/(c_v ac) share a division
    double c2o = (1.0 + G.delta) * G.R * Tb - 2.0 * G.a * rb * ob * ob;
    double ac = G.R * Tb - 2.0 * G.a * rb * ob * ob;
    const double rD = rcp_nr(ob * c2o * ac);
    double iob = rD * (c2o * ac);
    double c2 = c2o * iob * iob;
    double ic2 = ob * ob * (rD * (ob * ac));
    double iac = rD * (ob * c2o);
    Eig<D> E;
#pragma unroll
    for (int j = 0; j < D; ++j) E.n[j] = mm[j] * iL;
    if constexpr (D == 2) {
      E.tg[0][0] = -E.n[1];
      E.tg[0][1] = E.n[0];
    } else if constexpr (D == 3) {
      double sxy = sqrt(E.n[0] * E.n[0] + E.n[1] * E.n[1]);
      double ct = 1.0, st = 0.0;
      if (sxy > 0.0) {
        double is = 1.0 / sxy;
        ct = E.n[0] * is;
        st = E.n[1] * is;
      }
      E.tg[0][0] = -st;
      E.tg[0][1] = ct;
      E.tg[0][2] = 0.0;
      E.tg[1][0] = -E.n[2] * ct;
      E.tg[1][1] = -E.n[2] * st;
      E.tg[1][2] = sxy;
    }
    double un = 0.0, vv = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      un += E.n[j] * vb[j];
      vv += vb[j] * vb[j];
    }
    E.un = un;
#pragma unroll
    for (int t2 = 0; t2 < D - 1; ++t2) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) s += E.tg[t2][j] * vb[j];
      E.ut[t2] = s;
    }
    double Eb = rb * (G.cv * Tb - G.a * rb) + 0.5 * rb * vv;
    E.H = (Eb + pb) * ilr;
    E.c = sqrt_nr(c2);
    E.c2G = c2 * G.cv * ob * G.iR;  // c^2 / Gamma with Gamma = R/(c_v (1 - b rho))
    double S0 = 0.5 * rb * Tb * ic2, S1 = G.R * G.R * rb * Tb * Tb * ic2 * (iac * G.delta * G.iR), St = rb * Tb;
    if (!(S0 > 0.0) || !(S1 > 0.0)) bad = 1u;
    E.st = sqrt_nr(fabs(St));
    E.s0 = E.st * (E.c * ic2) * 0.70710678118654752;  // sqrt(S0) = sqrt(St / 2) / c
    E.s1 = sqrt_nr(fabs(S1));
    double Lam = fmax(fabs(mtb + L * (un - E.c)), fmax(fabs(mtb + L * un), fabs(mtb + L * (un + E.c))));
    double W[6][NV];
    double As[NV];  // rounding scale of W at the two nodes of the interface
    // LDS item of node (interface - 3) along K: local coordinates (tx, ty, tz)
    const int qw0 = (tz * WY + ty) * WX + tx, qws = K == 0 ? 1 : (K == 1 ? WX : WX * WY);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      double V[NV];
      const int qw = qw0 + s * qws;
      {
        double iT = sV[(D + 1) * QW + qw];
        V[0] = sV[qw];
#pragma unroll
        for (int m = 0; m < D; ++m) V[1 + m] = sV[(1 + m) * QW + qw] * iT;
        V[D + 1] = -iT;
      }
      w_of<D>(E, V, W[s]);
      if (s == 2) wmag_of<D>(E, V, As);
      if (s == 3) {
        double A3[NV];
        wmag_of<D>(E, V, A3);
#pragma unroll
        for (int c = 0; c < NV; ++c) As[c] = As[c] + A3[c];
      }
    }
    // zero test of the plain jumps: 2^-40 of the magnitude of all the terms forming W at the two
    // nodes (a component's own terms can be rounding residue of exact zeros)
    double zs = 0.0;
#pragma unroll
    for (int c = 0; c < NV; ++c) zs += As[c];
    zs = ldexp(zs, -40);
    double y[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      // wm = W2 + nm/dm, wp = W3 + np/dp, so [W]^WENO = wp - wm = jn / (dp dm) with
      // jn = (W3 - W2) dp dm + np dm - nm dp, dp, dm > 0: one division per component
      double nm, dm, np, dp;
      mrweno5_cfrac(G, W[0][c], W[1][c], W[2][c], W[3][c], W[4][c], nm, dm);
      mrweno5_cfrac(G, W[5][c], W[4][c], W[3][c], W[2][c], W[1][c], np, dp);
      double j0 = W[3][c] - W[2][c];
      const double pd = dp * dm;
      const double jn = fma(j0, pd, np * dm - nm * dp);
      if (fabs(j0) <= zs) j0 = 0.0;
      y[c] = ((jn > 0.0 && j0 > 0.0) || (jn < 0.0 && j0 < 0.0)) ? jn * rcp_nr(pd) : 0.0;
    }
    // R y in the rotated frame, then rotate the momentum back (T^T)
    double b0 = E.s0 * y[0], b1 = E.s1 * y[1], b2 = E.s0 * y[D + 1];
    double dr = b0 + b1 + b2;
    double dn = b0 * (un - E.c) + b1 * un + b2 * (un + E.c);
    double dE = b0 * (E.H - un * E.c) + b1 * (E.H - E.c2G) + b2 * (E.H + un * E.c);
    double dt_[D > 1 ? D - 1 : 1];
#pragma unroll
    for (int t2 = 0; t2 < D - 1; ++t2) {
      dt_[t2] = E.ut[t2] * dr + E.st * y[2 + t2];
      dE += E.st * y[2 + t2] * E.ut[t2];
    }
    h = 0.5 * Lam;
    dd[0] = dr;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double mj = E.n[j] * dn;
#pragma unroll
      for (int t2 = 0; t2 < D - 1; ++t2) mj += E.tg[t2][j] * dt_[t2];
      dd[1 + j] = mj;
    }
    dd[D + 1] = dE;
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double *P1 = sP + (c * 3 + 0) * Q, *P2 = sP + (c * 3 + 1) * Q, *P3 = sP + (c * 3 + 2) * Q;
    Fl[c] = AL1 * P1[qi] + AL2 * (P2[qi] + P2[qi - qs]) + AL3 * (P3[qi] + P3[qi - qs] + P3[qi - 2 * qs]);
    if (c < NV) Fl[c] -= h * dd[c];
  }
  if (bad) raise_flag(flags, ESVDW_F_MEANCONSTRAINT);
  return true;
}

// flux_tile_eval, the fluxes written to Fo (component-major, nif interfaces per component)
template <int D, int K, int TX, int TY, int TZ, int PX = TX, int PY = TY, bool ST = false>
__device__ __forceinline__ void flux_tile(const Geo &G, const double *__restrict__ nd, double *__restrict__ Fo,
                                          long nif, unsigned *flags, int bx0, int by0, int bz0,
                                          double *__restrict__ sP) {
  double Fl[D + 3];
  int a0, a1, a2;
  if (!flux_tile_eval<D, K, TX, TY, TZ, PX, PY, ST>(G, nd, flags, bx0, by0, bz0, sP, Fl, a0, a1, a2)) return;
  const int e0 = G.n[0] + (K == 0), e1 = G.n[1] + (K == 1);
  const long ti = ((long)a2 * e1 + a1) * e0 + a0;
#pragma unroll
  for (int c = 0; c < D + 3; ++c) Fo[(long)c * nif + ti] = Fl[c];
}


// =============================== update ==========================================

// operands of the SSP-RK3 stage combination at node slot t: dt (set by the caller, the same for
// every node), the stage input and (stages 1 and 2) the base values; loaded apart from the
// combination so that a kernel can issue the loads early (mode 0 loads nothing)
template <int D> struct UpdIn {
  double yin[D + 3], yb[D + 3], dt;
};
template <int D>
__device__ __forceinline__ void update_load(const Geo &G, long t, int mode, int s, const double *__restrict__ base_JU,
                                            const double *__restrict__ base_J, const double *__restrict__ in_JU,
                                            const double *__restrict__ in_J, UpdIn<D> &u) {
  constexpr int NV = D + 2;
  if (mode != 1) return;
#pragma unroll
  for (int c = 0; c <= NV; ++c) {
    const double *inp = c < NV ? in_JU + (long)c * G.N : in_J;
    const double *bp = c < NV ? base_JU + (long)c * G.N : base_J;
    u.yin[c] = inp[t];
    u.yb[c] = s != 0 ? bp[t] : 0.0;
  }
}

// RK-stage output at node slot t from the semi-discrete RHS L (nv + 1 values) and the operands
// u.  mode 0: write dJU, dJ.  mode 1: SSP-RK3 stage s combination.
template <int D>
__device__ __forceinline__ void update_store(const Geo &G, const double (&L)[D + 3], const UpdIn<D> &u, long t,
                                             int mode, int s, double *__restrict__ out_JU, double *__restrict__ out_J,
                                             unsigned *flags) {
  constexpr int NV = D + 2;
  bool nan = false;
  if (mode == 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      out_JU[(long)c * G.N + t] = L[c];
      nan |= isnan(L[c]);
    }
    out_J[t] = L[NV];
    nan |= isnan(L[NV]);
  } else {
    // the fused multiply-adds are written out so that the rounding does not depend on which
    // product the compiler would contract in a given kernel
#pragma unroll
    for (int c = 0; c <= NV; ++c) {
      const double y = fma(u.dt, L[c], u.yin[c]);
      double o;
      if (s == 0) o = y;
      else if (s == 1) o = fma(0.25, y, 0.75 * u.yb[c]);
      else o = fma(2.0 / 3.0, y, (1.0 / 3.0) * u.yb[c]);
      nan |= isnan(o);
      if (c < NV) out_JU[(long)c * G.N + t] = o;
      else out_J[t] = o;
    }
  }
  if (nan) raise_flag(flags, ESVDW_F_NAN);
}

// RK-stage output at node slot t from the semi-discrete RHS L, its operands loaded here
template <int D>
__device__ __forceinline__ void update_combine(const Geo &G, const double (&L)[D + 3], long t, int mode, int s,
                                               const double *__restrict__ dtp, const double *__restrict__ base_JU,
                                               const double *__restrict__ base_J, const double *__restrict__ in_JU,
                                               const double *__restrict__ in_J, double *__restrict__ out_JU,
                                               double *__restrict__ out_J, unsigned *flags) {
  UpdIn<D> u;
  u.dt = mode == 1 ? *dtp : 0.0;
  update_load<D>(G, t, mode, s, base_JU, base_J, in_JU, in_J, u);
  update_store<D>(G, L, u, t, mode, s, out_JU, out_J, flags);
}

// mode 0: write dJU, dJ.  mode 1: SSP-RK3 stage s combination with dt from the device.
template <int D>
__device__ __forceinline__ void update_point(const Geo &G, const double *__restrict__ F0,
                                             const double *__restrict__ F1, const double *__restrict__ F2, long nif0,
                                             long nif1, long nif2, int mode, int s, const double *__restrict__ dtp,
                                             const double *__restrict__ base_JU, const double *__restrict__ base_J,
                                             const double *__restrict__ in_JU, const double *__restrict__ in_J,
                                             double *__restrict__ out_JU, double *__restrict__ out_J, unsigned *flags,
                                             int i0, int i1, int i2) {
  constexpr int NV = D + 2;
  const long t = lin(G, i0, i1, i2);
  double L[NV + 1];
#pragma unroll
  for (int c = 0; c <= NV; ++c) L[c] = 0.0;
  {  // direction 0: interfaces (i0 - 1/2) at a0 = i0 and (i0 + 1/2) at a0 = i0 + 1
    long r = ((long)i2 * G.n[1] + i1) * (G.n[0] + 1) + i0;
#pragma unroll
    for (int c = 0; c <= NV; ++c) L[c] += (F0[(long)c * nif0 + r] - F0[(long)c * nif0 + r + 1]) * G.idxi[0];
  }
  if (D > 1) {
    long r = ((long)i2 * (G.n[1] + 1) + i1) * G.n[0] + i0;
#pragma unroll
    for (int c = 0; c <= NV; ++c) L[c] += (F1[(long)c * nif1 + r] - F1[(long)c * nif1 + r + G.n[0]]) * G.idxi[1];
  }
  if (D > 2) {
    long r = ((long)i2 * G.n[1] + i1) * G.n[0] + i0;
    long st = (long)G.n[0] * G.n[1];
#pragma unroll
    for (int c = 0; c <= NV; ++c) L[c] += (F2[(long)c * nif2 + r] - F2[(long)c * nif2 + r + st]) * G.idxi[2];
  }
  update_combine<D>(G, L, t, mode, s, dtp, base_JU, base_J, in_JU, in_J, out_JU, out_J, flags);
}


// 2D: the direction-0 interface fluxes of a 62 x 4 tile (rows of 64 threads, so that the
// pair-flux items are one per thread) and the update of the 61 x 4 nodes between them, in one
// block (the direction-1 fluxes are read from their buffer).  Tiles step by 61 nodes along x,
// so the tile's last interface is also computed by the next tile; in exchange the direction-0
// fluxes never go through memory and the separate update kernel is not needed.  The node's
// sums are those of update_point (direction 0, then direction 1).
#define FU_TX 62
#define FU_PX 64
#define FU_TY 4
// The tile whose first interface is (bx0, by0), for one 256-thread block; sP: FluxLds<2, 0, FU_TX,
// FU_TY, 1>::SIZE doubles of LDS.  mode 0: write dJU, dJ; mode 1: the SSP-RK3 stage s combination
// with dt from dtp; mout (mode 1): also mout = mx + mf dt mxd at the tile's nodes (mout may be mx).
// ST: the 2D backward-facing step; its solid nodes keep the step's base values (mode 1) or get a
// zero right-hand side (mode 0).  Every thread reaches the barriers.
template <bool ST>
__device__ __forceinline__ void flux_upd2_tile(const Geo &G, const double *__restrict__ nd,
                                               const double *__restrict__ F1, long nif1, int mode, int s,
                                               const double *__restrict__ dtp, const double *__restrict__ base_JU,
                                               const double *__restrict__ base_J, const double *__restrict__ in_JU,
                                               const double *__restrict__ in_J, double *__restrict__ out_JU,
                                               double *__restrict__ out_J, unsigned *flags, const double *mx,
                                               const double *mxd, double mf, double *mout, int bx0, int by0,
                                               double *__restrict__ sP) {
  static_assert(FluxLds<2, 0, FU_TX, FU_TY, 1>::SIZE >= 5 * 256, "the interface fluxes reuse the pair-flux LDS");
  double Fl[5];
  int a0, a1, a2;
  const bool ok = flux_tile_eval<2, 0, FU_TX, FU_TY, 1, FU_PX, FU_TY, ST>(G, nd, flags, bx0, by0, 0, sP, Fl, a0, a1, a2);
  const int tid = threadIdx.x, tx = tid % FU_PX, ty = tid / FU_PX;
  const int i0 = bx0 + tx, i1 = by0 + ty;
  const bool upd = tx < FU_TX - 1 && i0 < G.n[0] && i1 < G.n[1];
  const long t = (long)i1 * G.n[0] + i0;
  const bool solid = ST && upd && step_solid(G, i0, i1);
  // the update's operands are loaded before the two barriers below, so that their latency
  // overlaps the waits (the direction-0 fluxes of the tile are not yet in LDS)
  double f1l[5], f1h[5], mxv[2], mxdv[2];
  const double dtm = mout ? *dtp : 0.0;
  UpdIn<2> u;
  u.dt = mode == 1 ? *dtp : 0.0;
  if (upd && !solid) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      f1l[c] = F1[(long)c * nif1 + t];
      f1h[c] = F1[(long)c * nif1 + t + G.n[0]];
    }
    update_load<2>(G, t, mode, s, base_JU, base_J, in_JU, in_J, u);
  }
  if (upd && mout) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      mxv[j] = mx[(long)j * G.N + t];
      mxdv[j] = mxd[(long)j * G.N + t];
    }
  }
  __syncthreads();  // every thread has read its pair fluxes
  if (ok) {
#pragma unroll
    for (int c = 0; c < 5; ++c) sP[c * 256 + tid] = Fl[c];
  }
  __syncthreads();
  if (!upd) return;
  if (mout) {
#pragma unroll
    for (int j = 0; j < 2; ++j) mout[(long)j * G.N + t] = fma(mf * dtm, mxdv[j], mxv[j]);
  }
  if (solid) {
#pragma unroll
    for (int c = 0; c < 4; ++c) out_JU[(long)c * G.N + t] = mode == 1 ? base_JU[(long)c * G.N + t] : 0.0;
    out_J[t] = mode == 1 ? base_J[t] : 0.0;
    return;
  }
  double L[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) L[c] = 0.0;
#pragma unroll
  for (int c = 0; c < 5; ++c) L[c] += (sP[c * 256 + tid] - sP[c * 256 + tid + 1]) * G.idxi[0];
#pragma unroll
  for (int c = 0; c < 5; ++c) L[c] += (f1l[c] - f1h[c]) * G.idxi[1];
  update_store<2>(G, L, u, t, mode, s, out_JU, out_J, flags);
}

// =============================== CFL =============================================

// CFL spectral-radius sum at node (i0, i1, i2): sum_k (|v . m_k| + |m_k| c) / (J dxi_k) with
// m_k = J grad xi_k; metrics of the mesh x computed in place (1D/2D) or read from met (3D)
// the same sum with the metrics mm[k][j] of the node given
// the CFL sum from a node's primitive values and metrics
template <int D>
__device__ __forceinline__ double cfl_rate_prim(const Geo &G, double iJ, double rho, const double (&v)[D], double T,
                                                const double (&mm)[D][D]) {
  double s = 0.0;
  double c = sqrt(eos_c2(G, rho, T));
#pragma unroll
  for (int k = 0; k < D; ++k) {
    double L2 = 0.0, vn = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double m = mm[k][j];
      L2 += m * m;
      vn += m * v[j];
    }
    s += (fabs(vn) + sqrt(L2) * c) * iJ * G.idxi[k];
  }
  return s;
}

template <int D>
__device__ __forceinline__ double cfl_rate_m(const Geo &G, const double *__restrict__ JU, const double *__restrict__ J,
                                             long t, const double (&mm)[D][D]) {
  double iJ, rho, v[D], T;
  node_prim<D>(G, JU, J, t, iJ, rho, v, T);
  return cfl_rate_prim<D>(G, iJ, rho, v, T, mm);
}

template <int D>
__device__ __forceinline__ double cfl_rate(const Geo &G, const double *__restrict__ JU, const double *__restrict__ J,
                                           const double *__restrict__ x, const double *__restrict__ met, int i0,
                                           int i1, int i2) {
  const long t = lin(G, i0, i1, i2);
  double mm[D][D];
  if constexpr (D == 2) {
    metrics2(G, x, nullptr, 0.0, i0, i1, mm);
  } else {
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
      for (int j = 0; j < D; ++j)
        mm[k][j] = D == 3 ? met[(long)(k * D + j) * G.N + t] : metric_at<D>(G, x, nullptr, 0.0, nullptr, 0, k, j, i0, i1, i2);
  }
  return cfl_rate_m<D>(G, JU, J, t, mm);
}
