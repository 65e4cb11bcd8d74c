// api.hip -- the C ABI declared in include/esvdw.h: argument validation, context
// scratch, and the orchestration of the kernel launches.
#include <stdlib.h>
#include <string.h>

#include "common.h"
#include "kernels.h"

#define HIPOK(x) ((x) == hipSuccess)

int params_valid(const esvdw_params *p) {
  if (!p || p->dim < 1 || p->dim > 3) return 0;
  for (int k = 0; k < p->dim; ++k) {
    if (p->n[k] < 6) return 0;
    if (!(p->hi[k] > p->lo[k])) return 0;
    if (p->bc[k] != ESVDW_BC_PERIODIC && p->bc[k] != ESVDW_BC_OUTFLOW) return 0;
    if (p->bc[k] == ESVDW_BC_PERIODIC && (p->walls & (ESVDW_WALL_LO(k) | ESVDW_WALL_HI(k)))) return 0;
  }
  if (p->walls < 0 || (p->walls >> (2 * p->dim)) != 0) return 0;
  if (!(p->R > 0.0) || !(p->cv > 0.0) || p->a < 0.0 || p->b < 0.0) return 0;
  if (!(p->weno_lin[0] > 0.0) || p->weno_lin[1] < 0.0 || p->weno_lin[2] < 0.0 || !(p->weno_eps > 0.0)) return 0;
  if (!(p->cfl > 0.0) && !(p->dt_fixed > 0.0)) return 0;
  if (p->monitor_kind != ESVDW_MON_VDW && p->monitor_kind != ESVDW_MON_SINE) return 0;
  if (p->kappa < 0 || p->kappa > 2 || p->n_filter < 0 || p->mu < 0) return 0;
  // the flux kernels address a field of the padded node buffer with 32-bit byte offsets
  double pn = 1.0;
  for (int k = 0; k < p->dim; ++k) {
    long pk = (long)p->n[k] + 2 * GH;
    if (k == 0) pk = (pk + 15) & ~15L;
    pn *= (double)pk;
  }
  if (pn * 8.0 >= 4294967296.0) return 0;
  if (p->step[0] != 0 || p->step[1] != 0) {
    if (p->dim != 2 || p->bc[0] != ESVDW_BC_OUTFLOW || p->bc[1] != ESVDW_BC_OUTFLOW || !p->fixed_mu) return 0;
    if (p->step[0] < 3 || p->step[1] < 3 || p->step[0] + 3 > p->n[0] || p->step[1] + 3 > p->n[1]) return 0;
  }
  if (p->inflow) {
    if (p->dim != 2 || p->bc[0] != ESVDW_BC_OUTFLOW || (p->walls & ESVDW_WALL_LO(0))) return 0;
    const double rho = p->inflow_prim[0], ob = 1.0 - p->b * rho;
    if (!(rho > 0.0) || !(ob > 0.0)) return 0;
    const double T = (p->inflow_prim[3] + p->a * rho * rho) * ob / (rho * p->R);
    if (!(p->R * T - 2.0 * p->a * rho * ob * ob > 0.0)) return 0;
  }
  return 1;
}

void make_geo(const esvdw_params *p, Geo *G) {
  memset(G, 0, sizeof(*G));
  G->dim = p->dim;
  G->nv = p->dim + 2;
  G->N = 1;
  G->PN = 1;
  for (int k = 0; k < 3; ++k) {
    bool act = k < p->dim;
    G->n[k] = act ? p->n[k] : 1;
    G->g[k] = act ? GH : 0;
    G->P[k] = G->n[k] + 2 * G->g[k];
    if (k == 0) {
      G->E0 = G->P[0];
      G->P[0] = (G->P[0] + 15) & ~15;  // whole 128-byte lines per row
    }
    G->lo[k] = act ? p->lo[k] : 0.0;
    G->hi[k] = act ? p->hi[k] : 1.0;
    G->dxi[k] = (G->hi[k] - G->lo[k]) / G->n[k];
    G->idxi[k] = 1.0 / G->dxi[k];
    G->period[k] = G->hi[k] - G->lo[k];
    G->bc[k] = act ? p->bc[k] : ESVDW_BC_PERIODIC;
    G->walls = p->walls;
    G->N *= G->n[k];
    G->PN *= G->P[k];
  }
  G->R = p->R;
  G->cv = p->cv;
  G->a = p->a;
  G->b = p->b;
  G->delta = p->R / p->cv;
  G->iR = 1.0 / p->R;
  if (p->step[0] > 0 && p->step[1] > 0) {
    G->s0 = p->step[0];
    G->s1 = p->step[1];
  }
  if (p->inflow) {
    const double rho = p->inflow_prim[0];
    G->inflow = 1;
    G->qin[0] = rho;
    G->qin[1] = p->inflow_prim[1];
    G->qin[2] = p->inflow_prim[2];
    G->qin[3] = (p->inflow_prim[3] + p->a * rho * rho) * (1.0 - p->b * rho) / (rho * p->R);
  }
  for (int k = 0; k < 7; ++k) G->lmc[k] = 1.0 / (15 - 2 * k);
  G->lmc[7] = 1.0 / 17;
  G->wl0 = p->weno_lin[0];
  G->wl1 = p->weno_lin[1];
  G->wl2 = p->weno_lin[2];
  G->weps = p->weno_eps;
  G->iwl0 = 1.0 / p->weno_lin[0];
  G->diss = p->dissipation;
}

template <typename T> static int dalloc(T **ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) return 1;
  return HIPOK(hipMalloc((void **)ptr, count * sizeof(T)));
}

extern "C" {

const char *esvdw_strerror(int code) {
  switch (code) {
    case ESVDW_OK: return "ok";
    case ESVDW_EINVAL: return "invalid argument";
    case ESVDW_EHIP: return "HIP error";
    case ESVDW_ENOTIMPL: return "not implemented";
    case ESVDW_ESCRATCH: return "problem too large for the static scratch of a no-allocation entry point";
    default: return "unknown error";
  }
}

void esvdw_destroy(esvdw_ctx *c) {
  if (!c) return;
  void *bufs[] = {c->node_mem, c->flux[0], c->flux[1], c->flux[2], c->dprod, c->met, c->stA, c->stB, c->xdot, c->xmu,
                  c->xtmp, c->omega, c->omega2, c->mterm, c->rhoG, c->scal, c->part, c->flags};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  free(c);
}

int esvdw_create(const esvdw_params *p, esvdw_ctx **out) {
  if (!out) return ESVDW_EINVAL;
  *out = nullptr;
  if (!params_valid(p)) return ESVDW_EINVAL;
  esvdw_ctx *c = (esvdw_ctx *)calloc(1, sizeof(esvdw_ctx));
  if (!c) return ESVDW_EHIP;
  c->p = *p;
  make_geo(p, &c->G);
  (void)hipGetDevice(&c->dev);
  const Geo &G = c->G;
  int D = G.dim, nv = G.nv;
  c->NF = D == 1 ? NF_<1>::COUNT : (D == 2 ? NF_<2>::COUNT : NF_<3>::COUNT);
  long N = G.N;
  // node buffer: rows of whole cache lines, shifted so that node g0 (the first interior node)
  // of every row starts a 128-byte line
  bool ok = dalloc(&c->node_mem, (size_t)c->NF * G.PN + 16);
  if (ok) c->node = c->node_mem + (16 - G.g[0]) % 16;
  for (int k = 0; k < 3; ++k) {
    c->nif[k] = 0;
    if (k < D) {
      c->nif[k] = N / G.n[k] * (G.n[k] + 1);
      ok = ok && dalloc(&c->flux[k], (size_t)(nv + 1) * c->nif[k]);
    }
  }
  c->dpN = 0;
  if (D == 3) {
    c->dpN = (long)(G.n[0] + 12) * (G.n[1] + 12) * (G.n[2] + 12);
    ok = ok && dalloc(&c->dprod, (size_t)9 * c->dpN);
  }
  ok = ok && dalloc(&c->met, (size_t)(D * D + D) * N);
  ok = ok && dalloc(&c->stA, (size_t)(nv + 1) * N) && dalloc(&c->stB, (size_t)(nv + 1) * N);
  ok = ok && dalloc(&c->xdot, (size_t)D * N) && dalloc(&c->xmu, (size_t)D * N) && dalloc(&c->xtmp, (size_t)D * N);
  ok = ok && dalloc(&c->omega, (size_t)N) && dalloc(&c->omega2, (size_t)N) && dalloc(&c->mterm, (size_t)3 * N);
  ok = ok && dalloc(&c->rhoG, (size_t)2 * N) && dalloc(&c->scal, (size_t)SC_N) && dalloc(&c->flags, 1);
  {
    dim3 g, b;
    node_grid(G.n[0], G.n[1], G.n[2], g, b);
    c->npart = (long)g.x * g.y * g.z + 1;
  }
  ok = ok && dalloc(&c->part, (size_t)4 * c->npart);
  if (ok) ok = HIPOK(hipMemset(c->flags, 0, sizeof(unsigned))) && HIPOK(hipMemset(c->scal, 0, SC_N * sizeof(double)));
  if (ok) ok = HIPOK(hipDeviceSynchronize());
  if (!ok) {
    esvdw_destroy(c);
    return ESVDW_EHIP;
  }
  *out = c;
  return ESVDW_OK;
}

int esvdw_get_status(esvdw_ctx *c, unsigned *flags_host, int clear) {
  if (!c || !flags_host) return ESVDW_EINVAL;
  if (!HIPOK(hipDeviceSynchronize())) return ESVDW_EHIP;
  if (!HIPOK(hipMemcpy(flags_host, c->flags, sizeof(unsigned), hipMemcpyDeviceToHost))) return ESVDW_EHIP;
  if (clear && !HIPOK(hipMemset(c->flags, 0, sizeof(unsigned)))) return ESVDW_EHIP;
  return ESVDW_OK;
}

int init_mesh(esvdw_ctx *c, double *x, double *J, int uniform, hipStream_t st) {
  if (!c || !x || !J) return ESVDW_EINVAL;
  if (uniform && launch_uniform_mesh(c, x, st)) return ESVDW_EHIP;
  if (launch_metrics(c, x, nullptr, c->met, nullptr, J, st)) return ESVDW_EHIP;
  return ESVDW_OK;
}

int init_state(esvdw_ctx *c, const double *prim, const double *J, double *JU, hipStream_t st) {
  if (!c || !prim || !J || !JU) return ESVDW_EINVAL;
  return launch_init_state(c, prim, J, JU, st) ? ESVDW_EHIP : ESVDW_OK;
}

int compute_metrics(esvdw_ctx *c, const double *x, const double *xdot, double *met, double *xit, hipStream_t st) {
  if (!c || !x || !met) return ESVDW_EINVAL;
  return launch_metrics(c, x, xdot, met, xit, nullptr, st) ? ESVDW_EHIP : ESVDW_OK;
}

int es_rhs(esvdw_ctx *c, const double *JU, const double *J, const double *met, const double *xit, double *dJU,
           double *dJ, hipStream_t st) {
  if (!c || !JU || !J || !met || !dJU || !dJ) return ESVDW_EINVAL;
  if (dJU == JU || dJ == J) return ESVDW_EINVAL;
  return launch_rhs(c, JU, J, met, xit, nullptr, nullptr, 0.0, 0, 0, nullptr, nullptr, nullptr, dJU, dJ, st)
             ? ESVDW_EHIP
             : ESVDW_OK;
}

int rk_stage(esvdw_ctx *c, int s, const double *dt_dev, const double *JU0, const double *J0, const double *JUs,
             const double *Js, const double *x_n, const double *xdot, double *JUout, double *Jout, double *x_next,
             hipStream_t st) {
  if (!c || s < 0 || s > 2 || !dt_dev || !JU0 || !J0 || !JUs || !Js || !x_n || !JUout || !Jout) return ESVDW_EINVAL;
  if (JUout == JUs || Jout == Js) return ESVDW_EINVAL;
  static const double cst[3] = {0.0, 1.0, 0.5};
  const double *xs = x_n;
  if (xdot && s > 0) {
    // stage mesh x_n + c_s dt xdot, materialised in the context (dt lives on the device)
    if (launch_axpy_mesh(c, x_n, xdot, dt_dev, cst[s], c->xtmp, st)) return ESVDW_EHIP;
    xs = c->xtmp;
  }
  if (launch_rhs(c, JUs, Js, nullptr, nullptr, xs, xdot, 0.0, 1, s, dt_dev, JU0, J0, JUout, Jout, st))
    return ESVDW_EHIP;
  if (s == 2 && x_next && xdot)
    if (launch_axpy_mesh(c, x_n, xdot, dt_dev, 1.0, x_next, st) || launch_step_fill_mesh(c->G, x_next, st))
      return ESVDW_EHIP;
  return ESVDW_OK;
}

int mesh_monitor(esvdw_ctx *c, const double *JU, const double *J, double *omega, hipStream_t st) {
  if (!c || !JU || !J || !omega) return ESVDW_EINVAL;
  return launch_monitor(c, JU, J, omega, st) ? ESVDW_EHIP : ESVDW_OK;
}

int mesh_jacobi(esvdw_ctx *c, const double *omega, double *x, int nsweep, double *resid_dev, hipStream_t st) {
  if (!c || !omega || !x || nsweep < 0) return ESVDW_EINVAL;
  return launch_jacobi(c, omega, x, nsweep, resid_dev, st) ? ESVDW_EHIP : ESVDW_OK;
}

int mesh_sor(esvdw_ctx *c, const double *omega, double *x, int nsweep, double relax, double *resid_dev,
             hipStream_t st) {
  if (!c || !omega || !x || nsweep < 0 || !(relax > 0.0 && relax < 2.0) || c->G.s0 > 0) return ESVDW_EINVAL;
  for (int k = 0; k < c->G.dim; ++k)
    if (c->G.bc[k] == ESVDW_BC_PERIODIC && c->G.n[k] % 2) return ESVDW_EINVAL;
  return launch_sor(c, omega, x, nsweep, relax, resid_dev, st) ? ESVDW_EHIP : ESVDW_OK;
}

int mesh_limiter(esvdw_ctx *c, const double *x_n, const double *x_mu, double *gamma_dev, hipStream_t st) {
  if (!c || !x_n || !x_mu || !gamma_dev) return ESVDW_EINVAL;
  return launch_limiter(c, x_n, x_mu, gamma_dev, st) ? ESVDW_EHIP : ESVDW_OK;
}

int cfl_dt(esvdw_ctx *c, const double *JU, const double *J, const double *x, double *dt_dev, hipStream_t st) {
  if (!c || !JU || !J || !x) return ESVDW_EINVAL;
  return launch_cfl(c, JU, J, x, dt_dev, st) ? ESVDW_EHIP : ESVDW_OK;
}

int cfl_dt_noalloc(const esvdw_params *p, const double *JU, const double *J, const double *x, double *dt_dev,
                   hipStream_t st) {
  if (!params_valid(p) || p->dim > 2 || !JU || !J || !x || !dt_dev) return ESVDW_EINVAL;
  Geo G;
  make_geo(p, &G);
  return launch_cfl_noalloc(G, p->cfl, p->dt_fixed, JU, J, x, dt_dev, st);
}

int redistribute_mesh(esvdw_ctx *c, const double *JU, const double *J, const double *x_n, const double *warm_dx,
                      double *xdot, double *dt_dev, double *resid_dev, int *sweeps_dev, hipStream_t st) {
  if (!c || !JU || !J || !x_n || !xdot || !dt_dev) return ESVDW_EINVAL;
  const esvdw_params &p = c->p;
  long n = (long)c->G.dim * c->G.N;
  long nbc = 0;  // the CFL partials formed with the monitor (2D), else 0
  if (launch_monitor_cfl(c, JU, J, x_n, c->omega, &nbc, st)) return ESVDW_EHIP;
  // x^[0] = x_n (+ warm_dx); with a fixed sweep count and no warm start the first sweep reads x_n
  const bool from_xn = p.fixed_mu && !warm_dx;
  if (warm_dx) {
    if (launch_add(x_n, warm_dx, c->xmu, n, st)) return ESVDW_EHIP;
  } else if (!from_xn && launch_copy(x_n, c->xmu, n, st)) return ESVDW_EHIP;
  int sweeps = 0;
  if (p.fixed_mu) {
    if (launch_jacobi_from(c, c->omega, from_xn ? x_n : nullptr, c->xmu, p.mu, resid_dev, st)) return ESVDW_EHIP;
    sweeps = p.mu;
  } else {
    // tolerance mode: batches of sweeps, host-side test of the device residual
    double res = 0.0;
    int batch = 8;
    while (sweeps < p.mu) {
      int k = batch < p.mu - sweeps ? batch : p.mu - sweeps;
      if (launch_jacobi(c, c->omega, c->xmu, k, c->scal + SC_N - 1, st)) return ESVDW_EHIP;
      sweeps += k;
      if (!HIPOK(hipMemcpyAsync(&res, c->scal + SC_N - 1, sizeof(double), hipMemcpyDeviceToHost, st))) return ESVDW_EHIP;
      if (!HIPOK(hipStreamSynchronize(st))) return ESVDW_EHIP;
      if (res < p.mesh_tol) break;
      if (batch < 256) batch *= 2;
    }
    if (!(res < p.mesh_tol)) {
      unsigned f = ESVDW_F_NOTCONVERGED, cur = 0;
      if (!HIPOK(hipMemcpy(&cur, c->flags, sizeof(unsigned), hipMemcpyDeviceToHost))) return ESVDW_EHIP;
      cur |= f;
      if (!HIPOK(hipMemcpy(c->flags, &cur, sizeof(unsigned), hipMemcpyHostToDevice))) return ESVDW_EHIP;
    }
    if (resid_dev && launch_copy(c->scal + SC_N - 1, resid_dev, 1, st)) return ESVDW_EHIP;
  }
  if (sweeps_dev && launch_set_int(sweeps_dev, sweeps, st)) return ESVDW_EHIP;
  if (launch_limiter_cfl(c, x_n, c->xmu, JU, J, dt_dev, nbc, st)) return ESVDW_EHIP;
  if (launch_xdot(c, x_n, c->xmu, c->scal + SC_GAMMA, dt_dev, xdot, st)) return ESVDW_EHIP;
  return ESVDW_OK;
}

int mesh_converged(esvdw_ctx *c, double *xmu_out, hipStream_t st) {
  if (!c || !xmu_out) return ESVDW_EINVAL;
  return launch_copy(c->xmu, xmu_out, (long)c->G.dim * c->G.N, st) ? ESVDW_EHIP : ESVDW_OK;
}

int esvdw_step(esvdw_ctx *c, double *JU, double *J, double *x, int moving, double *dt_dev, hipStream_t st) {
  if (!c || !JU || !J || !x || !dt_dev) return ESVDW_EINVAL;
  long N = c->G.N;
  int nv = c->G.nv;
  const double *xd = nullptr;
  if (moving) {
    int r = redistribute_mesh(c, JU, J, x, nullptr, c->xdot, dt_dev, nullptr, nullptr, st);
    if (r) return r;
    xd = c->xdot;
  } else if (launch_cfl(c, JU, J, x, dt_dev, st)) {
    return ESVDW_EHIP;
  }
  double *aU = c->stA, *aJ = c->stA + (long)nv * N, *bU = c->stB, *bJ = c->stB + (long)nv * N;
  if (!xd) {
    int r = rk_stage(c, 0, dt_dev, JU, J, JU, J, x, xd, aU, aJ, nullptr, st);
    if (!r) r = rk_stage(c, 1, dt_dev, JU, J, aU, aJ, x, xd, bU, bJ, nullptr, st);
    if (!r) r = rk_stage(c, 2, dt_dev, JU, J, bU, bJ, x, xd, JU, J, nullptr, st);
    return r;
  }
  // moving mesh: the three rk_stage calls.  In 2D the node kernel forms each stage's mesh
  // x_n + c_s dt xdot (c = 0, 1, 1/2) itself, at the source nodes with the update kernel's
  // arithmetic; elsewhere each stage's update kernel forms the next stage's mesh instead of a
  // separate launch (the stage-1 update overwrites the stage mesh its own node kernel has read).
  // The stage-2 update forms x^{n+1} = x_n + dt xdot in place.
  if (c->G.dim == 2) {
    if (launch_rhs_mesh(c, JU, J, nullptr, nullptr, x, xd, 0.0, 0.0, 1, 0, dt_dev, JU, J, aU, aJ, nullptr, nullptr,
                        0.0, nullptr, st) ||
        launch_rhs_mesh(c, aU, aJ, nullptr, nullptr, x, xd, 0.0, 1.0, 1, 1, dt_dev, JU, J, bU, bJ, nullptr, nullptr,
                        0.0, nullptr, st) ||
        launch_rhs_mesh(c, bU, bJ, nullptr, nullptr, x, xd, 0.0, 0.5, 1, 2, dt_dev, JU, J, JU, J, x, xd, 1.0, x, st) ||
        launch_step_fill_mesh(c->G, x, st))
      return ESVDW_EHIP;
    return ESVDW_OK;
  }
  if (launch_rhs_mesh(c, JU, J, nullptr, nullptr, x, xd, 0.0, 0.0, 1, 0, dt_dev, JU, J, aU, aJ, x, xd, 1.0, c->xtmp,
                      st) ||
      launch_rhs_mesh(c, aU, aJ, nullptr, nullptr, c->xtmp, xd, 0.0, 0.0, 1, 1, dt_dev, JU, J, bU, bJ, x, xd, 0.5,
                      c->xtmp, st) ||
      launch_rhs_mesh(c, bU, bJ, nullptr, nullptr, c->xtmp, xd, 0.0, 0.0, 1, 2, dt_dev, JU, J, JU, J, x, xd, 1.0, x,
                      st) ||
      launch_step_fill_mesh(c->G, x, st))
    return ESVDW_EHIP;
  return ESVDW_OK;
}

int esvdw_bench_kernel(esvdw_ctx *c, int which, int reps, hipStream_t st) {
  if (!c || reps < 0) return ESVDW_EINVAL;
  if (which >= 1 && which <= 3) {
    if (which > c->G.dim) return ESVDW_EINVAL;
    for (int r = 0; r < reps; ++r)
      if (launch_flux_only(c, which - 1, st)) return ESVDW_EHIP;
    return ESVDW_OK;
  }
  if (which == 6) {
    long n = (long)(c->G.nv + 1) * c->G.N;
    for (int r = 0; r < reps; ++r)
      if (launch_copy(c->stA, c->stB, n, st)) return ESVDW_EHIP;
    return ESVDW_OK;
  }
  if (which == 5) {
    for (int r = 0; r < reps; ++r)
      if (launch_jacobi(c, c->omega, c->xmu, 1, nullptr, st)) return ESVDW_EHIP;
    return ESVDW_OK;
  }
  return ESVDW_EINVAL;
}

int mlp_features(esvdw_ctx *c, const double *JU, const double *J, float *feat, hipStream_t st) {
  if (!c || !JU || !J || !feat) return ESVDW_EINVAL;
  if (c->G.dim != 2) return ESVDW_EINVAL;
  return launch_mlp_feat(c, JU, J, feat, st) ? ESVDW_EHIP : ESVDW_OK;
}

int mlp_infer(esvdw_ctx *c, const float *feat, const float *params, double *warm_dx, hipStream_t st) {
  if (!c || !feat || !params || !warm_dx) return ESVDW_EINVAL;
  if (c->G.dim != 2) return ESVDW_EINVAL;
  return launch_mlp_infer(c, feat, params, warm_dx, st) ? ESVDW_EHIP : ESVDW_OK;
}

int mlp_grad(esvdw_ctx *c, const float *feats, const float *targets, const int *samples, long nsamples, float scale,
             const float *params, float *grad, float *loss_dev, hipStream_t st) {
  if (!c || !feats || !targets || !samples || !params || !grad || !loss_dev || nsamples < 1) return ESVDW_EINVAL;
  if (c->G.dim != 2) return ESVDW_EINVAL;
  return launch_mlp_grad(c, feats, targets, samples, nsamples, scale, params, grad, loss_dev, st) ? ESVDW_EHIP
                                                                                                 : ESVDW_OK;
}

int mlp_adam(float *params, const float *grad, float *m, float *v, int step, float lr, hipStream_t st) {
  if (!params || !grad || !m || !v || step < 1) return ESVDW_EINVAL;
  return launch_mlp_adam(params, grad, m, v, step, lr, st) ? ESVDW_EHIP : ESVDW_OK;
}

}  // extern "C"
