// kernels.h -- launchers shared between the translation units of the library
#pragma once
#include "common.h"

int params_valid(const esvdw_params *p);
void make_geo(const esvdw_params *p, Geo *G);

int launch_dprod(esvdw_ctx *c, const double *xn, const double *xd, double cdt, hipStream_t st);
int launch_metrics(esvdw_ctx *c, const double *x, const double *xd, double *met, double *xit, double *J,
                   hipStream_t st);
int launch_rhs(esvdw_ctx *c, const double *JU, const double *J, const double *met, const double *xit,
               const double *xn, const double *xd, double cdt, int mode, int s, const double *dtp,
               const double *bJU, const double *bJ, double *oJU, double *oJ, hipStream_t st);
// launch_rhs whose update kernel also writes the next stage's mesh mout = mx + mf dt mxd per node
int launch_rhs_mesh(esvdw_ctx *c, const double *JU, const double *J, const double *met, const double *xit,
                    const double *xn, const double *xd, double cdt, double cs, int mode, int s, const double *dtp,
                    const double *bJU, const double *bJ, double *oJU, double *oJ, const double *mx, const double *mxd,
                    double mf, double *mout, hipStream_t st);
int launch_uniform_mesh(esvdw_ctx *c, double *x, hipStream_t st);
int launch_init_state(esvdw_ctx *c, const double *prim, const double *J, double *JU, hipStream_t st);
int launch_axpy_mesh(esvdw_ctx *c, const double *x, const double *xd, const double *dtp, double f, double *out,
                     hipStream_t st);
int launch_set_int(int *p, int v, hipStream_t st);

int launch_set_scalars(esvdw_ctx *c, hipStream_t st);
int launch_monitor(esvdw_ctx *c, const double *JU, const double *J, double *omega, hipStream_t st);
int launch_monitor_cfl(esvdw_ctx *c, const double *JU, const double *J, const double *xn, double *omega, long *nbc,
                       hipStream_t st);
int launch_jacobi(esvdw_ctx *c, const double *omega, double *x, int nsweep, double *resid_dev, hipStream_t st);
// nsweep sweeps from the iterate x0 (not modified; nullptr = x), the result in x
int launch_jacobi_from(esvdw_ctx *c, const double *omega, const double *x0, double *x, int nsweep, double *resid_dev,
                       hipStream_t st);
int launch_sor(esvdw_ctx *c, const double *omega, double *x, int nsweep, double relax, double *resid_dev,
               hipStream_t st);
int launch_limiter(esvdw_ctx *c, const double *xn, const double *xmu, double *gamma_dev, hipStream_t st);
// launch_limiter (gamma into the context's scalars) followed by launch_cfl, the two final
// reductions in one launch
int launch_limiter_cfl(esvdw_ctx *c, const double *xn, const double *xmu, const double *JU, const double *J,
                       double *dt_dev, long nbc_ready, hipStream_t st);
int launch_cfl(esvdw_ctx *c, const double *JU, const double *J, const double *x, double *dt_dev, hipStream_t st);
// launch_cfl on the library's static per-device scratch (1D/2D); returns an ESVDW_* code
int launch_cfl_noalloc(const Geo &G, double cfl, double dt_fixed, const double *JU, const double *J,
                       const double *x, double *dt_dev, hipStream_t st);
int launch_xdot(esvdw_ctx *c, const double *xn, const double *xmu, const double *gam, const double *dtp, double *xdot,
                hipStream_t st);
int launch_copy(const double *src, double *dst, long n, hipStream_t st);
// backward-facing step: values at the solid nodes (no-ops without a step)
int launch_step_fill_state(const Geo &G, double *JU, double *J, hipStream_t st);
int launch_step_fill_scalar(const Geo &G, double *w, hipStream_t st);
int launch_step_fill_mesh(const Geo &G, double *x, hipStream_t st);
int launch_add(const double *a, const double *b, double *dst, long n, hipStream_t st);
int launch_flux_only(esvdw_ctx *c, int K, hipStream_t st);
int launch_grad_rho_terms(esvdw_ctx *c, const double *JU, const double *J, hipStream_t st);
int launch_mlp_feat(esvdw_ctx *c, const double *JU, const double *J, float *feat, hipStream_t st);
int launch_mlp_infer(esvdw_ctx *c, const float *feat, const float *P, double *warm, hipStream_t st);
int launch_mlp_grad(esvdw_ctx *c, const float *feats, const float *tgt, const int *samples, long nsamp, float scale,
                    const float *P, float *grad, float *loss, hipStream_t st);
int launch_mlp_adam(float *P, const float *grad, float *m, float *v, int step, float lr, hipStream_t st);
