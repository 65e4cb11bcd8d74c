/*
 * esvdw.h -- C ABI of the MI355X (gfx950) library for the high-order entropy-stable
 * finite-difference scheme on adaptive moving meshes for the Euler equations with the
 * van der Waals equation of state (S. Li, H. Tang, arXiv 2407.05568).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All arrays are DEVICE pointers to caller-owned, contiguous FP64 memory, laid out
 *    field-major over the interior nodes: a[var][z][y][x], x fastest, no ghost layers.
 *    N = n[0]*n[1]*n[2] (unused directions have n = 1); nv = dim + 2 conserved variables
 *    (rho, rho v_1..v_dim, E).  Boundary conditions are applied inside the library.
 *  - Nodes are cell-centred in the computational box: xi_i = lo + (i + 1/2) dxi,
 *    dxi = (hi - lo)/n, matching the fixed uniform computational mesh of Section 3.
 *  - Every call is asynchronous on the given stream, never synchronises the host and
 *    allocates nothing (scratch belongs to the context); sequences of calls can be captured
 *    into a HIP graph.  Device scalars (dt, residuals, sweep counts) go to caller device
 *    pointers.
 *  - The int return value reports synchronous errors only: ESVDW_OK, ESVDW_EINVAL (null
 *    pointer, bad size or option), ESVDW_EHIP (a HIP launch failed).  Numerical conditions
 *    found by the kernels (inadmissible states, failure of the mean-value constraint of
 *    Theorem 3.1, NaN, mesh iteration not converged) are OR-ed into a device status word that
 *    esvdw_get_status() reads back.
 *  - Units are general: p = rho R T/(1 - b rho) - a rho^2, e = c_v T - a rho (eq. vdWEOS).
 *    The paper's dimensionless units are (R, c_v, a, b) = (1, 1/delta, 9/8, 1/3); the
 *    "reduced" units (8/3, (8/3)/delta, 3, 1/3) make the critical point (1, 1, 1).
 */
#ifndef ESVDW_H
#define ESVDW_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ESVDW_OK 0
#define ESVDW_EINVAL (-1)
#define ESVDW_EHIP (-2)
#define ESVDW_ENOTIMPL (-3)
#define ESVDW_ESCRATCH (-4) /* the problem exceeds a no-allocation entry point's static scratch */

#define ESVDW_F_INADMISSIBLE 1u   /* a node state violates eq. coefflimit / eq. Tlimit */
#define ESVDW_F_MEANCONSTRAINT 2u /* D <= 0 (Theorem 3.1) or a non-positive S^2 entry */
#define ESVDW_F_NAN 4u            /* a NaN reached an output */
#define ESVDW_F_NOTCONVERGED 8u   /* tolerance-mode mesh iteration hit its sweep cap */
#define ESVDW_F_BARRIER 16u       /* a batched stage kernel gave up waiting at a grid barrier */

#define ESVDW_BC_PERIODIC 0
#define ESVDW_BC_OUTFLOW 1 /* state: zero gradient; mesh: mirror about the boundary face */
/* esvdw_params.walls bits: a face of an outflow direction k may instead be a reflecting (slip)
 * wall (Examples 5.4-5.5 have walls): state ghosts mirror the interior about the face with the
 * velocity component normal to it reversed; the mesh mirrors as for outflow. */
#define ESVDW_WALL_LO(k) (1 << (2 * (k)))
#define ESVDW_WALL_HI(k) (1 << (2 * (k) + 1))

#define ESVDW_MON_VDW 0  /* monitor of Section 4 (squared gradient terms + |Delta G|^2) */
#define ESVDW_MON_SINE 1 /* monitor of Example 5.1 (|grad rho|, |Delta rho|) */
#define ESVDW_VAR_RHO 0
#define ESVDW_VAR_G 1

typedef struct esvdw_params {
  int dim;              /* 1, 2 or 3 */
  int n[3];             /* interior nodes per direction (>= 6 in active directions) */
  double lo[3], hi[3];  /* computational box (equal to the physical box at t = 0) */
  int bc[3];            /* ESVDW_BC_* per direction */
  double R, cv, a, b;   /* gas constant, heat capacity, van der Waals a >= 0, b >= 0 */
  int dissipation;      /* 0: entropy-conservative flux only; 1: entropy-stable flux */
  double weno_lin[3];   /* MR-WENO linear weights of the 5-, 3-, 1-point levels (Section 5) */
  double weno_eps;      /* MR-WENO epsilon (1e-10) */
  double cfl;           /* eq. cfl; 0.4 in 1D/2D and 0.3 in 3D in the paper */
  double dt_fixed;      /* > 0: use this time step instead of eq. cfl */
  int monitor_kind;     /* ESVDW_MON_* */
  int kappa;            /* number of gradient terms in the vdW monitor (0..2) */
  int mon_var[2];       /* ESVDW_VAR_* of each gradient term */
  double alpha[3];      /* alpha_1..alpha_{kappa+1} (sine monitor: alpha_1, alpha_2) */
  int n_filter;         /* low-pass filter passes (3..10, 20 in the smooth tests) */
  int mu;               /* Jacobi sweeps (fixed mode) or the sweep cap (tolerance mode) */
  double mesh_tol;      /* tolerance of the Jacobi stop test (max node update) */
  int fixed_mu;         /* 1: exactly mu sweeps; 0: stop once the update is < mesh_tol */
  int walls;            /* ESVDW_WALL_LO / _HI bits (outflow directions only; 0: none) */
  /* Backward-facing step (Example 5.5; 2D, both directions outflow, fixed_mu = 1): the nodes
   * i0 < step[0], i1 < step[1] (step[k] >= 3) form a solid block whose two faces are
   * reflecting walls; the fluid is the L-shaped rest, with at least 3 nodes beyond the block in
   * each direction.  Seen along a direction, the 3 solid nodes next to a face stand for the
   * mirror images of the fluid nodes across it; the solid nodes keep their state (those next to
   * the step hold the images, for the monitor), the mesh holds the images of the fluid mesh
   * there, and the 6 x 6 nodes around the corner form a lattice mirror-symmetric about both
   * faces (the mesh iteration moves it as a whole).  step = {0, 0}: no step. */
  int step[2];
  int inflow;           /* 1: the lo face of direction 0 (outflow, not a wall; 2D) holds the fixed
                           state inflow_prim in its ghost layers */
  double inflow_prim[4]; /* rho, v_1, v_2, p of the inflow state (admissible) */
} esvdw_params;

typedef struct esvdw_ctx esvdw_ctx;

/* Validates the parameters and allocates the context's scratch on the current device.
 * Ownership of *out passes to the caller (release with esvdw_destroy).  EINVAL on bad
 * parameters (among them a grid whose padded node count, with 3 ghost layers per side and the
 * x rows rounded up to 16, reaches 2^29: the kernels address a field with 32-bit byte offsets),
 * EHIP on allocation failure. */
int esvdw_create(const esvdw_params *p, esvdw_ctx **out);
void esvdw_destroy(esvdw_ctx *ctx);

/* Synchronises the device, copies the status word (ESVDW_F_* bits) to *flags_host and
 * clears it when clear != 0. */
int esvdw_get_status(esvdw_ctx *ctx, unsigned *flags_host, int clear);
const char *esvdw_strerror(int code);

/* Mesh at t = 0 (Section 3.2).  If uniform != 0, x (dim fields) is first set to the uniform
 * mesh x = xi.  J (1 field) receives the discrete Jacobian det(dx/dxi) evaluated with the
 * same sixth-order central operators delta_k as the metrics (eq. SCLCoeff): in 2D
 * (delta_1[x_1] delta_2[x_2] - delta_2[x_1] delta_1[x_2])/(dxi_1 dxi_2). */
int init_mesh(esvdw_ctx *ctx, double *x, double *J, int uniform, hipStream_t stream);

/* JU = J U(prim) with prim = (rho, v_1..v_dim, p) fields and U = (rho, rho v, E),
 * E = rho e + rho |v|^2/2 (eq. ConserLaw2, eq. vdWEOS). */
int init_state(esvdw_ctx *ctx, const double *prim, const double *J, double *JU, hipStream_t stream);

/* Discrete metrics of Section 3.2 at the interior nodes: met[(k*dim + j)] = J dxi_k/dx_j
 * (eq. SCLCoeff; conservative nested form in 3D) and xit[k] = J dxi_k/dt =
 * -sum_j xdot_j J dxi_k/dx_j (eq. VCLCoeff).  xdot may be NULL (static mesh: xit = 0). */
int compute_metrics(esvdw_ctx *ctx, const double *x, const double *xdot, double *met, double *xit,
                    hipStream_t stream);

/* Semi-discrete right-hand side, eq. semi_U and eq. semi_J: dJU (nv fields) and dJ (1 field)
 * from the state (JU, J) and interior metrics (met, xit as written by compute_metrics; xit
 * may be NULL).  The interface flux is the sixth-order EC flux (eq. ECFlux_curv_2p built on
 * the two-point flux eq. ECfluxMM) minus, if dissipation is on, the scaled-eigenvector
 * MR-WENO dissipation of eq. HOstable.  Ghost metrics follow the boundary symmetry. */
int es_rhs(esvdw_ctx *ctx, const double *JU, const double *J, const double *met, const double *xit,
           double *dJU, double *dJ, hipStream_t stream);

/* One third-order SSP Runge-Kutta stage s in {0, 1, 2} (Shu-Osher form) on the moving mesh:
 * the RHS of the stage input (JUs, Js) is evaluated on the stage mesh x_n + c_s dt xdot,
 * c = (0, 1, 1/2), with metrics computed in place from that mesh, then
 *   s=0: out = in + dt L;  s=1: out = 3/4 base + 1/4 (in + dt L);  s=2: out = 1/3 base + 2/3 (in + dt L)
 * with base = (JU0, J0).  dt_dev: device pointer to dt.  xdot may be NULL (static mesh).
 * (JUout, Jout) may alias the base but not the stage input.  If s == 2 and x_next is not
 * NULL, x_next = x_n + dt xdot (x_next may alias x_n). */
int rk_stage(esvdw_ctx *ctx, int s, const double *dt_dev, const double *JU0, const double *J0,
             const double *JUs, const double *Js, const double *x_n, const double *xdot, double *JUout,
             double *Jout, double *x_next, hipStream_t stream);

/* Mesh redistribution between time steps (Section 4): monitor omega from U^n (eq.
 * van der Waalsmonitor or eq. van der Waalssinmonitor), n_filter low-pass passes, Jacobi
 * iteration of the discretised eq. mesh_EL from x^[0] = x_n (+ warm_dx if not NULL) for mu
 * sweeps (or to mesh_tol), the movement limiter Delta_gamma, the time step of eq. cfl (or
 * dt_fixed), and finally xdot = Delta_gamma (x^[mu] - x_n)/dt.  Outputs: xdot (dim fields),
 * *dt_dev, *resid_dev (max node update of the last sweep), *sweeps_dev (sweeps done); any of
 * resid_dev / sweeps_dev may be NULL.  In tolerance mode the call synchronises the stream
 * between sweep batches (not capturable). */
int redistribute_mesh(esvdw_ctx *ctx, const double *JU, const double *J, const double *x_n,
                      const double *warm_dx, double *xdot, double *dt_dev, double *resid_dev,
                      int *sweeps_dev, hipStream_t stream);

/* Building blocks of redistribute_mesh, exposed for tests and the learned warm start.
 * mesh_monitor: omega (1 field) = filtered monitor from (JU, J).
 * mesh_jacobi: nsweep Jacobi sweeps on x (dim fields, updated in place) with fixed omega;
 *   *resid_dev = max node update of the last sweep (may be NULL).
 * mesh_limiter: *gamma_dev = Delta_gamma for the move x_n -> x_mu.
 * cfl_dt: *dt_dev = CFL / max_i sum_k L_k (|v . n_k| + c)/(J dxi_k) on the mesh x. */
int mesh_monitor(esvdw_ctx *ctx, const double *JU, const double *J, double *omega, hipStream_t stream);
int mesh_jacobi(esvdw_ctx *ctx, const double *omega, double *x, int nsweep, double *resid_dev,
                hipStream_t stream);
/* Red-black successive over-relaxation for the same discretised eq. mesh_EL (Section 4) as
 * mesh_jacobi, with the same fixed point: an alternative solver for the mesh iteration
 * (Gauss-Seidel for relax = 1).  A sweep updates the nodes with i0 + i1 + i2 even, then the odd
 * ones, in place; each node solves its own equation with the other colour held fixed (at an
 * outflow wall its mirror image is itself: normal coordinate 2 wall - x, tangential x) and moves
 * to x + relax (v - x).  nsweep sweeps on x (dim fields) with fixed omega; *resid_dev = the
 * largest |v - x| of the last sweep (may be NULL).  ESVDW_EINVAL unless 0 < relax < 2 and every
 * periodic direction has an even node count (the wrap must join opposite colours), and for a
 * problem with the backward-facing step (not supported). */
int mesh_sor(esvdw_ctx *ctx, const double *omega, double *x, int nsweep, double relax, double *resid_dev,
             hipStream_t stream);
int mesh_limiter(esvdw_ctx *ctx, const double *x_n, const double *x_mu, double *gamma_dev, hipStream_t stream);
/* mesh_converged: copies into xmu_out (dim fields) the Jacobi result x^[mu] of the last
 *   redistribute_mesh call on this context, before the movement limiter (Section 4); the
 *   target of the learned warm start.  Stream-ordered after that call. */
int mesh_converged(esvdw_ctx *ctx, double *xmu_out, hipStream_t stream);
int cfl_dt(esvdw_ctx *ctx, const double *JU, const double *J, const double *x, double *dt_dev,
           hipStream_t stream);

/* cfl_dt for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): needs no context and calls no allocating
 * routine.  The same kernels and reduction order as cfl_dt with a context made from *p, so the
 * two give bit-identical dt.  Its per-block maxima live in a static device array of 65544 doubles
 * (512 KiB) that each GPU the library runs on holds until the process ends; it is looked up on
 * the first call on a device.  Limits: dim 1 or 2 (3D needs the metric scratch of a context), at
 * most 65536 blocks (1D: ceil(n0/256); 2D: tiles of 64 x 16 nodes, ceil(n0/64) ceil(n1/16), e.g.
 * 16384^2);
 * ESVDW_ESCRATCH beyond that, ESVDW_EINVAL for bad parameters or pointers.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (concurrent streams or threads) race
 * and must be serialised by the caller.  *dt_dev: the time step (device pointer). */
int cfl_dt_noalloc(const esvdw_params *p, const double *JU, const double *J, const double *x, double *dt_dev,
                   hipStream_t stream);

/* One complete time step in place: redistribute_mesh (fixed mu) when moving != 0, else the
 * CFL time step on the fixed mesh; three rk_stage calls using the context's stage buffers;
 * x <- x + dt xdot.  *dt_dev receives dt.  Capturable into a HIP graph. */
int esvdw_step(esvdw_ctx *ctx, double *JU, double *J, double *x, int moving, double *dt_dev,
               hipStream_t stream);

/* Measurement hook: launches one internal kernel `reps` times on `stream` with the
 * context's current scratch contents, so that a caller can bracket it with stream events.
 * which = 1, 2, 3: the interface-flux kernel of direction 1, 2, 3 (reads the node data left
 * by the last RHS evaluation, writes the context's flux buffer); which = 5: one Jacobi sweep
 * of the context's mesh-iteration buffers; which = 6: a plain copy of 2 (dim + 3) N doubles
 * between the context's stage buffers (reads and writes 16 (dim + 3) N bytes: a reference for
 * memory-traffic counters).  Call only after a step or RHS on this context.
 * EINVAL for an unknown kernel or a direction beyond dim. */
int esvdw_bench_kernel(esvdw_ctx *ctx, int which, int reps, hipStream_t stream);

/* ---- learned warm start for the mesh equations (2D) --------------------------------------
 * A 50 -> 64 -> 64 -> 2 ReLU MLP proposes the displacement x* - x^n (in units of dxi) of the
 * converged mesh from node features; the plain Jacobi iteration of redistribute_mesh then
 * starts from x^n + warm_dx and decides convergence (the network is never trusted alone).
 * Parameters: MLP_NPARAM = 9360 FP32 values, packed W1[64][64] (inputs 50..63 unused), b1[64],
 * W2[64][64], b2[64], W3[64][16] (outputs 2..15 unused), b3[16]; W[k][j] maps input k to
 * output j.  Matrix products run on BF16 operands with FP32 accumulation. */
#define ESVDW_MLP_NPARAM 9360

/* feat (2 N floats): f1 = |grad_xi rho|^2 / max |grad_xi rho|^2 (second-order central
 * differences, as in the monitor of Section 4) and f2 = tanh G (eq. fundamental) per node. */
int mlp_features(esvdw_ctx *ctx, const double *JU, const double *J, float *feat, hipStream_t stream);

/* warm_dx (2 N doubles) = dxi * MLP(5 x 5 stencil of (f1, f2), boundary values replicated),
 * clipped to +-64 dxi per component (a guard only: the Jacobi iteration that follows is
 * linear in x and converges from any start). */
int mlp_infer(esvdw_ctx *ctx, const float *feat, const float *params, double *warm_dx, hipStream_t stream);

/* Training gradient: for the sample list samples[2 s] = frame, samples[2 s + 1] = node index
 * (s < nsamples) over frames stored frame-major in feats ([frame][2][N] floats, as written by
 * mlp_features) and targets ([frame][2][N] floats, displacement / dxi), computes
 * loss = scale * sum_s |MLP(s) - target(s)|^2 into *loss_dev and its gradient with respect to
 * params into grad (MLP_NPARAM floats, overwritten). */
int mlp_grad(esvdw_ctx *ctx, const float *feats, const float *targets, const int *samples, long nsamples,
             float scale, const float *params, float *grad, float *loss_dev, hipStream_t stream);

/* One Adam step (beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias-corrected at step >= 1) on the FP32
 * parameters with moment buffers m, v (MLP_NPARAM floats each, zero-initialised by the caller). */
int mlp_adam(float *params, const float *grad, float *m, float *v, int step, float lr, hipStream_t stream);

/* ---- Batched independent 2D problems ------------------------------------------------------
 * A batch advances ninst independent 2D problems, each with its own esvdw_params (grid size,
 * EOS constants R, c_v, a, b, boundary conditions, scheme parameters; dim must be 2), with one
 * launch of a persistent kernel per SSP-RK3 stage for all of them (the scheme of Sections
 * 3.1-3.3 at every node, the CFL step of Section 5 per instance).
 * Caller arrays are pooled device arrays in FP64: instance i owns nodes [off[i], off[i+1]) and
 * a pool with F fields stores instance i's fields contiguously from base + F off[i], in the
 * single-problem layout ([field][y][x], N_i nodes per field).  Pools: x (2 fields), xdot (2),
 * J (1), JU (4), prim (4: rho, v1, v2, p).  dt: ninst doubles. */
typedef struct esvdw_batch esvdw_batch;

/* Creates a batch (allocates its device scratch).  Returns ESVDW_EINVAL for an invalid or
 * non-2D parameter set. */
int esvdw_batch_create(int ninst, const esvdw_params *params, esvdw_batch **out);
void esvdw_batch_destroy(esvdw_batch *b);
/* Node offsets of the instances in the pools (off: ninst + 1 longs, may be NULL); returns the
 * total node count. */
long esvdw_batch_offsets(const esvdw_batch *b, long *off);
/* Uniform meshes and their Jacobians for every instance (as init_mesh with uniform = 1). */
int esvdw_batch_init_mesh(esvdw_batch *b, double *x, double *J, hipStream_t stream);
/* Conserved variables JU = J U(prim) for every instance (as init_state). */
int esvdw_batch_init_state(esvdw_batch *b, const double *prim, const double *J, double *JU, hipStream_t stream);
/* One SSP-RK3 stage s of every instance, in the semantics of rk_stage: step base (JU0, J0),
 * stage input (JUs, Js), output (JUout, Jout) (may alias the base but not the stage input).
 * Stage 0 first computes each instance's CFL step dt[i] = cfl / max over nodes of the
 * spectral-radius sum on (JU0, J0, x) (or dt_fixed) and stages 1, 2 read it.  xdot (may be
 * NULL: fixed meshes) is the mesh velocity of the step: stage s uses the mesh x + c_s dt xdot,
 * and stage 2 advances x in place to x + dt xdot. */
int esvdw_batch_stage(esvdw_batch *b, int s, const double *JU0, const double *J0, const double *JUs,
                      const double *Js, double *JUout, double *Jout, double *x, const double *xdot, double *dt,
                      hipStream_t stream);
/* Mesh redistribution of every instance (Section 4), as redistribute_mesh with a fixed sweep
 * count: monitor omega from (JU, J) with each instance's monitor parameters and per-instance
 * maxima, n_filter low-pass passes, mu Jacobi sweeps from x^[0] = x, the movement limiter (one
 * Delta_gamma per instance), the CFL step dt[i] (as in esvdw_batch_stage) and
 * xdot = Delta_gamma (x^[mu] - x)/dt (pool of 2 fields).  x is not modified.  Requires that all
 * instances use fixed_mu = 1 and share n_filter and mu (ESVDW_EINVAL otherwise).  A moving-mesh
 * step is esvdw_batch_redistribute followed by esvdw_batch_step with this xdot. */
int esvdw_batch_redistribute(esvdw_batch *b, const double *JU, const double *J, const double *x, double *xdot,
                             double *dt, hipStream_t stream);
/* One full SSP-RK3 step of every instance in place (three esvdw_batch_stage launches through
 * the batch's own stage buffers); capturable in a HIP graph. */
int esvdw_batch_step(esvdw_batch *b, double *JU, double *J, double *x, const double *xdot, double *dt,
                     hipStream_t stream);
/* Launch variants: count, and the choice used by later launches.  Variants 0 .. count/2 - 1 run
 * each stage as one launch of a persistent kernel (grid barriers between its phases);
 * count/2 .. count - 1 run the same phases as separate launches (CFL and dt at stage 0, node
 * data, direction-1 fluxes, then the direction-0 fluxes together with the update), each at its
 * own occupancy.  Within a mode, variants differ in the interface-tile shapes.  Results agree
 * across variants to rounding (measured: within 1e-15 of the field maximum); only speed
 * differs. */
int esvdw_batch_variants(void);
int esvdw_batch_set_variant(esvdw_batch *b, int variant);
/* Synchronises the device, copies the batch's status word (ESVDW_F_* bits) and clears it. */
int esvdw_batch_get_status(esvdw_batch *b, unsigned *flags_host);

#ifdef __cplusplus
}
#endif
#endif
