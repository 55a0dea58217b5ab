/*
 * sa_iga.h - C ABI of the MI355X (gfx950) semi-analytical isogeometric
 * thermal model for laser powder bed fusion.
 *
 * The model (Yang, Ji, Moeller, Ayas, "Efficient thermal simulation in metal
 * additive manufacturing via semi-analytical isogeometric analysis"):
 *
 *   T = T~ + T^                                             (Eq. 6)
 *   T~(x,t) = sum over switched-on point sources I of
 *       s E_I / (rho c_p [4 pi alpha D_I]^{3/2}) exp(-|x - x_I|^2 / (4 alpha D_I)),
 *       D_I = t - t_I + r^2/(8 alpha),  alpha = k/(rho c_p)   (Eqs. 2, 7, 8)
 *   T^ solves the heat equation with the transferred data   (Eqs. 9-11)
 *       -k dT^/dn = k dT~/dn on the lateral (NEUMANN) faces,
 *       T^ = T_c - T~ on the bottom (DIRICHLET) face,
 *   discretised with NURBS (Eqs. 13-18) and stepped with the theta-scheme
 *       (M/dt + theta K) u^{n+1} = (M/dt - (1-theta) K) u^n
 *                                  + theta F^{n+1} + (1-theta) F^n   (Eq. 20)
 *   F_A = sum_q R_A(x_q) (-k grad T~(x_q) . n_q) w_q dS_q  over NEUMANN faces (Eq. 18).
 *
 * Every function returns an int status (sa_status).  On failure the message
 * is available from sa_iga_last_error() (thread-local); objects are left in
 * their previous state unless stated otherwise.  No C++ exception crosses
 * this boundary.
 *
 * Conventions fixed by this interface (the FP64 oracle used by the tests
 * follows the same ones):
 *   - Units are SI (m, s, W, J, K).
 *   - Parametric faces f = 0..5 are xi0=0, xi0=1, xi1=0, xi1=1, xi2=0, xi2=1.
 *   - DOF (control point) index A = a0 + n0*(a1 + n1*a2).
 *   - Boundary quadrature points: face 0 first, then 1, ..., 5; on face f
 *     with fixed direction d and in-face directions a < b, the points form a
 *     row-major grid over (b, a) (a fastest); along each in-face direction
 *     they are ordered by element, then by the quad_face Gauss points of
 *     that element.
 *   - Source i of a path is switched on at tick_i * delta with
 *     delta = dt / sources_per_step; theta-step n -> n+1 ends at
 *     t = (n+1) dt and includes the sources with tick <= (n+1)*sources_per_step.
 *     Causality is decided on these integers; the age t - t_i is formed as
 *     ((n+1)*sources_per_step - tick_i) * delta.
 *   - The initial state is u = T_c (every control value), F = 0.
 *   - The Dirichlet values at t^{n+1} are the L2 projection of T_c - T~ on
 *     the trace space of the control variables of the DIRICHLET faces.
 */
#ifndef SA_IGA_H
#define SA_IGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sa_iga sa_iga;   /* opaque; owns its device memory */

enum sa_status {
  SA_OK = 0,
  SA_EINVAL = -1,    /* invalid argument (NULL, sizes, knots, weights, ticks, theta) */
  SA_ENOMEM = -2,    /* host or device allocation failed */
  SA_EDEVICE = -3,   /* HIP runtime error or no gfx950 device */
  SA_ENOCONV = -4,   /* PCG did not reach pcg_rtol within pcg_max_iter */
  SA_ERANGE = -5,    /* query point outside [0,1]^3 or path index out of range */
  SA_ESTATE = -6     /* object in a sticky error state (earlier ENOCONV / NaN) */
};

enum sa_face_role {
  SA_FACE_NEUMANN = 0,       /* lateral, adiabatic: takes the flux load F (Eq. 10) */
  SA_FACE_DIRICHLET = 1,     /* bottom: T = T_c (Eq. 11) */
  SA_FACE_SOURCE_PLANE = 2,  /* top: holds the sources; adiabatic by Eq. 8, no load */
  SA_FACE_INTERFACE = 3      /* multi-patch models only (sa_mp_setup): glued to a face of another
                                patch; no boundary points, no load */
};

enum sa_precision {
  SA_PREC_FP64 = 0,          /* every source in FP64 */
  SA_PREC_FP32_FAR = 1,      /* sources older than tau_near summed in FP32 (exp2),
                                FP32 tile partials accumulated in FP64; near
                                sources, loads and the solve in FP64 */
  SA_PREC_SURROGATE = 2      /* far sources replaced by the learned network (sa_mlp), near
                                sources in FP64.  A path's network is audited against the
                                exact FP64 far sum on the first step with far sources and
                                then every audit_every steps; before its first passing
                                audit, and after a failing one, the path sums its far
                                sources as SA_PREC_FP32_FAR does */
};

enum sa_precond {
  SA_PRECOND_JACOBI = 0,
  SA_PRECOND_FD = 1          /* fast diagonalisation of a Kronecker approximation */
};

typedef struct {
  int32_t degree[3];           /* p_d >= 1 */
  int32_t n_ctrl[3];           /* n_d >= p_d + 1 */
  const double *knots[3];      /* n_d + p_d + 1 values, non-decreasing, open
                                  (p_d+1 repeated end knots), from 0 to 1 */
  const double *ctrl_xyzw;     /* [n2][n1][n0][4]: x, y, z (m), weight > 0 */
  int32_t face_role[6];        /* sa_face_role per parametric face */
  int32_t quad_vol[3];         /* Gauss points per element per direction (1..16) */
  int32_t quad_face;           /* Gauss points per direction on faces (1..16) */
} sa_patch;

typedef struct {
  double k;                    /* conductivity W/(m K) > 0 */
  double rho;                  /* density kg/m^3 > 0 */
  double cp;                   /* heat capacity J/(kg K) > 0 */
  double T0;                   /* platform and initial temperature T_c (K) */
} sa_material;

typedef struct {
  double theta;                /* theta-scheme parameter in [0,1]; default 0.5 */
  double kernel_scale;         /* s in the kernel; default 1 (Eq. 8 as printed) */
  int32_t precision;           /* sa_precision; default SA_PREC_FP64 */
  double tau_near;             /* near/far age split (s) for FP32_FAR/SURROGATE; default 2e-4 */
  double pcg_rtol;             /* stop when |r| <= pcg_rtol |rhs|; default 1e-13 */
  int32_t pcg_max_iter;        /* default 2000 */
  int32_t preconditioner;      /* sa_precond; default SA_PRECOND_FD */
  int32_t timing;              /* nonzero: time every stage with HIP events (sa_stats) */
  int32_t points_per_lane;     /* kernel-sum register blocking (1, 2, 4); 0 = tuned default */
  int32_t waves_per_group;     /* kernel-sum waves per workgroup (1, 2, 4, 8); 0 = tuned default */
  int32_t chunk_sources;       /* sources per source chunk of the sum; 0 = tuned default */
  /* SA_PREC_SURROGATE only: the far-history network (see sa_mlp below).
   * surrogate_weights [surrogate_len] = {T_scale (K), G_scale (K/m),
   * E_scale (J), then the sa_mlp_n_params() FP32 parameters}; copied at set-up. */
  const float *surrogate_weights;
  int64_t surrogate_len;
  int32_t audit_every;         /* audit a path's network on its first step with far sources,
                                  then every this many steps (>= 1); default 50 */
  double audit_frac;           /* fraction of the boundary points audited; default 0.01 */
  double audit_tol;            /* K: largest far-temperature error an audit passes; default 0.5 */
} sa_solver_options;

typedef struct {
  int32_t n_paths;             /* independent scan strategies on the same patch */
  const int64_t *src_offset;   /* [n_paths+1]; path p owns rows src_offset[p] .. src_offset[p+1]-1 */
  const double *xyz;           /* [N][3] source positions (m) */
  const int64_t *tick;         /* [N] activation ticks >= 1, non-decreasing within a path */
  const double *energy;        /* [N] source energies (J) */
  const int32_t *n_steps;      /* [n_paths] theta-steps of each path (>= 0) */
  double dt;                   /* theta-step length (s) > 0 */
  int32_t sources_per_step;    /* ticks per theta-step >= 1 */
  double spot_radius;          /* r (m) >= 0: D = age + r^2/(8 alpha) */
  const sa_solver_options *opt;  /* NULL = defaults */
} sa_scan_path;

typedef struct {
  int32_t n_ctrl[3];
  int64_t n_dof;
  int64_t n_bpts;              /* boundary quadrature points (all six faces) */
  int64_t face_offset[7];      /* points of face f: face_offset[f] .. face_offset[f+1]-1 */
  int32_t n_paths;
  int64_t n_sources;
  int64_t n_dirichlet;         /* control variables fixed by DIRICHLET faces */
  int32_t tensor_faces;        /* planar faces whose points form a grid along Cartesian axes: their
                                  kernel sums run as matrix products (the Gaussian of Eq. 8 factorises) */
  int64_t generic_points;      /* boundary points of the other faces (summed pair by pair) */
  int32_t blocked_steps;       /* steps per source-side block of a one-path call (1: every step alone):
                                  the sums, load vectors and Dirichlet data of that many steps go
                                  through one launch each */
  int32_t sum_groups_per_cu_batch; /* matrix-core sum: workgroups per compute unit of a launch of four
                                  paths or more (0: no tensor faces) */
  int32_t block_lds_pad;       /* matrix-core sum of a blocked call: extra LDS bytes per workgroup, which
                                  leaves compute-unit room to the solver kernels beside it */
  int32_t batch_lds_pad;       /* the same for a launch of four paths or more (default 10000; 0
                                  without tensor faces) */
} sa_info;

enum sa_stage {
  SA_STAGE_COEFF = 0,          /* per-step source coefficients */
  SA_STAGE_SUM = 1,            /* kernel sum at the boundary points (dominant) */
  SA_STAGE_REDUCE = 2,         /* chunk reduction, flux and Dirichlet densities */
  SA_STAGE_LOAD = 3,           /* load-vector and projection right-hand-side gathers */
  SA_STAGE_DIRICHLET = 4,      /* projection solve */
  SA_STAGE_RHS = 5,            /* theta-scheme right-hand side */
  SA_STAGE_PCG = 6,            /* theta-scheme solve */
  SA_STAGE_NET = 7,            /* far-history network and its audits (SA_PREC_SURROGATE) */
  SA_N_STAGES = 8
};

typedef struct {
  int64_t steps;               /* theta-steps advanced, summed over paths */
  int64_t pairs;               /* source x point pairs evaluated, summed */
  int64_t pairs_near;          /* of which in FP64 (all of them with SA_PREC_FP64) */
  int64_t pcg_iterations;      /* summed over steps and paths */
  int32_t pcg_last_iterations;
  double pcg_last_relres;
  int64_t dirichlet_iterations;
  double stage_ms[SA_N_STAGES];        /* device time per stage (timing != 0) */
  int64_t stage_launches[SA_N_STAGES]; /* kernel launches per stage (timing != 0) */
  /* SA_PREC_SURROGATE */
  int64_t net_steps;           /* path-steps whose far part came from the network */
  int64_t pairs_net;           /* far source x point pairs the network replaced */
  int64_t audits;              /* audits run */
  int64_t audit_failures;      /* audits above audit_tol (the path then sums its far sources) */
  double audit_max_err;        /* largest audited error of the far temperature (K) */
  int64_t rollbacks;           /* calls whose steps were run again with a second PCG iteration
                                  (one iteration did not reach the tolerance on some step) */
  double host_enqueue_ms;      /* host time sa_iga_step spent from its first launch to its last one
                                  (before the final status check and synchronisation): issuing the
                                  launches, copies and events, and any wait inside the call (audits,
                                  a PCG fallback's synchronisation); an upper bound of the host's
                                  share, on which the device need not wait while it stays below the
                                  device time of the same steps */
} sa_stats;

/* Fill *opt with the defaults listed above. */
int sa_iga_default_options(sa_solver_options *opt);

/*
 * Build the model on the current HIP device: basis and quadrature tables,
 * M and K (Eqs. 16-17), boundary tables (Eq. 18), source tables, state
 * u^0 = T_c, F^0 = 0.  All input arrays are copied; the caller keeps
 * ownership.  *out receives a new object (NULL on failure).
 * Errors: SA_EINVAL (invalid patch/material/scan/options), SA_ENOMEM,
 * SA_EDEVICE (no device or HIP failure).
 */
int sa_iga_setup(const sa_patch *patch, const sa_material *mat, const sa_scan_path *scan,
                 sa_iga **out);

/*
 * Advance every path by n_steps theta-steps (Eq. 20); a path that has done
 * its n_steps[p] steps stays as it is.  Starts after the work already queued
 * on the object's stream and returns after the last step is complete.  With
 * the fused solvers the source side of each step (kernel sum; reduction, load
 * vector and Dirichlet data) runs on two internal streams, one step ahead of
 * the theta-step solves on the object's stream; the results are bitwise those
 * of the serial order (environment variable SA_IGA_SERIAL at set-up selects
 * that order).  A call that advances one path (or up to four at one step
 * parity) on the matrix-core sum runs in blocks of sa_info.blocked_steps
 * steps, whose sums, load vectors and Dirichlet data go through one launch
 * each; the results are bitwise those of one step at a time.  Where the fast-diagonalisation solve is exact (an affine
 * axis-aligned block with the FD preconditioner) a theta-step is one
 * application of it, u^{n+1} = x0 + P r0; its residual against the tolerance
 * is formed by the next step's right-hand side passes or, for a path's last
 * step of the call, by a check pass before the call returns.  If a step
 * missed the tolerance, the state goes back to the call's start and the
 * steps run again with two PCG iterations each (sa_stats.rollbacks), which
 * stays the object's form from then on.  SA_ENOCONV if a solve did not
 * converge (the object then enters the sticky error state SA_ESTATE).
 */
int sa_iga_step(sa_iga *h, int32_t n_steps);

/* Steps done so far by path `path`. */
int sa_iga_get_step(sa_iga *h, int32_t path, int64_t *step);

/*
 * Temperature T = T~ + T^ (Eq. 21) and optionally its gradient at n
 * parametric points xi [n][3] in [0,1]^3 of path `path`, at its current
 * time.  T [n] and gradT [n][3] (may be NULL) are host arrays.
 * SA_ERANGE if a point lies outside [0,1]^3 or path is out of range.
 */
int sa_iga_eval_temperature(sa_iga *h, int32_t path, int64_t n, const double *xi,
                            double *T, double *gradT);

/*
 * T = T~ + T^ (Eq. 21) and optionally its gradient at n PHYSICAL points
 * x [n][3] (m, host) of path `path` at its current time: each point is first
 * mapped back to the parametric domain (the inverse of the geometry map:
 * the nearest element centre, then Newton steps on x(xi) = x kept in
 * [0,1]^3, to 1e-13 of the patch size).  A point that is not reached lies
 * outside the patch and gets NaN in T, gradT and xi.  T [n], gradT [n][3]
 * and xi [n][3] (the parametric points) are host arrays; gradT and xi may be
 * NULL.
 */
int sa_iga_eval_temperature_at(sa_iga *h, int32_t path, int64_t n, const double *x, double *T, double *gradT,
                               double *xi);

/*
 * Net heat-loss rate along a boundary edge (Sec. 3.1, the check of the
 * adiabatic condition, Tables 3-4): at `quad` (1..16) Gauss points per
 * element of the edge where parametric face `face` meets face `edge_face`
 * (faces of different directions, e.g. a lateral face and the top), at path
 * `path`'s current time,
 *   q~ = -k grad T~ . n,  q^ = -k grad T^ . n      (n: outward unit normal of `face`)
 * and the line integrals integrals[0] = int |q~ + q^| ds, integrals[1] =
 * int |q~| ds over the edge.  Host outputs, any may be NULL: x [n][3] the
 * points, normal [n][3], ds [n] the arc-length weights, q_tilde [n], q_hat [n].
 * *n_pts: on input the capacity of the per-point arrays, on output the
 * number of points n (elements along the edge x quad); with every output
 * NULL the call only sets *n_pts.  SA_EINVAL for faces that do not meet,
 * quad out of range or arrays shorter than n (*n_pts is then set to n).
 */
int sa_iga_heat_loss(sa_iga *h, int32_t path, int32_t face, int32_t edge_face, int32_t quad, int64_t *n_pts,
                     double *x, double *normal, double *ds, double *q_tilde, double *q_hat, double *integrals);

/*
 * Copy the current fields of path `path` to host arrays (any may be NULL):
 * T_gp [n_bpts] and grad_gp [3][n_bpts] (component-major) = T~ and
 * grad T~ at the boundary points at the path's current time (as summed by
 * the last step), F [n_dof] = the load vector F^n, du [n_dof] = the control
 * values of T^ minus T_c at step n (the state is carried as this deviation,
 * so it is returned without the T_c offset; add T_c for T^).
 */
int sa_iga_get_boundary_fields(sa_iga *h, int32_t path, double *T_gp, double *grad_gp,
                               double *F, double *du);

/*
 * Device-pointer variants of the two queries above, for zero-copy use of
 * caller-owned device memory (e.g. torch tensors): every array argument is
 * a DEVICE pointer with the layout of the host version, the work is
 * enqueued on the object's stream (sa_iga_set_stream) after the steps
 * already queued there, and the call returns without waiting; order the use
 * of the outputs after that stream.
 *
 * sa_iga_eval_temperature_device: T = T~ + T^ (Eq. 21) and optionally its
 * gradient at n parametric points xi [n][3] of path `path` at its current
 * time; T [n], gradT [n][3] (may be NULL).  The basis functions are
 * evaluated on the device, so a point outside [0,1]^3 cannot be refused: it
 * gets NaN in T and gradT.  The call may allocate device memory (a
 * workspace the object keeps and grows to the largest query).
 * sa_iga_get_boundary_fields_device: the copies of
 * sa_iga_get_boundary_fields (T_gp [n_bpts], grad_gp [3][n_bpts], F
 * [n_dof], du [n_dof], any may be NULL), device to device.
 */
int sa_iga_eval_temperature_device(sa_iga *h, int32_t path, int64_t n, const double *xi, double *T,
                                   double *gradT);
int sa_iga_get_boundary_fields_device(sa_iga *h, int32_t path, double *T_gp, double *grad_gp, double *F,
                                      double *du);

/* Boundary quadrature tables (host arrays, any may be NULL): x [n_bpts][3],
 * outward unit normals n [n_bpts][3], weights w dS [n_bpts]. */
int sa_iga_get_boundary_points(sa_iga *h, double *x, double *normal, double *wdS);

/* y = M x (which = 0) or y = K x (which = 1) with the assembled matrices of
 * Eqs. 16-17; x, y are host arrays of n_dof values. */
int sa_iga_apply_operator(sa_iga *h, int32_t which, const double *x, double *y);

/*
 * Evaluate T~ and grad T~ (Eqs. 7-8) of path `path` at time step*dt at n
 * physical points x [n][3] (host arrays), with the precision form of the
 * object.  T [n], grad [3][n] (component-major, may be NULL).
 */
int sa_iga_eval_source_field(sa_iga *h, int32_t path, int64_t step, int64_t n,
                             const double *x, double *T, double *grad);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * evaluation of sa_iga_eval_source_field with DEVICE arrays x [n][3],
 * T [n] and grad [3][n] (component-major; may be NULL), n <= 4096 points
 * per call (SA_EINVAL beyond: split the query).  It calls no allocating
 * routine: everything besides the inputs and outputs lives in a fixed
 * 11 MiB device scratch area that the library holds on each GPU it runs on
 * until the process ends.  The work is enqueued on the object's stream
 * (sa_iga_set_stream) and the call returns without waiting; order the use
 * of T and grad after that stream.  Every call on a GPU, of any object,
 * shares that GPU's scratch area, so calls that can run at the same time on
 * one GPU race: keep them on one stream.  The source history is split into
 * at most 64 chunks, so the sums agree with sa_iga_eval_source_field's to
 * rounding (not bitwise).  SA_EDEVICE if the scratch area could not be
 * located at set-up.
 */
int sa_iga_eval_source_field_noalloc(sa_iga *h, int32_t path, int64_t step, int64_t n, const double *x,
                                     double *T, double *grad);

/*
 * Tile-shape tuner of the kernel sum (Eqs. 7-8).  For every tile shape
 * (points per lane 1, 2, 4 x waves per workgroup 1, 2, 4, 8) it runs one
 * untimed and `reps` timed theta-steps (reps >= 1) of all paths from the
 * middle of their scans through the whole step pipeline, so the timing holds
 * the overlap of the sum with the solves; the fastest shape becomes the
 * object's points_per_lane and waves_per_group.  The state (steps, u, F,
 * Dirichlet values, boundary fields, statistics, audit flags) is restored
 * afterwards.  The split of the source history into chunks does not depend on
 * the tile shape, so later results are bitwise those of any other shape.
 * When every boundary point lies on a tensor face (sa_info.generic_points
 * == 0) the pair-by-pair kernel does not run and only the default shape
 * (2 points per lane, 4 waves) is timed.  With tensor faces the launch shape
 * of the matrix-core sum is tuned the same way: with four paths or more its
 * workgroups per compute unit (4, 6, 8, 12), then its LDS padding (0, 10000,
 * 38000 bytes: three, two or one workgroup per compute unit), and for the
 * blocked calls of up to four paths its LDS padding (the same three) and
 * block length
 * (4, 8 steps; timed at a quarter, half and three quarters of the scans, the
 * better of two runs of at least 48 steps at each); the set-up shape is kept
 * unless another is at least 3 % faster.  The choice is reported in
 * sa_info (sum_groups_per_cu_batch, batch_lds_pad, block_lds_pad,
 * blocked_steps) and, like
 * the tile shape, changes no result bit.  Outputs (each may be NULL): the
 * chosen shape and its time per step of all paths in ms (0 when no path has
 * sources and more than one step: nothing to time).  SA_ESTATE in the sticky
 * error state.
 */
int sa_iga_autotune(sa_iga *h, int32_t reps, int32_t *points_per_lane, int32_t *waves_per_group,
                    double *ms_per_step);

/* Turn the per-stage HIP-event timing of later steps on (nonzero) or off. */
int sa_iga_set_timing(sa_iga *h, int32_t on);

int sa_iga_get_info(sa_iga *h, sa_info *info);
int sa_iga_get_stats(sa_iga *h, sa_stats *stats);
int sa_iga_reset_stats(sa_iga *h);

/*
 * Checkpoint of the mutable state of every path: its step, u^n, F^n, the
 * Dirichlet values, T~, grad T~ at the boundary points and, in the
 * surrogate form, its audit state (whether its far part comes from the
 * network or the exact sum, and the step of its next audit).  With
 * buf == NULL, *len receives the size needed.  sa_iga_load restores a
 * checkpoint taken from an object with the same patch and number of paths
 * (SA_EINVAL if the sizes differ or a step exceeds that path's n_steps) and
 * clears the sticky error state; sa_iga_get_boundary_fields then returns
 * bitwise what it returned when the checkpoint was taken.  Neither call
 * changes the statistics.
 */
int sa_iga_save(sa_iga *h, void *buf, size_t *len);
int sa_iga_load(sa_iga *h, const void *buf, size_t len);

/*
 * Far-history data of path `path` at time step*dt (training set generation
 * for the network): the exact FP64 far field (sources with tick <
 * step*sources_per_step - floor(tau_near/delta), Eqs. 7-8) at every boundary
 * point, T [n_bpts] and grad [3][n_bpts] (component-major), and the network
 * inputs X [n_bpts][70] (FP32): normalised position, normal, far energy per
 * 4 x 4 x 4 bin of the control-net bounding box divided by e_scale.  All three
 * are DEVICE pointers on the object's stream (X may be NULL); the call returns
 * when they are written.
 */
int sa_iga_far_field(sa_iga *h, int32_t path, int64_t step, double e_scale, float *X, double *T,
                     double *grad);

/* Use the given hipStream_t (NULL = the object's own stream) for all work;
 * sa_iga_step also uses internal streams, ordered after the work queued on
 * this stream before the call and joined back into it at the end.  The own
 * stream and the internal streams are a set of three per device that the
 * library shares among all its objects (work of different objects on them is
 * ordered, never concurrent) and keeps until the process ends. */
int sa_iga_set_stream(sa_iga *h, void *hip_stream);

/* Message of the last failure on this thread ("" if none). */
const char *sa_iga_last_error(void);

/* Free the object and its device memory.  NULL is ignored. */
void sa_iga_destroy(sa_iga *h);

/*
 * Far-history network (surrogate form).  Inputs x [70] as documented for
 * sa_iga_far_field; outputs y [4] = (T~_far / T_scale, grad T~_far / G_scale).
 *   z1 = W1 x + b1, h1 = gelu(z1)            W1 [256][70], FP32
 *   z_l = W_l h_{l-1} + b_l, h_l = gelu(z_l)  l = 2, 3, 4; W_l [256][256]
 *   y = W5 h4 + b5                           W5 [4][256], FP32
 * gelu(z) = z (1 + erf(z / sqrt 2)) / 2, evaluated in the tanh form of
 * Hendrycks & Gimpel (2016), z (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))) / 2,
 * within 4.7e-4 of it everywhere; the backward pass differentiates that same
 * tanh form.  The layers 2..4 run on the matrix
 * cores with bfloat16 operands (h_{l-1} and W_l rounded to nearest even) and
 * FP32 accumulation, h1..h4 are stored in bfloat16.  Parameters are one FP32
 * vector in the order W1, b1, W2, b2, W3, b3, W4, b4, W5, b5 (row-major,
 * sa_mlp_n_params() values).  The trainer holds FP32 master weights and Adam
 * moments (beta1 0.9, beta2 0.999, eps 1e-8) on the current device; its
 * loss is the mean of (y - t)^2 over rows and outputs.  X, Y, T below are
 * DEVICE pointers (row-major [B][70], [B][4], [B][4]) used on the trainer's
 * stream; every call returns when its results are written.
 */
typedef struct sa_mlp sa_mlp;
int64_t sa_mlp_n_params(void);
int sa_mlp_create(const float *params, int64_t n, sa_mlp **out);      /* params: host */
int sa_mlp_get_params(sa_mlp *h, float *params, int64_t n);           /* params: host */
int sa_mlp_forward(sa_mlp *h, int64_t B, const float *X, float *Y);
/* gradients of the loss (host grad [n_params] in parameter order, may be NULL) */
int sa_mlp_gradients(sa_mlp *h, int64_t B, const float *X, const float *T, float *grad, double *loss);
/* one Adam step with learning rate lr on the batch; *loss = loss before the step */
int sa_mlp_train_step(sa_mlp *h, int64_t B, const float *X, const float *T, float lr, double *loss);
int sa_mlp_set_stream(sa_mlp *h, void *hip_stream);
void sa_mlp_destroy(sa_mlp *h);

/*
 * Multi-patch models (the parts of Sec. 3.3 built from several patches).
 * NURBS patches meet face to face with matching knot vectors and control
 * points along the shared faces, which carry the role SA_FACE_INTERFACE on
 * both sides.  The caller numbers the control points globally; a shared
 * control point has one index, so the spline space is continuous (C0)
 * across the interfaces.  Eqs. 16-18 and 11 are assembled patch by patch
 * into the global numbering (every element and every boundary point belongs
 * to one patch); the kernel sum (Eqs. 7-8), the transferred data (Eqs.
 * 10-11) and the theta-scheme (Eq. 20) are those of the single-patch model.
 * On the device: the kernel sum pair by pair at every boundary point (FP64,
 * or FP32 for the sources older than tau_near), the load vector and the
 * projection right-hand side as CSR gathers, the Dirichlet projection and
 * the theta-step as CSR operators solved by preconditioned CG to pcg_rtol
 * (the theta-step on the free unknowns, the Dirichlet columns moved to the
 * right-hand side).  The preconditioner is additive Schwarz over the
 * patches, z = sum_p S_p^T A_p^-1 S_p r with A_p^-1 the fast-diagonalisation
 * solve of patch p's own operator (exact on an affine patch) and S_p the
 * restriction to its control points, with SA_PRECOND_FD (the default; else
 * where a patch has no such solve) or Jacobi.  An object holds any number of
 * scan paths (scan strategies on the same part), each with its own state;
 * sa_mp_step advances them one after another, and every query names its
 * path.
 */
typedef struct sa_multipatch sa_multipatch;   /* opaque; owns its device memory */

typedef struct {
  int32_t n_patches;
  int32_t n_paths;
  int64_t n_dof;               /* global control points */
  int64_t n_bpts;              /* boundary points (the non-interface faces of every patch, patch by
                                  patch, each patch's in the single-patch order) */
  int64_t n_dirichlet;         /* control variables fixed by DIRICHLET faces */
  int64_t n_free;
  int64_t nnz;                 /* non-zeros of the global M (and K) */
  /* of the path named in sa_mp_get_info: */
  int64_t step;                /* steps taken */
  int64_t n_steps;             /* steps of its scan */
  int64_t pcg_iterations;      /* total over the steps taken (theta-steps) */
  int64_t dirichlet_iterations;  /* total over the steps taken (projections) */
  double pcg_last_relres;      /* |r| / |b| of the last theta-step */
} sa_mp_info;

/*
 * Build a multi-patch model on the current HIP device.
 *   patches [n_patches]: as for sa_iga_setup, with SA_FACE_INTERFACE allowed;
 *   index_map: the global index of every control point, patch after patch,
 *     each patch's control points in the order A = a0 + n0 (a1 + n1 a2);
 *     the indices cover 0 .. n_dof - 1, every one used;
 *   scan: one or more paths, as for sa_iga_setup; the options (scan->opt,
 *     NULL = defaults) take
 *     precision SA_PREC_FP64 or SA_PREC_FP32_FAR; preconditioner
 *     SA_PRECOND_FD (additive Schwarz) or SA_PRECOND_JACOBI.
 * All input arrays are copied.  Errors: SA_EINVAL (invalid patch, role,
 * index map, scan or options), SA_ENOMEM, SA_EDEVICE.
 */
int sa_mp_setup(const sa_patch *patches, int32_t n_patches, const int64_t *index_map, const sa_material *mat,
                const sa_scan_path *scan, sa_multipatch **out);

/* Advance every path n_steps theta-steps (fewer at the end of its scan),
 * path 0 first.  SA_ENOCONV if a CG solve does not reach pcg_rtol within
 * pcg_max_iter iterations: that path keeps the state of its last completed
 * step, the paths before it have taken their steps, the paths after it none
 * of them. */
int sa_mp_step(sa_multipatch *h, int32_t n_steps);

/* The model's sizes and, for path `path`, its step and solver statistics.
 * SA_ERANGE if the path index is out of range (here and in the queries
 * below). */
int sa_mp_get_info(const sa_multipatch *h, int32_t path, sa_mp_info *info);

/* Host copies of path `path`'s current fields (any may be NULL), as
 * sa_iga_get_boundary_fields: T_gp [n_bpts], grad_gp [3][n_bpts]
 * (component-major), F [n_dof], du [n_dof] (global numbering). */
int sa_mp_get_boundary_fields(sa_multipatch *h, int32_t path, double *T_gp, double *grad_gp, double *F, double *du);

/* Boundary quadrature tables (host arrays, any may be NULL): x [n_bpts][3],
 * outward unit normals [n_bpts][3], weights w dS [n_bpts]. */
int sa_mp_get_boundary_points(sa_multipatch *h, double *x, double *normal, double *wdS);

/* T and grad T (Eq. 21) of path `path` at n parametric points xi [n][3] of
 * patch `patch` (host arrays: T [n], grad [n][3]) at its current step: the basis
 * contraction with the control values and the kernel sum at the mapped
 * points on the device.  SA_ERANGE if a point lies outside [0,1]^3 or the
 * patch index is out of range. */
int sa_mp_eval_temperature(sa_multipatch *h, int32_t path, int32_t patch, int64_t n, const double *xi, double *T,
                           double *grad);

/* T and grad T (Eq. 21) of path `path` at n PHYSICAL points x [n][3] (m) at
 * its current step: each point is mapped back to the parametric domain of the first
 * patch (in patch order) that holds it, by the inverse map of
 * sa_iga_eval_temperature_at (nearest element centre, then Newton steps in
 * [0,1]^3 to 1e-13 of the patch size), then evaluated as by
 * sa_mp_eval_temperature.  A point on an interface goes to the lower patch
 * index (T is continuous there; grad T is the one-sided value of that
 * patch).  A point in no patch gets NaN in T and grad, -1 in patch.  Host
 * arrays: T [n], grad [n][3], patch [n], xi [n][3] (the parametric points);
 * grad, patch and xi may be NULL. */
int sa_mp_eval_temperature_at(sa_multipatch *h, int32_t path, int64_t n, const double *x, double *T, double *grad,
                              int32_t *patch, double *xi);

/* The net heat-loss rate of sa_iga_heat_loss (Sec. 3.1, Tables 3-4) along
 * an edge of patch `patch`: the edge where its parametric face `face` meets
 * its face `edge_face`, at `quad` Gauss points per element, for path `path`
 * at its current step; T^ from the global control values.  Arguments, outputs and errors as
 * for sa_iga_heat_loss (SA_ERANGE for a patch index out of range). */
int sa_mp_heat_loss(sa_multipatch *h, int32_t path, int32_t patch, int32_t face, int32_t edge_face, int32_t quad,
                    int64_t *n_pts, double *x, double *normal, double *ds, double *q_tilde, double *q_hat,
                    double *integrals);

/* Free the object and its device memory.  NULL is ignored. */
void sa_mp_destroy(sa_multipatch *h);

#ifdef __cplusplus
}
#endif

#endif /* SA_IGA_H */
