/*
 * ocfd — MI355X (gfx950) library for the right-hand side and time march of
 * the finite-difference compressible Navier-Stokes solver described by Dang,
 * Liu, Guo, Duan & Li, "Direct numerical simulation of compressible turbulence
 * accelerated by GPU. Part 1: OpenCFD-SCU", arXiv:2209.15333.
 *
 * One GPU holds the whole single-block curvilinear grid.  Each substep (one
 * stage of the third-order Runge-Kutta scheme, eq 45) evaluates
 *   dU/dt = J * [ -d(F - Fv)/dxi - d(G - Gv)/deta - d(H - Hv)/dzeta ]   (eq 1)
 * with Steger-Warming splitting of the inviscid fluxes (eq 19-30), seventh-order
 * WENO or hybrid reconstruction along each grid direction (Sec. 2.2.3,
 * component-wise or in characteristic variables, Sec. 2.2.2), and sixth- or
 * eighth-order central viscous and heat-flux terms (eq 9-16, Sec. 2.3).
 *
 * Conventions shared by every entry point
 *  - Arrays are structure-of-arrays, field-major, x fastest: field f of node
 *    (i,j,k) is at  f*N + i + nx*(j + ny*k),  N = nx*ny*nz.
 *  - Pointers named *_dev are device pointers; the library never frees them.
 *    Host pointers are named *_host.
 *  - All device work is enqueued on the solver's HIP stream and returns
 *    before it finishes, except where an entry point says it synchronises.
 *  - Every int-returning entry point returns OCFD_OK (0) on success or a
 *    negative OCFD_ERR_* code; the text of the last error of a solver is
 *    available from ocfd_last_error.  No C++ exception crosses this interface.
 *  - One solver must not be used from two host threads at the same time.
 */
#ifndef OCFD_H
#define OCFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OCFD_OK 0
#define OCFD_ERR_BADARG (-1)      /* null pointer, out-of-range parameter */
#define OCFD_ERR_BADSIZE (-2)     /* grid size or workspace size not accepted */
#define OCFD_ERR_HIP (-3)         /* a HIP runtime call failed */
#define OCFD_ERR_UNSUPPORTED (-4) /* option combination not built */
#define OCFD_ERR_STATE (-5)       /* call out of order (e.g. advance before set_state) */
#define OCFD_ERR_NONFINITE (-6)   /* ocfd_advance's state check found a non-finite conserved value or a
                                     density or pressure <= 0 (ocfd_substeps_done names the substep) */
#define OCFD_ERR_CFL (-7)         /* ocfd_advance's state check found the CFL number above cfl_max */

/* Inviscid schemes (Sec. 2.2.3, Table 2). */
#define OCFD_SCHEME_WENO7 0   /* seventh-order WENO at every interface */
#define OCFD_SCHEME_HYBRID 1  /* sensor-selected low-dissipation / WENO7 (eq 41-43); with
                                 three_way, WENO5 above theta2 */
/* Low-dissipation stencil of the hybrid scheme. */
#define OCFD_LOWDISS_UD7 0    /* seventh-order upwind, eq 41 */
#define OCFD_LOWDISS_C8 1     /* eighth-order central */

/* Arithmetic of the inviscid path.  MIXED: Steger-Warming split, smoothness
   indicators and reconstruction in FP32; metrics, the interface-flux
   difference (sum of the two FP32 halves taken in FP64), viscous terms, the
   Runge-Kutta accumulation and reductions stay FP64. */
#define OCFD_PREC_FP64 0
#define OCFD_PREC_MIXED 1

/* Pressure and density features of the learned sensor (ocfd_params.sensor_inputs). */
#define OCFD_INPUTS_JUMP 0
#define OCFD_INPUTS_CURV 1

/* Shock sensor of the hybrid scheme. */
#define OCFD_SENSOR_PLAIN 0    /* modified Jameson pressure sensor, eq 42-43 */
#define OCFD_SENSOR_LEARNED 1  /* perceptron on local flow features (ocfd_sensor_* below) */

/* Boundary kinds of the faces of a non-periodic direction (Sec. 2.4 names
   the kinds used by the compression-ramp case).  Applied after every
   Runge-Kutta stage, face by face in the order xi-, xi+, eta-, eta+, zeta-,
   zeta+; a face node's dU/dt is zero (except on NRBC faces), its value is
   set by its face:
   INFLOW: the conserved state given by ocfd_set_inflow;
   EXTRAP: rho, velocity and p of the first interior node;
   WALL:   no slip, T = Tw, p of the first interior node, rho = gamma Ma^2 p / Tw;
   NONE:   the face keeps its value;
   NRBC:   characteristic nonreflecting face (Sec. 6.1 names nonreflecting
           conditions at the ramp's exit and upper boundary; the reading is
           Thompson 1987 with the local one-dimensional relations of Poinsot &
           Lele 1992): its nodes are advanced by the Runge-Kutta stage with
           the fluxes of the directions they are interior to plus, along the
           face normal, the time derivative carried by the outgoing
           characteristic waves (one-sided second-order differences; incoming
           wave amplitudes zero) and the metric-derivative part of the normal
           flux derivative; no normal viscous term.  A node that also lies on
           a face of another kind takes that face's value. */
#define OCFD_BC_NONE 0
#define OCFD_BC_INFLOW 1
#define OCFD_BC_EXTRAP 2
#define OCFD_BC_WALL 3
#define OCFD_BC_NRBC 4

/* Parts of the right-hand side for ocfd_dudt (bit mask). */
#define OCFD_PART_XI 1
#define OCFD_PART_ETA 2
#define OCFD_PART_ZETA 4
#define OCFD_PART_VISC 8
#define OCFD_PART_ALL 15

/* Entries of ocfd_reduce's output. */
#define OCFD_RED_SUM0 0     /* 0..4: sum over nodes of U_m / J (conserved totals, eq 5) */
#define OCFD_RED_CFL 5      /* max over nodes of dt * sum_d (|u~_d| + c |grad xi_d|) / h_d */
#define OCFD_RED_PMIN 6     /* min pressure */
#define OCFD_RED_RHOMIN 7   /* min density */
#define OCFD_RED_NONFINITE 8 /* number of non-finite conserved values */
#define OCFD_RED_WENO0 9    /* 9..11: fraction of the interfaces of xi, eta, zeta whose stencil in the
                               last right-hand side was WENO (WENO7, WENO5 or a bounded-end closure);
                               1 for the WENO7 scheme; NaN for a hybrid solver that has not evaluated
                               one since its creation or its last ocfd_set_flags (the paper reports
                               over 90% low-dissipation, Sec. 2.2.3) */
#define OCFD_RED_COUNT 12

/* Kernel classes timed by the profiling counters (OCFD_K_VISC: the viscous
   fluxes and their divergence; OCFD_K_PRIM: the plain sensor's pressure). */
#define OCFD_K_SWEEP_XI 0
#define OCFD_K_SWEEP_ETA 1
#define OCFD_K_SWEEP_ZETA 2
#define OCFD_K_VISC 3
#define OCFD_K_PRIM 4
#define OCFD_K_OTHER 5
#define OCFD_K_COUNT 6

/* Run parameters.  The physical inputs are those the paper names in Sec. 2.1
   (eq 17-18): gamma, Re, Ma, Pr and the Sutherland reference temperature. */
typedef struct ocfd_params {
  int32_t nx, ny, nz;      /* nodes per direction; each >= 1 */
  int32_t periodic[3];     /* 1: direction xi/eta/zeta is periodic; 0: bounded (needs >= 8 nodes) */
  int32_t bc[6];           /* OCFD_BC_* of the faces xi-, xi+, eta-, eta+, zeta-, zeta+ of bounded
                              directions (ignored for periodic ones); at most one INFLOW face */
  double period[3];        /* coordinate d grows by period[d] across the seam of direction d */
  double h[3];             /* computational spacing of xi, eta, zeta (> 0) */
  double gamma, Re, Ma, Pr;
  double Tref, suth;       /* Sutherland law mu = T^1.5 (1 + S)/(T + S), S = suth/Tref (eq 15) */
  double Tw;               /* wall temperature / reference temperature (WALL faces, > 0) */
  double theta1, theta2;   /* sensor thresholds of eq 43 */
  double weno_eps;         /* epsilon of the WENO nonlinear weights */
  int32_t viscous;         /* 0: Euler; 6 or 8: sixth- or eighth-order central viscous terms (Sec. 2.3:
                              node gradients and the derivative of the viscous fluxes; on bounded
                              lines second-order one-sided at the end node, then second-, fourth-
                              and sixth-order central toward the interior) */
  int32_t scheme;          /* OCFD_SCHEME_* */
  int32_t lowdiss;         /* OCFD_LOWDISS_* */
  int32_t precision;       /* OCFD_PREC_* */
  int32_t sensor;          /* hybrid only: OCFD_SENSOR_PLAIN (eq 42-43) or OCFD_SENSOR_LEARNED */
  int32_t sensor_every;    /* learned sensor: re-evaluate the flags every this many substeps (>= 1) */
  int32_t audit_every;     /* learned sensor: compare with the plain sensor every this many substeps (0: never) */
  int32_t three_way;       /* hybrid with the plain sensor: interfaces with max theta > theta2 take
                              fifth-order WENO (eq 43, Table 2), 0 or 1 */
  int32_t characteristic;  /* 1: WENO interfaces (WENO7, WENO5 and the boundary closures) are
                              reconstructed in characteristic variables (Sec. 2.2.2, eq 31-40):
                              split fluxes carried by S of the interface state (the mean of the
                              conserved variables of its two nodes, eq 32; normal: the unit vector
                              of the mean of their metric rows) to characteristic variables,
                              reconstructed field by field, carried back by S^-1; 0: component
                              by component.  Linear stencils give the same flux either way. */
  int32_t check_every;     /* ocfd_advance checks the state after every this many substeps (counted
                              from ocfd_set_state; 0: never): non-finite conserved values, density or
                              pressure <= 0 (OCFD_ERR_NONFINITE), CFL number above cfl_max
                              (OCFD_ERR_CFL); each check synchronises the stream */
  int32_t flag_window;     /* plain sensor, how node values of theta decide interface j+1/2 (eq 43 applies
                              theta "at positions"): 0: the maximum over the nodes j-3 .. j+4 of its
                              stencil; 1: the maximum of theta_j and theta_j+1 */
  int32_t sensor_inputs;   /* learned sensor, the pressure and density features of a node:
                              OCFD_INPUTS_JUMP: normalised first differences across the node;
                              OCFD_INPUTS_CURV: the plain sensor's normalised second differences
                              (eq 42), so its own value is among the inputs */
  double cfl_max;          /* > 0: CFL limit of the state check (the CFL number as OCFD_RED_CFL);
                              0: no CFL check */
} ocfd_params;

typedef struct ocfd_solver ocfd_solver;

/* Fill *p with defaults: gamma 1.4, Pr 0.72, Tref 288.15 K, suth 110.4 K,
   Tw 1, theta 0.02/0.1, eps 1e-6, periodic, WENO7, viscous order 6. */
int ocfd_params_default(ocfd_params* p);

/* Bytes of device workspace a solver with these parameters needs (0 if the
   parameters are invalid).  The workspace holds the metrics [10][N], three
   state buffers [5][N], the right-hand-side sum [5][N], the node pressure [N]
   and sensor [N] and the viscous fluxes [12][N], all FP64, the learned-sensor
   buffers (node features, two flag fields, network and optimiser state), the
   inflow face [5][face] and small reduction buffers. */
size_t ocfd_workspace_bytes(const ocfd_params* p);

/* Create a solver.  stream: a hipStream_t (NULL: the default stream).  The
   solver copies *p.  Errors: BADARG (null pointer / invalid parameter),
   UNSUPPORTED (the learned sensor with three_way: the network decides two
   ways only). */
int ocfd_create(const ocfd_params* p, void* stream, ocfd_solver** out);

/* Hand the solver caller-owned device memory of at least
   ocfd_workspace_bytes bytes, aligned to 256 bytes.  The caller keeps
   ownership and must keep it alive until ocfd_destroy.  Errors: BADARG,
   BADSIZE (too small). */
int ocfd_bind_workspace(ocfd_solver* s, void* workspace_dev, size_t bytes);

/* Compute the metrics from node coordinates xyz_dev [3][N] (x, y, z) with the
   conservative form of eq 3 evaluated by eighth-order central differences;
   1/J = det d(x,y,z)/d(xi,eta,zeta) (eq 4).  Errors: BADARG, STATE (no
   workspace). */
int ocfd_set_grid(ocfd_solver* s, const double* xyz_dev);

/* Inflow state of the INFLOW face: conserved variables inflow_dev [5][face],
   the face indexed by its two other node indices, the lower direction fastest
   (xi- face: j + ny*k).  Copied into the workspace.  Errors: BADARG,
   UNSUPPORTED (no INFLOW face), STATE (no workspace).  ocfd_advance returns
   STATE while an INFLOW face has no state. */
int ocfd_set_inflow(ocfd_solver* s, const double* inflow_dev);

/* Copy metrics [10][N] = xi_x/J, xi_y/J, xi_z/J, eta_x/J, ..., zeta_z/J, 1/J
   in or out of the solver. */
int ocfd_set_metrics(ocfd_solver* s, const double* met_dev);
int ocfd_get_metrics(ocfd_solver* s, double* met_dev);

/* Set the conserved state U_dev [5][N] = rho, rho u, rho v, rho w, E (eq 5)
   and restart the Runge-Kutta cycle at stage 0; the substep count (which
   times the learned sensor's evaluations, its audits and the state checks)
   restarts at 0. */
int ocfd_set_state(ocfd_solver* s, const double* U_dev);
/* Copy out the current state (the value the next substep starts from). */
int ocfd_get_state(ocfd_solver* s, double* U_dev);
/* Mid-step restart: the state at the start of the current step and the stage
   (0, 1, 2).  set_step_state takes the current state, the step-start state
   and the stage, and sets the substep count to the stage. */
int ocfd_get_step_state(ocfd_solver* s, double* Un_dev, int32_t* stage_host);
int ocfd_set_step_state(ocfd_solver* s, const double* U_dev, const double* Un_dev, int32_t stage);

/* Advance n substeps of eq 45 with time step dt: substep k of a step sets
   U(k) = a_k U^n + b_k (U(k-1) + dt L(U(k-1))), (a,b) = (0,1), (3/4,1/4),
   (1/3,2/3), then sets the faces of bounded directions (OCFD_BC_*).  With
   check_every > 0 the state is checked after every substep whose count is a
   multiple of it; a failed check stops the advance there (the state is the
   one that failed).  Errors: BADARG (n < 0, dt not finite), STATE,
   NONFINITE, CFL. */
int ocfd_advance(ocfd_solver* s, int32_t n_substeps, double dt);
/* Substeps completed since ocfd_set_state (or the stage given to
   ocfd_set_step_state); after OCFD_ERR_NONFINITE or OCFD_ERR_CFL, the substep
   whose result failed the check.  -1 for a null solver. */
int64_t ocfd_substeps_done(const ocfd_solver* s);

/* dudt_dev [5][N] = L(U_dev) = dU/dt for the parts selected by the
   OCFD_PART_* mask, without touching the solver's state (zero on the faces of
   bounded directions).  U_dev must not alias dudt_dev. */
int ocfd_dudt(ocfd_solver* s, const double* U_dev, double* dudt_dev, int32_t parts);

/* Global sums and extrema of the current state (entries OCFD_RED_*), written
   to out_host[OCFD_RED_COUNT].  Deterministic order.  Synchronises the
   stream. */
int ocfd_reduce(ocfd_solver* s, double dt, double* out_host);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the
   reduction of ocfd_reduce without a solver, a workspace or a host copy.
   Inputs: the grid and gas parameters *p (sizes, periodic, h, gamma are
   read), the state U_dev [5][N] and the metrics met_dev [10][N] (layout of
   ocfd_set_metrics).  Output: out_dev, a device buffer of OCFD_RED_COUNT
   doubles; entries OCFD_RED_SUM0 .. OCFD_RED_NONFINITE as ocfd_reduce, the
   WENO entries 0 (no flags are seen).  Enqueued on `stream` (a hipStream_t,
   NULL: the default stream) on the current device, without synchronising.
   Allocates nothing: its partial records live in a fixed array of
   1024 x OCFD_RED_COUNT doubles (96 KiB) of device memory, one per GPU,
   held until the process ends; every grid this library accepts needs at
   most 1024 records (more would return BADSIZE).  Calls that overlap on one
   GPU (two streams, two threads) share that array and race: serialise them.
   Errors: BADARG (null pointer, dt not finite, invalid sizes, h or gamma),
   BADSIZE, HIP (the array's address or the launch); the reason is printed
   to stderr. */
int ocfd_reduce_static(const ocfd_params* p, const double* U_dev, const double* met_dev, double dt,
                       double* out_dev, void* stream);

/* Per-interface scheme flags flags_dev [3][N] (byte: 0 low-dissipation,
   1 WENO7, 2 WENO5) used by the hybrid scheme instead of the sensor, or NULL
   to go back to the sensor.  The caller keeps the buffer alive while set.
   Resets the WENO fractions of ocfd_reduce to NaN until the next
   right-hand side. */
int ocfd_set_flags(ocfd_solver* s, const uint8_t* flags_dev);

/* Kernel timing: when enabled, every launch is bracketed by HIP events on the
   solver's stream.  profile_read synchronises and returns, per kernel class
   OCFD_K_*, the summed milliseconds and the launch counts since the last
   enable. */
int ocfd_profile(ocfd_solver* s, int32_t enable);
int ocfd_profile_read(ocfd_solver* s, double* ms_host, int64_t* count_host);
const char* ocfd_kernel_name(int32_t kernel_class);

/* ---- Learned shock sensor ------------------------------------------------
   A perceptron 32 -> 64 -> 64 -> 64 (ReLU each) -> 1 (sigmoid) maps, for interface
   j+1/2 along a direction, four features of each of the 8 nodes j-3..j+4
   (Delta div u / c and Delta |curl u| / c with Delta = (1/J)^(1/3); the
   pressure and the density jump summed over the three directions and divided
   by theta1, each the normalised first difference |q+ - q-| / (q+ + q-)
   across the node, or with sensor_inputs = OCFD_INPUTS_CURV the normalised
   second difference |q- - 2q + q+| / (q- + 2q + q+) of eq 42) to the
   probability that the interface needs WENO.  It replaces
   the pressure sensor of eq 42-43 in the hybrid scheme: an interface takes
   WENO7 iff p >= tau.  Inference and training run on bf16 matrix cores with
   FP32 accumulation and FP32 master weights.  Parameters: one flat FP32 array
   of ocfd_sensor_nparams() = 10497 values: W1 [32 inputs][64 units],
   b1 [64], W2 [64][64], b2 [64], W3 [64][64], b3 [64], w4 [64], b4 [1].
   On a bounded line the end nodes take a one-sided velocity difference over
   one spacing and add no jump term along that line; interfaces whose 8-node
   window leaves the grid (j < 3 or j > n-5) take the masked WENO5 closure
   whatever their flag: their learned flag is 1 and they are neither sampled
   nor audited. */
int32_t ocfd_sensor_nparams(void);
int ocfd_sensor_set_params(ocfd_solver* s, const float* params_host);
int ocfd_sensor_get_params(ocfd_solver* s, float* params_host);
/* Decision thresholds tau_d of the interfaces of direction d (default 0.5):
   set_threshold gives all three directions the same value in [0, 1];
   ocfd_sensor_calibrate sets them per direction; set_thresholds and
   get_thresholds copy tau_host[3] in and out.  Errors: BADARG (null pointer,
   a value outside [0, 1]). */
int ocfd_sensor_set_threshold(ocfd_solver* s, double tau);
int ocfd_sensor_set_thresholds(ocfd_solver* s, const double* tau_host);
int ocfd_sensor_get_thresholds(ocfd_solver* s, double* tau_host);
/* Flags [3][N] of the state U_dev by the plain sensor (0 low-dissipation,
   1 WENO7, 2 WENO5 when three_way) or by the network (0 / 1), written to
   flags_dev.  Errors: STATE (network not set). */
int ocfd_sensor_flags(ocfd_solver* s, const double* U_dev, int32_t which, uint8_t* flags_dev);
/* Caller-owned device buffer for training samples: each sample is 32 bf16
   inputs, a label byte (bit 0: WENO; bits 1-2: the interface's direction),
   a weight and bookkeeping, ocfd_sensor_sample_bytes(cap) bytes for cap
   samples. */
size_t ocfd_sensor_sample_bytes(int64_t capacity);
int ocfd_sensor_bind_samples(ocfd_solver* s, void* samples_dev, size_t bytes);
/* Append samples from the current state labelled by the plain sensor: an
   interface is kept with probability keep_weno (label 1) or keep_low
   (label 0) by a counter-based hash of (seed, direction, node), in node order.
   *total_host receives the number of stored samples.  Synchronises. */
int ocfd_sensor_collect(ocfd_solver* s, uint64_t seed, double keep_weno, double keep_low, int64_t* total_host);
/* Train on the first (1 - holdout) of the stored samples: `epochs` passes of
   mini-batches of `batch` samples in a seeded random order, Adam with
   learning rate lr, weighted binary cross-entropy with class balance (each
   WENO sample weighs n_low / n_weno, at most 1000; the weights are written
   into the sample buffer).  stats_host[4] = loss of the first and of the last
   epoch, number of steps, training samples.  Synchronises. */
int ocfd_sensor_train(ocfd_solver* s, int32_t epochs, int32_t batch, float lr, uint64_t seed, double holdout,
                      double* stats_host);
/* Set the thresholds from the held-out samples (the last `holdout` fraction
   of the buffer): tau_d = margin * the k-th least probability over the
   held-out WENO samples of direction d, k = floor(miss * their count) (a
   direction with none takes the value over all directions).  miss = 0 keeps
   every held-out WENO interface; miss > 0 lets that fraction of them fall
   below the threshold before the margin is applied (the margin usually
   keeps most of them).  0 < holdout < 1, 0 < margin <= 1, 0 <= miss < 0.5,
   else OCFD_ERR_BADARG.  out_host[4] = the smallest tau_d, recall, false-
   positive rate, held-out samples.  Synchronises. */
int ocfd_sensor_calibrate(ocfd_solver* s, double holdout, double margin, double miss, double* out_host);
/* Loss and gradient over n given samples with the current weights (no
   update): grad_host[nparams] then the loss.  X_dev: [n][32] bf16 bit
   patterns; y_dev: label bytes (bit 0 read); w_dev: weights.  Synchronises. */
int ocfd_sensor_grad(ocfd_solver* s, const uint16_t* X_dev, const uint8_t* y_dev, const float* w_dev, int64_t n,
                     float* grad_host);
/* Audit counters of the learned sensor since the solver started:
   out_host[6] = audits run, interfaces compared, plain WENO interfaces,
   learned WENO interfaces, missed WENO interfaces (fell back to WENO),
   mismatches.  */
int ocfd_sensor_audit(ocfd_solver* s, double* out_host);

const char* ocfd_last_error(const ocfd_solver* s);
void ocfd_destroy(ocfd_solver* s);

#ifdef __cplusplus
}
#endif
#endif
