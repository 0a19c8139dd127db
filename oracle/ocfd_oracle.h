/*
 * Plain FP64 CPU oracle for the right-hand side and Runge-Kutta update of the
 * curvilinear compressible Navier-Stokes solver of Dang et al., "Direct
 * numerical simulation of compressible turbulence accelerated by GPU. Part 1:
 * OpenCFD-SCU" (arXiv:2209.15333), Section 2.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the independent checker of the GPU
 * library.  It shares no source, header, table or helper with the GPU path and
 * must never be linked into it.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.
 *
 * Everything is straightforward loops in double precision, compiled without
 * floating-point contraction.  Arrays are structure-of-arrays, field-major:
 * a field f of a node (i,j,k) lives at  f*N + i + nx*(j + ny*k),  N = nx*ny*nz.
 */
#ifndef OCFD_ORACLE_H
#define OCFD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Scheme selections. */
enum { OR_WENO7 = 0, OR_HYBRID = 1 };      /* inviscid scheme (Sec. 2.2.3) */
enum { OR_UD7 = 0, OR_C8 = 1 };            /* low-dissipation stencil of the hybrid */
/* Per-interface flag values (one byte per interface). */
enum { OR_FLAG_LOW = 0, OR_FLAG_WENO7 = 1, OR_FLAG_WENO5 = 2 };
/* Boundary kinds for the faces of non-periodic directions (ramp workloads).
   OR_BC_NRBC: characteristic nonreflecting face (Thompson 1987; the local
   one-dimensional inviscid relations of Poinsot & Lele 1992): its nodes are
   advanced in time like interior nodes, with the normal-direction terms
   replaced by the outgoing characteristic wave amplitudes and the incoming
   ones set to zero. */
enum { OR_BC_NONE = 0, OR_BC_INFLOW = 1, OR_BC_EXTRAP = 2, OR_BC_WALL = 3, OR_BC_NRBC = 4 };

typedef struct {
  int32_t nx, ny, nz;
  int32_t periodic[3];   /* 1 if direction xi/eta/zeta is periodic */
  int32_t bc[6];         /* face kinds: xi-, xi+, eta-, eta+, zeta-, zeta+ */
  double period[3];      /* coordinate d is translated by period[d] across the seam of direction d */
  double h[3];           /* computational spacing of xi, eta, zeta */
  double gamma, Re, Ma, Pr;
  double Tref, suth;     /* Sutherland constant and reference temperature, kelvin (eq 15) */
  double Tw;             /* isothermal wall temperature / reference temperature */
  double theta1, theta2; /* sensor thresholds (eq 43) */
  double eps;            /* WENO epsilon */
  int32_t viscous;       /* 0: Euler; 6 or 8: sixth- or eighth-order central viscous terms (Sec. 2.3) */
  int32_t scheme;        /* OR_WENO7 or OR_HYBRID */
  int32_t lowdiss;       /* OR_UD7 or OR_C8 */
  int32_t three_way;     /* hybrid with the WENO5 tier above theta2 */
  int32_t characteristic; /* reconstruct in characteristic variables (Sec. 2.2.2) */
  int32_t flag_window;   /* sensor window of interface j+1/2: 0 nodes j-3..j+4; 1 nodes j, j+1 */
  int32_t nthreads;      /* OpenMP threads (0: runtime default) */
} or_params;

/* Parts of the right-hand side (bit mask). */
#define OR_PART_XI   1
#define OR_PART_ETA  2
#define OR_PART_ZETA 4
#define OR_PART_VISC 8
#define OR_PART_ALL  15

/* ---- building blocks exposed for the identity tests ---- */
/* Steger-Warming split (eq 19-30) of one node: primitive state rho,u,v,w,p;
   alpha = metric row / J.  Writes f+ (fp) and f- (fm), 5 each. */
void or_sw_split(const or_params* P, double rho, double u, double v, double w, double p,
                 const double alpha[3], double fp[5], double fm[5]);
/* Reconstructions at j+1/2 of a left-biased stencil (the f+ direction). */
double or_weno7(const double f[7], double eps);            /* f_{j-3..j+3} */
double or_weno5(const double f[5], double eps, const int valid[3]); /* f_{j-2..j+2}; valid substencils */
double or_ud7(const double f[7]);                          /* eq 41 */
double or_c8(const double f[8]);                           /* f_{j-3..j+4}, central */
/* Eigenvector matrices of the flux Jacobian along the unit normal n at the
   conserved state U (Sec. 2.2.2, eq 34-40), row-major 5x5: S (rows: left
   eigenvectors, eigenvalues u_n, u_n, u_n, u_n - c, u_n + c) and its inverse
   Sinv (columns: right eigenvectors). */
void or_char_matrices(const or_params* P, const double U[5], const double n[3], double S[25], double Sinv[25]);

/* ---- whole-field operations ---- */
/* Metrics by the conservative forms of eq 3 (xyz: [3][N] -> met: [10][N] =
   xi_x/J, xi_y/J, xi_z/J, eta_x/J, ..., zeta_z/J, 1/J). */
int or_metrics(const or_params* P, const double* xyz, double* met);
/* Node sensor theta (eq 42-43) and per-interface flags [3][N]. */
int or_sensor(const or_params* P, const double* U, double* theta, uint8_t* flags);
/* dU/dt = L(U) at every node.  flags: [3][N] or NULL (NULL: computed from the
   sensor in hybrid mode; WENO7 everywhere otherwise). */
int or_dudt(const or_params* P, const double* met, const double* U, const uint8_t* flags,
            int32_t parts, double* dudt);
/* The same quantity evaluated only at the listed nodes (linear node index);
   out: [npts][5].  Bitwise equal to or_dudt at those nodes. */
int or_dudt_points(const or_params* P, const double* met, const double* U, const uint8_t* flags,
                   int32_t parts, int64_t npts, const int64_t* nodes, double* out);
/* n Runge-Kutta substeps (eq 45).  U: current stage value (in/out); Un: value
   at the start of the step (in/out); *stage in {0,1,2} (in/out).  Boundary
   conditions are applied after every stage.  flags: as in or_dudt. */
int or_advance(const or_params* P, const double* met, double* U, double* Un, int32_t* stage,
               int32_t n, double dt, const double* inflow);
/* out[0..4] = sum of U_m/J; out[5] = max CFL number; out[6] = min p;
   out[7] = min rho; out[8] = count of non-finite values. */
int or_reduce(const or_params* P, const double* met, const double* U, double dt, double* out);
/* Apply the boundary conditions of the non-periodic faces to U in place, face
   by face (xi-, xi+, eta-, eta+, zeta-, zeta+); NRBC faces are left as the
   time step made them.  inflow: conserved variables
   [5][face] of the inflow face, the face indexed by its two other node
   indices with the lower direction fastest (NULL if there is none). */
int or_apply_bc(const or_params* P, double* U, const double* inflow);
/* Normal-direction part of dU/dt at node (i,j,k) on face (d, side) of a
   nonreflecting face: out[5], the time derivative of the conserved variables
   from the characteristic wave amplitudes (incoming ones zero). */
int or_nrbc_normal(const or_params* P, const double* met, const double* U, int32_t i, int32_t j, int32_t k,
                   int32_t d, int32_t side, double* out);

#ifdef __cplusplus
}
#endif
#endif
