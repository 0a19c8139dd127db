/*
 * Plain FP64 CPU oracle of the OpenCFD-SCU right-hand side and time march
 * (arXiv:2209.15333, Section 2).  TEST INFRASTRUCTURE ONLY: it is the checker
 * of the GPU library, shares no code with it, and is loaded only by the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark.
 *
 * Written for reading, not for speed: every step is a loop over nodes or
 * interfaces in the order the method states it.  Build flags keep the
 * arithmetic literal (-O2 -ffp-contract=off -fno-fast-math).
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes of the repository):
 *  - energy (eq 8) is E = p/(gamma-1) + rho|u|^2/2;
 *  - in eq 12 the heat flux of component i uses dT/dx_i; in eq 13 the stress
 *    is (mu/Re)(du_i/dx_j + du_j/dx_i - 2/3 delta_ij div u);
 *  - Sutherland (eq 15) uses the dimensional constant suth/Tref and eq 16 is
 *    the sound speed, so c^2 = T/Ma^2 = gamma p/rho;
 *  - the Steger-Warming vector (eq 23) uses k_1,k_2,k_3 in the three momentum
 *    rows, the energy row (gamma-1)l1|u|^2 + W + l4|u-ck|^2/2 + l5|u+ck|^2/2,
 *    f+ built from the l+ of eq 29 and f- from the l-; with this form f+ + f-
 *    equals the flux of eq 6 exactly;
 *  - the metrics of eq 3 are evaluated in their conservative (Thomas-Lombard)
 *    form with the eighth-order central operator;
 *  - the seventh-order WENO (Table 2, scheme 4) is the Balsara-Shu/Jiang-Shu
 *    scheme with linear weights (1,12,18,4)/35, p = 2 and the smoothness
 *    indicators of the Jiang-Shu integral definition;
 *  - a hybrid interface takes the low-dissipation stencil when the sensor
 *    theta of every node of its 8-node stencil is <= theta1 (eq 43);
 *  - in characteristic variables (Sec. 2.2.2) the split fluxes f+ and f- of
 *    the window are both carried by the S of the interface, reconstructed
 *    field by field with the stencil the interface would use component-wise,
 *    and their sum carried back by S^-1; the eigenvalues of eq 33 enter only
 *    through the split.  The interface normal is the unit vector of the mean
 *    of the two nodes' metric rows of the sweep direction.
 */
#include "ocfd_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Grid indexing                                                        */
/* ------------------------------------------------------------------ */

/* Honour the requested OpenMP thread count (0 keeps the runtime default). */
static void set_threads(const or_params* P) {
#ifdef _OPENMP
  if (P->nthreads > 0) omp_set_num_threads(P->nthreads);
#else
  (void)P;
#endif
}

static long n_nodes(const or_params* P) { return (long)P->nx * P->ny * P->nz; }
static int dim_n(const or_params* P, int d) { return d == 0 ? P->nx : (d == 1 ? P->ny : P->nz); }
static long lin(const or_params* P, const int c[3]) { return c[0] + (long)P->nx * (c[1] + (long)P->ny * c[2]); }
static void unlin(const or_params* P, long id, int c[3]) {
  c[0] = (int)(id % P->nx);
  c[1] = (int)((id / P->nx) % P->ny);
  c[2] = (int)(id / ((long)P->nx * P->ny));
}
static int floordiv(int a, int n) { return (a >= 0) ? a / n : -((-a + n - 1) / n); }

/* Node c shifted by m along direction d.  Returns 0 if the node lies outside a
   non-periodic direction.  *wraps counts seam crossings (negative leftwards). */
static int shifted(const or_params* P, const int c[3], int d, int m, long* id, int* wraps) {
  int n = dim_n(P, d);
  int q[3] = {c[0], c[1], c[2]};
  int t = c[d] + m;
  int w = 0;
  if (P->periodic[d]) {
    w = floordiv(t, n);
    t -= w * n;
  } else if (t < 0 || t >= n) {
    return 0;
  }
  q[d] = t;
  *id = lin(P, q);
  if (wraps) *wraps = w;
  return 1;
}

/* ------------------------------------------------------------------ */
/* Central first derivatives (Sec. 2.3 and the metric evaluation)       */
/* ------------------------------------------------------------------ */

/* Coefficients a_m of  sum_m a_m (f_{j+m} - f_{j-m}) / h  for orders 2..8. */
static const double C2c[1] = {0.5};
static const double C4c[2] = {2.0 / 3.0, -1.0 / 12.0};
static const double C6c[3] = {3.0 / 4.0, -3.0 / 20.0, 1.0 / 60.0};
static const double C8c[4] = {4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};

/* Derivative of a sampled function along one line.  vals[m + R] holds f_{j+m}
   for m in [-R, R]; pos is the node position along the line and n its length;
   maxhalf is the half width of the interior operator (3: sixth order, 4: eighth
   order).  Near a non-periodic end the order drops as Sec. 2.3 describes:
   one-sided second order at the end node, then second-, fourth- and sixth-order
   central differences at the next nodes. */
static double line_derivative(const double* vals, int R, int pos, int n, int periodic, int maxhalf, double h) {
  const double* f = vals + R; /* f[m] = f_{j+m} */
  int half = maxhalf;
  if (!periodic) {
    int dist = pos < n - 1 - pos ? pos : n - 1 - pos; /* distance to the nearer end */
    if (dist == 0) {
      if (pos == 0) return (-3.0 * f[0] + 4.0 * f[1] - f[2]) / (2.0 * h);
      return (3.0 * f[0] - 4.0 * f[-1] + f[-2]) / (2.0 * h);
    }
    if (dist < half) half = dist;
  }
  const double* a = half == 1 ? C2c : half == 2 ? C4c : half == 3 ? C6c : C8c;
  double s = 0.0;
  for (int m = 1; m <= half; ++m) s += a[m - 1] * (f[m] - f[-m]);
  return s / h;
}

/* ------------------------------------------------------------------ */
/* Metrics (eq 2-4), conservative form                                   */
/* ------------------------------------------------------------------ */

/* Coordinate `coord` at node c shifted by m along d, unwrapped across the seam
   of a periodic direction: coordinate d grows by period[d] per crossing. */
static double coord_shift(const or_params* P, const double* xyz, int coord, const int c[3], int d, int m, int* ok) {
  long id; int w;
  *ok = shifted(P, c, d, m, &id, &w);
  if (!*ok) return 0.0;
  double v = xyz[(long)coord * n_nodes(P) + id];
  if (coord == d) v += w * P->period[d];
  return v;
}

int or_metrics(const or_params* P, const double* xyz, double* met) {
  set_threads(P);
  const long N = n_nodes(P);
  /* inner[3*c + d] = d(coordinate c)/d(direction d) */
  double* inner = (double*)malloc(sizeof(double) * 9 * N);
  if (!inner) return -1;
#pragma omp parallel for schedule(static)
  for (long id = 0; id < N; ++id) {
    int c[3]; unlin(P, id, c);
    for (int co = 0; co < 3; ++co)
      for (int d = 0; d < 3; ++d) {
        double vals[9]; int ok;
        for (int m = -4; m <= 4; ++m) vals[m + 4] = coord_shift(P, xyz, co, c, d, m, &ok);
        inner[(long)(3 * co + d) * N + id] =
            line_derivative(vals, 4, c[d], dim_n(P, d), P->periodic[d], 4, P->h[d]);
      }
  }
  /* Metric of row r (xi, eta, zeta) and column co (x, y, z):
       (r_co)/J = D_t( (a)_s * b ) - D_s( (a)_t * b ),
     with (s, t) = (r+1, r+2) and (a, b) = (co+1, co+2) taken cyclically; this
     is eq 3 written as a divergence (e.g. xi_x/J = (y_eta z)_zeta - (y_zeta z)_eta). */
#pragma omp parallel for schedule(static)
  for (long id = 0; id < N; ++id) {
    int c[3]; unlin(P, id, c);
    for (int r = 0; r < 3; ++r)
      for (int co = 0; co < 3; ++co) {
        int s = (r + 1) % 3, t = (r + 2) % 3;
        int a = (co + 1) % 3, b = (co + 2) % 3;
        double term[2];
        for (int pass = 0; pass < 2; ++pass) {
          int dir = pass == 0 ? t : s;       /* outer derivative direction */
          int inn = pass == 0 ? s : t;       /* inner derivative direction */
          double vals[9];
          for (int m = -4; m <= 4; ++m) {
            long nid; int w, ok;
            ok = shifted(P, c, dir, m, &nid, &w);
            if (!ok) { vals[m + 4] = 0.0; continue; }
            double bc = coord_shift(P, xyz, b, c, dir, m, &ok);
            vals[m + 4] = inner[(long)(3 * a + inn) * N + nid] * bc;
          }
          term[pass] = line_derivative(vals, 4, c[dir], dim_n(P, dir), P->periodic[dir], 4, P->h[dir]);
        }
        met[(long)(3 * r + co) * N + id] = term[0] - term[1];
      }
    /* 1/J = det d(x,y,z)/d(xi,eta,zeta)  (eq 4) */
    double g[3][3];
    for (int co = 0; co < 3; ++co)
      for (int d = 0; d < 3; ++d) g[co][d] = inner[(long)(3 * co + d) * N + id];
    met[9 * N + id] = g[0][0] * (g[1][1] * g[2][2] - g[1][2] * g[2][1])
                    - g[0][1] * (g[1][0] * g[2][2] - g[1][2] * g[2][0])
                    + g[0][2] * (g[1][0] * g[2][1] - g[1][1] * g[2][0]);
  }
  free(inner);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Primitive variables (eq 5, 8, 16)                                    */
/* ------------------------------------------------------------------ */

typedef struct { double rho, u, v, w, p, c, T; } prim_t;

static prim_t primitive(const or_params* P, const double* U, long N, long id) {
  prim_t q;
  q.rho = U[id];
  q.u = U[N + id] / q.rho;
  q.v = U[2 * N + id] / q.rho;
  q.w = U[3 * N + id] / q.rho;
  q.p = (P->gamma - 1.0) * (U[4 * N + id] - 0.5 * q.rho * (q.u * q.u + q.v * q.v + q.w * q.w));
  q.c = sqrt(P->gamma * q.p / q.rho);
  q.T = P->gamma * P->Ma * P->Ma * q.p / q.rho;
  return q;
}

/* ------------------------------------------------------------------ */
/* Steger-Warming flux-vector splitting (eq 19-30)                      */
/* ------------------------------------------------------------------ */

/* The vector of eq 23 for eigenvalues (l1, l4, l5). */
static void sw_vector(double g, double rho, double u, double v, double w, double c,
                      const double k[3], double l1, double l4, double l5, double f[5]) {
  double s = rho / (2.0 * g);
  double um = u - c * k[0], vm = v - c * k[1], wm = w - c * k[2];
  double up = u + c * k[0], vp = v + c * k[1], wp = w + c * k[2];
  double W = (3.0 - g) * (l4 + l5) * c * c / (2.0 * (g - 1.0));      /* eq 26 */
  f[0] = s * (2.0 * (g - 1.0) * l1 + l4 + l5);
  f[1] = s * (2.0 * (g - 1.0) * l1 * u + l4 * um + l5 * up);
  f[2] = s * (2.0 * (g - 1.0) * l1 * v + l4 * vm + l5 * vp);
  f[3] = s * (2.0 * (g - 1.0) * l1 * w + l4 * wm + l5 * wp);
  f[4] = s * ((g - 1.0) * l1 * (u * u + v * v + w * w) + W
              + 0.5 * l4 * (um * um + vm * vm + wm * wm)
              + 0.5 * l5 * (up * up + vp * vp + wp * wp));
}

void or_sw_split(const or_params* P, double rho, double u, double v, double w, double p,
                 const double alpha[3], double fp[5], double fm[5]) {
  double g = P->gamma;
  double c = sqrt(g * p / rho);
  double sigma = sqrt(alpha[0] * alpha[0] + alpha[1] * alpha[1] + alpha[2] * alpha[2]); /* eq 22 */
  double V = alpha[0] * u + alpha[1] * v + alpha[2] * w;                                  /* eq 21 */
  double k[3] = {alpha[0] / sigma, alpha[1] / sigma, alpha[2] / sigma};                  /* eq 27 */
  double l[3] = {V, V - c * sigma, V + c * sigma};                                        /* eq 20 */
  double lp[3], lm[3];
  for (int i = 0; i < 3; ++i) {                                                           /* eq 29 */
    lp[i] = 0.5 * (l[i] + fabs(l[i]));
    lm[i] = 0.5 * (l[i] - fabs(l[i]));
  }
  sw_vector(g, rho, u, v, w, c, k, lp[0], lp[1], lp[2], fp);
  sw_vector(g, rho, u, v, w, c, k, lm[0], lm[1], lm[2], fm);
}

/* ------------------------------------------------------------------ */
/* Interface reconstructions (Sec. 2.2.3, Table 2, eq 41)               */
/* ------------------------------------------------------------------ */

/* Seventh-order WENO at j+1/2 from f_{j-3..j+3} (left-biased). */
double or_weno7(const double f[7], double eps) {
  const double *a = f; /* a[0] = f_{j-3} */
  double q[4], b[4];
  q[0] = (-3.0 * a[0] + 13.0 * a[1] - 23.0 * a[2] + 25.0 * a[3]) / 12.0;
  q[1] = (a[1] - 5.0 * a[2] + 13.0 * a[3] + 3.0 * a[4]) / 12.0;
  q[2] = (-a[2] + 7.0 * a[3] + 7.0 * a[4] - a[5]) / 12.0;
  q[3] = (3.0 * a[3] + 13.0 * a[4] - 5.0 * a[5] + a[6]) / 12.0;
  b[0] = (547.0 * a[0] * a[0] - 3882.0 * a[0] * a[1] + 4642.0 * a[0] * a[2] - 1854.0 * a[0] * a[3]
          + 7043.0 * a[1] * a[1] - 17246.0 * a[1] * a[2] + 7042.0 * a[1] * a[3]
          + 11003.0 * a[2] * a[2] - 9402.0 * a[2] * a[3] + 2107.0 * a[3] * a[3]) / 240.0;
  b[1] = (267.0 * a[1] * a[1] - 1642.0 * a[1] * a[2] + 1602.0 * a[1] * a[3] - 494.0 * a[1] * a[4]
          + 2843.0 * a[2] * a[2] - 5966.0 * a[2] * a[3] + 1922.0 * a[2] * a[4]
          + 3443.0 * a[3] * a[3] - 2522.0 * a[3] * a[4] + 547.0 * a[4] * a[4]) / 240.0;
  b[2] = (547.0 * a[2] * a[2] - 2522.0 * a[2] * a[3] + 1922.0 * a[2] * a[4] - 494.0 * a[2] * a[5]
          + 3443.0 * a[3] * a[3] - 5966.0 * a[3] * a[4] + 1602.0 * a[3] * a[5]
          + 2843.0 * a[4] * a[4] - 1642.0 * a[4] * a[5] + 267.0 * a[5] * a[5]) / 240.0;
  b[3] = (2107.0 * a[3] * a[3] - 9402.0 * a[3] * a[4] + 7042.0 * a[3] * a[5] - 1854.0 * a[3] * a[6]
          + 11003.0 * a[4] * a[4] - 17246.0 * a[4] * a[5] + 4642.0 * a[4] * a[6]
          + 7043.0 * a[5] * a[5] - 3882.0 * a[5] * a[6] + 547.0 * a[6] * a[6]) / 240.0;
  const double d[4] = {1.0 / 35.0, 12.0 / 35.0, 18.0 / 35.0, 4.0 / 35.0};
  double al[4], sum = 0.0;
  for (int r = 0; r < 4; ++r) {
    al[r] = d[r] / ((eps + b[r]) * (eps + b[r]));
    sum += al[r];
  }
  double out = 0.0;
  for (int r = 0; r < 4; ++r) out += (al[r] / sum) * q[r];
  return out;
}

/* Fifth-order WENO at j+1/2 from f_{j-2..j+2}.  A substencil with valid[r]=0
   (it would use a node outside a non-periodic domain, Sec. 2.2.4) gets weight
   zero and the remaining nonlinear weights are renormalised. */
double or_weno5(const double f[5], double eps, const int valid[3]) {
  const double* a = f;
  double q[3], b[3];
  q[0] = (2.0 * a[0] - 7.0 * a[1] + 11.0 * a[2]) / 6.0;
  q[1] = (-a[1] + 5.0 * a[2] + 2.0 * a[3]) / 6.0;
  q[2] = (2.0 * a[2] + 5.0 * a[3] - a[4]) / 6.0;
  b[0] = 13.0 / 12.0 * (a[0] - 2.0 * a[1] + a[2]) * (a[0] - 2.0 * a[1] + a[2])
       + 0.25 * (a[0] - 4.0 * a[1] + 3.0 * a[2]) * (a[0] - 4.0 * a[1] + 3.0 * a[2]);
  b[1] = 13.0 / 12.0 * (a[1] - 2.0 * a[2] + a[3]) * (a[1] - 2.0 * a[2] + a[3])
       + 0.25 * (a[1] - a[3]) * (a[1] - a[3]);
  b[2] = 13.0 / 12.0 * (a[2] - 2.0 * a[3] + a[4]) * (a[2] - 2.0 * a[3] + a[4])
       + 0.25 * (3.0 * a[2] - 4.0 * a[3] + a[4]) * (3.0 * a[2] - 4.0 * a[3] + a[4]);
  const double d[3] = {0.1, 0.6, 0.3};
  double al[3], sum = 0.0;
  for (int r = 0; r < 3; ++r) {
    al[r] = valid[r] ? d[r] / ((eps + b[r]) * (eps + b[r])) : 0.0;
    sum += al[r];
  }
  double out = 0.0;
  for (int r = 0; r < 3; ++r) out += (al[r] / sum) * q[r];
  return out;
}

/* Seventh-order upwind, eq 41. */
double or_ud7(const double f[7]) {
  return (-3.0 * f[0] + 25.0 * f[1] - 101.0 * f[2] + 319.0 * f[3] + 214.0 * f[4] - 38.0 * f[5] + 4.0 * f[6]) / 420.0;
}

/* Eighth-order central interface value over f_{j-3..j+4}: its difference is the
   eighth-order central first derivative. */
double or_c8(const double f[8]) {
  return (-3.0 * f[0] + 29.0 * f[1] - 139.0 * f[2] + 533.0 * f[3] + 533.0 * f[4] - 139.0 * f[5] + 29.0 * f[6] - 3.0 * f[7]) / 840.0;
}

/* ------------------------------------------------------------------ */
/* Characteristic variables (Sec. 2.2.2, eq 31-40)                      */
/* ------------------------------------------------------------------ */

void or_char_matrices(const or_params* P, const double U[5], const double n[3], double S[25], double Sinv[25]) {
  const double g = P->gamma;
  const double rho = U[0], u = U[1] / rho, v = U[2] / rho, w = U[3] / rho;
  const double V = 0.5 * (u * u + v * v + w * w);                      /* eq 25 */
  const double p = (g - 1.0) * (U[4] - rho * V);
  const double c = sqrt(g * p / rho);
  const double H = V + c * c / (g - 1.0);                              /* eq 36 */
  const double kap = (g - 1.0) / (c * c), kap1 = 0.5 * kap, chi = 1.0 / (2.0 * c); /* eq 37 */
  double l[3], m[3];
  if (fabs(n[2]) <= fabs(n[1])) {                                      /* eq 39 */
    double r = sqrt(n[0] * n[0] + n[1] * n[1]);
    l[0] = -n[1] / r; l[1] = n[0] / r; l[2] = 0.0;
  } else {
    double r = sqrt(n[0] * n[0] + n[2] * n[2]);
    l[0] = -n[2] / r; l[1] = 0.0; l[2] = n[0] / r;
  }
  m[0] = n[1] * l[2] - n[2] * l[1];                                    /* eq 40 */
  m[1] = n[2] * l[0] - n[0] * l[2];
  m[2] = n[0] * l[1] - n[1] * l[0];
  const double un = u * n[0] + v * n[1] + w * n[2];                    /* eq 38 */
  const double ul = u * l[0] + v * l[1] + w * l[2];
  const double um = u * m[0] + v * m[1] + w * m[2];
  const double vel[3] = {u, v, w};
  /* S^-1 (eq 34), column by column: the entropy wave, the two shear waves,
     the acoustic waves u_n - c and u_n + c. */
  Sinv[0 * 5 + 0] = 1.0; Sinv[0 * 5 + 1] = 0.0; Sinv[0 * 5 + 2] = 0.0; Sinv[0 * 5 + 3] = 1.0; Sinv[0 * 5 + 4] = 1.0;
  for (int i = 0; i < 3; ++i) {
    Sinv[(1 + i) * 5 + 0] = vel[i];
    Sinv[(1 + i) * 5 + 1] = l[i];
    Sinv[(1 + i) * 5 + 2] = m[i];
    Sinv[(1 + i) * 5 + 3] = vel[i] - c * n[i];
    Sinv[(1 + i) * 5 + 4] = vel[i] + c * n[i];
  }
  Sinv[4 * 5 + 0] = V; Sinv[4 * 5 + 1] = ul; Sinv[4 * 5 + 2] = um;
  Sinv[4 * 5 + 3] = H - c * un; Sinv[4 * 5 + 4] = H + c * un;
  /* S (eq 35), row by row. */
  S[0 * 5 + 0] = 1.0 - kap * V;
  S[1 * 5 + 0] = -ul;
  S[2 * 5 + 0] = -um;
  S[3 * 5 + 0] = kap1 * V + chi * un;
  S[4 * 5 + 0] = kap1 * V - chi * un;
  for (int i = 0; i < 3; ++i) {
    S[0 * 5 + 1 + i] = kap * vel[i];
    S[1 * 5 + 1 + i] = l[i];
    S[2 * 5 + 1 + i] = m[i];
    S[3 * 5 + 1 + i] = -chi * n[i] - kap1 * vel[i];
    S[4 * 5 + 1 + i] = chi * n[i] - kap1 * vel[i];
  }
  S[0 * 5 + 4] = -kap; S[1 * 5 + 4] = 0.0; S[2 * 5 + 4] = 0.0; S[3 * 5 + 4] = kap1; S[4 * 5 + 4] = kap1;
}

/* Numerical flux at the interface between window nodes 3 and 4 (j and j+1),
   component by component.  fpw/fmw[t][m]: split fluxes of window node j-3+t;
   ok[t]: node exists. */
static void interface_flux_comp(const or_params* P, const double fpw[8][5], const double fmw[8][5],
                                const int ok[8], int flag, double F[5]) {
  int all = 1;
  for (int t = 0; t < 8; ++t) all &= ok[t];
  for (int m = 0; m < 5; ++m) {
    double a[8], b[8]; /* a: f+ window; b: f- window mirrored about j+1/2 (b[t] = f-_{j+4-t}) */
    for (int t = 0; t < 8; ++t) { a[t] = fpw[t][m]; b[t] = fmw[7 - t][m]; }
    if (!all || flag == OR_FLAG_WENO5) {
      /* Fifth-order WENO with the out-of-domain substencils masked (Sec. 2.2.4). */
      int vp[3], vm[3];
      for (int r = 0; r < 3; ++r) {
        vp[r] = ok[1 + r] && ok[2 + r] && ok[3 + r];       /* f+: nodes j-2+r .. j+r */
        vm[r] = ok[6 - r] && ok[5 - r] && ok[4 - r];       /* f-: nodes j+3-r .. j+1-r */
      }
      F[m] = or_weno5(a + 1, P->eps, vp) + or_weno5(b + 1, P->eps, vm);
    } else if (flag == OR_FLAG_LOW) {
      if (P->lowdiss == OR_C8) {
        double s[8];
        for (int t = 0; t < 8; ++t) s[t] = fpw[t][m] + fmw[t][m];
        F[m] = or_c8(s);
      } else {
        F[m] = or_ud7(a) + or_ud7(b);
      }
    } else {
      F[m] = or_weno7(a, P->eps) + or_weno7(b, P->eps);
    }
  }
}

/* Numerical flux at j+1/2.  S, Sinv: NULL for the component-wise
   reconstruction; otherwise the split fluxes of the window are carried to the
   characteristic variables of the interface state by S, reconstructed field by
   field with the same stencil choice, and carried back by S^-1 (eq 31). */
static void interface_flux(const or_params* P, const double fpw[8][5], const double fmw[8][5],
                           const int ok[8], int flag, const double* S, const double* Sinv, double F[5]) {
  if (!S) {
    interface_flux_comp(P, fpw, fmw, ok, flag, F);
    return;
  }
  double cpw[8][5], cmw[8][5], G[5];
  for (int t = 0; t < 8; ++t)
    for (int k = 0; k < 5; ++k) {
      double a = 0.0, b = 0.0;
      for (int m = 0; m < 5; ++m) {
        a += S[k * 5 + m] * fpw[t][m];
        b += S[k * 5 + m] * fmw[t][m];
      }
      cpw[t][k] = a;
      cmw[t][k] = b;
    }
  interface_flux_comp(P, cpw, cmw, ok, flag, G);
  for (int m = 0; m < 5; ++m) {
    double a = 0.0;
    for (int k = 0; k < 5; ++k) a += Sinv[m * 5 + k] * G[k];
    F[m] = a;
  }
}

/* The characteristic matrices of interface c+1/2 along d: the interface state
   is the mean of the conserved variables of its two nodes (eq 32), the normal
   the unit vector of the mean of their metric rows of direction d. */
static void interface_char(const or_params* P, const double* met, const double* U, const int c[3], int d,
                           double S[25], double Sinv[25]) {
  const long N = n_nodes(P);
  const long i0 = lin(P, c);
  long i1;
  shifted(P, c, d, 1, &i1, NULL);
  double Ua[5], a[3];
  for (int m = 0; m < 5; ++m) Ua[m] = 0.5 * (U[(long)m * N + i0] + U[(long)m * N + i1]);
  for (int q = 0; q < 3; ++q) a[q] = 0.5 * (met[(long)(3 * d + q) * N + i0] + met[(long)(3 * d + q) * N + i1]);
  const double r = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  const double nrm[3] = {a[0] / r, a[1] / r, a[2] / r};
  or_char_matrices(P, Ua, nrm, S, Sinv);
}

/* ------------------------------------------------------------------ */
/* Shock sensor (eq 42-43) and interface flags                          */
/* ------------------------------------------------------------------ */

static double node_pressure(const or_params* P, const double* U, long N, long id) {
  return primitive(P, U, N, id).p;
}

static double node_theta(const or_params* P, const double* U, const int c[3]) {
  const long N = n_nodes(P);
  double th = 0.0;
  for (int d = 0; d < 3; ++d) {
    long im, ip, i0 = lin(P, c);
    /* A node on a non-periodic end has no second difference: phi = 0 there. */
    if (!shifted(P, c, d, -1, &im, NULL) || !shifted(P, c, d, 1, &ip, NULL)) continue;
    double pm = node_pressure(P, U, N, im), p0 = node_pressure(P, U, N, i0), pp = node_pressure(P, U, N, ip);
    th += fabs(-pm + 2.0 * p0 - pp) / (pm + 2.0 * p0 + pp);
  }
  return th;
}

/* Flag of the interface j+1/2 along d (eq 43) from the largest sensor value
   of its window: the 8 stencil nodes j-3 .. j+4, or with flag_window = 1 the
   two nodes j and j+1 (the paper applies theta "at positions" without naming
   them; both readings give every interface one flag, as conservation needs). */
static int interface_flag(const or_params* P, const double* theta, const int c[3], int d) {
  double mx = 0.0;
  const int lo = P->flag_window == 1 ? 0 : -3, hi = P->flag_window == 1 ? 1 : 4;
  for (int m = lo; m <= hi; ++m) {
    long id;
    if (!shifted(P, c, d, m, &id, NULL)) continue;
    if (theta[id] > mx) mx = theta[id];
  }
  if (mx <= P->theta1) return OR_FLAG_LOW;
  if (P->three_way && mx > P->theta2) return OR_FLAG_WENO5;
  return OR_FLAG_WENO7;
}

int or_sensor(const or_params* P, const double* U, double* theta, uint8_t* flags) {
  set_threads(P);
  const long N = n_nodes(P);
#pragma omp parallel for schedule(static)
  for (long id = 0; id < N; ++id) {
    int c[3]; unlin(P, id, c);
    theta[id] = node_theta(P, U, c);
  }
  if (flags) {
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
      int c[3]; unlin(P, id, c);
      for (int d = 0; d < 3; ++d) flags[(long)d * N + id] = (uint8_t)interface_flag(P, theta, c, d);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Pieces of the right-hand side                                        */
/* ------------------------------------------------------------------ */

/* Split fluxes of node id for direction d (alpha = row d of the metrics / J). */
static void node_split(const or_params* P, const double* met, const prim_t* q, long N, long id, int d,
                       double fp[5], double fm[5]) {
  double alpha[3] = {met[(long)(3 * d) * N + id], met[(long)(3 * d + 1) * N + id], met[(long)(3 * d + 2) * N + id]};
  or_sw_split(P, q[id].rho, q[id].u, q[id].v, q[id].w, q[id].p, alpha, fp, fm);
}

/* Does node c have an interface at c+1/2 along d? */
static int has_right_interface(const or_params* P, const int c[3], int d) {
  return P->periodic[d] || c[d] < dim_n(P, d) - 1;
}

/* Numerical flux at c+1/2 along d, the split fluxes computed on the spot. */
static void flux_at(const or_params* P, const double* met, const double* U, const prim_t* q, const uint8_t* flags,
                    const int c[3], int d, double F[5]) {
  const long N = n_nodes(P);
  double fpw[8][5], fmw[8][5];
  int ok[8];
  for (int t = 0; t < 8; ++t) {
    long id;
    ok[t] = shifted(P, c, d, t - 3, &id, NULL);
    if (ok[t]) node_split(P, met, q, N, id, d, fpw[t], fmw[t]);
    else for (int m = 0; m < 5; ++m) fpw[t][m] = fmw[t][m] = 0.0;
  }
  double S[25], Si[25];
  if (P->characteristic) interface_char(P, met, U, c, d, S, Si);
  interface_flux(P, fpw, fmw, ok, flags ? flags[(long)d * N + lin(P, c)] : OR_FLAG_WENO7,
                 P->characteristic ? S : NULL, P->characteristic ? Si : NULL, F);
}

/* Viscous flux vectors F_v, G_v, H_v (eq 9-14) at node c: Fv[d][0..3] are the
   momentum and energy components of the viscous flux of direction d. */
static void viscous_flux_at(const or_params* P, const double* met, const prim_t* q, const int c[3], double Fv[3][4]) {
  const long N = n_nodes(P);
  const long id = lin(P, c);
  /* Derivatives of u, v, w, T along xi, eta, zeta (sixth or eighth order,
     Sec. 2.3). */
  const int vh = P->viscous / 2;
  double dq[4][3];
  for (int d = 0; d < 3; ++d) {
    double vals[4][9];
    for (int m = -4; m <= 4; ++m) {
      long nid;
      if (m < -vh || m > vh || !shifted(P, c, d, m, &nid, NULL)) {
        for (int s = 0; s < 4; ++s) vals[s][m + 4] = 0.0;
        continue;
      }
      vals[0][m + 4] = q[nid].u; vals[1][m + 4] = q[nid].v; vals[2][m + 4] = q[nid].w; vals[3][m + 4] = q[nid].T;
    }
    for (int s = 0; s < 4; ++s)
      dq[s][d] = line_derivative(vals[s], 4, c[d], dim_n(P, d), P->periodic[d], vh, P->h[d]);
  }
  /* Chain rule: d/dx_col = sum_d (metric_{d,col}/J) / (1/J) * d/d(direction d). */
  double Jinv = met[9 * N + id];
  double g[4][3]; /* g[s][col] */
  for (int s = 0; s < 4; ++s)
    for (int col = 0; col < 3; ++col) {
      double acc = 0.0;
      for (int d = 0; d < 3; ++d) acc += (met[(long)(3 * d + col) * N + id] / Jinv) * dq[s][d];
      g[s][col] = acc;
    }
  double T = q[id].T;
  double S = P->suth / P->Tref;
  double mu = T * sqrt(T) * (1.0 + S) / (T + S);                                   /* eq 15 */
  double kc = mu / ((P->gamma - 1.0) * P->Ma * P->Ma * P->Pr * P->Re);              /* eq 14 */
  double div = g[0][0] + g[1][1] + g[2][2];
  double tau[3][3];                                                                  /* eq 13 */
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      tau[a][b] = (mu / P->Re) * (g[a][b] + g[b][a] - (a == b ? 2.0 / 3.0 * div : 0.0));
  double vel[3] = {q[id].u, q[id].v, q[id].w};
  double Th[3];                                                                      /* eq 12 */
  for (int a = 0; a < 3; ++a)
    Th[a] = vel[0] * tau[0][a] + vel[1] * tau[1][a] + vel[2] * tau[2][a] + kc * g[3][a];
  for (int d = 0; d < 3; ++d) {                                                      /* eq 9-11 */
    double m0 = met[(long)(3 * d) * N + id], m1 = met[(long)(3 * d + 1) * N + id], m2 = met[(long)(3 * d + 2) * N + id];
    for (int b = 0; b < 3; ++b) Fv[d][b] = m0 * tau[0][b] + m1 * tau[1][b] + m2 * tau[2][b];
    Fv[d][3] = m0 * Th[0] + m1 * Th[1] + m2 * Th[2];
  }
}

/* Is node c on a face whose kind sets its value after the stage (every kind
   but the nonreflecting one)?  Such nodes have dU/dt = 0. */
static int on_set_face(const or_params* P, const int c[3]) {
  for (int d = 0; d < 3; ++d) {
    if (P->periodic[d]) continue;
    int n = dim_n(P, d);
    if (c[d] == 0 && P->bc[2 * d] != OR_BC_NRBC) return 1;
    if (c[d] == n - 1 && P->bc[2 * d + 1] != OR_BC_NRBC) return 1;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Characteristic nonreflecting faces (Thompson 1987; Poinsot & Lele    */
/* 1992).  The paper imposes nonreflecting conditions at the exit and  */
/* the upper boundary of the ramp (Sec. 6.1) without formulas.          */
/* ------------------------------------------------------------------ */

/* Normal-direction part of dU/dt at a node of face (d, side).  Along the
   grid line the Euler equations in primitive variables q = (rho, u, v, w, p)
   read  dq/dt + s A_n dq/dxi = ...  with s = |grad xi_d| and A_n the Jacobian
   along the unit normal n = grad xi_d / s (metric derivatives dropped).  Its
   characteristic wave amplitudes, with dq/dxi the one-sided second-order
   difference into the grid and u_n = u.n:
     L1 = s (u_n - c) (dp - rho c du_n)        L5 = s (u_n + c) (dp + rho c du_n)
     L2 = s u_n (c^2 drho - dp)                Lt = s u_n (du - n (n.du))
   A wave entering the grid (speed < 0 on the upper face, > 0 on the lower)
   has amplitude zero.  Then
     drho/dt = -(L2 + (L5 + L1)/2) / c^2,   dp/dt = -(L5 + L1)/2,
     du/dt = -(n (L5 - L1) / (2 rho c) + Lt),
   carried to the conserved variables (eq 5, 8).  The part of the normal flux
   derivative that the frozen normal leaves out, -J sum_a d(xi_a/J)/dxi F_a
   (F_a the Cartesian inviscid flux of eq 6), is added as it stands (one-sided
   second-order difference of the metrics): on a curved grid it balances the
   metric derivatives of the transverse fluxes, so a uniform stream stays
   uniform at the face. */
static void nrbc_normal(const or_params* P, const double* met, const double* U, const int c[3], int d, int side,
                        double out[5]) {
  const long N = n_nodes(P);
  const long id = lin(P, c);
  const double h = P->h[d];
  /* primitives of the node and of the next two nodes into the grid */
  double q[3][5];
  for (int t = 0; t < 3; ++t) {
    int ct[3] = {c[0], c[1], c[2]};
    ct[d] += side ? -t : t;
    prim_t r = primitive(P, U, N, lin(P, ct));
    q[t][0] = r.rho; q[t][1] = r.u; q[t][2] = r.v; q[t][3] = r.w; q[t][4] = r.p;
  }
  /* dq/dxi_d by the one-sided second-order difference */
  double dq[5];
  for (int m = 0; m < 5; ++m) {
    double one = (-3.0 * q[0][m] + 4.0 * q[1][m] - q[2][m]) / (2.0 * h);
    dq[m] = side ? -one : one;
  }
  const double Jinv = met[9 * N + id];
  double gx[3];
  for (int a = 0; a < 3; ++a) gx[a] = met[(long)(3 * d + a) * N + id] / Jinv;   /* grad xi_d */
  const double sg = sqrt(gx[0] * gx[0] + gx[1] * gx[1] + gx[2] * gx[2]);
  const double n[3] = {gx[0] / sg, gx[1] / sg, gx[2] / sg};
  const double rho = q[0][0], u[3] = {q[0][1], q[0][2], q[0][3]}, p = q[0][4];
  const double cs = sqrt(P->gamma * p / rho);
  const double un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
  const double du[3] = {dq[1], dq[2], dq[3]};
  const double dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
  const double lam1 = sg * (un - cs), lam2 = sg * un, lam5 = sg * (un + cs);
  /* a wave enters through the upper face when its speed is negative, through
     the lower face when it is positive */
  #define OUTGOING(l) (side ? (l) >= 0.0 : (l) <= 0.0)
  const double L1 = OUTGOING(lam1) ? lam1 * (dq[4] - rho * cs * dun) : 0.0;
  const double L5 = OUTGOING(lam5) ? lam5 * (dq[4] + rho * cs * dun) : 0.0;
  const double L2 = OUTGOING(lam2) ? lam2 * (cs * cs * dq[0] - dq[4]) : 0.0;
  double Lt[3];
  for (int a = 0; a < 3; ++a) Lt[a] = OUTGOING(lam2) ? lam2 * (du[a] - n[a] * dun) : 0.0;
  #undef OUTGOING
  const double drho = -(L2 + 0.5 * (L5 + L1)) / (cs * cs);
  const double dp = -0.5 * (L5 + L1);
  double dvel[3];
  for (int a = 0; a < 3; ++a) dvel[a] = -(n[a] * (L5 - L1) / (2.0 * rho * cs) + Lt[a]);
  out[0] = drho;
  for (int a = 0; a < 3; ++a) out[1 + a] = u[a] * drho + rho * dvel[a];
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  out[4] = dp / (P->gamma - 1.0) + 0.5 * uu * drho + rho * (u[0] * dvel[0] + u[1] * dvel[1] + u[2] * dvel[2]);
  /* metric-derivative part */
  const double E = U[4 * N + id];
  for (int a = 0; a < 3; ++a) {
    double mt[3];
    for (int t = 0; t < 3; ++t) {
      int ct[3] = {c[0], c[1], c[2]};
      ct[d] += side ? -t : t;
      mt[t] = met[(long)(3 * d + a) * N + lin(P, ct)];
    }
    double dm = (-3.0 * mt[0] + 4.0 * mt[1] - mt[2]) / (2.0 * h);
    if (side) dm = -dm;
    const double Fa[5] = {rho * u[a], rho * u[0] * u[a] + (a == 0 ? p : 0.0), rho * u[1] * u[a] + (a == 1 ? p : 0.0),
                          rho * u[2] * u[a] + (a == 2 ? p : 0.0), (E + p) * u[a]};
    for (int m = 0; m < 5; ++m) out[m] -= dm * Fa[m] / Jinv;
  }
}

int or_nrbc_normal(const or_params* P, const double* met, const double* U, int32_t i, int32_t j, int32_t k,
                   int32_t d, int32_t side, double* out) {
  int c[3] = {i, j, k};
  if (d < 0 || d > 2 || P->periodic[d] || c[d] != (side ? dim_n(P, d) - 1 : 0)) return -1;
  nrbc_normal(P, met, U, c, d, side, out);
  return 0;
}

/* dU/dt at node c from its interface fluxes and viscous fluxes:
   Fl[d] = flux at c-1/2, Fr[d] = flux at c+1/2 along d;
   Fvn[d][m+4][s] = viscous flux component s of direction d at node c+m e_d.
   A node on a face whose kind sets it after the stage gets 0.  A node on
   nonreflecting faces only takes the usual terms along the directions it is
   interior to and, along each direction it is an end of, the characteristic
   normal part of that face instead (no normal viscous term). */
static void assemble(const or_params* P, const double* met, const double* U, const int c[3], int32_t parts,
                     const double Fl[3][5], const double Fr[3][5], const double Fvn[3][9][4], double out[5]) {
  const long N = n_nodes(P);
  double rhs[5] = {0, 0, 0, 0, 0};
  if (on_set_face(P, c)) { for (int m = 0; m < 5; ++m) out[m] = 0.0; return; }
  int end[3] = {0, 0, 0};   /* end[d]: 1 lower end, 2 upper end of a bounded line */
  for (int d = 0; d < 3; ++d)
    if (!P->periodic[d]) end[d] = c[d] == 0 ? 1 : (c[d] == dim_n(P, d) - 1 ? 2 : 0);
  for (int d = 0; d < 3; ++d) {
    if (end[d]) continue;
    if (parts & (1 << d))
      for (int m = 0; m < 5; ++m) rhs[m] -= (Fr[d][m] - Fl[d][m]) / P->h[d];
    if ((parts & OR_PART_VISC) && P->viscous)
      for (int s = 0; s < 4; ++s) {
        double vals[9];
        for (int t = 0; t < 9; ++t) vals[t] = Fvn[d][t][s];
        rhs[s + 1] += line_derivative(vals, 4, c[d], dim_n(P, d), P->periodic[d], P->viscous / 2, P->h[d]);
      }
  }
  double Jinv = met[9 * N + lin(P, c)];
  for (int m = 0; m < 5; ++m) out[m] = rhs[m] / Jinv;   /* L(U) of eq 44 for U, not U/J */
  for (int d = 0; d < 3; ++d) {
    if (!end[d] || !(parts & (1 << d))) continue;
    double nb[5];
    nrbc_normal(P, met, U, c, d, end[d] == 2, nb);
    for (int m = 0; m < 5; ++m) out[m] += nb[m];
  }
}

static prim_t* all_primitives(const or_params* P, const double* U) {
  const long N = n_nodes(P);
  prim_t* q = (prim_t*)malloc(sizeof(prim_t) * N);
  if (!q) return NULL;
#pragma omp parallel for schedule(static)
  for (long id = 0; id < N; ++id) q[id] = primitive(P, U, N, id);
  return q;
}

static uint8_t* default_flags(const or_params* P, const double* U, const uint8_t* flags, int* owned) {
  *owned = 0;
  if (flags || P->scheme != OR_HYBRID) return (uint8_t*)flags;
  const long N = n_nodes(P);
  double* theta = (double*)malloc(sizeof(double) * N);
  uint8_t* f = (uint8_t*)malloc(3 * N);
  or_sensor(P, U, theta, f);
  free(theta);
  *owned = 1;
  return f;
}

int or_dudt(const or_params* P, const double* met, const double* U, const uint8_t* flags_in,
            int32_t parts, double* dudt) {
  set_threads(P);
  const long N = n_nodes(P);
  prim_t* q = all_primitives(P, U);
  int owned;
  uint8_t* flags = default_flags(P, U, flags_in, &owned);
  /* Interface fluxes F[d][m][node]: the flux at node+1/2 along d. */
  double* F = (double*)calloc(15 * (size_t)N, sizeof(double));
  double* fp = (double*)malloc(sizeof(double) * 5 * N);
  double* fm = (double*)malloc(sizeof(double) * 5 * N);
  double* Fv = (double*)calloc(12 * (size_t)N, sizeof(double));
  if (!q || !F || !fp || !fm || !Fv) return -1;
  for (int d = 0; d < 3; ++d) {
    if (!(parts & (1 << d))) continue;
    /* Split fluxes at every node (eq 30) ... */
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
      double a[5], b[5];
      node_split(P, met, q, N, id, d, a, b);
      for (int m = 0; m < 5; ++m) { fp[(long)m * N + id] = a[m]; fm[(long)m * N + id] = b[m]; }
    }
    /* ... then the numerical flux at every interface. */
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
      int c[3]; unlin(P, id, c);
      if (!has_right_interface(P, c, d)) continue;
      double fpw[8][5], fmw[8][5];
      int ok[8];
      for (int t = 0; t < 8; ++t) {
        long nid;
        ok[t] = shifted(P, c, d, t - 3, &nid, NULL);
        for (int m = 0; m < 5; ++m) {
          fpw[t][m] = ok[t] ? fp[(long)m * N + nid] : 0.0;
          fmw[t][m] = ok[t] ? fm[(long)m * N + nid] : 0.0;
        }
      }
      double Fi[5], S[25], Si[25];
      if (P->characteristic) interface_char(P, met, U, c, d, S, Si);
      interface_flux(P, fpw, fmw, ok, flags ? flags[(long)d * N + id] : OR_FLAG_WENO7,
                     P->characteristic ? S : NULL, P->characteristic ? Si : NULL, Fi);
      for (int m = 0; m < 5; ++m) F[(long)(5 * d + m) * N + id] = Fi[m];
    }
  }
  if ((parts & OR_PART_VISC) && P->viscous) {
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
      int c[3]; unlin(P, id, c);
      double v[3][4];
      viscous_flux_at(P, met, q, c, v);
      for (int d = 0; d < 3; ++d)
        for (int s = 0; s < 4; ++s) Fv[(long)(4 * d + s) * N + id] = v[d][s];
    }
  }
#pragma omp parallel for schedule(static)
  for (long id = 0; id < N; ++id) {
    int c[3]; unlin(P, id, c);
    double Fl[3][5], Fr[3][5], Fvn[3][9][4];
    for (int d = 0; d < 3; ++d) {
      long nl;
      int okl = shifted(P, c, d, -1, &nl, NULL);
      for (int m = 0; m < 5; ++m) {
        Fr[d][m] = F[(long)(5 * d + m) * N + id];
        Fl[d][m] = okl ? F[(long)(5 * d + m) * N + nl] : 0.0;
      }
      for (int t = 0; t < 9; ++t) {
        long nid;
        int ok = t - 4 >= -P->viscous / 2 && t - 4 <= P->viscous / 2 && shifted(P, c, d, t - 4, &nid, NULL);
        for (int s = 0; s < 4; ++s) Fvn[d][t][s] = ok ? Fv[(long)(4 * d + s) * N + nid] : 0.0;
      }
    }
    double o[5];
    assemble(P, met, U, c, parts, Fl, Fr, Fvn, o);
    for (int m = 0; m < 5; ++m) dudt[(long)m * N + id] = o[m];
  }
  free(q); free(F); free(fp); free(fm); free(Fv);
  if (owned) free(flags);
  return 0;
}

int or_dudt_points(const or_params* P, const double* met, const double* U, const uint8_t* flags_in,
                   int32_t parts, int64_t npts, const int64_t* nodes, double* out) {
  set_threads(P);
  prim_t* q = all_primitives(P, U);
  int owned;
  uint8_t* flags = default_flags(P, U, flags_in, &owned);
  if (!q) return -1;
#pragma omp parallel for schedule(dynamic)
  for (int64_t s = 0; s < npts; ++s) {
    int c[3]; unlin(P, (long)nodes[s], c);
    double Fl[3][5], Fr[3][5], Fvn[3][9][4];
    for (int d = 0; d < 3; ++d) {
      for (int m = 0; m < 5; ++m) Fl[d][m] = Fr[d][m] = 0.0;
      if (parts & (1 << d)) {
        if (has_right_interface(P, c, d)) flux_at(P, met, U, q, flags, c, d, Fr[d]);
        long nl;
        if (shifted(P, c, d, -1, &nl, NULL)) {
          int cl[3]; unlin(P, nl, cl);
          flux_at(P, met, U, q, flags, cl, d, Fl[d]);
        }
      }
      for (int t = 0; t < 9; ++t) {
        long nid;
        for (int k = 0; k < 4; ++k) Fvn[d][t][k] = 0.0;
        if (!((parts & OR_PART_VISC) && P->viscous)) continue;
        if (t - 4 < -P->viscous / 2 || t - 4 > P->viscous / 2) continue;
        if (!shifted(P, c, d, t - 4, &nid, NULL)) continue;
        int cn[3]; unlin(P, nid, cn);
        double v[3][4];
        viscous_flux_at(P, met, q, cn, v);
        for (int k = 0; k < 4; ++k) Fvn[d][t][k] = v[d][k];
      }
    }
    assemble(P, met, U, c, parts, Fl, Fr, Fvn, out + 5 * s);
  }
  free(q);
  if (owned) free(flags);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Boundary conditions of the non-periodic faces                        */
/* ------------------------------------------------------------------ */

/* Conserved variables from rho, velocity and p (eq 5, 8). */
static void conserved(const or_params* P, double rho, double u, double v, double w, double p, double out[5]) {
  out[0] = rho; out[1] = rho * u; out[2] = rho * v; out[3] = rho * w;
  out[4] = p / (P->gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w);
}

/* Boundary readings (the paper names the kinds but gives no formulas):
   inflow: the stored inflow state is imposed;  extrapolation: primitive
   variables copied from the first interior node;  isothermal wall: zero
   velocity, T = Tw, p from the first interior node, rho = gamma Ma^2 p / Tw. */
int or_apply_bc(const or_params* P, double* U, const double* inflow) {
  const long N = n_nodes(P);
  for (int d = 0; d < 3; ++d) {
    if (P->periodic[d]) continue;
    for (int side = 0; side < 2; ++side) {
      int kind = P->bc[2 * d + side];
      if (kind == OR_BC_NONE || kind == OR_BC_NRBC) continue;
      int n = dim_n(P, d);
      for (long id = 0; id < N; ++id) {
        int c[3]; unlin(P, id, c);
        if (c[d] != (side ? n - 1 : 0)) continue;
        int ci[3] = {c[0], c[1], c[2]};
        ci[d] = side ? n - 2 : 1;
        long ii = lin(P, ci);
        prim_t qi = primitive(P, U, N, ii);
        double o[5];
        if (kind == OR_BC_INFLOW && inflow) {
          /* inflow: conserved variables on this face, [5][face], the face
             indexed by its two other node indices, lower direction fastest */
          int e0 = d == 0 ? 1 : 0, e1 = d == 2 ? 1 : 2;
          long nf = (long)dim_n(P, e0) * dim_n(P, e1);
          long fi = c[e0] + (long)dim_n(P, e0) * c[e1];
          for (int m = 0; m < 5; ++m) o[m] = inflow[(long)m * nf + fi];
        } else if (kind == OR_BC_WALL) {
          double rho = P->gamma * P->Ma * P->Ma * qi.p / P->Tw;
          conserved(P, rho, 0.0, 0.0, 0.0, qi.p, o);
        } else {
          conserved(P, qi.rho, qi.u, qi.v, qi.w, qi.p, o);
        }
        for (int m = 0; m < 5; ++m) U[(long)m * N + id] = o[m];
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Third-order Runge-Kutta (eq 45)                                      */
/* ------------------------------------------------------------------ */

int or_advance(const or_params* P, const double* met, double* U, double* Un, int32_t* stage,
               int32_t n, double dt, const double* inflow) {
  set_threads(P);
  const long N = n_nodes(P);
  double* L = (double*)malloc(sizeof(double) * 5 * N);
  if (!L) return -1;
  static const double A[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
  static const double B[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};
  for (int s = 0; s < n; ++s) {
    int k = *stage;
    if (k == 0) memcpy(Un, U, sizeof(double) * 5 * N);
    int rc = or_dudt(P, met, U, NULL, OR_PART_ALL, L);
    if (rc) { free(L); return rc; }
#pragma omp parallel for schedule(static)
    for (long i = 0; i < 5 * N; ++i) U[i] = A[k] * Un[i] + B[k] * (U[i] + dt * L[i]);
    or_apply_bc(P, U, inflow);
    *stage = (k + 1) % 3;
  }
  free(L);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Global sums and extrema                                              */
/* ------------------------------------------------------------------ */

int or_reduce(const or_params* P, const double* met, const double* U, double dt, double* out) {
  const long N = n_nodes(P);
  for (int m = 0; m < 5; ++m) {
    /* Neumaier-compensated sum of U_m/J */
    double s = 0.0, comp = 0.0;
    for (long id = 0; id < N; ++id) {
      double x = U[(long)m * N + id] * met[9 * N + id];
      double t = s + x;
      if (fabs(s) >= fabs(x)) comp += (s - t) + x;
      else comp += (x - t) + s;
      s = t;
    }
    out[m] = s + comp;
  }
  double cfl = 0.0, pmin = INFINITY, rmin = INFINITY, bad = 0.0;
  for (long id = 0; id < N; ++id) {
    for (int m = 0; m < 5; ++m)
      if (!isfinite(U[(long)m * N + id])) bad += 1.0;
    prim_t q = primitive(P, U, N, id);
    double local = 0.0;
    for (int d = 0; d < 3; ++d) {
      double a0 = met[(long)(3 * d) * N + id], a1 = met[(long)(3 * d + 1) * N + id], a2 = met[(long)(3 * d + 2) * N + id];
      double sig = sqrt(a0 * a0 + a1 * a1 + a2 * a2) / met[9 * N + id];
      double V = (a0 * q.u + a1 * q.v + a2 * q.w) / met[9 * N + id];
      local += (fabs(V) + q.c * sig) / P->h[d];
    }
    local *= dt;
    if (local > cfl) cfl = local;
    if (q.p < pmin) pmin = q.p;
    if (q.rho < rmin) rmin = q.rho;
  }
  out[5] = cfl; out[6] = pmin; out[7] = rmin; out[8] = bad;
  return 0;
}
