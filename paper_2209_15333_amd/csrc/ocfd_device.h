// Device helpers shared by the kernels of the ocfd library: periodic index
// wrapping, the Steger-Warming split, the interface reconstructions and the
// central first derivative with its closures.
#pragma once

#include "ocfd_internal.h"

namespace ocfd {

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------

// Position p (possibly outside [0, n)) wrapped into a periodic line of n nodes.
__device__ __forceinline__ int wrap(int p, int n) {
  while (p < 0) p += n;
  while (p >= n) p -= n;
  return p;
}

// The same for -n <= p < 2n (one conditional step each way).
__device__ __forceinline__ int wrap1(int p, int n) {
  p += (p < 0) ? n : 0;
  p -= (p >= n) ? n : 0;
  return p;
}

// Steger-Warming split of one node (eq 19-30).  The vector of eq 23, with the
// three momentum rows using k1, k2, k3 and the energy row
// (g-1) l1 |u|^2 + W + l4 |u - c k|^2 / 2 + l5 |u + c k|^2 / 2, is rearranged
// with B = l4 + l5 and D = c (l5 - l4) into
//   f0 = s (2(g-1) l1 + B)
//   f_i = s ((2(g-1) l1 + B) u_i + D k_i)
//   f4 = s (|u|^2 ((g-1) l1 + B/2) + B c^2 / (g-1) + D (u.k)),  s = rho / (2 g),
// evaluated once with the positive and once with the negative eigenvalue
// parts of eq 29.
template <typename R>
__device__ __forceinline__ R rcp_r(R x);
// FP64: the hardware reciprocal estimate refined by two Newton-Raphson steps
// r <- r + r (1 - x r) (error squared at each step), within an ulp or two of
// 1/x for the normal, finite x the kernels pass (six instructions against
// about twelve for a correctly rounded division).
template <>
__device__ __forceinline__ double rcp_r<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
  r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
  return r;
}
template <>
__device__ __forceinline__ float rcp_r<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// R is the precision of the split and of the reconstruction: double for the
// FP64 path, float for the mixed form.
template <typename R>
__device__ __forceinline__ void sw_split(const Phys& ph, R rho, R ir, R u, R v, R w, R p, R a0, R a1, R a2, R* fp,
                                         R* fm) {
  const R gm1 = (R)ph.gm1;
  const R c2 = (R)ph.gamma * p * ir;
  const R c = sqrt(c2);
  const R sig = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
  const R isig = rcp_r<R>(sig);
  const R k0 = a0 * isig, k1 = a1 * isig, k2 = a2 * isig;
  const R V = a0 * u + a1 * v + a2 * w;
  const R cs = c * sig;
  const R l4 = V - cs, l5 = V + cs;
  const R q2 = u * u + v * v + w * w;
  const R uk = V * isig;
  const R s = rho * (R)ph.inv_2g;
  const R c2g = c2 * (R)ph.inv_gm1;
  const R half = (R)0.5;
#pragma unroll
  for (int sgn = 0; sgn < 2; ++sgn) {
    const R L1 = sgn == 0 ? half * (V + fabs(V)) : half * (V - fabs(V));
    const R L4 = sgn == 0 ? half * (l4 + fabs(l4)) : half * (l4 - fabs(l4));
    const R L5 = sgn == 0 ? half * (l5 + fabs(l5)) : half * (l5 - fabs(l5));
    const R A = (R)2 * gm1 * L1;
    const R B = L4 + L5;
    const R D = c * (L5 - L4);
    const R AB = A + B;
    R* f = sgn == 0 ? fp : fm;
    f[0] = s * AB;
    f[1] = s * (AB * u + D * k0);
    f[2] = s * (AB * v + D * k1);
    f[3] = s * (AB * w + D * k2);
    f[4] = s * (q2 * (gm1 * L1 + half * B) + B * c2g + D * uk);
  }
}

// Seventh-order WENO value at j+1/2 from a0..a6 = f_{j-3..j+3} (left-biased;
// Table 2 scheme 4 with the Jiang-Shu smoothness indicators).
//
// The four cubic candidates share the first, second and third differences
// D_k = a_{k+1} - a_k, E_k = D_{k+1} - D_k, G_k = E_{k+1} - E_k.  For candidate
// r (cells j-3+r .. j+r) the derivatives of its polynomial at the centre of
// cell j are d3 = G_r, d2 = E_r + (2, 1, 0, -1)_r G_r and
// d1 = D_r + (5/2, 3/2, 1/2, -1/2)_r E_r + (43, 7, -5, 7)_r/24 G_r, and the
// indicator sum_{l=1..3} int_cell (p^(l))^2 equals
//   (d1 + d3/24)^2 + 13/12 d2^2 + 781/720 d3^2,
// a sum of squares that avoids the cancellation of the expanded quadratic
// form.  The candidate values at j+1/2 follow from the same differences.  The
// four weight divisions are folded into one: w_r = d_r prod_{s != r} (eps + beta_s)^2
// with d = (1, 12, 18, 4)/35 (the common 1/35 cancels).
template <typename R>
__device__ __forceinline__ R weno7(R a0, R a1, R a2, R a3, R a4, R a5, R a6, R eps) {
  const R D0 = a1 - a0, D1 = a2 - a1, D2 = a3 - a2, D3 = a4 - a3, D4 = a5 - a4, D5 = a6 - a5;
  const R E0 = D1 - D0, E1 = D2 - D1, E2 = D3 - D2, E3 = D4 - D3, E4 = D5 - D4;
  const R G0 = E1 - E0, G1 = E2 - E1, G2 = E3 - E2, G3 = E4 - E3;
  // t_r = d1 + d3/24 and d2 of each candidate
  const R t0 = D0 + (R)2.5 * E0 + (R)(11.0 / 6.0) * G0, s0 = E0 + (R)2 * G0;
  const R t1 = D1 + (R)1.5 * E1 + (R)(1.0 / 3.0) * G1, s1 = E1 + G1;
  const R t2 = D2 + (R)0.5 * E2 - (R)(1.0 / 6.0) * G2, s2 = E2;
  const R t3 = D3 - (R)0.5 * E3 + (R)(1.0 / 3.0) * G3, s3 = E3 - G3;
  const R C2 = (R)(13.0 / 12.0), C3 = (R)(781.0 / 720.0);
  R e0 = eps + (t0 * t0 + C2 * s0 * s0 + C3 * G0 * G0);
  R e1 = eps + (t1 * t1 + C2 * s1 * s1 + C3 * G1 * G1);
  R e2 = eps + (t2 * t2 + C2 * s2 * s2 + C3 * G2 * G2);
  R e3 = eps + (t3 * t3 + C2 * s3 * s3 + C3 * G3 * G3);
  e0 *= e0;
  e1 *= e1;
  e2 *= e2;
  e3 *= e3;
  // candidate values at j+1/2 relative to a3 = f_j: for every candidate
  // q_r - f_j = (0.5 D + (4/3, 5/6, 1/3, -1/6)_r E + (13/12, 1/4, -1/12, 1/12)_r G)
  // = t_r / 2 + s_r / 12 (the same differences as the indicator)
  const R c12 = (R)(1.0 / 12.0);
  const R q0 = (R)0.5 * t0 + c12 * s0;
  const R q1 = (R)0.5 * t1 + c12 * s1;
  const R q2 = (R)0.5 * t2 + c12 * s2;
  const R q3 = (R)0.5 * t3 + c12 * s3;
  if (sizeof(R) == 4) {
    // FP32: the weights d_r / (eps + beta_r)^2 from four reciprocals; the
    // folded product of three (eps + beta)^2 factors can leave the float range.
    const R i0 = rcp_r<R>(e0), i1 = rcp_r<R>(e1), i2 = rcp_r<R>(e2), i3 = rcp_r<R>(e3);
    const R w0 = i0, w1 = (R)12 * i1, w2 = (R)18 * i2, w3 = (R)4 * i3;
    return a3 + (w0 * q0 + w1 * q1 + w2 * q2 + w3 * q3) * rcp_r<R>(w0 + w1 + w2 + w3);
  }
  const R e01 = e0 * e1, e23 = e2 * e3;
  const R w0 = e1 * e23;
  const R w1 = (R)12 * e0 * e23;
  const R w2 = (R)18 * e3 * e01;
  const R w3 = (R)4 * e2 * e01;
  return a3 + (w0 * q0 + w1 * q1 + w2 * q2 + w3 * q3) * rcp_r<R>(w0 + w1 + w2 + w3);
}

// Seventh-order upwind value at j+1/2 (eq 41).
template <typename R>
__device__ __forceinline__ R ud7(R a0, R a1, R a2, R a3, R a4, R a5, R a6) {
  return ((R)-3 * a0 + (R)25 * a1 - (R)101 * a2 + (R)319 * a3 + (R)214 * a4 - (R)38 * a5 + (R)4 * a6) *
         (R)(1.0 / 420.0);
}

// Eighth-order central value at j+1/2 over g_{j-3..j+4}.
template <typename R>
__device__ __forceinline__ R c8(R g0, R g1, R g2, R g3, R g4, R g5, R g6, R g7) {
  return ((R)-3 * (g0 + g7) + (R)29 * (g1 + g6) - (R)139 * (g2 + g5) + (R)533 * (g3 + g4)) * (R)(1.0 / 840.0);
}

// Fifth-order WENO at j+1/2 from a0..a4 = f_{j-2..j+2} (Table 2 scheme 2),
// substencil r (nodes j-2+r .. j+r) given weight zero when v_r is false
// (it would reach outside a non-periodic domain, Sec. 2.2.4) and the other
// nonlinear weights renormalised.  Masked inputs must be finite.
template <typename R>
__device__ __forceinline__ R weno5m(R a0, R a1, R a2, R a3, R a4, R eps, bool v0, bool v1, bool v2) {
  const R q0 = ((R)2 * a0 - (R)7 * a1 + (R)11 * a2) * (R)(1.0 / 6.0);
  const R q1 = (-a1 + (R)5 * a2 + (R)2 * a3) * (R)(1.0 / 6.0);
  const R q2 = ((R)2 * a2 + (R)5 * a3 - a4) * (R)(1.0 / 6.0);
  const R c13 = (R)(13.0 / 12.0), c14 = (R)0.25;
  const R s0 = a0 - (R)2 * a1 + a2, t0 = a0 - (R)4 * a1 + (R)3 * a2;
  const R s1 = a1 - (R)2 * a2 + a3, t1 = a1 - a3;
  const R s2 = a2 - (R)2 * a3 + a4, t2 = (R)3 * a2 - (R)4 * a3 + a4;
  R e0 = eps + (c13 * s0 * s0 + c14 * t0 * t0);
  R e1 = eps + (c13 * s1 * s1 + c14 * t1 * t1);
  R e2 = eps + (c13 * s2 * s2 + c14 * t2 * t2);
  const R w0 = v0 ? (R)0.1 / (e0 * e0) : (R)0;
  const R w1 = v1 ? (R)0.6 / (e1 * e1) : (R)0;
  const R w2 = v2 ? (R)0.3 / (e2 * e2) : (R)0;
  return (w0 * q0 + w1 * q1 + w2 * q2) / (w0 + w1 + w2);
}

// Characteristic variables of one interface (Sec. 2.2.2, eq 31-40).  The
// interface state is the mean of the conserved variables of the two nodes
// (eq 32); the normal n is the unit vector of the mean of their metric rows of
// the sweep direction; l and m complete the frame as eq 39-40 choose them.
// The products with S (eq 35) and S^-1 (eq 34) are regrouped around the terms
// their rows share:
//   a = V f0 - u.f + f4,  b = u_n f0 - n.f      (f = (f1, f2, f3))
//   S f = (f0 - kappa a, l.f - u_l f0, m.f - u_m f0, kappa1 a + chi b, kappa1 a - chi b)
// and with s = g3 + g4, d = c (g4 - g3):
//   S^-1 g = (g0 + s, u_i (g0 + s) + l_i g1 + m_i g2 + n_i d, V g0 + u_l g1 + u_m g2 + H s + u_n d).
// The state, frame and coefficients are formed in FP64 and held in R.
template <typename R>
struct CharFrame {
  R u[3], n[3], l[3], m[3];
  R V, H, un, ul, um, c, kap, kap1, chi;

  __device__ __forceinline__ void init(const Phys& ph, const double* Ua, const double* a) {
    const double ir = rcp_r<double>(Ua[0]);
    const double vu = Ua[1] * ir, vv = Ua[2] * ir, vw = Ua[3] * ir;
    const double Vd = 0.5 * (vu * vu + vv * vv + vw * vw);               // eq 25
    const double p = ph.gm1 * (Ua[4] - Ua[0] * Vd);
    const double c2 = ph.gamma * p * ir;
    const double cd = sqrt(c2);
    const double is = rcp_r<double>(sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]));
    const double n0 = a[0] * is, n1 = a[1] * is, n2 = a[2] * is;
    double l0, l1, l2;
    if (fabs(n2) <= fabs(n1)) {                                          // eq 39
      const double r = rcp_r<double>(sqrt(n0 * n0 + n1 * n1));
      l0 = -n1 * r; l1 = n0 * r; l2 = 0.0;
    } else {
      const double r = rcp_r<double>(sqrt(n0 * n0 + n2 * n2));
      l0 = -n2 * r; l1 = 0.0; l2 = n0 * r;
    }
    const double m0 = n1 * l2 - n2 * l1, m1 = n2 * l0 - n0 * l2, m2 = n0 * l1 - n1 * l0;   // eq 40
    const double kd = ph.gm1 * rcp_r<double>(c2);                        // eq 37
    u[0] = (R)vu; u[1] = (R)vv; u[2] = (R)vw;
    n[0] = (R)n0; n[1] = (R)n1; n[2] = (R)n2;
    l[0] = (R)l0; l[1] = (R)l1; l[2] = (R)l2;
    m[0] = (R)m0; m[1] = (R)m1; m[2] = (R)m2;
    V = (R)Vd;
    H = (R)(Vd + c2 * ph.inv_gm1);                                      // eq 36
    un = (R)(vu * n0 + vv * n1 + vw * n2);                              // eq 38
    ul = (R)(vu * l0 + vv * l1 + vw * l2);
    um = (R)(vu * m0 + vv * m1 + vw * m2);
    c = (R)cd;
    kap = (R)kd;
    kap1 = (R)(0.5 * kd);
    chi = (R)(0.5 * rcp_r<double>(cd));
  }
  // w = S f
  __device__ __forceinline__ void to_char(const R* f, R* w) const {
    const R uf = u[0] * f[1] + u[1] * f[2] + u[2] * f[3];
    const R a = V * f[0] - uf + f[4];
    const R b = un * f[0] - (n[0] * f[1] + n[1] * f[2] + n[2] * f[3]);
    w[0] = f[0] - kap * a;
    w[1] = (l[0] * f[1] + l[1] * f[2] + l[2] * f[3]) - ul * f[0];
    w[2] = (m[0] * f[1] + m[1] * f[2] + m[2] * f[3]) - um * f[0];
    w[3] = kap1 * a + chi * b;
    w[4] = kap1 * a - chi * b;
  }
  // F = S^-1 g
  __device__ __forceinline__ void from_char(const R* g, R* F) const {
    const R s = g[3] + g[4];
    const R d = c * (g[4] - g[3]);
    const R gs = g[0] + s;
    F[0] = gs;
#pragma unroll
    for (int i = 0; i < 3; ++i) F[1 + i] = u[i] * gs + l[i] * g[1] + m[i] * g[2] + n[i] * d;
    F[4] = V * g[0] + ul * g[1] + um * g[2] + H * s + un * d;
  }
};

// First derivative (times h) at node position pos of a line of n nodes from
// values val(m) = f_{pos+m}.  Periodic lines and interior nodes use the central
// operator of half width maxhalf; toward a non-periodic end the order drops as
// Sec. 2.3 describes: one-sided second order at the end node, then central of
// half width 1, 2, 3 at the next nodes.
template <class F>
__device__ __forceinline__ double line_deriv(F val, int pos, int n, bool periodic, int maxhalf) {
  int half = maxhalf;
  if (!periodic) {
    const int dist = pos < n - 1 - pos ? pos : n - 1 - pos;
    if (dist == 0)
      return pos == 0 ? 0.5 * (-3.0 * val(0) + 4.0 * val(1) - val(2)) : 0.5 * (3.0 * val(0) - 4.0 * val(-1) + val(-2));
    if (dist < half) half = dist;
  }
  if (half == 1) return 0.5 * (val(1) - val(-1));
  if (half == 2) return (2.0 / 3.0) * (val(1) - val(-1)) - (1.0 / 12.0) * (val(2) - val(-2));
  if (half == 3)
    return 0.75 * (val(1) - val(-1)) - 0.15 * (val(2) - val(-2)) + (1.0 / 60.0) * (val(3) - val(-3));
  return 0.8 * (val(1) - val(-1)) - 0.2 * (val(2) - val(-2)) + (4.0 / 105.0) * (val(3) - val(-3)) -
         (1.0 / 280.0) * (val(4) - val(-4));
}

}  // namespace ocfd
