// HIP kernels (gfx950) of the ocfd library: one Runge-Kutta substep of the
// curvilinear compressible Navier-Stokes solver of Dang et al.,
// arXiv:2209.15333, Section 2.
//
// Data layout: structure-of-arrays, field-major, x fastest (see ocfd.h).
// Every kernel keeps FP64 arithmetic.
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
template <>
__device__ __forceinline__ double rcp_r<double>(double x) { return 1.0 / x; }
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
  // candidate values at j+1/2 relative to a3 = f_j
  const R q0 = (R)0.5 * D0 + (R)(4.0 / 3.0) * E0 + (R)(13.0 / 12.0) * G0;
  const R q1 = (R)0.5 * D1 + (R)(5.0 / 6.0) * E1 + (R)0.25 * G1;
  const R q2 = (R)0.5 * D2 + (R)(1.0 / 3.0) * E2 - (R)(1.0 / 12.0) * G2;
  const R q3 = (R)0.5 * D3 - (R)(1.0 / 6.0) * E3 + (R)(1.0 / 12.0) * G3;
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
  return a3 + (w0 * q0 + w1 * q1 + w2 * q2 + w3 * q3) / (w0 + w1 + w2 + w3);
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

// ---------------------------------------------------------------------------
// Directional sweep
// ---------------------------------------------------------------------------
//
// A workgroup owns SW_W neighbouring grid lines along direction DIR and
// marches along them in chunks of SW_S nodes.  Per chunk:
//   1. each thread loads one node, recovers the primitives and splits the
//      flux (eq 19-30) into an LDS ring of split fluxes (node m -> slot m%32);
//   2. each thread reconstructs one interface j+1/2 (WENO7, or the hybrid's
//      low-dissipation stencil) from the ring;
//   3. each thread forms one node's flux difference (F(j+1/2) - F(j-1/2))/h,
//      adds the sixth-order derivative of the viscous flux of this direction
//      and applies the mode (store, accumulate, Runge-Kutta update, dU/dt).
// The flux of the chunk's last interface is carried to the next chunk, so
// every interface is reconstructed exactly once, and the first node of a
// periodic line is finished after the last chunk with the wrapped flux.
// Lines are periodic (the wrap of node positions happens at load time).

constexpr int SW_W = 16;
constexpr int SW_S = 16;
constexpr int SW_T = SW_W * SW_S;
constexpr int RING = 32;

template <int DIR, int MODE, bool HYB, typename R>
__global__ __launch_bounds__(SW_T) void k_sweep(const SweepArgs A) {
  constexpr int CD = (DIR == 0) ? 1 : 0;  // direction across the lines of the group
  constexpr int OD = (DIR == 2) ? 1 : 2;  // remaining direction
  constexpr int NVAL = HYB ? 11 : 10;     // f+ (5), f- (5), node sensor
  constexpr int SLOT = NVAL * SW_W + 1;   // padded against bank conflicts
  constexpr int FHS = 5 * SW_W + 1;
  __shared__ R ring[RING * SLOT];
  __shared__ double fh[(SW_S + 1) * FHS];  // fh[0]: carried flux; fh[s+1]: interface j0+s
  __shared__ double fh0[FHS];             // flux at 1/2, for node 0 of a periodic line
  __shared__ int wl_n;                    // hybrid: WENO work list of this chunk
  __shared__ short wl[SW_T];

  const int n = A.g.n[DIR];
  const int ncol = A.g.n[CD];
  const long long sd = A.g.s[DIR];
  const long long sc = A.g.s[CD];
  const long long N = A.g.N;
  const int col0 = blockIdx.x * SW_W;
  const long long base = (long long)blockIdx.y * A.g.s[OD] + (long long)col0 * sc;
  const int t = threadIdx.x;
  // Global-facing mapping: consecutive threads walk the contiguous index.
  const int gs = (DIR == 0) ? (t & (SW_S - 1)) : (t / SW_W);
  const int gc = (DIR == 0) ? (t / SW_S) : (t & (SW_W - 1));
  // LDS-facing mapping for the reconstruction: lines fastest.
  const int rs = t / SW_W;
  const int rc = t & (SW_W - 1);
  const bool gcol_ok = col0 + gc < ncol;
  const bool rcol_ok = col0 + rc < ncol;
  const double ih = A.ph.ih[DIR];
  const R eps = (R)A.ph.eps;
  const bool per = A.g.periodic[DIR] != 0;

  // Raw inputs of one node: conserved variables, row DIR of the metrics / J,
  // node sensor.  Fetched one chunk ahead so the loads overlap the
  // reconstruction of the current chunk.
  struct NodeIn {
    double U[5];
    double a[3];
    double th;
  };
  auto fetch = [&](int m, int col) {
    NodeIn r;
    const int jm = !per ? m : (n >= 8 ? wrap1(m, n) : wrap(m, n));
    const long long id = base + (long long)col * sc + (long long)jm * sd;
#pragma unroll
    for (int q = 0; q < 5; ++q) r.U[q] = A.U[q * N + id];
#pragma unroll
    for (int q = 0; q < 3; ++q) r.a[q] = A.met[(3 * DIR + q) * N + id];
    r.th = (HYB && A.theta) ? A.theta[id] : 0.0;
    return r;
  };
  // Primitive recovery and Steger-Warming split of node m into the ring.
  auto split_store = [&](int m, int col, const NodeIn& in) {
    const double rho = in.U[0];
    const double ir = 1.0 / rho;
    const double u = in.U[1] * ir;
    const double v = in.U[2] * ir;
    const double w = in.U[3] * ir;
    const double p = A.ph.gm1 * (in.U[4] - 0.5 * rho * (u * u + v * v + w * w));
    R fp[5], fm[5];
    sw_split<R>(A.ph, (R)rho, (R)ir, (R)u, (R)v, (R)w, (R)p, (R)in.a[0], (R)in.a[1], (R)in.a[2], fp, fm);
    R* slot = ring + (m & (RING - 1)) * SLOT + col;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      slot[q * SW_W] = fp[q];
      slot[(5 + q) * SW_W] = fm[q];
    }
    if (HYB) slot[10 * SW_W] = (R)in.th;
  };

  // Output of node j of line col from its two interface fluxes (inv: this
  // node has both interfaces along DIR, i.e. it is not an end of a
  // non-periodic line).
  auto emit = [&](int j, int col, const double* Fr, const double* Fl, bool inv) {
    const long long id = base + (long long)col * sc + (long long)j * sd;
    double r[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) r[q] = (A.inviscid && inv) ? -(Fr[q * SW_W] - Fl[q * SW_W]) * ih : 0.0;
    if (A.viscous) {
      if (per) {
        // offsets of the six neighbours along the line (wrapped at the seam)
        auto off = [&](int k) {
          const int p = j + k;
          return (long long)((n >= 8 ? wrap1(p, n) : wrap(p, n)) - j) * sd;
        };
        const long long o1p = off(1), o1m = off(-1), o2p = off(2), o2m = off(-2), o3p = off(3), o3m = off(-3);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double* F = A.Fv + (long long)(4 * DIR + q) * N + id;
          const double d = 0.75 * (F[o1p] - F[o1m]) - 0.15 * (F[o2p] - F[o2m]) + (1.0 / 60.0) * (F[o3p] - F[o3m]);
          r[q + 1] += d * ih;
        }
      } else if (inv) {
        // sixth order inside, then fourth and second order toward the ends (Sec. 2.3)
        const int dist = min(j, n - 1 - j);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double* F = A.Fv + (long long)(4 * DIR + q) * N + id;
          double d;
          if (dist == 1)
            d = 0.5 * (F[sd] - F[-sd]);
          else if (dist == 2)
            d = (2.0 / 3.0) * (F[sd] - F[-sd]) - (1.0 / 12.0) * (F[2 * sd] - F[-2 * sd]);
          else
            d = 0.75 * (F[sd] - F[-sd]) - 0.15 * (F[2 * sd] - F[-2 * sd]) + (1.0 / 60.0) * (F[3 * sd] - F[-3 * sd]);
          r[q + 1] += d * ih;
        }
      }
    }
    if (MODE == MODE_SET) {
#pragma unroll
      for (int q = 0; q < 5; ++q) A.rhs[q * N + id] = r[q];
    } else if (MODE == MODE_ADD) {
#pragma unroll
      for (int q = 0; q < 5; ++q) A.rhs[q * N + id] += r[q];
    } else {
      // nodes on a face of a non-periodic direction take dU/dt = 0 (their
      // value is set by the boundary condition after the stage)
      bool bnd = false;
      if (!A.g.periodic[0] || !A.g.periodic[1] || !A.g.periodic[2]) {
        const int p0 = (int)(id % A.g.n[0]), p1 = (int)((id / A.g.n[0]) % A.g.n[1]),
                  p2 = (int)(id / ((long long)A.g.n[0] * A.g.n[1]));
        bnd = (!A.g.periodic[0] && (p0 == 0 || p0 == A.g.n[0] - 1)) ||
              (!A.g.periodic[1] && (p1 == 0 || p1 == A.g.n[1] - 1)) ||
              (!A.g.periodic[2] && (p2 == 0 || p2 == A.g.n[2] - 1));
      }
      const double ij = 1.0 / A.met[9 * N + id];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const double L = bnd ? 0.0 : (A.rhs[q * N + id] + r[q]) * ij;
        if (MODE == MODE_RK)
          A.out[q * N + id] = A.a * A.Un[q * N + id] + A.b * (A.U[q * N + id] + A.dt * L);
        else
          A.out[q * N + id] = L;
      }
    }
  };

  const int nchunks = (n + SW_S - 1) / SW_S;
  // Chunk c reconstructs interfaces JB + 16c + s (s = 0..15) and loads nodes
  // JB + 16c + 4 .. JB + 16c + 19.  Periodic lines: JB = -4, so every load
  // window starts on a 16-node (128-byte) boundary, n interfaces.  Non-periodic
  // lines: JB = 0, interfaces 0 .. n-2, nodes outside [0, n-1] never loaded.
  const int JB = per ? -4 : 0;
  const int nif = per ? n : n - 1;          // interfaces of the line
  const int mmax = n - 1;                   // last node the chunks load (the prologue covers JB-3 .. JB+3)
  // Prologue: nodes JB-3 .. JB+3 of every line.
  if (A.inviscid && t < 7 * SW_W) {
    const int pm = (DIR == 0) ? (t % 7) : (t / SW_W);
    const int pc = (DIR == 0) ? (t / 7) : (t % SW_W);
    const int m = JB + pm - 3;
    if (col0 + pc < ncol && (per || (m >= 0 && m < n))) split_store(m, pc, fetch(m, pc));
  }
  NodeIn ahead;
  bool have = A.inviscid && gcol_ok && JB + 4 + gs <= mmax;
  if (have) ahead = fetch(JB + 4 + gs, gc);
  // Reconstruction of interface j of line col into dst (WENO7 or low-dissipation stencil).
  auto reconstruct = [&](int j, int col, bool low, double* dst) {
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const R* P = ring + col + q * SW_W;
      const R* M = ring + col + (5 + q) * SW_W;
#define RP(o) P[((j + (o)) & (RING - 1)) * SLOT]
#define RM(o) M[((j + (o)) & (RING - 1)) * SLOT]
      double F;
      if (!per && (j < 3 || j > n - 5)) {
        // stencil leaves the domain: masked WENO5 (out-of-domain values
        // replaced by the centre value so the masked terms stay finite)
        auto fp = [&](int o) { const int m = j + o; return (m >= 0 && m < n) ? RP(o) : RP(0); };
        auto fm = [&](int o) { const int m = j + o; return (m >= 0 && m < n) ? RM(o) : RM(1); };
        auto in = [&](int o) { const int m = j + o; return m >= 0 && m < n; };
        // f+: substencils j-2..j, j-1..j+1, j..j+2; f- (mirrored): j+3..j+1, j+2..j, j+1..j-1
        F = (double)weno5m<R>(fp(-2), fp(-1), fp(0), fp(1), fp(2), eps, in(-2), in(-1), in(2)) +
            (double)weno5m<R>(fm(3), fm(2), fm(1), fm(0), fm(-1), eps, in(3), in(2), in(-1));
      } else if (HYB && low) {
        if (A.lowdiss == OCFD_LOWDISS_C8)
          F = (double)c8<R>(RP(-3) + RM(-3), RP(-2) + RM(-2), RP(-1) + RM(-1), RP(0) + RM(0), RP(1) + RM(1),
                            RP(2) + RM(2), RP(3) + RM(3), RP(4) + RM(4));
        else
          F = (double)ud7<R>(RP(-3), RP(-2), RP(-1), RP(0), RP(1), RP(2), RP(3)) +
              (double)ud7<R>(RM(4), RM(3), RM(2), RM(1), RM(0), RM(-1), RM(-2));
      } else {
        F = (double)weno7<R>(RP(-3), RP(-2), RP(-1), RP(0), RP(1), RP(2), RP(3), eps) +
            (double)weno7<R>(RM(4), RM(3), RM(2), RM(1), RM(0), RM(-1), RM(-2), eps);
      }
#undef RP
#undef RM
      dst[q * SW_W] = F;
    }
  };

  for (int c = 0; c < nchunks; ++c) {
    const int j0 = JB + c * SW_S;
    if (have) split_store(j0 + 4 + gs, gc, ahead);
    if (HYB && t == 0) wl_n = 0;
    __syncthreads();
    have = A.inviscid && gcol_ok && c + 1 < nchunks && j0 + SW_S + 4 + gs <= mmax;
    if (have) ahead = fetch(j0 + SW_S + 4 + gs, gc);
    const int j = j0 + rs;
    const bool act = A.inviscid && rcol_ok && c * SW_S + rs < nif;
    if (HYB) {
      // Low-dissipation interfaces are done in place; WENO interfaces go to a
      // work list so that whole waves run the WENO code (no divergence).
      if (act) {
        bool low;
        if (!per && (j < 3 || j > n - 5)) {
          low = false;   // boundary closure: always the WENO5 path
        } else if (A.flags) {
          low = A.flags[DIR * N + base + (long long)rc * sc + (long long)(n >= 8 ? wrap1(j, n) : wrap(j, n)) * sd] == 0;
        } else {
          R mx = (R)0;
#pragma unroll
          for (int o = -3; o <= 4; ++o) mx = fmax(mx, ring[((j + o) & (RING - 1)) * SLOT + 10 * SW_W + rc]);
          low = mx <= (R)A.ph.theta1;
        }
        if (low)
          reconstruct(j, rc, true, fh + (rs + 1) * FHS + rc);
        else
          wl[atomicAdd(&wl_n, 1)] = (short)t;
      }
      __syncthreads();
      if (t < wl_n) {
        const int tt = wl[t];
        const int s2 = tt / SW_W, c2 = tt & (SW_W - 1);
        reconstruct(j0 + s2, c2, false, fh + (s2 + 1) * FHS + c2);
      }
    } else if (act) {
      reconstruct(j, rc, false, fh + (rs + 1) * FHS + rc);
    }
    __syncthreads();
    if (c == 0 && t < 5 * SW_W) fh0[(t / SW_W) * SW_W + (t % SW_W)] = fh[FHS + (t / SW_W) * SW_W + (t % SW_W)];
    if (per) {
      if (gcol_ok && c * SW_S + gs < n && (c > 0 || gs > 0))
        emit(n >= 8 ? wrap1(j0 + gs, n) : wrap(j0 + gs, n), gc, fh + (gs + 1) * FHS + gc, fh + gs * FHS + gc, true);
    } else {
      const int jn = j0 + gs;
      if (gcol_ok && jn < n) emit(jn, gc, fh + (gs + 1) * FHS + gc, fh + gs * FHS + gc, jn > 0 && jn < n - 1);
    }
    __syncthreads();
    if (t < 5 * SW_W) {
      const int last = min(SW_S, nif - c * SW_S);
      if (last > 0) fh[(t / SW_W) * SW_W + (t % SW_W)] = fh[last * FHS + (t / SW_W) * SW_W + (t % SW_W)];
    }
  }
  __syncthreads();
  // The periodic line's first node (JB) with the wrapped flux carried out of the last chunk.
  if (per && gs == 0 && gcol_ok) emit(wrap(JB, n), gc, fh0 + gc, fh + gc, true);
}

template <int DIR, int MODE>
static hipError_t launch_sweep_t(const SweepArgs& a, hipStream_t st) {
  constexpr int CD = (DIR == 0) ? 1 : 0;
  constexpr int OD = (DIR == 2) ? 1 : 2;
  dim3 grid((a.g.n[CD] + SW_W - 1) / SW_W, a.g.n[OD]);
  if (a.mixed) {
    if (a.hybrid)
      hipLaunchKernelGGL((k_sweep<DIR, MODE, true, float>), grid, dim3(SW_T), 0, st, a);
    else
      hipLaunchKernelGGL((k_sweep<DIR, MODE, false, float>), grid, dim3(SW_T), 0, st, a);
  } else {
    if (a.hybrid)
      hipLaunchKernelGGL((k_sweep<DIR, MODE, true, double>), grid, dim3(SW_T), 0, st, a);
    else
      hipLaunchKernelGGL((k_sweep<DIR, MODE, false, double>), grid, dim3(SW_T), 0, st, a);
  }
  return hipGetLastError();
}

template <int DIR>
static hipError_t launch_sweep_d(int mode, const SweepArgs& a, hipStream_t st) {
  switch (mode) {
    case MODE_SET: return launch_sweep_t<DIR, MODE_SET>(a, st);
    case MODE_ADD: return launch_sweep_t<DIR, MODE_ADD>(a, st);
    case MODE_RK: return launch_sweep_t<DIR, MODE_RK>(a, st);
    default: return launch_sweep_t<DIR, MODE_DUDT>(a, st);
  }
}

hipError_t launch_sweep(int dir, int mode, const SweepArgs& a, hipStream_t st) {
  if (dir == 0) return launch_sweep_d<0>(mode, a, st);
  if (dir == 1) return launch_sweep_d<1>(mode, a, st);
  return launch_sweep_d<2>(mode, a, st);
}

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

// ---------------------------------------------------------------------------
// Primitive variables and viscous fluxes (eq 9-16, Sec. 2.3)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_prim(const Geo g, const Phys ph, const double* __restrict__ U,
                                              double* __restrict__ W) {
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= g.N) return;
  const long long N = g.N;
  const double rho = U[id];
  const double ir = 1.0 / rho;
  const double u = U[N + id] * ir, v = U[2 * N + id] * ir, w = U[3 * N + id] * ir;
  const double p = ph.gm1 * (U[4 * N + id] - 0.5 * rho * (u * u + v * v + w * w));
  W[id] = u;
  W[N + id] = v;
  W[2 * N + id] = w;
  W[3 * N + id] = ph.gamma * ph.Ma2 * p * ir;  // T = gamma Ma^2 p / rho (eq 16-17)
}

hipError_t launch_prim(const Geo& g, const Phys& ph, const double* U, double* W, hipStream_t st) {
  hipLaunchKernelGGL(k_prim, dim3((unsigned)((g.N + 255) / 256)), dim3(256), 0, st, g, ph, U, W);
  return hipGetLastError();
}

// Viscous flux vectors of the three directions at every node: derivatives of
// u, v, w, T along xi, eta, zeta; Cartesian gradients by the chain rule with
// the node metrics; Sutherland viscosity (eq 15), heat conductivity (eq 14),
// stresses (eq 13) and stress work plus heat flux (eq 12); the flux of
// direction d is (row d of the metrics / J) applied to tau and Theta (eq 9-11).
// Output Fv[4*d + q][N], q = momentum x, y, z, energy.
//
// A workgroup owns a 64 x 4 tile of (xi, eta) columns and marches along zeta
// through one segment of planes, keeping each column's seven-plane window of
// u, v, w, T in registers, so every plane is read from memory once per
// segment.  Neighbours along xi and eta are read directly (they sit in the
// same or adjacent rows of the plane).  Tiles are numbered so that the eight
// XCDs each receive a contiguous range (round-robin dispatch), which keeps a
// whole segment of neighbouring tiles on one L2.
constexpr int VT_X = 64;
constexpr int VT_Y = 4;

__global__ __launch_bounds__(256, 3) void k_visc_flux(const Geo g, const Phys ph, const double* __restrict__ W,
                                                   const double* __restrict__ met, double* __restrict__ Fv,
                                                   int ntx, int nty, int nseg, int zseg) {
  const int per = gridDim.x / 8;
  const int L = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (L >= ntx * nty * nseg) return;
  const int tx = L % ntx, ty = (L / ntx) % nty, zs = L / (ntx * nty);
  const int i = tx * VT_X + (threadIdx.x & (VT_X - 1));
  const int j = ty * VT_Y + threadIdx.x / VT_X;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  if (i >= nx || j >= ny) return;
  const int k0 = zs * zseg;
  const int k1 = min(nz, k0 + zseg);
  const long long N = g.N;
  const long long sz = g.s[2];
  const long long colid = i + (long long)nx * j;
  const bool px = g.periodic[0], py = g.periodic[1], pz = g.periodic[2];
  // plane index of k (wrapped when zeta is periodic, clamped otherwise: the
  // clamped planes are loaded but never used by the boundary closure)
  auto zi = [&](int k) { return pz ? wrap(k, nz) : min(max(k, 0), nz - 1); };
  double zw[4][7];
#pragma unroll
  for (int o = -3; o <= 2; ++o) {
    const long long id = colid + (long long)zi(k0 + o) * sz;
#pragma unroll
    for (int q = 0; q < 4; ++q) zw[q][o + 3] = W[q * N + id];
  }
  // neighbour offsets along xi and eta (periodic lines; a non-periodic line
  // uses the closure of line_deriv with direct offsets)
  const long long xp1 = wrap(i + 1, nx) - i, xm1 = wrap(i - 1, nx) - i;
  const long long xp2 = wrap(i + 2, nx) - i, xm2 = wrap(i - 2, nx) - i;
  const long long xp3 = wrap(i + 3, nx) - i, xm3 = wrap(i - 3, nx) - i;
  const long long yp1 = (long long)(wrap(j + 1, ny) - j) * nx, ym1 = (long long)(wrap(j - 1, ny) - j) * nx;
  const long long yp2 = (long long)(wrap(j + 2, ny) - j) * nx, ym2 = (long long)(wrap(j - 2, ny) - j) * nx;
  const long long yp3 = (long long)(wrap(j + 3, ny) - j) * nx, ym3 = (long long)(wrap(j - 3, ny) - j) * nx;
  for (int k = k0; k < k1; ++k) {
    const long long idn = colid + (long long)zi(k + 3) * sz;
#pragma unroll
    for (int q = 0; q < 4; ++q) zw[q][6] = W[q * N + idn];
    const long long id = colid + (long long)k * sz;
    double dq[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double* f = W + q * N + id;
      if (px)
        dq[q][0] = (0.75 * (f[xp1] - f[xm1]) - 0.15 * (f[xp2] - f[xm2]) + (1.0 / 60.0) * (f[xp3] - f[xm3])) * ph.ih[0];
      else
        dq[q][0] = line_deriv([&](int m) { return f[m]; }, i, nx, false, 3) * ph.ih[0];
      if (py)
        dq[q][1] = (0.75 * (f[yp1] - f[ym1]) - 0.15 * (f[yp2] - f[ym2]) + (1.0 / 60.0) * (f[yp3] - f[ym3])) * ph.ih[1];
      else
        dq[q][1] = line_deriv([&](int m) { return f[(long long)m * nx]; }, j, ny, false, 3) * ph.ih[1];
      if (pz)
        dq[q][2] = (0.75 * (zw[q][4] - zw[q][2]) - 0.15 * (zw[q][5] - zw[q][1]) + (1.0 / 60.0) * (zw[q][6] - zw[q][0])) *
                   ph.ih[2];
      else
        dq[q][2] = line_deriv([&](int m) { return zw[q][3 + m]; }, k, nz, false, 3) * ph.ih[2];
    }
    const double ij = 1.0 / met[9 * N + id];
    double m[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) m[r] = met[r * N + id];
    double gr[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        gr[q][c] = (m[c] * ij) * dq[q][0] + (m[3 + c] * ij) * dq[q][1] + (m[6 + c] * ij) * dq[q][2];
    const double T = zw[3][3];
    const double mu = T * sqrt(T) * (1.0 + ph.suth) / (T + ph.suth);
    const double kc = mu * ph.kcoef;
    const double mr = mu * ph.inv_Re;
    const double div = gr[0][0] + gr[1][1] + gr[2][2];
    double tau[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) tau[a][b] = mr * (gr[a][b] + gr[b][a] - (a == b ? (2.0 / 3.0) * div : 0.0));
    const double u = zw[0][3], v = zw[1][3], w = zw[2][3];
    double th[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) th[a] = u * tau[0][a] + v * tau[1][a] + w * tau[2][a] + kc * gr[3][a];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double m0 = m[3 * d], m1 = m[3 * d + 1], m2 = m[3 * d + 2];
#pragma unroll
      for (int b = 0; b < 3; ++b) Fv[(4 * d + b) * N + id] = m0 * tau[0][b] + m1 * tau[1][b] + m2 * tau[2][b];
      Fv[(4 * d + 3) * N + id] = m0 * th[0] + m1 * th[1] + m2 * th[2];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int o = 0; o < 6; ++o) zw[q][o] = zw[q][o + 1];
  }
}

hipError_t launch_visc_flux(const Geo& g, const Phys& ph, const double* W, const double* met, double* Fv,
                            hipStream_t st) {
  const int ntx = (g.n[0] + VT_X - 1) / VT_X;
  const int nty = (g.n[1] + VT_Y - 1) / VT_Y;
  // Enough segments along zeta for ~2048 workgroups.
  int nseg = (2048 + ntx * nty - 1) / (ntx * nty);
  nseg = nseg < 1 ? 1 : (nseg > g.n[2] ? g.n[2] : nseg);
  const int zseg = (g.n[2] + nseg - 1) / nseg;
  nseg = (g.n[2] + zseg - 1) / zseg;
  const long long tiles = (long long)ntx * nty * nseg;
  const unsigned nb = (unsigned)(8 * ((tiles + 7) / 8));
  hipLaunchKernelGGL(k_visc_flux, dim3(nb), dim3(256), 0, st, g, ph, W, met, Fv, ntx, nty, nseg, zseg);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Boundary conditions of a face of a bounded direction.  The paper names the
// kinds (inflow, extrapolated outflow and far field, isothermal no-slip wall)
// without formulas; the readings: INFLOW imposes the stored state, EXTRAP
// copies rho, velocity and p from the first interior node, WALL sets zero
// velocity, T = Tw and p from the first interior node (rho = gamma Ma^2 p / Tw,
// eq 16-17).  One thread per face node; the face is indexed by its two other
// node indices, the lower direction fastest.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_bc(const Geo g, const Phys ph, double* __restrict__ U, int d, int side,
                                            int kind, double Tw, const double* __restrict__ inflow) {
  const int e0 = d == 0 ? 1 : 0, e1 = d == 2 ? 1 : 2;
  const long long nf = (long long)g.n[e0] * g.n[e1];
  const long long f = (long long)blockIdx.x * 256 + threadIdx.x;
  if (f >= nf) return;
  int c[3];
  c[e0] = (int)(f % g.n[e0]);
  c[e1] = (int)(f / g.n[e0]);
  c[d] = side ? g.n[d] - 1 : 0;
  const long long N = g.N;
  const long long id = c[0] + g.s[1] * c[1] + g.s[2] * c[2];
  double o[5];
  if (kind == OCFD_BC_INFLOW) {
#pragma unroll
    for (int q = 0; q < 5; ++q) o[q] = inflow[q * nf + f];
  } else {
    const long long ii = id + (side ? -g.s[d] : g.s[d]);
    const double rho = U[ii];
    const double u = U[N + ii] / rho, v = U[2 * N + ii] / rho, w = U[3 * N + ii] / rho;
    const double ke = 0.5 * rho * (u * u + v * v + w * w);
    const double p = ph.gm1 * (U[4 * N + ii] - ke);
    if (kind == OCFD_BC_WALL) {
      o[0] = ph.gamma * ph.Ma2 * p / Tw;
      o[1] = o[2] = o[3] = 0.0;
      o[4] = p / ph.gm1;
    } else {
      o[0] = rho;
      o[1] = rho * u;
      o[2] = rho * v;
      o[3] = rho * w;
      o[4] = p / ph.gm1 + ke;
    }
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) U[q * N + id] = o[q];
}

hipError_t launch_bc(const Geo& g, const Phys& ph, double* U, int d, int side, int kind, double Tw,
                     const double* inflow, hipStream_t st) {
  const long long nf = (long long)g.n[d == 0 ? 1 : 0] * g.n[d == 2 ? 1 : 2];
  hipLaunchKernelGGL(k_bc, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, st, g, ph, U, d, side, kind, Tw,
                     inflow);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Shock sensor (eq 42-43): theta = sum_d |-p_- + 2p - p_+| / (p_- + 2p + p_+)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double node_p(const Phys& ph, const double* U, long long N, long long id) {
  const double rho = U[id];
  const double u = U[N + id] / rho, v = U[2 * N + id] / rho, w = U[3 * N + id] / rho;
  return ph.gm1 * (U[4 * N + id] - 0.5 * rho * (u * u + v * v + w * w));
}

__global__ __launch_bounds__(256) void k_sensor(const Geo g, const Phys ph, const double* __restrict__ U,
                                                double* __restrict__ theta) {
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= g.N) return;
  const int i = (int)(id % g.n[0]);
  const int j = (int)((id / g.n[0]) % g.n[1]);
  const int k = (int)(id / ((long long)g.n[0] * g.n[1]));
  const int pos[3] = {i, j, k};
  const double p0 = node_p(ph, U, g.N, id);
  double th = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    // a node at the end of a non-periodic line has no second difference there
    if (!g.periodic[d] && (pos[d] == 0 || pos[d] == g.n[d] - 1)) continue;
    const long long im = id + (long long)(wrap(pos[d] - 1, g.n[d]) - pos[d]) * g.s[d];
    const long long ip = id + (long long)(wrap(pos[d] + 1, g.n[d]) - pos[d]) * g.s[d];
    const double pm = node_p(ph, U, g.N, im), pp = node_p(ph, U, g.N, ip);
    th += fabs(-pm + 2.0 * p0 - pp) / (pm + 2.0 * p0 + pp);
  }
  theta[id] = th;
}

hipError_t launch_sensor(const Geo& g, const Phys& ph, const double* U, double* theta, hipStream_t st) {
  hipLaunchKernelGGL(k_sensor, dim3((unsigned)((g.N + 255) / 256)), dim3(256), 0, st, g, ph, U, theta);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Metrics (eq 2-4) in the conservative form, eighth-order central operator
// ---------------------------------------------------------------------------

// Coordinate co at node pos + m along d (linear index id at pos), unwrapped
// across the seam of a periodic direction: coordinate d grows by period[d].
__device__ __forceinline__ double coord_at(const Geo& g, const Phys& ph, const double* xyz, int co, long long id,
                                           const int* pos, int d, int m) {
  const int p = pos[d] + m;
  const int w = g.periodic[d] ? wrap(p, g.n[d]) : p;
  double x = xyz[co * g.N + id + (long long)(w - pos[d]) * g.s[d]];
  if (co == d && g.periodic[d]) x += (double)((p - w) / g.n[d]) * ph.period[d];
  return x;
}

__global__ __launch_bounds__(256) void k_metric_inner(const Geo g, const Phys ph, const double* __restrict__ xyz,
                                                      double* __restrict__ inner) {
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= g.N) return;
  const int pos[3] = {(int)(id % g.n[0]), (int)((id / g.n[0]) % g.n[1]), (int)(id / ((long long)g.n[0] * g.n[1]))};
  for (int co = 0; co < 3; ++co)
    for (int d = 0; d < 3; ++d) {
      auto val = [&](int m) { return coord_at(g, ph, xyz, co, id, pos, d, m); };
      inner[(3 * co + d) * g.N + id] = line_deriv(val, pos[d], g.n[d], g.periodic[d], 4) * ph.ih[d];
    }
}

hipError_t launch_metric_inner(const Geo& g, const Phys& ph, const double* xyz, double* inner, hipStream_t st) {
  hipLaunchKernelGGL(k_metric_inner, dim3((unsigned)((g.N + 255) / 256)), dim3(256), 0, st, g, ph, xyz, inner);
  return hipGetLastError();
}

// Row r (xi, eta, zeta), column co (x, y, z):
//   (r_co)/J = D_t(a_s * b) - D_s(a_t * b)
// with (s, t) = (r+1, r+2) and (a, b) = (co+1, co+2) cyclic; for example
// xi_x/J = (y_eta z)_zeta - (y_zeta z)_eta.  The outer derivative uses the
// same eighth-order operator (with its boundary closure), and the coordinate
// b is unwrapped across a seam of the derivative direction.  1/J is the
// determinant of the inner derivatives (eq 4).
__global__ __launch_bounds__(256) void k_metric_outer(const Geo g, const Phys ph, const double* __restrict__ xyz,
                                                      const double* __restrict__ inner, double* __restrict__ met) {
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= g.N) return;
  const int pos[3] = {(int)(id % g.n[0]), (int)((id / g.n[0]) % g.n[1]), (int)(id / ((long long)g.n[0] * g.n[1]))};
  for (int r = 0; r < 3; ++r)
    for (int co = 0; co < 3; ++co) {
      const int s = (r + 1) % 3, t = (r + 2) % 3;
      const int a = (co + 1) % 3, b = (co + 2) % 3;
      double term[2];
      for (int pass = 0; pass < 2; ++pass) {
        const int dir = pass == 0 ? t : s;
        const int inn = pass == 0 ? s : t;
        const double* ia = inner + (3 * a + inn) * g.N;
        auto val = [&](int m) {
          const int p = pos[dir] + m;
          const int w = g.periodic[dir] ? wrap(p, g.n[dir]) : p;
          return ia[id + (long long)(w - pos[dir]) * g.s[dir]] * coord_at(g, ph, xyz, b, id, pos, dir, m);
        };
        term[pass] = line_deriv(val, pos[dir], g.n[dir], g.periodic[dir], 4) * ph.ih[dir];
      }
      met[(3 * r + co) * g.N + id] = term[0] - term[1];
    }
  double q[3][3];
  for (int co = 0; co < 3; ++co)
    for (int d = 0; d < 3; ++d) q[co][d] = inner[(3 * co + d) * g.N + id];
  met[9 * g.N + id] = q[0][0] * (q[1][1] * q[2][2] - q[1][2] * q[2][1]) -
                      q[0][1] * (q[1][0] * q[2][2] - q[1][2] * q[2][0]) +
                      q[0][2] * (q[1][0] * q[2][1] - q[1][1] * q[2][0]);
}

hipError_t launch_metric_outer(const Geo& g, const Phys& ph, const double* xyz, const double* inner, double* met,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_metric_outer, dim3((unsigned)((g.N + 255) / 256)), dim3(256), 0, st, g, ph, xyz, inner, met);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reductions: conserved totals, CFL, extrema, non-finite count
// ---------------------------------------------------------------------------

constexpr int RED_T = 256;
constexpr int RED_MAXB = 1024;
constexpr int NRED = OCFD_RED_COUNT;

int reduce_blocks(const Geo& g) {
  long long b = (g.N + RED_T * 16 - 1) / (RED_T * 16);
  if (b < 1) b = 1;
  if (b > RED_MAXB) b = RED_MAXB;
  return (int)b;
}

// Combine two partial records (sums add; CFL max; p, rho min; count add).
__device__ __forceinline__ void red_combine(double* a, const double* b) {
  for (int q = 0; q < 5; ++q) a[q] += b[q];
  a[5] = fmax(a[5], b[5]);
  a[6] = fmin(a[6], b[6]);
  a[7] = fmin(a[7], b[7]);
  a[8] += b[8];
}

__device__ void block_reduce(double (*sh)[RED_T], double* acc, double* out) {
  const int t = threadIdx.x;
  for (int q = 0; q < NRED; ++q) sh[q][t] = acc[q];
  __syncthreads();
  for (int w = RED_T / 2; w > 0; w >>= 1) {
    if (t < w) {
      double a[NRED], b[NRED];
      for (int q = 0; q < NRED; ++q) {
        a[q] = sh[q][t];
        b[q] = sh[q][t + w];
      }
      red_combine(a, b);
      for (int q = 0; q < NRED; ++q) sh[q][t] = a[q];
    }
    __syncthreads();
  }
  if (t < NRED) out[t] = sh[t][0];
}

__global__ __launch_bounds__(RED_T) void k_reduce_partial(const Geo g, const Phys ph, const double* __restrict__ U,
                                                          const double* __restrict__ met, double dt,
                                                          double* __restrict__ partial) {
  __shared__ double sh[NRED][RED_T];
  const long long N = g.N;
  double acc[NRED] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, INFINITY, INFINITY, 0.0};
  for (long long id = (long long)blockIdx.x * RED_T + threadIdx.x; id < N; id += (long long)gridDim.x * RED_T) {
    const double jinv = met[9 * N + id];
    double Uq[5];
    for (int q = 0; q < 5; ++q) {
      Uq[q] = U[q * N + id];
      acc[q] += Uq[q] * jinv;
      if (!isfinite(Uq[q])) acc[8] += 1.0;
    }
    const double rho = Uq[0];
    const double u = Uq[1] / rho, v = Uq[2] / rho, w = Uq[3] / rho;
    const double p = ph.gm1 * (Uq[4] - 0.5 * rho * (u * u + v * v + w * w));
    const double c = sqrt(ph.gamma * p / rho);
    double local = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double a0 = met[(3 * d) * N + id], a1 = met[(3 * d + 1) * N + id], a2 = met[(3 * d + 2) * N + id];
      const double sig = sqrt(a0 * a0 + a1 * a1 + a2 * a2) / jinv;
      const double V = (a0 * u + a1 * v + a2 * w) / jinv;
      local += (fabs(V) + c * sig) * ph.ih[d];
    }
    acc[5] = fmax(acc[5], local * dt);
    acc[6] = fmin(acc[6], p);
    acc[7] = fmin(acc[7], rho);
  }
  block_reduce(sh, acc, partial + (long long)blockIdx.x * NRED);
}

__global__ __launch_bounds__(RED_T) void k_reduce_final(const double* __restrict__ partial, int nb,
                                                        double* __restrict__ out) {
  __shared__ double sh[NRED][RED_T];
  double acc[NRED] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, INFINITY, INFINITY, 0.0};
  for (int b = threadIdx.x; b < nb; b += RED_T) red_combine(acc, partial + (long long)b * NRED);
  block_reduce(sh, acc, out);
}

hipError_t launch_reduce(const Geo& g, const Phys& ph, const double* U, const double* met, double dt,
                         double* partial, int nblocks, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partial, dim3(nblocks), dim3(RED_T), 0, st, g, ph, U, met, dt, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_T), 0, st, partial, nblocks, out);
  return hipGetLastError();
}

}  // namespace ocfd
