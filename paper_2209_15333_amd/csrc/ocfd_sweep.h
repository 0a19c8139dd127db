// Directional sweep kernel of the ocfd library (one Runge-Kutta substep of
// the curvilinear compressible Navier-Stokes solver of Dang et al.,
// arXiv:2209.15333, Section 2).  Included by one translation unit per
// direction and reconstruction variables, each instantiating launch_sweep_dc.
#pragma once

#include "ocfd_device.h"

namespace ocfd {

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
//      (FP32 and hybrid sweeps) adds the central derivative of the viscous
//      flux of this direction, and applies the mode (store, accumulate,
//      Runge-Kutta update, dU/dt).
// The flux of the chunk's last interface is carried to the next chunk, so
// every interface is reconstructed exactly once, and the first node of a
// periodic line is finished after the last chunk with the wrapped flux.
// BND selects the boundary code compiled in: 0 all three directions
// periodic; 1 this direction periodic, another bounded (faces of the other
// directions take dU/dt = 0 in the last sweep); 2 this direction bounded
// (masked WENO5 at interfaces whose stencil leaves the line, reduced-order
// viscous derivative toward the ends, no wrap).  Periodic lines wrap node
// positions at load time.  The hybrid scheme reads one flag byte per
// interface (0: low-dissipation stencil), computed beforehand by a sensor.
// CHR reconstructs the WENO interfaces in characteristic variables (Sec.
// 2.2.2): the split fluxes of the window are carried to the characteristic
// variables of the interface by S, reconstructed field by field and carried
// back by S^-1.  A linear stencil commutes with the fixed S, so the hybrid's
// low-dissipation interfaces skip the two products (an exact identity).

constexpr int SW_W = 16;
constexpr int SW_S = 16;
constexpr int SW_T = SW_W * SW_S;
constexpr int RING = 32;
// Ring slots of a kernel: the FP32 eta and zeta sweeps keep 24 (a chunk
// reads the 23 nodes j0 - 3 .. j0 + 19 and finishes with the viscous fluxes
// of j0 - 4 .. j0 + 19), which with their 24-slot viscous-flux ring brings a
// workgroup under 40 KB of LDS: four workgroups per CU instead of three,
// within 128 registers without spills.  On bounded lines that needs the
// loads of each chunk's nodes issued when they are split rather than one
// chunk ahead (with the prefetch they took 137 registers and spilled at
// 128), and holds for the first and summing sweeps only.  Measured on the
// developed 2048 x 256 x 256 ramp: zeta (periodic span) 6.06 -> 5.44 ms, eta
// (bounded) 6.01 -> 5.41 ms; eta and zeta at 256^3 2-4% faster.  The WENO7
// Runge-Kutta ones of periodic lines, and the Runge-Kutta and dU/dt ones of
// bounded lines, would spill too: they keep 32 slots and three workgroups.
template <int DIR, int MODE, bool HYB, typename R, int BND, bool CHR>
constexpr int ring_slots() {
  return (sizeof(R) == 4 && DIR != 0 && !CHR &&
          (BND != 2 ? (HYB || MODE != MODE_RK) : (MODE == MODE_SET || MODE == MODE_ADD))) ? 24 : RING;
}

// Occupancy floor: the FP64 characteristic kernels need it stated (two waves
// per SIMD on bounded lines, three otherwise), or the compiler may go past
// 256 registers and drop to one wave (measured: the bounded hybrid
// Runge-Kutta one did, 10% slower); the 24-slot sweeps ask for the four
// waves their LDS allows.
template <int DIR, int MODE, bool HYB, typename R, int BND, bool CHR>
__global__ __launch_bounds__(SW_T) __attribute__((amdgpu_waves_per_eu(
    (CHR && sizeof(R) == 8) ? (BND == 2 ? 2 : 3) : (ring_slots<DIR, MODE, HYB, R, BND, CHR>() == 24 ? 4 : 1))))
void k_sweep(const SweepArgs A) {
  constexpr int CD = (DIR == 0) ? 1 : 0;  // direction across the lines of the group
  constexpr int OD = (DIR == 2) ? 1 : 2;  // remaining direction
  constexpr int NVAL = 10;                // f+ (5), f- (5)
  constexpr bool per = BND != 2;          // this direction periodic
  constexpr bool anyb = BND != 0;         // some direction bounded
  constexpr int SLOT = NVAL * SW_W + 1;   // padded against bank conflicts
  constexpr int FHS = 5 * SW_W + 1;
  constexpr int FVS = 4 * SW_W + 1;
  // Viscous-flux neighbours staged in an LDS ring (16.6 KB per workgroup, 12.5
  // KB with 24 slots):
  // the FP32 and hybrid sweeps add the derivative of the viscous fluxes of
  // their direction in the finishing step; the FP64 WENO7 sweep keeps three
  // workgroups per CU instead and has no viscous code (a separate kernel
  // writes the viscous divergence it accumulates onto).
  constexpr bool FVR = HYB || sizeof(R) == 4;
  constexpr int NR = ring_slots<DIR, MODE, HYB, R, BND, CHR>();
  // slot of node m (m >= -8: the prologue and the viscous neighbours of a
  // periodic line reach 8 nodes before its first)
  auto slot = [](int m) -> int {
    if constexpr (NR == 32)
      return m & 31;
    else
      return (int)((unsigned)(m + 48) % 24u);
  };
  __shared__ R ring[NR * SLOT];
  __shared__ double fh[(SW_S + 1) * FHS];  // fh[0]: carried flux; fh[s+1]: interface j0+s
  __shared__ double fh0[FHS];             // flux at 1/2, for node 0 of a periodic line
  __shared__ double cyb[FHS];             // carried flux of odd chunks (even chunks: fh[0])
  // hybrid: this chunk's work list, WENO entries from the front (wl_n of them)
  // and, in the FP32 xi sweeps, low-dissipation ones from the back (wl_l)
  __shared__ int wl_n, wl_l;
  __shared__ short wl[SW_T];
  // the viscous flux of direction DIR of every ring node (FVR kernels in
  // viscous runs: [ring slots][4 * SW_W + 1] doubles, dynamic; zero bytes otherwise)
  extern __shared__ double fvr[];

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

  // Raw inputs of one node: conserved variables and row DIR of the metrics / J.
  // Fetched one chunk ahead so the loads overlap the reconstruction of the
  // current chunk.
  struct NodeIn {
    double U[5];
    double a[3];
    double fv[4];
  };
  auto fetch = [&](int m, int col) {
    NodeIn r;
    const int jm = !per ? m : (n >= 8 ? wrap1(m, n) : wrap(m, n));
    const long long id = base + (long long)col * sc + (long long)jm * sd;
#pragma unroll
    for (int q = 0; q < 5; ++q) r.U[q] = A.U[q * N + id];
#pragma unroll
    for (int q = 0; q < 3; ++q) r.a[q] = A.met[(3 * DIR + q) * N + id];
    if (FVR && A.viscous) {
#pragma unroll
      for (int q = 0; q < 4; ++q) r.fv[q] = A.Fv[(long long)(4 * DIR + q) * N + id];
    }
    return r;
  };
  // Primitive recovery and Steger-Warming split of node m into the ring.
  auto split_store = [&](int m, int col, const NodeIn& in) {
    if (A.inviscid) {
      const double rho = in.U[0];
      const double ir = rcp_r<double>(rho);
      const double u = in.U[1] * ir;
      const double v = in.U[2] * ir;
      const double w = in.U[3] * ir;
      const double p = A.ph.gm1 * (in.U[4] - 0.5 * rho * (u * u + v * v + w * w));
      R fp[5], fm[5];
      sw_split<R>(A.ph, (R)rho, (R)ir, (R)u, (R)v, (R)w, (R)p, (R)in.a[0], (R)in.a[1], (R)in.a[2], fp, fm);
      R* sl = ring + slot(m) * SLOT + col;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        sl[q * SW_W] = fp[q];
        sl[(5 + q) * SW_W] = fm[q];
      }
    }
    if (FVR && A.viscous) {
      double* fs = fvr + slot(m) * FVS + col;
#pragma unroll
      for (int q = 0; q < 4; ++q) fs[q * SW_W] = in.fv[q];
    }
  };

  // What the finishing step of a node reads besides the fluxes: the sum of
  // the previous sweeps, U^n, U and 1/J as the mode needs them.  Loaded at the
  // start of the chunk so that the loads overlap the split and the
  // reconstruction (barriers wait for LDS only, not for global loads).
  struct EmitIn {
    double s[5];
    double un[5];
    double u[5];
    double ij;
  };
  auto emit_load = [&](int j, int col, bool with_u) {
    EmitIn e;
    const long long id = base + (long long)col * sc + (long long)j * sd;
    // the sum, U^n and 1/J are read once per sweep: non-temporal loads keep
    // them from displacing reused lines (the load windows, U) in L2
    if (MODE != MODE_SET) {
#pragma unroll
      for (int q = 0; q < 5; ++q) e.s[q] = __builtin_nontemporal_load(A.rhs + q * N + id);
    }
    if (MODE == MODE_RK) {
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        e.un[q] = __builtin_nontemporal_load(A.Un + q * N + id);
        if (with_u) e.u[q] = A.U[q * N + id];
      }
    }
    if (MODE == MODE_RK || MODE == MODE_DUDT) e.ij = __builtin_nontemporal_load(A.met + 9 * N + id);
    return e;
  };

  // Output of node j of line col from its two interface fluxes (inv: this
  // node has both interfaces along DIR, i.e. it is not an end of a
  // non-periodic line).
  // jr: the node's unwrapped position, which indexes the rings; ringfv: its
  // viscous-flux neighbours are in the LDS ring (false only for the first node
  // of a periodic line, finished after the last chunk, which reads them from
  // memory).
  auto emit = [&](int j, int jr, int col, const double* Fr, const double* Fl, bool inv, bool ringfv,
                  const EmitIn& e) {
    const long long id = base + (long long)col * sc + (long long)j * sd;
    double r[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) r[q] = (A.inviscid && inv) ? -(Fr[q * SW_W] - Fl[q * SW_W]) * ih : 0.0;
    if (FVR && A.viscous && inv) {
      // F(q, k): component q of the viscous flux at node jr + k
      auto F = [&](int q, int k) {
        if (ringfv) return fvr[slot(jr + k) * FVS + q * SW_W + col];
        const int p = j + k;
        const int w = per ? (n >= 8 ? wrap1(p, n) : wrap(p, n)) : p;
        return A.Fv[(long long)(4 * DIR + q) * N + id + (long long)(w - j) * sd];
      };
      // sixth or eighth order inside, then sixth, fourth and second order
      // toward the ends of a bounded line (Sec. 2.3)
      const int vh = A.ph.vh;
      const int dist = per ? vh : min(min(j, n - 1 - j), vh);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double d;
        if (dist == 1)
          d = 0.5 * (F(q, 1) - F(q, -1));
        else if (dist == 2)
          d = (2.0 / 3.0) * (F(q, 1) - F(q, -1)) - (1.0 / 12.0) * (F(q, 2) - F(q, -2));
        else if (dist == 3)
          d = 0.75 * (F(q, 1) - F(q, -1)) - 0.15 * (F(q, 2) - F(q, -2)) + (1.0 / 60.0) * (F(q, 3) - F(q, -3));
        else
          d = 0.8 * (F(q, 1) - F(q, -1)) - 0.2 * (F(q, 2) - F(q, -2)) + (4.0 / 105.0) * (F(q, 3) - F(q, -3)) -
              (1.0 / 280.0) * (F(q, 4) - F(q, -4));
        r[q + 1] += d * ih;
      }
    }
    // outputs are written once per sweep: non-temporal stores
    if (MODE == MODE_SET) {
#pragma unroll
      for (int q = 0; q < 5; ++q) __builtin_nontemporal_store(r[q], A.rhs + q * N + id);
    } else if (MODE == MODE_ADD) {
#pragma unroll
      for (int q = 0; q < 5; ++q) __builtin_nontemporal_store(e.s[q] + r[q], A.rhs + q * N + id);
    } else {
      // nodes on a face whose kind sets them after the stage take dU/dt = 0
      // (every kind but the nonreflecting one, whose nodes keep the terms of
      // the directions they are interior to; the normal part is added by
      // k_nrbc)
      bool bnd = false;
      if (anyb) {
        int pq[3];
        node_position(A.g, id, pq);
        const int p0 = pq[0], p1 = pq[1], p2 = pq[2];
        bnd = (p0 == 0 && A.g.setface[0]) || (p0 == A.g.n[0] - 1 && A.g.setface[1]) ||
              (p1 == 0 && A.g.setface[2]) || (p1 == A.g.n[1] - 1 && A.g.setface[3]) ||
              (p2 == 0 && A.g.setface[4]) || (p2 == A.g.n[2] - 1 && A.g.setface[5]);
      }
      const double ij = 1.0 / e.ij;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const double L = bnd ? 0.0 : (e.s[q] + r[q]) * ij;
        if (MODE == MODE_RK)
          __builtin_nontemporal_store(A.a * e.un[q] + A.b * (e.u[q] + A.dt * L), A.out + q * N + id);
        else
          __builtin_nontemporal_store(L, A.out + q * N + id);
      }
    }
  };

  const int nchunks = (n + SW_S - 1) / SW_S;
  // Chunk c reconstructs interfaces JB + 16c + s (s = 0..15), loads nodes
  // JB + 16c + 4 .. JB + 16c + 19 and finishes nodes JB + 16c .. JB + 16c + 15.
  // Periodic lines choose JB so that the wider of the two access streams
  // starts on a 16-node (128-byte) boundary along xi: the finishing accesses
  // (sum, U^n, U, 1/J, output) in the last sweep along xi (JB = 0), the
  // loads otherwise (JB = -4); n interfaces.  Bounded lines: JB = 0,
  // interfaces 0 .. n-2, nodes outside [0, n-1] never loaded.
  constexpr int JBP = (DIR == 0 && (MODE == MODE_RK || MODE == MODE_DUDT)) ? 0 : -4;
  const int JB = per ? JBP : 0;
  const int nif = per ? n : n - 1;             // interfaces of the line
  const int mmax = per ? JB + n + 3 : n - 1;   // last node the chunks load (the prologue covers JB-3 .. JB+3)
  // Prologue: nodes JB-3 .. JB+3 of every line.
  const bool load = A.inviscid || A.viscous;   // the rings are filled for either part
  if (load && t < 7 * SW_W) {
    const int pm = (DIR == 0) ? (t % 7) : (t / SW_W);
    const int pc = (DIR == 0) ? (t / 7) : (t % SW_W);
    const int m = JB + pm - 3;
    if (col0 + pc < ncol && (per || (m >= 0 && m < n))) split_store(m, pc, fetch(m, pc));
  }
  // Characteristic kernels, and the 24-slot sweeps of bounded lines, fetch
  // each chunk's nodes when they split them instead of one chunk ahead: the
  // registers go to the longer reconstruction, or to the fourth wave.
  // The xi sweeps with JB = 0 split nodes 16c + 4 .. 16c + 19 in chunk c,
  // which straddle two 128-byte lines of every array; loaded that way, the
  // second half of each line is evicted from L2 before the next chunk reads
  // it and is fetched again.  The FP32 ones, and the FP64 hybrid ones of
  // periodic lines, load whole aligned 16-node blocks instead: blk holds
  // block c (node 16c + gs of this lane), ahead block c + 1; lanes 4..15
  // split their node of block c, lanes 0..3 theirs of block c + 1.  Measured
  // per Runge-Kutta xi sweep: FP32 hybrid 7.68 -> 7.16 ms on the developed
  // 2048 x 256 x 256 ramp, 825 -> 759 us on 256^3 turbulence, FP64 hybrid
  // there 866 -> 838 us; the other FP64 kernels lost to the 24 extra
  // registers (the bounded hybrid one 9.70 -> 9.96 ms, the periodic WENO7
  // one 798 -> 891 us, down to two waves per SIMD).
  constexpr bool NOPF = CHR || (NR == 24 && BND == 2);
  constexpr bool ALN = DIR == 0 && !CHR && (BND == 2 || JBP == 0) && (sizeof(R) == 4 || (HYB && BND != 2));
  NodeIn ahead, blk;
  bool have, have_blk = false;
  if (ALN) {
    have_blk = load && gcol_ok && gs <= mmax;
    if (have_blk) blk = fetch(gs, gc);
    have = load && gcol_ok && SW_S + gs <= mmax;
    if (have) ahead = fetch(SW_S + gs, gc);
  } else {
    have = load && gcol_ok && JB + 4 + gs <= mmax;
    if (!NOPF && have) ahead = fetch(JB + 4 + gs, gc);
  }
  // Hybrid: the flag of the interface this thread reconstructs in chunk c is
  // loaded during chunk c - 1, after that chunk's prefetch, so waiting for
  // it never waits for the prefetch (loads complete in issue order).
  auto flag_of = [&](int c) -> int {
    const int jj = JB + c * SW_S + rs;
    if (!(A.inviscid && rcol_ok && c * SW_S + rs < nif)) return 0;
    if (!per && (jj < 3 || jj > n - 5)) return 1;   // boundary closure: always the masked WENO5 path
    return A.flags[DIR * N + base + (long long)rc * sc + (long long)(n >= 8 ? wrap1(jj, n) : wrap(jj, n)) * sd];
  };
  int kflag = 0;
  if (HYB) kflag = flag_of(0);
  // The same in characteristic variables (kind 1 or 2, or a boundary closure).
  auto reconstruct_char = [&](int j, int col, int kind, double* dst) {
    const int w0 = per ? (n >= 8 ? wrap1(j, n) : wrap(j, n)) : j;
    const int w1 = per ? (n >= 8 ? wrap1(j + 1, n) : wrap(j + 1, n)) : j + 1;
    const long long i0 = base + (long long)col * sc + (long long)w0 * sd;
    const long long i1 = base + (long long)col * sc + (long long)w1 * sd;
    double Ua[5], a[3];
#pragma unroll
    for (int q = 0; q < 5; ++q) Ua[q] = 0.5 * (A.U[q * N + i0] + A.U[q * N + i1]);
#pragma unroll
    for (int q = 0; q < 3; ++q) a[q] = 0.5 * (A.met[(3 * DIR + q) * N + i0] + A.met[(3 * DIR + q) * N + i1]);
    CharFrame<R> fr;
    fr.init(A.ph, Ua, a);
    // characteristic values of node j + o of the f+ (sg 0) or f- (sg 1) ring
    auto proj = [&](int sg, int o, R* w) {
      const R* B = ring + col + sg * 5 * SW_W + slot(j + o) * SLOT;
      R f[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) f[q] = B[q * SW_W];
      fr.to_char(f, w);
    };
    // One projected 7-node window per sign serves every stencil: WENO7 takes
    // positions 0..6 (f+ nodes j-3 .. j+3, f- mirrored j+4 .. j-2), WENO5
    // positions 1..5.  At the ends of a bounded line (masked WENO5) the
    // substencils that leave it get weight zero and out-of-domain nodes take
    // the centre node's values (finite).
    const bool closure = !per && (j < 3 || j > n - 5);
    const bool w5 = closure || (HYB && kind == 2);
    auto in = [&](int o) { const int m = j + o; return !closure || (m >= 0 && m < n); };
    R G[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) G[k] = (R)0;
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
      R wv[5][7];
#pragma unroll
      for (int t = 0; t < 7; ++t) {
        const int o = sg == 0 ? t - 3 : 4 - t;
        R w[5];
        proj(sg, in(o) ? o : (sg == 0 ? 0 : 1), w);
#pragma unroll
        for (int k = 0; k < 5; ++k) wv[k][t] = w[k];
      }
      if (w5) {
        const bool v0 = sg == 0 ? in(-2) : in(3), v1 = sg == 0 ? in(-1) : in(2), v2 = sg == 0 ? in(2) : in(-1);
#pragma unroll
        for (int k = 0; k < 5; ++k) G[k] += weno5m<R>(wv[k][1], wv[k][2], wv[k][3], wv[k][4], wv[k][5], eps, v0, v1, v2);
      } else {
#pragma unroll
        for (int k = 0; k < 5; ++k)
          G[k] += weno7<R>(wv[k][0], wv[k][1], wv[k][2], wv[k][3], wv[k][4], wv[k][5], wv[k][6], eps);
      }
    }
    R F[5];
    fr.from_char(G, F);
#pragma unroll
    for (int q = 0; q < 5; ++q) dst[q * SW_W] = (double)F[q];
  };
  // Reconstruction of interface j of line col into dst: kind 0 the
  // low-dissipation stencil, 1 WENO7, 2 WENO5 (three-way hybrid).
  auto reconstruct = [&](int j, int col, int kind, double* dst) {
    if (CHR && kind != 0) {
      reconstruct_char(j, col, kind, dst);
      return;
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const R* P = ring + col + q * SW_W;
      const R* M = ring + col + (5 + q) * SW_W;
#define RP(o) P[slot(j + (o)) * SLOT]
#define RM(o) M[slot(j + (o)) * SLOT]
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
      } else if (HYB && kind == 0) {
        if (A.lowdiss == OCFD_LOWDISS_C8)
          F = (double)c8<R>(RP(-3) + RM(-3), RP(-2) + RM(-2), RP(-1) + RM(-1), RP(0) + RM(0), RP(1) + RM(1),
                            RP(2) + RM(2), RP(3) + RM(3), RP(4) + RM(4));
        else
          F = (double)ud7<R>(RP(-3), RP(-2), RP(-1), RP(0), RP(1), RP(2), RP(3)) +
              (double)ud7<R>(RM(4), RM(3), RM(2), RM(1), RM(0), RM(-1), RM(-2));
      } else if (HYB && kind == 2) {
        F = (double)weno5m<R>(RP(-2), RP(-1), RP(0), RP(1), RP(2), eps, true, true, true) +
            (double)weno5m<R>(RM(3), RM(2), RM(1), RM(0), RM(-1), eps, true, true, true);
      } else {
        F = (double)weno7<R>(RP(-3), RP(-2), RP(-1), RP(0), RP(1), RP(2), RP(3), eps) +
            (double)weno7<R>(RM(4), RM(3), RM(2), RM(1), RM(0), RM(-1), RM(-2), eps);
      }
#undef RP
#undef RM
      dst[q * SW_W] = F;
    }
  };

  // The xi Runge-Kutta sweeps with aligned blocks take U of the node they
  // finish (node 16c + gs) from the block this lane loaded for the split
  // instead of reading it again.
  constexpr bool UROW = ALN && MODE == MODE_RK;
  for (int c = 0; c < nchunks; ++c) {
    const int j0 = JB + c * SW_S;
    // the node this thread finishes in this chunk (periodic: node JB is
    // finished after the last chunk), and its inputs
    const int jraw = j0 + gs;
    const bool fin = gcol_ok && (per ? (c * SW_S + gs < n && (c > 0 || gs > 0)) : jraw < n);
    const int jfin = per ? (n >= 8 ? wrap1(jraw, n) : wrap(jraw, n)) : jraw;
    // characteristic kernels load the finishing step's inputs just before it,
    // which keeps 32 registers free through the longer reconstruction
    const bool urow = UROW && load;
    EmitIn ein;
    if (!CHR && fin) ein = emit_load(jfin, gc, !urow);
    if (ALN) {
      // a finished node is loaded (j0 + gs <= mmax) wherever fin holds
      if (urow) {
#pragma unroll
        for (int q = 0; q < 5; ++q) ein.u[q] = blk.U[q];
      }
      const bool lo = gs < 4;
      if (lo ? have : have_blk) split_store(j0 + gs + (lo ? SW_S : 0), gc, lo ? ahead : blk);
    } else if (have) {
      split_store(j0 + 4 + gs, gc, NOPF ? fetch(j0 + 4 + gs, gc) : ahead);
    }
    if (HYB && t == 0) {
      wl_n = 0;
      wl_l = 0;
    }
    __syncthreads();
    if (ALN) {
      blk = ahead;
      have_blk = have;
      have = load && gcol_ok && j0 + 2 * SW_S + gs <= mmax;
      if (have) ahead = fetch(j0 + 2 * SW_S + gs, gc);
    } else {
      have = load && gcol_ok && c + 1 < nchunks && j0 + SW_S + 4 + gs <= mmax;
      if (!NOPF && have) ahead = fetch(j0 + SW_S + 4 + gs, gc);
    }
    const int j = j0 + rs;
    const bool act = A.inviscid && rcol_ok && c * SW_S + rs < nif;
    if (HYB) {
      const int kind = kflag;
      if (c + 1 < nchunks) kflag = flag_of(c + 1);
      // The FP32 xi sweeps of bounded lines use one list for both kinds: the
      // compiler then keeps that kernel within three waves per SIMD (136
      // registers then, 162 with the aligned block loads) instead of 195
      // registers and two, 9.5 -> 7.9 ms per Runge-Kutta sweep on the
      // 2048 x 256 x 256 ramp at 0.63 WENO, 7.5 -> 7.0 ms at 0.003 (measured);
      // the other sweeps are slower with it.
      constexpr bool ONE_LIST = sizeof(R) == 4 && DIR == 0 && BND == 2;
      if (!ONE_LIST) {
        // Low-dissipation interfaces are done in place; WENO interfaces go to
        // a work list so that whole waves run the WENO code (no divergence).
        if (act) {
          if (kind == 0)
            reconstruct(j, rc, 0, fh + (rs + 1) * FHS + rc);
          else
            wl[atomicAdd(&wl_n, 1)] = (short)(t | (kind == 2 ? 512 : 0));
        }
        __syncthreads();
        if (t < wl_n) {
          const int tt = wl[t] & 511;
          const int s2 = tt / SW_W, c2 = tt & (SW_W - 1);
          reconstruct(j0 + s2, c2, (wl[t] & 512) ? 2 : 1, fh + (s2 + 1) * FHS + c2);
        }
      } else {
        if (act) {
          if (kind == 0)
            wl[SW_T - 1 - atomicAdd(&wl_l, 1)] = (short)t;
          else
            wl[atomicAdd(&wl_n, 1)] = (short)(t | (kind == 2 ? 512 : 0));
        }
        __syncthreads();
        if (wl_n < 64) {
          // at most one wave of WENO interfaces: the low-dissipation ones in place
          if (act && kind == 0) reconstruct(j, rc, 0, fh + (rs + 1) * FHS + rc);
          if (t < wl_n) {
            const int tt = wl[t] & 511;
            const int s2 = tt / SW_W, c2 = tt & (SW_W - 1);
            reconstruct(j0 + s2, c2, (wl[t] & 512) ? 2 : 1, fh + (s2 + 1) * FHS + c2);
          }
        } else {
          // WENO entries from the front, low-dissipation ones from the back:
          // whole waves run one kind (at most one wave holds both)
          const bool weno = t < wl_n;
          if (weno || t >= SW_T - wl_l) {
            const int tt = wl[t] & 511;
            const int s2 = tt / SW_W, c2 = tt & (SW_W - 1);
            reconstruct(j0 + s2, c2, weno ? ((wl[t] & 512) ? 2 : 1) : 0, fh + (s2 + 1) * FHS + c2);
          }
        }
      }
    } else if (act) {
      reconstruct(j, rc, 1, fh + (rs + 1) * FHS + rc);
    }
    __syncthreads();
    if (c == 0 && t < 5 * SW_W) fh0[(t / SW_W) * SW_W + (t % SW_W)] = fh[FHS + (t / SW_W) * SW_W + (t % SW_W)];
    // The flux carried into chunk c (its interface j0 - 1) alternates between
    // fh[0] and cyb, so the carry for chunk c + 1 can be written while other
    // threads still finish chunk c's nodes: no barrier is needed between the
    // finishing step and the next chunk, except where the next chunk's
    // viscous-flux ring stores overwrite slots the finishing step still reads.
    double* const cy_in = (c & 1) ? cyb : fh;
    double* const cy_out = (c & 1) ? fh : cyb;
    if (CHR && fin) ein = emit_load(jfin, gc, true);
    if (fin)
      emit(jfin, jraw, gc, fh + (gs + 1) * FHS + gc, gs == 0 ? cy_in + gc : fh + gs * FHS + gc,
           per || (jraw > 0 && jraw < n - 1), FVR, ein);
    if (t < 5 * SW_W) {
      const int last = min(SW_S, nif - c * SW_S);
      if (last > 0) cy_out[(t / SW_W) * SW_W + (t % SW_W)] = fh[last * FHS + (t / SW_W) * SW_W + (t % SW_W)];
    }
    if (FVR) __syncthreads();
  }
  __syncthreads();
  // The periodic line's first node (JB) with the wrapped flux carried out of the last chunk.
  if (per && gs == 0 && gcol_ok) {
    const int j = wrap(JB, n);
    emit(j, JB, gc, fh0 + gc, ((nchunks & 1) ? cyb : fh) + gc, true, false, emit_load(j, gc, true));
  }
}

// Dynamic LDS: the viscous-flux ring of the FP32 and hybrid kernels.
template <int DIR, int MODE, bool HYB, typename R, int BND, bool CHR>
static void launch_sweep_k(const SweepArgs& a, dim3 grid, hipStream_t st) {
  const size_t lds = (a.viscous && (a.mixed || a.hybrid))
                         ? (size_t)ring_slots<DIR, MODE, HYB, R, BND, CHR>() * (4 * SW_W + 1) * sizeof(double)
                         : 0;
  hipLaunchKernelGGL((k_sweep<DIR, MODE, HYB, R, BND, CHR>), grid, dim3(SW_T), lds, st, a);
}
template <int DIR, int MODE, int BND, bool CHR>
static void launch_sweep_b(const SweepArgs& a, dim3 grid, hipStream_t st) {
  if (a.mixed) {
    if (a.hybrid)
      launch_sweep_k<DIR, MODE, true, float, BND, CHR>(a, grid, st);
    else
      launch_sweep_k<DIR, MODE, false, float, BND, CHR>(a, grid, st);
  } else {
    if (a.hybrid)
      launch_sweep_k<DIR, MODE, true, double, BND, CHR>(a, grid, st);
    else
      launch_sweep_k<DIR, MODE, false, double, BND, CHR>(a, grid, st);
  }
}

template <int DIR, int MODE, bool CHR>
static hipError_t launch_sweep_t(const SweepArgs& a, hipStream_t st) {
  constexpr int CD = (DIR == 0) ? 1 : 0;
  constexpr int OD = (DIR == 2) ? 1 : 2;
  dim3 grid((a.g.n[CD] + SW_W - 1) / SW_W, a.g.n[OD]);
  const bool all = a.g.periodic[0] && a.g.periodic[1] && a.g.periodic[2];
  if (!a.g.periodic[DIR])
    launch_sweep_b<DIR, MODE, 2, CHR>(a, grid, st);
  else if (all)
    launch_sweep_b<DIR, MODE, 0, CHR>(a, grid, st);
  else
    launch_sweep_b<DIR, MODE, 1, CHR>(a, grid, st);
  return hipGetLastError();
}

// One translation unit per direction and reconstruction variables (component
// or characteristic) instantiates this, so the variants compile in parallel.
template <int DIR, bool CHR>
hipError_t launch_sweep_dc(int mode, const SweepArgs& a, hipStream_t st) {
  if (a.hybrid && a.inviscid && !a.flags) return hipErrorInvalidValue;   // hybrid needs interface flags
  // only the FP32 and hybrid sweeps (LDS ring) add the viscous derivative;
  // the FP64 WENO7 ones take it from the viscous divergence kernel
  if (a.viscous && !a.hybrid && !a.mixed) return hipErrorInvalidValue;
  switch (mode) {
    case MODE_SET: return launch_sweep_t<DIR, MODE_SET, CHR>(a, st);
    case MODE_ADD: return launch_sweep_t<DIR, MODE_ADD, CHR>(a, st);
    case MODE_RK: return launch_sweep_t<DIR, MODE_RK, CHR>(a, st);
    default: return launch_sweep_t<DIR, MODE_DUDT, CHR>(a, st);
  }
}

}  // namespace ocfd
