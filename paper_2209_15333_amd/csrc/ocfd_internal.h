// Private declarations of the ocfd HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ocfd.h"

namespace ocfd {

// Learned-sensor perceptron 32 -> 64 -> 64 -> 64 -> 1: offsets in the flat
// FP32 parameter array (W1 [input][unit], b1, W2 [input][unit], b2, W3, b3,
// w4, b4).
constexpr int MLP_IN = 32;
constexpr int MLP_H = 64;
constexpr int MLP_W1 = 0;
constexpr int MLP_B1 = MLP_W1 + MLP_IN * MLP_H;
constexpr int MLP_W2 = MLP_B1 + MLP_H;
constexpr int MLP_B2 = MLP_W2 + MLP_H * MLP_H;
constexpr int MLP_W3 = MLP_B2 + MLP_H;
constexpr int MLP_B3 = MLP_W3 + MLP_H * MLP_H;
constexpr int MLP_W4 = MLP_B3 + MLP_H;
constexpr int MLP_B4 = MLP_W4 + MLP_H;
constexpr int MLP_NPARAM = MLP_B4 + 1;

// Division of 32-bit unsigned integers by an invariant divisor d >= 1:
// x / d = (umulhi(x, mul) + x) >> shift with shift = ceil(log2 d) and
// mul = floor(2^32 (2^shift - d) / d) + 1 (Granlund and Montgomery,
// "Division by invariant integers using multiplication", 1994).
struct FastDiv {
  uint32_t mul;
  uint32_t shift;
};

inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  const unsigned long long m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
  return FastDiv{(uint32_t)m, l};
}

// Grid geometry: node counts and element strides of xi, eta, zeta (N < 2^31).
struct Geo {
  int n[3];
  long long s[3];
  long long N;
  int periodic[3];
  int setface[6];   // face f of a bounded direction whose kind sets its nodes after a stage (all but NRBC)
  FastDiv div[2];   // by n[0] and by n[1]
};

// Column tiles for kernels that march along zeta: 64 x 4 (xi, eta) columns
// per workgroup, zeta cut into segments so that about 2048 workgroups run;
// tiles are numbered so that each of the 8 XCDs (which receive workgroups
// round robin) gets a contiguous range of neighbouring tiles.
struct ZMarch {
  int ntx, nty, nseg, zseg;
  unsigned blocks;
};

inline ZMarch make_zmarch(const int n[3]) {
  ZMarch z;
  z.ntx = (n[0] + 63) / 64;
  z.nty = (n[1] + 3) / 4;
  int nseg = (2048 + z.ntx * z.nty - 1) / (z.ntx * z.nty);
  nseg = nseg < 1 ? 1 : (nseg > n[2] ? n[2] : nseg);
  z.zseg = (n[2] + nseg - 1) / nseg;
  z.nseg = (n[2] + z.zseg - 1) / z.zseg;
  const long long tiles = (long long)z.ntx * z.nty * z.nseg;
  z.blocks = (unsigned)(8 * ((tiles + 7) / 8));
  return z;
}

// This thread's column (i, j) and zeta range [k0, k1); false if it has none.
__device__ __forceinline__ bool zmarch_column(const ZMarch& z, const int n[3], int* i, int* j, int* k0, int* k1) {
  const int per = gridDim.x / 8;
  const int L = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (L >= z.ntx * z.nty * z.nseg) return false;
  const int tx = L % z.ntx, ty = (L / z.ntx) % z.nty, zs = L / (z.ntx * z.nty);
  *i = tx * 64 + (threadIdx.x & 63);
  *j = ty * 4 + threadIdx.x / 64;
  if (*i >= n[0] || *j >= n[1]) return false;
  *k0 = zs * z.zseg;
  *k1 = min(n[2], *k0 + z.zseg);
  return true;
}

// Node position (i, j, k) of the linear index id (< 2^31).
__device__ __forceinline__ void node_position(const Geo& g, long long id, int pos[3]) {
  const uint32_t x = (uint32_t)id;
  const uint32_t q0 = (uint32_t)(((unsigned long long)__umulhi(x, g.div[0].mul) + x) >> g.div[0].shift);
  const uint32_t q1 = (uint32_t)(((unsigned long long)__umulhi(q0, g.div[1].mul) + q0) >> g.div[1].shift);
  pos[0] = (int)(x - q0 * (uint32_t)g.n[0]);
  pos[1] = (int)(q0 - q1 * (uint32_t)g.n[1]);
  pos[2] = (int)q1;
}

// Physical constants as the kernels use them.
struct Phys {
  double gamma, gm1;        // gamma, gamma - 1
  double inv_gm1, inv_2g;   // 1 / (gamma - 1), 1 / (2 gamma)
  double Ma2;               // Ma^2
  double inv_Re;            // 1 / Re
  double kcoef;             // 1 / ((gamma-1) Ma^2 Pr Re): heat conductivity per unit mu (eq 14)
  double suth;              // Sutherland constant / Tref (eq 15)
  double eps;               // WENO epsilon
  double theta1, theta2;    // sensor thresholds (eq 43)
  int three_way;            // plain sensor marks max theta > theta2 with flag 2 (WENO5)
  int flag_window;          // plain sensor window of interface j+1/2: 0 nodes j-3 .. j+4; 1 nodes j, j+1
  int curv_inputs;          // learned sensor: second differences (eq 42) as the jump features
  int vh;                   // half width of the interior viscous central stencil (3: sixth, 4: eighth order)
  double h[3], ih[3];       // computational spacing and its inverse
  double period[3];
};

// What the last sweep of a substep does with the summed right-hand side.
enum SweepMode : int {
  MODE_SET = 0,    // rhs = this direction's contribution
  MODE_ADD = 1,    // rhs += contribution
  MODE_RK = 2,     // U_out = a U_n + b (U + dt (rhs + contribution) / (1/J))
  MODE_DUDT = 3,   // out = (rhs + contribution) / (1/J)
};

struct SweepArgs {
  Geo g;
  Phys ph;
  const double* U;       // state the right-hand side is evaluated from
  const double* met;     // [10][N]
  const double* Fv;      // [12][N] viscous fluxes (or null when inviscid-only / Euler)
  const uint8_t* flags;  // [3][N] interface flags of the hybrid scheme (0: low-dissipation stencil)
  double* rhs;           // [5][N]
  const double* Un;      // RK: state at the start of the step
  double* out;           // RK: new state; DUDT: dU/dt
  double a, b, dt;       // RK coefficients
  int inviscid;          // add the inviscid flux difference of this direction
  int viscous;           // add the viscous flux derivative of this direction
  int hybrid;            // 0: WENO7 everywhere; 1: sensor / flags select the stencil
  int lowdiss;           // OCFD_LOWDISS_*
  int mixed;             // 1: split and reconstruction in FP32 (difference, RK in FP64)
  int characteristic;    // 1: WENO interfaces reconstructed in characteristic variables
};

// Kernel launch entry points (ocfd_kernels.hip).  All return hipError_t of the launch.
hipError_t launch_sweep(int dir, int mode, const SweepArgs& a, hipStream_t st);
// One direction's sweep, component-wise (CHR false) or in characteristic
// variables (instantiated in ocfd_sweep_{xi,eta,zeta}[_char].hip).
template <int DIR, bool CHR>
hipError_t launch_sweep_dc(int mode, const SweepArgs& a, hipStream_t st);
// rhs [5][N] = divergence of the viscous fluxes Fv [12][N] (mass row 0).
hipError_t launch_visc_div(const Geo& g, const Phys& ph, const double* Fv, double* rhs, hipStream_t st);
// Fv [12][N] (viscous fluxes of xi, eta, zeta; momentum x, y, z, energy) of U.
hipError_t launch_visc_flux(const Geo& g, const Phys& ph, const double* U, const double* met, double* Fv,
                            hipStream_t st);
// One face (d, side) of a bounded direction set by boundary kind `kind`.
hipError_t launch_bc(const Geo& g, const Phys& ph, double* U, int d, int side, int kind, double Tw,
                     const double* inflow, hipStream_t st);
// out [5][N] += coef * (normal-direction part of dU/dt) on the nodes of the
// nonreflecting face (d, side), from the state U.
hipError_t launch_nrbc(const Geo& g, const Phys& ph, const double* U, const double* met, double* out, int d, int side,
                       double coef, hipStream_t st);
// theta [N] of eq 42 from node pressures P [N].
hipError_t launch_sensor(const Geo& g, const double* P, double* theta, hipStream_t st);
// P [N] = pressure of U.
hipError_t launch_pressure(const Geo& g, const Phys& ph, const double* U, double* P, hipStream_t st);
hipError_t launch_metric_inner(const Geo& g, const Phys& ph, const double* xyz, double* inner, hipStream_t st);
hipError_t launch_metric_outer(const Geo& g, const Phys& ph, const double* xyz, const double* inner, double* met,
                               hipStream_t st);
// Most workgroups of the reduction (reduce_blocks never exceeds it): the
// partial buffer holds RED_MAX_BLOCKS records of OCFD_RED_COUNT doubles.
constexpr int RED_MAX_BLOCKS = 1024;
hipError_t launch_reduce(const Geo& g, const Phys& ph, const double* U, const double* met, double dt,
                         const uint8_t* flags, double* partial, int nblocks, double* out, hipStream_t st);
int reduce_blocks(const Geo& g);

// Sensors (ocfd_sensor.hip).
// Interface flags from theta: 0 low-dissipation (max theta over the window
// <= theta1; the window is nodes j-3 .. j+4, or j and j+1 when flag_window is
// 1), 1 WENO7, 2 WENO5 (three_way and max theta > theta2).
hipError_t launch_plain_flags(const Geo& g, const Phys& ph, const double* theta, uint8_t* flags, hipStream_t st);
hipError_t launch_features(const Geo& g, const Phys& ph, const double* U, const double* met, uint16_t* feat,
                           hipStream_t st);
// Decision thresholds of the learned sensor, one per direction.
struct Tau3 {
  float t[3];
};
hipError_t launch_mlp_flags(const Geo& g, const uint16_t* feat, const float* P, const Tau3& tau, uint8_t* flags,
                            hipStream_t st);
hipError_t launch_mlp_prob(const uint16_t* X, long long S, const float* P, float* prob, hipStream_t st);
hipError_t launch_mlp_grad(const uint16_t* X, const uint8_t* y, const float* w, const int* idx, long long nb,
                           float Wsum, const float* P, float* partial, int nblocks, float* grad, float* Pmut,
                           float* m, float* v, float lr, int t, double* eloss, hipStream_t st);
hipError_t launch_collect_count(const Geo& g, const uint8_t* flags, uint64_t seed, uint32_t thr_pos, uint32_t thr_neg,
                                unsigned long long* counts, int nblocks, hipStream_t st);
hipError_t launch_collect_write(const Geo& g, const uint8_t* flags, const uint16_t* feat, uint64_t seed, uint32_t thr_pos,
                                uint32_t thr_neg, const unsigned long long* offs, long long cap, uint16_t* X,
                                uint8_t* y, float* w, int nblocks, hipStream_t st);
hipError_t launch_flags_or(uint8_t* a, const uint8_t* b, long long n, hipStream_t st);
hipError_t launch_flag_stats(const Geo& g, const uint8_t* fa, const uint8_t* fb, unsigned long long* out,
                             int nblocks, hipStream_t st);

}  // namespace ocfd
