// Shock sensors of the hybrid scheme (Sec. 2.2.3, eq 42-43) and the learned
// sensor that can replace the pressure sensor: node features, per-interface
// flags, a 32-64-64-64-1 perceptron evaluated and trained with bf16 matrix-core
// (MFMA) instructions, sample collection, calibration and audit.
//
// MFMA operand layout used throughout (v_mfma_f32_16x16x32_bf16, one wave):
//   A (16 x 32): lane l holds row l%16, columns 8*(l/16) .. 8*(l/16)+7;
//   B (32 x 16): lane l holds column l%16, rows 8*(l/16) .. 8*(l/16)+7;
//   C (16 x 16): lane l holds column l%16, rows 4*(l/16) .. 4*(l/16)+3.
// and for v_mfma_f32_16x16x16bf16_1k the same with 4 values per lane.
// Activations are kept transposed (hidden unit x sample), so a layer's C
// registers are the next layer's B operand after a fixed relabelling of the
// hidden units: in the K-chunk of units 32c .. 32c+31, k-slot 8g+q of lane
// group g holds unit 32c + 4g+q (q < 4) or 32c + 16+4g+q-4 (q >= 4).  The
// relabelling is applied to the weights instead.
#include "ocfd_internal.h"

namespace ocfd {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v2s __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int wrapn(int p, int n) {
  while (p < 0) p += n;
  while (p >= n) p -= n;
  return p;
}

// Hidden unit held in k-slot q (0..7) of lane group g.
__device__ __forceinline__ int unit_of(int g, int q) { return q < 4 ? 4 * g + q : 16 + 4 * g + (q - 4); }

__device__ __forceinline__ v4f mfma32(const v8bf& a, const v8bf& b, const v4f& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ v4f mfma16(const v4bf& a, const v4bf& b, const v4f& c) {
  v4s as, bs;
  __builtin_memcpy(&as, &a, 8);
  __builtin_memcpy(&bs, &b, 8);
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(as, bs, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Plain sensor flags: interface j+1/2 along d is low-dissipation iff the node
// sensor theta is <= theta1 at every node of its window; otherwise WENO7, or
// WENO5 in the three-way hybrid when the window maximum exceeds theta2.  The
// window (the paper applies theta "at positions" without saying which) is
// the interface's stencil, nodes j-3 .. j+4 (W0 = -3, W1 = 4), or its two
// nodes j, j+1 (W0 = 0, W1 = 1).
// ---------------------------------------------------------------------------
// A workgroup owns a 64 x 4 tile of (xi, eta) columns (ZMarch numbering) and
// marches it along zeta through one segment.  Per plane it stages an LDS patch
// of theta covering the tile widened by the window along xi and eta
// ((64 + W1 - W0) x (4 + W1 - W0) values, read one plane ahead into
// registers), from which each thread takes the xi and eta window maxima of
// its column; the zeta window is a register window of the column's own
// theta.  Positions outside a bounded line count as 0 (theta >= 0, so the
// maximum is the one over the nodes that exist).
template <int W0, int W1>
__global__ __launch_bounds__(256) void k_plain_flags(const Geo g, const ZMarch zm, double theta1, double theta2,
                                                     int three_way, const double* __restrict__ theta,
                                                     uint8_t* __restrict__ flags) {
  constexpr int WN = W1 - W0 + 1;
  constexpr int PX = 64 + WN - 1, PY = 4 + WN - 1, NP = PX * PY;
  constexpr int NPT = (NP + 255) / 256;   // patch values per thread
  __shared__ double patch[NP];
  const int per = gridDim.x / 8;
  const int L = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (L >= zm.ntx * zm.nty * zm.nseg) return;   // uniform over the workgroup
  const int tx = L % zm.ntx, ty = (L / zm.ntx) % zm.nty, zs = L / (zm.ntx * zm.nty);
  const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
  const int i = tx * 64 + lx, j = ty * 4 + ly;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const bool own = i < nx && j < ny;
  const int k0 = zs * zm.zseg;
  const int k1 = min(nz, k0 + zm.zseg);
  const bool px_ = g.periodic[0], py_ = g.periodic[1], pz = g.periodic[2];
  const long long sz = g.s[2];
  // this thread's patch entries: their in-plane offsets (-1: outside a bounded line)
  long long poff[NPT];
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int v = threadIdx.x + 256 * q;
    poff[q] = -1;
    if (v < NP) {
      int gx = tx * 64 + W0 + v % PX, gy = ty * 4 + W0 + v / PX;
      bool ok = true;
      if (px_) gx = wrapn(gx, nx); else ok = ok && gx >= 0 && gx < nx;
      if (py_) gy = wrapn(gy, ny); else ok = ok && gy >= 0 && gy < ny;
      if (ok) poff[q] = gx + (long long)nx * gy;
    }
  }
  auto patch_load = [&](double* r, int k) {
#pragma unroll
    for (int q = 0; q < NPT; ++q) r[q] = poff[q] >= 0 ? theta[poff[q] + (long long)k * sz] : 0.0;
  };
  const long long col = own ? i + (long long)nx * j : 0;
  auto zval = [&](int k) {
    if (!own) return 0.0;
    if (pz) return theta[col + (long long)(nz >= 8 ? k + (k < 0 ? nz : 0) - (k >= nz ? nz : 0) : wrapn(k, nz)) * sz];
    return (k < 0 || k >= nz) ? 0.0 : theta[col + (long long)k * sz];
  };
  double w[WN];
#pragma unroll
  for (int o = 0; o < WN - 1; ++o) w[o] = zval(k0 + W0 + o);
  double nxt[NPT];
  patch_load(nxt, k0);
  auto flag = [&](double mx) -> uint8_t { return mx <= theta1 ? 0 : ((three_way && mx > theta2) ? 2 : 1); };
  for (int k = k0; k < k1; ++k) {
#pragma unroll
    for (int q = 0; q < NPT; ++q)
      if (threadIdx.x + 256 * q < NP) patch[threadIdx.x + 256 * q] = nxt[q];
    w[WN - 1] = zval(k + W1);
    __syncthreads();
    if (k + 1 < k1) patch_load(nxt, k + 1);
    if (own) {
      double mx = 0.0, my = 0.0, mz = 0.0;
#pragma unroll
      for (int o = 0; o < WN; ++o) {
        mx = fmax(mx, patch[(ly - W0) * PX + lx + o]);
        my = fmax(my, patch[(ly + o) * PX + lx - W0]);
        mz = fmax(mz, w[o]);
      }
      const long long id = col + (long long)k * sz;
      flags[id] = flag(mx);
      flags[g.N + id] = flag(my);
      flags[2 * g.N + id] = flag(mz);
    }
#pragma unroll
    for (int o = 0; o < WN - 1; ++o) w[o] = w[o + 1];
    __syncthreads();
  }
}

hipError_t launch_plain_flags(const Geo& g, const Phys& ph, const double* theta, uint8_t* flags, hipStream_t st) {
  const ZMarch zm = make_zmarch(g.n);
  if (ph.flag_window == 1)
    hipLaunchKernelGGL((k_plain_flags<0, 1>), dim3(zm.blocks), dim3(256), 0, st, g, zm, ph.theta1, ph.theta2,
                       ph.three_way, theta, flags);
  else
    hipLaunchKernelGGL((k_plain_flags<-3, 4>), dim3(zm.blocks), dim3(256), 0, st, g, zm, ph.theta1, ph.theta2,
                       ph.three_way, theta, flags);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Node features [4][N]: Delta div(u)/c and Delta |curl u|/c (Delta = (1/J)^(1/3),
// the local cell size), and the pressure and density jumps: the normalised
// first differences across the node summed over the three directions,
//   sum_d |q+ - q-| / (q+ + q-),
// divided by the sensor threshold theta1 (a jump, not the plain sensor's
// second difference: the label the network learns is not one of its
// inputs); with the CURV inputs the normalised second differences
//   sum_d |q- - 2q + q+| / (q- + 2q + q+) / theta1
// instead (the plain sensor's own node value, eq 42).  Velocity derivatives:
// second-order central differences (one-sided over one spacing at the end of
// a bounded line), chain rule with the node metrics.  A bounded direction adds
// no jump term at its end nodes.
// ---------------------------------------------------------------------------
// Primitives (rho, u, v, w, p) of node id.
__device__ __forceinline__ void prim5(const Phys& ph, const double* __restrict__ U, long long N, long long id,
                                      double q[5]) {
  const double rho = U[id];
  const double ir = 1.0 / rho;
  q[0] = rho;
  q[1] = U[N + id] * ir;
  q[2] = U[2 * N + id] * ir;
  q[3] = U[3 * N + id] * ir;
  q[4] = ph.gm1 * (U[4 * N + id] - 0.5 * rho * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]));
}

// Stored as bf16 (round to nearest even of the FP32 value), four per node
// (node-major, 8 bytes), the operand format of the perceptron.  Each thread
// marches one (xi, eta) column through a zeta segment with the primitives of
// planes k-1, k, k+1 in registers; xi and eta neighbours are read from the
// plane.
__global__ __launch_bounds__(256) void k_features(const Geo g, const ZMarch zm, const Phys ph,
                                                  const double* __restrict__ U, const double* __restrict__ met,
                                                  uint2* __restrict__ feat) {
  int i, j, k0, k1;
  if (!zmarch_column(zm, g.n, &i, &j, &k0, &k1)) return;
  const long long N = g.N;
  const int nz = g.n[2];
  const bool pz = g.periodic[2];
  const long long col = i + g.s[1] * j;
  auto plane = [&](int k) { return pz ? wrapn(k, nz) : min(max(k, 0), nz - 1); };
  // xi and eta neighbour positions (clamped at a bounded end) and spacings
  int qpx, qmx, qpy, qmy;
  {
    const bool bx = !g.periodic[0], by = !g.periodic[1];
    const int nx = g.n[0], ny = g.n[1];
    qpx = bx ? min(i + 1, nx - 1) : wrapn(i + 1, nx);
    qmx = bx ? max(i - 1, 0) : wrapn(i - 1, nx);
    qpy = by ? min(j + 1, ny - 1) : wrapn(j + 1, ny);
    qmy = by ? max(j - 1, 0) : wrapn(j - 1, ny);
  }
  const double isx = 1.0 / ((!g.periodic[0] ? (double)(qpx - qmx) : 2.0) * ph.h[0]);
  const double isy = 1.0 / ((!g.periodic[1] ? (double)(qpy - qmy) : 2.0) * ph.h[1]);
  const bool endx = !g.periodic[0] && (i == 0 || i == g.n[0] - 1);
  const bool endy = !g.periodic[1] && (j == 0 || j == g.n[1] - 1);
  const long long oxp = qpx - i, oxm = qmx - i, oyp = (long long)(qpy - j) * g.s[1], oym = (long long)(qmy - j) * g.s[1];
  const double it1 = 1.0 / ph.theta1;
  double zm1[5], z0[5], zp1[5];
  prim5(ph, U, N, col + (long long)plane(k0 - 1) * g.s[2], zm1);
  prim5(ph, U, N, col + (long long)k0 * g.s[2], z0);
  for (int k = k0; k < k1; ++k) {
    const long long id = col + (long long)k * g.s[2];
    prim5(ph, U, N, col + (long long)plane(k + 1) * g.s[2], zp1);
    const int kp = plane(k + 1), km = plane(k - 1);
    const bool endz = !pz && (k == 0 || k == nz - 1);
    const double isz = 1.0 / ((pz ? 2.0 : (double)(kp - km)) * ph.h[2]);
    double xp[5], xm[5], yp[5], ym[5];
    prim5(ph, U, N, id + oxp, xp);
    prim5(ph, U, N, id + oxm, xm);
    prim5(ph, U, N, id + oyp, yp);
    prim5(ph, U, N, id + oym, ym);
    double dvd[3][3];   // d(vel_a)/d(xi_d)
    for (int a = 0; a < 3; ++a) {
      dvd[a][0] = (xp[a + 1] - xm[a + 1]) * isx;
      dvd[a][1] = (yp[a + 1] - ym[a + 1]) * isy;
      dvd[a][2] = (zp1[a + 1] - zm1[a + 1]) * isz;
    }
    const bool curv = ph.curv_inputs;
    auto jump = [&](double m, double c, double pl) {
      return curv ? fabs(-m + 2.0 * c - pl) / (m + 2.0 * c + pl) : fabs(pl - m) / (pl + m);
    };
    double jp = 0.0, jr = 0.0;
    if (!endx) { jp += jump(xm[4], z0[4], xp[4]); jr += jump(xm[0], z0[0], xp[0]); }
    if (!endy) { jp += jump(ym[4], z0[4], yp[4]); jr += jump(ym[0], z0[0], yp[0]); }
    if (!endz) { jp += jump(zm1[4], z0[4], zp1[4]); jr += jump(zm1[0], z0[0], zp1[0]); }
    const double jinv = met[9 * N + id];
    const double ij = 1.0 / jinv;
    double gr[3][3];
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) {
        double sum = 0.0;
        for (int d = 0; d < 3; ++d) sum += (met[(3 * d + c) * N + id] * ij) * dvd[a][d];
        gr[a][c] = sum;
      }
    const double div = gr[0][0] + gr[1][1] + gr[2][2];
    const double wx = gr[2][1] - gr[1][2], wy = gr[0][2] - gr[2][0], wz = gr[1][0] - gr[0][1];
    const double vort = sqrt(wx * wx + wy * wy + wz * wz);
    const double dc = cbrt(fabs(jinv)) / sqrt(ph.gamma * z0[4] / z0[0]);   // Delta / c
    const __bf16 f[4] = {(__bf16)(float)(dc * div), (__bf16)(float)(dc * vort), (__bf16)(float)(jp * it1),
                         (__bf16)(float)(jr * it1)};
    uint2 out;
    __builtin_memcpy(&out, f, 8);
    feat[id] = out;
    for (int q = 0; q < 5; ++q) {
      zm1[q] = z0[q];
      z0[q] = zp1[q];
    }
  }
}

hipError_t launch_features(const Geo& g, const Phys& ph, const double* U, const double* met, uint16_t* feat,
                           hipStream_t st) {
  const ZMarch zm = make_zmarch(g.n);
  hipLaunchKernelGGL(k_features, dim3(zm.blocks), dim3(256), 0, st, g, zm, ph, U, met, (uint2*)feat);
  return hipGetLastError();
}

// Does the 8-node window j-3 .. j+4 of interface (d, node at pos) stay inside
// the grid?  Always on periodic lines; on a bounded line only for
// 3 <= j <= n-5 (the other interfaces use the masked WENO5 closure whatever
// their flag, and are neither sampled nor audited).
__device__ __forceinline__ bool window_inside(const Geo& g, int d, int pos) {
  return g.periodic[d] || (pos >= 3 && pos <= g.n[d] - 5);
}

__device__ __forceinline__ int node_pos(const Geo& g, long long id, int d) {
  int pos[3];
  node_position(g, id, pos);
  return pos[d];
}

// ---------------------------------------------------------------------------
// The perceptron
// ---------------------------------------------------------------------------

// Per-lane weight registers of one wave (forward pass).  Hidden unit u of a
// layer with 64 units lives in C tile u / 16, row u % 16; a K-chunk c of 32
// units (tiles 2c and 2c+1) feeds the next layer's B operand, k-slot 8g+q of
// lane group g holding unit 32c + unit_of(g, q), which is the lane's own C
// value of tile 2c (q < 4) or 2c+1 (q >= 4).
// The biases and output weights (read once per tile each) sit in LDS, which
// frees 64 registers per lane for the weights and the tile in flight.
struct MlpRegs {
  v8bf A1[4];      // W1^T tiles: row = unit 16m + l%16, k = inputs 8g .. 8g+7
  v8bf A2[4][2];   // W2^T: row = output unit 16m + l%16, k-chunk c: input unit 32c + unit_of(g, q)
  v8bf A3[4][2];   // W3^T, the same
};

// LDS copy of b1, b2, b3, w4 (64 each) and b4.
constexpr int LB_B1 = 0, LB_B2 = 64, LB_B3 = 128, LB_W4 = 192, LB_B4 = 256, LB_N = 260;

// Every thread of the block takes part; a barrier follows before use.
__device__ __forceinline__ void stage_bias(const float* __restrict__ P, float* lb) {
  for (int k = threadIdx.x; k < 257; k += blockDim.x)
    lb[k] = k < 64 ? P[MLP_B1 + k] : k < 128 ? P[MLP_B2 + k - 64] : k < 192 ? P[MLP_B3 + k - 128]
          : k < 256 ? P[MLP_W4 + k - 192] : P[MLP_B4];
}

// Values of units 16m + 4g .. 16m + 4g + 3 of one 64-vector in LDS.
__device__ __forceinline__ v4f lds4(const float* lb, int off, int m, int g) {
  return *(const v4f*)(lb + off + 16 * m + 4 * g);
}

// A operand of W^T (W [input][unit] of a 64-unit layer, row 16m + i, k-chunk c).
__device__ __forceinline__ void load_wt(const float* __restrict__ W, int m, int c, int g, int i, v8bf& A) {
  for (int q = 0; q < 8; ++q) A[q] = (__bf16)W[(32 * c + unit_of(g, q)) * MLP_H + 16 * m + i];
}

__device__ __forceinline__ void load_mlp(const float* __restrict__ P, MlpRegs& R) {
  const int l = threadIdx.x & 63, i = l & 15, g = l >> 4;
  for (int m = 0; m < 4; ++m) {
    for (int q = 0; q < 8; ++q) R.A1[m][q] = (__bf16)P[MLP_W1 + (8 * g + q) * MLP_H + 16 * m + i];
    for (int c = 0; c < 2; ++c) {
      load_wt(P + MLP_W2, m, c, g, i, R.A2[m][c]);
      load_wt(P + MLP_W3, m, c, g, i, R.A3[m][c]);
    }
  }
}

struct Fwd {
  v4f a1[4], a2[4], a3[4];  // pre-activations, C layout (unit 16m + 4g + r, sample l%16)
  v8bf h1[2], h2[2];        // relu(a1), relu(a2) as the B operands of layers 2 and 3 (K-chunks)
  float z;                  // output logit of sample l%16 (same in the four lane groups)
};

// max(a, 0) in one integer instruction: a negative float is a negative
// int32 and a non-negative one keeps its order as an int32.
__device__ __forceinline__ float relu(float a) { return __int_as_float(max(__float_as_int(a), 0)); }

// B operand of K-chunk c from C tiles 2c, 2c+1 (the relabelling above), of
// v (relu when relu is set).
// The ReLU is taken after the rounding, on the packed bf16 values (a
// negative bf16 is a negative int16): the same bits, half the instructions.
__device__ __forceinline__ v8bf chunk_b(const v4f* v, int c, bool use_relu) {
  unsigned w[4];
  for (int k = 0; k < 4; ++k) {
    const v4f& t = v[2 * c + k / 2];
    const v2bf p = __builtin_convertvector((v2f){t[2 * (k & 1)], t[2 * (k & 1) + 1]}, v2bf);
    __builtin_memcpy(&w[k], &p, 4);
  }
  if (use_relu) {
    for (int k = 0; k < 4; ++k) {
      v2s h;
      __builtin_memcpy(&h, &w[k], 4);
      h = __builtin_elementwise_max(h, (v2s)0);
      __builtin_memcpy(&w[k], &h, 4);
    }
  }
  v8bf b;
  __builtin_memcpy(&b, w, 16);
  return b;
}

// One 64-unit layer: out[m] = sum_c A[m][c] B[c] + bias.
__device__ __forceinline__ void layer64(const v8bf (*A)[2], const v8bf* B, const float* lb, int off, v4f* out) {
  const int g = (threadIdx.x & 63) >> 4;
  for (int m = 0; m < 4; ++m) out[m] = mfma32(A[m][1], B[1], mfma32(A[m][0], B[0], lds4(lb, off, m, g)));
}

// Forward pass of 16 samples held as the B operand x (inputs 8g..8g+7 of sample l%16).
__device__ __forceinline__ void mlp_forward(const MlpRegs& R, const float* lb, const v8bf& x, Fwd& F) {
  const int g = (threadIdx.x & 63) >> 4;
  for (int m = 0; m < 4; ++m) F.a1[m] = mfma32(R.A1[m], x, lds4(lb, LB_B1, m, g));
  for (int c = 0; c < 2; ++c) F.h1[c] = chunk_b(F.a1, c, true);
  layer64(R.A2, F.h1, lb, LB_B2, F.a2);
  for (int c = 0; c < 2; ++c) F.h2[c] = chunk_b(F.a2, c, true);
  layer64(R.A3, F.h2, lb, LB_B3, F.a3);
  float z = 0.f;
  for (int m = 0; m < 4; ++m) {
    const v4f w4 = lds4(lb, LB_W4, m, g);
    for (int r = 0; r < 4; ++r) z += w4[r] * relu(F.a3[m][r]);
  }
  // sum over the four lane groups (hidden units) of each sample
  z += __shfl_xor(z, 16);
  z += __shfl_xor(z, 32);
  F.z = z + lb[LB_B4];
}

__device__ __forceinline__ float sigmoidf(float z) { return __builtin_amdgcn_rcpf(1.f + __expf(-z)); }

// Learned flags of every interface: x of interface (d, node) = the four
// features of the 8 nodes j-3 .. j+4 along d, node-major.
// FAST: nx a multiple of 16 and every n >= 8.  A tile is then 16 consecutive
// nodes of one xi row, its position comes from the (wave-uniform) tile
// index, a periodic wrap is one conditional add, and the gather has no
// branch: the next tile's loads stay in flight while the current tile is
// evaluated (a load behind a branch makes the compiler wait for every load
// before the first MFMA).  The fast path runs three waves per SIMD (no
// spills): 1.27 ms against 1.59 ms at two waves for 50.3 M interfaces,
// measured; the general one two.
template <bool FAST>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FAST ? 3 : 2))) void k_mlp_flags(const Geo g, const uint2* __restrict__ feat,
                                                   const float* __restrict__ P, const Tau3 tau,
                                                   uint8_t* __restrict__ flags) {
  __shared__ __align__(16) float lb[LB_N];
  stage_bias(P, lb);
  MlpRegs R;
  load_mlp(P, R);
  __syncthreads();
  const int l = threadIdx.x & 63, j = l & 15, gg = l >> 4;
  const long long N = g.N;
  const long long tiles = (N + 15) / 16;
  const long long wave = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const long long nwaves = (long long)gridDim.x * 4;
  if (wave >= tiles) return;
  struct Tile {
    uint2 xv[2];     // inputs 8gg .. 8gg+7 = the four bf16 features of window nodes 2gg, 2gg+1
    long long id;
    bool ok, inside;
  };
  for (int d = 0; d < 3; ++d) {
    const int n = g.n[d];
    const int sd = (int)g.s[d];
    const bool per = g.periodic[d];
    auto gather = [&](long long T, Tile& tl) {
      int pos[3];
      if (FAST) {
        const int b = (int)(T * 16);
        node_position(g, b, pos);
        pos[0] += j;
        tl.id = b + j;
        tl.ok = true;
      } else {
        tl.id = T * 16 + j;
        tl.ok = tl.id < N;
        node_position(g, tl.ok ? tl.id : N - 1, pos);
      }
      const int idc = (int)(tl.ok ? tl.id : N - 1);
      tl.inside = window_inside(g, d, pos[d]);
      for (int tt = 0; tt < 2; ++tt) {
        int q = pos[d] + 2 * gg + tt - 3;
        if (FAST) {
          const int wr = q + (q < 0 ? n : 0) - (q >= n ? n : 0);
          const int cl = min(max(q, 0), n - 1);
          q = per ? wr : cl;
        } else if (per) {
          q = n >= 8 ? q + (q < 0 ? n : 0) - (q >= n ? n : 0) : wrapn(q, n);
        } else {
          q = min(max(q, 0), n - 1);
        }
        tl.xv[tt] = feat[idc + (q - pos[d]) * sd];
      }
    };
    // the next tile's inputs are loaded while the current one is evaluated;
    // the last iteration of a wave reloads its own last tile (never past the end)
    Tile cur, nxt;
    gather(wave, cur);
    for (long long T = wave; T < tiles; T += nwaves) {
      gather(T + nwaves < tiles ? T + nwaves : T, nxt);
      // keep the scheduler from sinking those loads into the MFMA chain
      __builtin_amdgcn_sched_barrier(0);
      v8bf x;
      __builtin_memcpy(&x, cur.xv, 16);
      Fwd F;
      mlp_forward(R, lb, x, F);
      if (cur.ok && gg == 0) flags[d * N + cur.id] = (!cur.inside || sigmoidf(F.z) >= tau.t[d]) ? 1 : 0;
      cur = nxt;
    }
  }
}

hipError_t launch_mlp_flags(const Geo& g, const uint16_t* feat, const float* P, const Tau3& tau, uint8_t* flags,
                            hipStream_t st) {
  const bool fast = (g.n[0] & 15) == 0 && g.n[0] >= 8 && g.n[1] >= 8 && g.n[2] >= 8;
  if (fast)
    hipLaunchKernelGGL(k_mlp_flags<true>, dim3(2048), dim3(256), 0, st, g, (const uint2*)feat, P, tau, flags);
  else
    hipLaunchKernelGGL(k_mlp_flags<false>, dim3(2048), dim3(256), 0, st, g, (const uint2*)feat, P, tau, flags);
  return hipGetLastError();
}

// Probabilities of stored samples X [S][32] (bf16 bits), in order.
__global__ __launch_bounds__(256) void k_mlp_prob(const uint16_t* __restrict__ X, long long S,
                                                  const float* __restrict__ P, float* __restrict__ prob) {
  __shared__ __align__(16) float lb[LB_N];
  stage_bias(P, lb);
  MlpRegs R;
  load_mlp(P, R);
  __syncthreads();
  const int l = threadIdx.x & 63, j = l & 15, gg = l >> 4;
  const long long tiles = (S + 15) / 16;
  for (long long T = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); T < tiles; T += (long long)gridDim.x * 4) {
    const long long s = T * 16 + j;
    const long long sc = s < S ? s : S - 1;
    v8bf x;
    __builtin_memcpy(&x, X + sc * 32 + 8 * gg, 16);
    Fwd F;
    mlp_forward(R, lb, x, F);
    if (s < S && gg == 0) prob[s] = sigmoidf(F.z);
  }
}

hipError_t launch_mlp_prob(const uint16_t* X, long long S, const float* P, float* prob, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_prob, dim3(256), dim3(256), 0, st, X, S, P, prob);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Training: gradient of the weighted binary cross-entropy over a batch
//   L = -sum_i w_i [y_i log p_i + (1 - y_i) log(1 - p_i)] / Wsum
// An iteration takes 64 samples, 16 per wave.  Each wave runs the forward pass and
// the backward pass of its samples through the layers (16x16x32 MFMAs with
// the transposed weights) and stages its inputs, hidden activations and
// pre-activation gradients as [unit][sample] bf16 rows in LDS.  Then the
// weight gradients dW[in][out] = sum_s act[in][s] delta[out][s] are forty
// 16x16 tiles (W1 8, W2 16, W3 16), ten per wave, each an MFMA chain over the
// iteration's 64 samples (4 x 16x16x16).  Bias, output-layer and loss terms are
// per-lane sums.  Every workgroup writes its partial gradient;
// k_mlp_reduce_adam sums them in a fixed order (deterministic).
// ---------------------------------------------------------------------------
constexpr int GT = 256;
constexpr int SPAD = 64 + 8;   // row stride (bf16) of the [unit][sample] staging

struct Stage {
  __bf16 x[MLP_IN][SPAD];
  __bf16 h1[MLP_H][SPAD];
  __bf16 h2[MLP_H][SPAD];
  __bf16 d1[MLP_H][SPAD];
  __bf16 d2[MLP_H][SPAD];
  __bf16 d3[MLP_H][SPAD];
};

// A operand of W (W [input][unit], 64 x 64) for the product W delta: row =
// input unit 16m + i, k-chunk c: output unit 32c + unit_of(g, q).
__device__ __forceinline__ void load_w(const float* __restrict__ W, int m, int c, int g, int i, v8bf& A) {
  for (int q = 0; q < 8; ++q) A[q] = (__bf16)W[(16 * m + i) * MLP_H + 32 * c + unit_of(g, q)];
}

__global__ __launch_bounds__(GT) void k_mlp_grad(const uint16_t* __restrict__ X, const uint8_t* __restrict__ y,
                                                 const float* __restrict__ w, const int* __restrict__ idx,
                                                 long long nb, float Wsum, const float* __restrict__ P,
                                                 float* __restrict__ partial) {
  __shared__ union {
    Stage st;
    float red[MLP_NPARAM + 1];
  } sh;
  __shared__ __align__(16) float lb[LB_N];
  stage_bias(P, lb);
  MlpRegs R;
  load_mlp(P, R);
  __syncthreads();
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, j = l & 15, gg = l >> 4;
  v8bf A2b[4][2], A3b[4][2];   // W2, W3 as the A operands of the back-propagation
  for (int m = 0; m < 4; ++m)
    for (int c = 0; c < 2; ++c) {
      load_w(P + MLP_W2, m, c, gg, j, A2b[m][c]);
      load_w(P + MLP_W3, m, c, gg, j, A3b[m][c]);
    }
  v4f acc[10];   // weight-gradient tiles t = wv + 4k (C layout: col = input unit, rows = output unit)
  for (int k = 0; k < 10; ++k) acc[k] = (v4f){0.f, 0.f, 0.f, 0.f};
  float gb1[4][4] = {}, gb2[4][4] = {}, gb3[4][4] = {}, gw4[4][4] = {};
  float gb4 = 0.f, loss = 0.f;
  const v4f zero = {0.f, 0.f, 0.f, 0.f};
  // Every wave runs the same number of iterations (barriers below are block-wide);
  // a wave past the last tile works on sample 0 with zero weight.
  const long long tiles = (nb + 15) / 16;
  for (long long T0 = (long long)blockIdx.x * 4; T0 < tiles; T0 += (long long)gridDim.x * 4) {
    const long long T = T0 + wv;
    const long long s = T * 16 + j;
    const bool ok = T < tiles && s < nb;
    const long long si = idx[ok ? s : 0];
    v8bf x;
    __builtin_memcpy(&x, X + si * 32 + 8 * gg, 16);
    Fwd F;
    mlp_forward(R, lb, x, F);
    const float p = sigmoidf(F.z);
    const float ys = (float)(y[si] & 1);   // bit 0: label (bits 1-2 of collected samples: direction)
    const float ws = ok ? w[si] : 0.f;
    const float dz = ws * (p - ys) / Wsum;
    if (gg == 0) loss += -ws * (ys * __logf(p + 1e-12f) + (1.f - ys) * __logf(1.f - p + 1e-12f)) / Wsum;
    if (gg == 0) gb4 += dz;
    // output layer and da3
    v4f da3[4], da2[4], da1[4];
    for (int m = 0; m < 4; ++m)
      for (int r = 0; r < 4; ++r) {
        gw4[m][r] += dz * fmaxf(F.a3[m][r], 0.f);
        da3[m][r] = F.a3[m][r] > 0.f ? dz * lb[LB_W4 + 16 * m + 4 * gg + r] : 0.f;
        gb3[m][r] += da3[m][r];
      }
    // da2 = (W3 da3) * (a2 > 0), da1 = (W2 da2) * (a1 > 0)
    v8bf db[2];
    for (int c = 0; c < 2; ++c) db[c] = chunk_b(da3, c, false);
    for (int m = 0; m < 4; ++m) {
      const v4f dh = mfma32(A3b[m][1], db[1], mfma32(A3b[m][0], db[0], zero));
      for (int r = 0; r < 4; ++r) {
        da2[m][r] = F.a2[m][r] > 0.f ? dh[r] : 0.f;
        gb2[m][r] += da2[m][r];
      }
    }
    for (int c = 0; c < 2; ++c) db[c] = chunk_b(da2, c, false);
    for (int m = 0; m < 4; ++m) {
      const v4f dh = mfma32(A2b[m][1], db[1], mfma32(A2b[m][0], db[0], zero));
      for (int r = 0; r < 4; ++r) {
        da1[m][r] = F.a1[m][r] > 0.f ? dh[r] : 0.f;
        gb1[m][r] += da1[m][r];
      }
    }
    // stage [unit][sample] rows of this wave's 16 samples
    const int col = 16 * wv + j;
    for (int m = 0; m < 4; ++m)
      for (int r = 0; r < 4; ++r) {
        const int u = 16 * m + 4 * gg + r;
        sh.st.h1[u][col] = (__bf16)fmaxf(F.a1[m][r], 0.f);
        sh.st.h2[u][col] = (__bf16)fmaxf(F.a2[m][r], 0.f);
        sh.st.d1[u][col] = (__bf16)da1[m][r];
        sh.st.d2[u][col] = (__bf16)da2[m][r];
        sh.st.d3[u][col] = (__bf16)da3[m][r];
      }
    for (int q = 0; q < 8; ++q) sh.st.x[8 * gg + q][col] = x[q];
    __syncthreads();
    // weight-gradient tiles: t < 8 W1 (4 output x 2 input tiles), 8 <= t < 24
    // W2, 24 <= t < 40 W3 (4 x 4); t is uniform within the wave
    for (int k = 0; k < 10; ++k) {
      const int t = wv + 4 * k;
      const int mat = t < 8 ? 1 : (t < 24 ? 2 : 3);
      const int tt = t < 8 ? t : (t < 24 ? t - 8 : t - 24);
      const int mo = mat == 1 ? tt / 2 : tt / 4, mi = mat == 1 ? tt % 2 : tt % 4;
      const __bf16(*act)[SPAD] = mat == 1 ? sh.st.x : (mat == 2 ? sh.st.h1 : sh.st.h2);
      const __bf16(*del)[SPAD] = mat == 1 ? sh.st.d1 : (mat == 2 ? sh.st.d2 : sh.st.d3);
      for (int kc = 0; kc < 4; ++kc) {
        v4bf a, b;
        for (int q = 0; q < 4; ++q) {
          a[q] = del[16 * mo + j][16 * kc + 4 * gg + q];
          b[q] = act[16 * mi + j][16 * kc + 4 * gg + q];
        }
        acc[k] = mfma16(a, b, acc[k]);
      }
    }
    __syncthreads();
  }
  // Bias, output-layer and loss terms: lane (j, gg) holds the sums over its
  // samples for the units of lane group gg; add the 16 lanes of each group by
  // butterfly shuffles (every lane takes part; fixed order, so deterministic).
  for (int m = 0; m < 4; ++m)
    for (int r = 0; r < 4; ++r)
      for (int o = 1; o < 16; o <<= 1) {
        gb1[m][r] += __shfl_xor(gb1[m][r], o);
        gb2[m][r] += __shfl_xor(gb2[m][r], o);
        gb3[m][r] += __shfl_xor(gb3[m][r], o);
        gw4[m][r] += __shfl_xor(gw4[m][r], o);
      }
  for (int o = 1; o < 16; o <<= 1) {
    gb4 += __shfl_xor(gb4, o);
    loss += __shfl_xor(loss, o);
  }
  // The staging is done with (barrier above); the same LDS now holds red[].
  for (int k = threadIdx.x; k < MLP_NPARAM + 1; k += GT) sh.red[k] = 0.f;
  __syncthreads();
  // Weight tiles: each entry belongs to one lane of one wave, so all waves
  // write at once.
  for (int k = 0; k < 10; ++k) {
    const int t = wv + 4 * k;
    const int mat = t < 8 ? 1 : (t < 24 ? 2 : 3);
    const int tt = t < 8 ? t : (t < 24 ? t - 8 : t - 24);
    const int mo = mat == 1 ? tt / 2 : tt / 4, mi = mat == 1 ? tt % 2 : tt % 4;
    const int off = mat == 1 ? MLP_W1 : (mat == 2 ? MLP_W2 : MLP_W3);
    for (int r = 0; r < 4; ++r) sh.red[off + (16 * mi + j) * MLP_H + 16 * mo + 4 * gg + r] = acc[k][r];
  }
  __syncthreads();
  // Bias terms: the waves in turn (fixed order).
  for (int wave = 0; wave < 4; ++wave) {
    if (wv == wave && j == 0) {
      for (int m = 0; m < 4; ++m)
        for (int r = 0; r < 4; ++r) {
          const int u = 16 * m + 4 * gg + r;
          sh.red[MLP_B1 + u] += gb1[m][r];
          sh.red[MLP_B2 + u] += gb2[m][r];
          sh.red[MLP_B3 + u] += gb3[m][r];
          sh.red[MLP_W4 + u] += gw4[m][r];
        }
      if (gg == 0) {
        sh.red[MLP_B4] += gb4;
        sh.red[MLP_NPARAM] += loss;
      }
    }
    __syncthreads();
  }
  for (int k = threadIdx.x; k < MLP_NPARAM + 1; k += GT)
    partial[(long long)blockIdx.x * (MLP_NPARAM + 1) + k] = sh.red[k];
}

// Sum the workgroups' partial gradients (fixed order) into grad[NPARAM + 1]
// (last entry: loss, also added to the epoch's running sum *eloss), then, if
// lr > 0, one Adam step on the FP32 master parameters (moments m, v; step
// count t).  One thread per parameter.
__global__ __launch_bounds__(256) void k_mlp_reduce_adam(const float* __restrict__ partial, int nblocks,
                                                         float* __restrict__ grad, float* __restrict__ P,
                                                         float* __restrict__ m, float* __restrict__ v, float lr,
                                                         int t, double* __restrict__ eloss) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k > MLP_NPARAM) return;
  float s = 0.f;
  for (int b = 0; b < nblocks; ++b) s += partial[(long long)b * (MLP_NPARAM + 1) + k];
  grad[k] = s;
  if (k == MLP_NPARAM) {
    *eloss += (double)s;
  } else if (lr > 0.f) {
    const float mk = b1 * m[k] + (1.f - b1) * s;
    const float vk = b2 * v[k] + (1.f - b2) * s * s;
    m[k] = mk;
    v[k] = vk;
    const float mh = mk / (1.f - powf(b1, (float)t));
    const float vh = vk / (1.f - powf(b2, (float)t));
    P[k] -= lr * mh / (sqrtf(vh) + eps);
  }
}

hipError_t launch_mlp_grad(const uint16_t* X, const uint8_t* y, const float* w, const int* idx, long long nb,
                           float Wsum, const float* P, float* partial, int nblocks, float* grad, float* Pmut,
                           float* m, float* v, float lr, int t, double* eloss, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_grad, dim3(nblocks), dim3(GT), 0, st, X, y, w, idx, nb, Wsum, P, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_reduce_adam, dim3((MLP_NPARAM + 1 + 255) / 256), dim3(256), 0, st, partial, nblocks, grad,
                     Pmut, m, v, lr, t, eloss);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sample collection from the current flags: interface (d, node) is taken if
// a counter-based hash of (seed, d, node) falls below the keep probability of
// its class.  Two passes (count per workgroup, then write at the scanned
// offset) keep the sample order deterministic.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t hash3(uint64_t seed, uint32_t d, uint64_t id) {
  // SplitMix64 finaliser of a combined counter
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (id * 4 + d + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (uint32_t)(z >> 32);
}

__device__ __forceinline__ bool keep_interface(const Geo& g, uint64_t seed, int d, long long id, uint8_t flag,
                                               uint32_t thr_pos, uint32_t thr_neg) {
  if (!window_inside(g, d, node_pos(g, id, d))) return false;
  const uint32_t h = hash3(seed, (uint32_t)d, (uint64_t)id);
  return flag ? h < thr_pos : h < thr_neg;
}

constexpr int CT = 256;

__global__ __launch_bounds__(CT) void k_collect_count(const Geo g, const uint8_t* __restrict__ flags, uint64_t seed,
                                                      uint32_t thr_pos, uint32_t thr_neg,
                                                      unsigned long long* __restrict__ counts) {
  __shared__ unsigned long long sh[CT];
  const long long total = 3 * g.N;
  const long long per = (total + gridDim.x - 1) / gridDim.x;
  const long long a = (long long)blockIdx.x * per, b = min(total, a + per);
  unsigned long long c = 0;
  for (long long k = a + threadIdx.x; k < b; k += CT) {
    const int d = (int)(k / g.N);
    const long long id = k % g.N;
    c += keep_interface(g, seed, d, id, flags[k], thr_pos, thr_neg) ? 1 : 0;
  }
  sh[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int i = 0; i < CT; ++i) s += sh[i];
    counts[blockIdx.x] = s;
  }
}

// Writes the kept samples of this workgroup's range, in index order, from
// offset offs[block] (offsets beyond cap are dropped).
__global__ __launch_bounds__(CT) void k_collect_write(const Geo g, const uint8_t* __restrict__ flags,
                                                      const uint2* __restrict__ feat, uint64_t seed, uint32_t thr_pos,
                                                      uint32_t thr_neg, const unsigned long long* __restrict__ offs,
                                                      long long cap, uint16_t* __restrict__ X,
                                                      uint8_t* __restrict__ y, float* __restrict__ w) {
  __shared__ unsigned long long base;
  __shared__ int sc[CT];
  const long long total = 3 * g.N;
  const long long per = (total + gridDim.x - 1) / gridDim.x;
  const long long a = (long long)blockIdx.x * per, b = min(total, a + per);
  if (threadIdx.x == 0) base = offs[blockIdx.x];
  __syncthreads();
  const long long N = g.N;
  for (long long k0 = a; k0 < b; k0 += CT) {
    const long long k = k0 + threadIdx.x;
    const bool in = k < b;
    const int d = in ? (int)(k / N) : 0;
    const long long id = in ? k % N : 0;
    const bool kp = in && keep_interface(g, seed, d, id, flags[in ? k : 0], thr_pos, thr_neg);
    sc[threadIdx.x] = kp ? 1 : 0;
    __syncthreads();
    // exclusive prefix of this pass (serial in one thread: 256 entries)
    if (threadIdx.x == 0) {
      int s = 0;
      for (int i = 0; i < CT; ++i) {
        const int c = sc[i];
        sc[i] = s;
        s += c;
      }
    }
    __syncthreads();
    if (kp) {
      const long long o = (long long)base + sc[threadIdx.x];
      if (o < cap) {
        int pos[3];
        node_position(g, id, pos);
        uint2 xs[8];
        for (int t = 0; t < 8; ++t)
          xs[t] = feat[id + (long long)(wrapn(pos[d] + t - 3, g.n[d]) - pos[d]) * g.s[d]];  // window inside
        uint2* dst = (uint2*)(X + o * 32);
        for (int t = 0; t < 8; ++t) dst[t] = xs[t];
        y[o] = (uint8_t)((flags[k] ? 1 : 0) | (d << 1));   // label, and the direction for calibration
        w[o] = 1.f;
      }
    }
    __syncthreads();
    if (threadIdx.x == CT - 1) base += sc[CT - 1] + (kp ? 1 : 0);
    __syncthreads();
  }
}

hipError_t launch_collect_count(const Geo& g, const uint8_t* flags, uint64_t seed, uint32_t thr_pos, uint32_t thr_neg,
                                unsigned long long* counts, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(k_collect_count, dim3(nblocks), dim3(CT), 0, st, g, flags, seed, thr_pos, thr_neg, counts);
  return hipGetLastError();
}

hipError_t launch_collect_write(const Geo& g, const uint8_t* flags, const uint16_t* feat, uint64_t seed, uint32_t thr_pos,
                                uint32_t thr_neg, const unsigned long long* offs, long long cap, uint16_t* X,
                                uint8_t* y, float* w, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(k_collect_write, dim3(nblocks), dim3(CT), 0, st, g, flags, (const uint2*)feat, seed, thr_pos,
                     thr_neg, offs,
                     cap, X, y, w);
  return hipGetLastError();
}

// Class counts of flag fields over the interfaces whose window stays inside
// the grid (per workgroup partials).
__global__ __launch_bounds__(CT) void k_flag_stats(const Geo g, const uint8_t* __restrict__ fa,
                                                   const uint8_t* __restrict__ fb, unsigned long long* __restrict__ out) {
  __shared__ unsigned long long sh[4][CT];
  unsigned long long c[4] = {0, 0, 0, 0};  // a=1, a=0&b=1, a=1&b=0, a!=b
  const long long total = 3 * g.N;
  for (long long k = (long long)blockIdx.x * CT + threadIdx.x; k < total; k += (long long)gridDim.x * CT) {
    const int d = (int)(k / g.N);
    if (!window_inside(g, d, node_pos(g, k % g.N, d))) continue;
    const uint8_t x = fa[k];
    c[0] += x ? 1 : 0;
    if (fb) {
      const uint8_t z = fb[k];
      c[1] += (!x && z) ? 1 : 0;
      c[2] += (x && !z) ? 1 : 0;
      c[3] += ((x != 0) != (z != 0)) ? 1 : 0;
    }
  }
  for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] = c[q];
  __syncthreads();
  if (threadIdx.x < 4) {
    unsigned long long s = 0;
    for (int i = 0; i < CT; ++i) s += sh[threadIdx.x][i];
    out[blockIdx.x * 4 + threadIdx.x] = s;
  }
}

hipError_t launch_flag_stats(const Geo& g, const uint8_t* fa, const uint8_t* fb, unsigned long long* out,
                             int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(k_flag_stats, dim3(nblocks), dim3(CT), 0, st, g, fa, fb, out);
  return hipGetLastError();
}

// a |= b elementwise (learned flags widened by the plain sensor's).
__global__ __launch_bounds__(256) void k_flags_or(uint8_t* __restrict__ a, const uint8_t* __restrict__ b,
                                                  long long n) {
  for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256) a[k] |= b[k];
}

hipError_t launch_flags_or(uint8_t* a, const uint8_t* b, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_flags_or, dim3(2048), dim3(256), 0, st, a, b, n);
  return hipGetLastError();
}

}  // namespace ocfd
