// HIP kernels (gfx950) of the ocfd library other than the directional
// sweeps: primitives and viscous fluxes, boundary conditions, the pressure
// sensor, metrics and reductions, for one Runge-Kutta substep of the
// curvilinear compressible Navier-Stokes solver of Dang et al.,
// arXiv:2209.15333, Section 2.
//
// Data layout: structure-of-arrays, field-major, x fastest (see ocfd.h).
// Every kernel keeps FP64 arithmetic.
#include "ocfd_device.h"

namespace ocfd {

hipError_t launch_sweep(int dir, int mode, const SweepArgs& a, hipStream_t st) {
  if (a.characteristic) {
    if (dir == 0) return launch_sweep_dc<0, true>(mode, a, st);
    if (dir == 1) return launch_sweep_dc<1, true>(mode, a, st);
    return launch_sweep_dc<2, true>(mode, a, st);
  }
  if (dir == 0) return launch_sweep_dc<0, false>(mode, a, st);
  if (dir == 1) return launch_sweep_dc<1, false>(mode, a, st);
  return launch_sweep_dc<2, false>(mode, a, st);
}

// ---------------------------------------------------------------------------
// Pressure and viscous fluxes (eq 9-16, Sec. 2.3)
// ---------------------------------------------------------------------------

// Pressure of every node, into P[N] (the plain sensor's input).
__global__ __launch_bounds__(256) void k_pressure(const Geo g, const Phys ph, const double* __restrict__ U,
                                                  double* __restrict__ P) {
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= g.N) return;
  const long long N = g.N;
  const double m1 = U[N + id], m2 = U[2 * N + id], m3 = U[3 * N + id];
  P[id] = ph.gm1 * (U[4 * N + id] - 0.5 * (m1 * m1 + m2 * m2 + m3 * m3) / U[id]);
}

hipError_t launch_pressure(const Geo& g, const Phys& ph, const double* U, double* P, hipStream_t st) {
  hipLaunchKernelGGL(k_pressure, dim3((unsigned)((g.N + 255) / 256)), dim3(256), 0, st, g, ph, U, P);
  return hipGetLastError();
}

// Viscous flux vectors of the three directions at every node, from the
// conserved variables: u, v, w, T of each node read (eq 5, 8, 16-17);
// derivatives of u, v, w, T along xi, eta, zeta; Cartesian gradients by the chain rule with
// the node metrics; Sutherland viscosity (eq 15), heat conductivity (eq 14),
// stresses (eq 13) and stress work plus heat flux (eq 12); the flux of
// direction d is (row d of the metrics / J) applied to tau and Theta (eq 9-11).
// Output Fv[4*d + q][N], q = momentum x, y, z, energy.
//
// A workgroup owns a VT_X x VT_Y tile of (xi, eta) columns and marches along zeta
// through one segment of planes, keeping each column's (2 VH + 1)-plane window
// of u, v, w, T in registers, so every plane is read from memory once per
// segment.  Neighbours along xi and eta come from an LDS patch of the current
// plane: the tile (from the register windows) and a ring VH nodes wide
// around it (read from memory one plane ahead into registers).  Tiles are
// numbered so that the eight XCDs each receive a contiguous range
// (round-robin dispatch), which keeps a whole segment of neighbouring tiles
// on one L2.
// Tile shapes (xi x eta columns of a workgroup of 256): 32 x 8 for the
// viscous fluxes (their U ring is five values a node, so the smaller ring
// pays) and for the eighth-order divergence; 64 x 4 for the sixth-order
// divergence (measured on MI355X at 256^3 and on the ramp).  At least three
// waves per SIMD (168 registers, no spills): the eighth-order fluxes took
// 8.09 ms at two waves and 7.44 ms at three on the 2048 x 256 x 256 ramp.

template <int VH, int VT_X, int VT_Y>
__global__ __launch_bounds__(256, 3) void k_visc_flux(const Geo g, const Phys ph, const double* __restrict__ U,
                                                   const double* __restrict__ met, double* __restrict__ Fv,
                                                   int ntx, int nty, int nseg, int zseg) {
  constexpr int ZW = 2 * VH + 1;          // planes of the zeta window
  constexpr int PX = VT_X + 2 * VH;       // patch width (xi) and height (eta)
  constexpr int PY = VT_Y + 2 * VH;
  constexpr int NR = PX * PY - VT_X * VT_Y;   // ring nodes around the tile
  constexpr int NH = (NR + 255) / 256;        // ring nodes per thread and plane
  __shared__ double patch[4][PY][PX];
  const int per = gridDim.x / 8;
  const int L = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (L >= ntx * nty * nseg) return;          // uniform over the workgroup
  const int tx = L % ntx, ty = (L / ntx) % nty, zs = L / (ntx * nty);
  const int lx = threadIdx.x & (VT_X - 1), ly = threadIdx.x / VT_X;
  const int i = tx * VT_X + lx;
  const int j = ty * VT_Y + ly;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const bool own = i < nx && j < ny;
  const int k0 = zs * zseg;
  const int k1 = min(nz, k0 + zseg);
  const long long N = g.N;
  const long long sz = g.s[2];
  const bool px = g.periodic[0], py = g.periodic[1], pz = g.periodic[2];
  // node positions of the patch, wrapped on periodic lines and clamped on
  // bounded ones (clamped entries are never read by the closures)
  auto xi_of = [&](int gi) { return px ? wrap(gi, nx) : min(max(gi, 0), nx - 1); };
  auto eta_of = [&](int gj) { return py ? wrap(gj, ny) : min(max(gj, 0), ny - 1); };
  // plane index of k (wrapped when zeta is periodic, clamped otherwise: the
  // clamped planes are loaded but never used by the boundary closure)
  auto zi = [&](int k) { return pz ? wrap(k, nz) : min(max(k, 0), nz - 1); };
  // this thread's column (a tile position outside the grid takes the wrapped
  // or clamped column, so its patch entry holds what a neighbour expects)
  const long long colid = xi_of(i) + (long long)nx * eta_of(j);
  // the ring around the tile: patch index and node position (xi + nx eta)
  // of each of its NR nodes, computed once per workgroup
  __shared__ int ring_at[NR];
  __shared__ int ring_pos[NR];
  for (int r = threadIdx.x; r < NR; r += 256) {
    int yy, xx;
    if (r < 2 * VH * PX) {          // full rows above and below the tile
      yy = r / PX;
      xx = r % PX;
      if (yy >= VH) yy += VT_Y;
    } else {                         // the VH columns left and right of it
      const int r2 = r - 2 * VH * PX;
      yy = VH + r2 / (2 * VH);
      const int c = r2 % (2 * VH);
      xx = c < VH ? c : VT_X + c;
    }
    ring_at[r] = yy * PX + xx;
    ring_pos[r] = xi_of(tx * VT_X + xx - VH) + nx * eta_of(ty * VT_Y + yy - VH);
  }
  __syncthreads();
  double* const pf = &patch[0][0][0];
  // u, v, w, T of a node from its conserved variables (eq 5, 8, 16-17)
  auto prim = [&](const double* c, double* o) {
    const double rho = c[0];
    const double ir = 1.0 / rho;
    const double u = c[1] * ir, v = c[2] * ir, w = c[3] * ir;
    const double p = ph.gm1 * (c[4] - 0.5 * rho * (u * u + v * v + w * w));
    o[0] = u;
    o[1] = v;
    o[2] = w;
    o[3] = ph.gamma * ph.Ma2 * p * ir;
  };
  // ring node s of this thread: r = thread + 256 s; its conserved variables
  // are read one plane ahead and turned into u, v, w, T when stored
  auto ring_load = [&](double (*ring)[5], int k) {
#pragma unroll
    for (int s = 0; s < NH; ++s) {
      const int r = threadIdx.x + 256 * s;
      if (r < NR) {
        const long long id = ring_pos[r] + (long long)k * sz;
#pragma unroll
        for (int c = 0; c < 5; ++c) ring[s][c] = U[c * N + id];
      }
    }
  };
  auto ring_store = [&](const double (*ring)[5]) {
#pragma unroll
    for (int s = 0; s < NH; ++s) {
      const int r = threadIdx.x + 256 * s;
      if (r < NR) {
        double o[4];
        prim(ring[s], o);
#pragma unroll
        for (int q = 0; q < 4; ++q) pf[q * (PX * PY) + ring_at[r]] = o[q];
      }
    }
  };
  // the zeta window of this column (u, v, w, T of planes k - VH .. k + VH)
  double zw[4][ZW];
  auto zload = [&](int k, int slot) {
    const long long id = colid + (long long)zi(k) * sz;
    double c[5], o[4];
#pragma unroll
    for (int q = 0; q < 5; ++q) c[q] = U[q * N + id];
    prim(c, o);
#pragma unroll
    for (int q = 0; q < 4; ++q) zw[q][slot] = o[q];
  };
#pragma unroll
  for (int o = -VH; o < VH; ++o) zload(k0 + o, o + VH);
  double ring[NH][5];
  ring_load(ring, k0);
  // interior central derivative of half width VH (sixth or eighth order)
  auto central = [&](auto val) {
    if constexpr (VH == 3)
      return 0.75 * (val(1) - val(-1)) - 0.15 * (val(2) - val(-2)) + (1.0 / 60.0) * (val(3) - val(-3));
    else
      return 0.8 * (val(1) - val(-1)) - 0.2 * (val(2) - val(-2)) + (4.0 / 105.0) * (val(3) - val(-3)) -
             (1.0 / 280.0) * (val(4) - val(-4));
  };
  for (int k = k0; k < k1; ++k) {
    zload(k + VH, ZW - 1);
    // the patch of plane k: the tile from the windows, the ring prefetched
#pragma unroll
    for (int q = 0; q < 4; ++q) patch[q][VH + ly][VH + lx] = zw[q][VH];
    ring_store(ring);
    __syncthreads();
    if (k + 1 < k1) ring_load(ring, k + 1);
    const long long id = colid + (long long)k * sz;
    if (own) {
      double dq[4][3];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double* rowx = &patch[q][VH + ly][VH + lx];
        if (px)
          dq[q][0] = central([&](int m) { return rowx[m]; }) * ph.ih[0];
        else
          dq[q][0] = line_deriv([&](int m) { return rowx[m]; }, i, nx, false, VH) * ph.ih[0];
        if (py)
          dq[q][1] = central([&](int m) { return rowx[m * PX]; }) * ph.ih[1];
        else
          dq[q][1] = line_deriv([&](int m) { return rowx[m * PX]; }, j, ny, false, VH) * ph.ih[1];
        if (pz)
          dq[q][2] = central([&](int m) { return zw[q][VH + m]; }) * ph.ih[2];
        else
          dq[q][2] = line_deriv([&](int m) { return zw[q][VH + m]; }, k, nz, false, VH) * ph.ih[2];
      }
      // metrics are read once and the fluxes written once: non-temporal, so
      // they do not push the planes of u, v, w, T (re-read as neighbours) out of L2
      const double ij = 1.0 / __builtin_nontemporal_load(met + 9 * N + id);
      double m[9];
#pragma unroll
      for (int r = 0; r < 9; ++r) m[r] = __builtin_nontemporal_load(met + r * N + id);
      double gr[4][3];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          gr[q][c] = (m[c] * ij) * dq[q][0] + (m[3 + c] * ij) * dq[q][1] + (m[6 + c] * ij) * dq[q][2];
      const double T = zw[3][VH];
      const double mu = T * sqrt(T) * (1.0 + ph.suth) / (T + ph.suth);
      const double kc = mu * ph.kcoef;
      const double mr = mu * ph.inv_Re;
      const double div = gr[0][0] + gr[1][1] + gr[2][2];
      double tau[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) tau[a][b] = mr * (gr[a][b] + gr[b][a] - (a == b ? (2.0 / 3.0) * div : 0.0));
      const double u = zw[0][VH], v = zw[1][VH], w = zw[2][VH];
      double th[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) th[a] = u * tau[0][a] + v * tau[1][a] + w * tau[2][a] + kc * gr[3][a];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double m0 = m[3 * d], m1 = m[3 * d + 1], m2 = m[3 * d + 2];
#pragma unroll
        for (int b = 0; b < 3; ++b)
          __builtin_nontemporal_store(m0 * tau[0][b] + m1 * tau[1][b] + m2 * tau[2][b], Fv + (4 * d + b) * N + id);
        __builtin_nontemporal_store(m0 * th[0] + m1 * th[1] + m2 * th[2], Fv + (4 * d + 3) * N + id);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int o = 0; o < ZW - 1; ++o) zw[q][o] = zw[q][o + 1];
  }
}

// Workgroups of a z-marching tile launch: ntx x nty tiles per plane, nseg
// segments of zseg planes, a multiple of 8 so the XCD-contiguous numbering
// is exact.  The kernels hold three workgroups per CU, so the workgroups run
// in rounds of three per CU; nseg minimises the rounds times the planes a
// workgroup reads (its zseg planes, and the 2 VH planes that open its zeta
// window at a quarter of a plane's cost: they load one column's U only).
// On the 2048 x 256 x 256 ramp that gives three segments (6144 workgroups,
// eight full rounds) instead of one (2048, the last round two-thirds full):
// eighth-order fluxes 7.33 -> 6.87 ms (measured).
struct TileGrid {
  int ntx, nty, nseg, zseg;
  unsigned nb;
};
static int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, v = 0;
    const bool ok = hipGetDevice(&dev) == hipSuccess &&
                    hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess;
    cus = ok && v > 0 ? v : 256;
  }
  return cus;
}
static TileGrid tile_grid(const Geo& g, int tx, int ty, int vh) {
  TileGrid t;
  t.ntx = (g.n[0] + tx - 1) / tx;
  t.nty = (g.n[1] + ty - 1) / ty;
  const long long per_plane = (long long)t.ntx * t.nty;
  const long long slots = 3LL * device_cus();
  double best = 0.0;
  int bseg = 1;
  for (int ns = 1; ns <= g.n[2] && ns <= 64; ++ns) {
    const int zs = (g.n[2] + ns - 1) / ns;
    const int nsg = (g.n[2] + zs - 1) / zs;
    const long long wg = per_plane * nsg;
    const double cost = (double)((wg + slots - 1) / slots) * (zs + 0.5 * vh);
    if (ns == 1 || cost < best) {
      best = cost;
      bseg = nsg;
    }
  }
  t.zseg = (g.n[2] + bseg - 1) / bseg;
  t.nseg = (g.n[2] + t.zseg - 1) / t.zseg;
  const long long tiles = per_plane * t.nseg;
  t.nb = (unsigned)(8 * ((tiles + 7) / 8));
  return t;
}

hipError_t launch_visc_flux(const Geo& g, const Phys& ph, const double* U, const double* met, double* Fv,
                            hipStream_t st) {
  const TileGrid t = tile_grid(g, 32, 8, ph.vh);
  if (ph.vh == 4)
    hipLaunchKernelGGL((k_visc_flux<4, 32, 8>), dim3(t.nb), dim3(256), 0, st, g, ph, U, met, Fv, t.ntx, t.nty, t.nseg,
                       t.zseg);
  else
    hipLaunchKernelGGL((k_visc_flux<3, 32, 8>), dim3(t.nb), dim3(256), 0, st, g, ph, U, met, Fv, t.ntx, t.nty, t.nseg,
                       t.zseg);
  return hipGetLastError();
}

// Divergence of the viscous fluxes (Sec. 2.3): rhs[0] = 0 and, for the
// momentum and energy rows, rhs[1+q] = sum_d (d/d xi_d of Fv[4d+q]) / h_d,
// each derivative of half width VH with the closures of line_deriv on
// bounded lines; at the end node of a bounded line the derivative along that
// line is 0 (a face node either takes dU/dt = 0, or on a nonreflecting face
// has no normal viscous term).  Each flux is differentiated along its own direction only: the
// zeta fluxes through a register window of the zeta march, the xi fluxes from
// an LDS row patch (the tile plus VH columns each side), the eta fluxes from
// an LDS column patch (the tile plus VH rows above and below, read from memory
// one plane ahead into registers).  Same tile scheme and XCD numbering as
// k_visc_flux, and the same three waves per SIMD.
template <int VH, int VT_X, int VT_Y>
__global__ __launch_bounds__(256, 3) void k_visc_div(const Geo g, const Phys ph, const double* __restrict__ Fv,
                                                  double* __restrict__ rhs, int ntx, int nty, int nseg, int zseg) {
  constexpr int ZW = 2 * VH + 1;
  constexpr int SX = VT_Y * (VT_X + 2 * VH);   // one field of the xi patch
  constexpr int SY = (VT_Y + 2 * VH) * VT_X;   // one field of the eta patch
  constexpr int NRX = VT_Y * 2 * VH;           // halo nodes of the xi patch
  constexpr int NRY = 2 * VH * VT_X;           // halo nodes of the eta patch
  constexpr int NR = NRX + NRY;
  constexpr int NH = (4 * NR + 255) / 256;     // halo values per thread and plane
  __shared__ double pbuf[4 * SX + 4 * SY];
  __shared__ int ring_at[NR];                  // offset of field 0 in pbuf
  __shared__ int ring_pos[NR];                 // node position xi + nx eta
  const int per = gridDim.x / 8;
  const int L = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (L >= ntx * nty * nseg) return;           // uniform over the workgroup
  const int tx = L % ntx, ty = (L / ntx) % nty, zs = L / (ntx * nty);
  const int lx = threadIdx.x & (VT_X - 1), ly = threadIdx.x / VT_X;
  const int i = tx * VT_X + lx;
  const int j = ty * VT_Y + ly;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const bool own = i < nx && j < ny;
  const int k0 = zs * zseg;
  const int k1 = min(nz, k0 + zseg);
  const long long N = g.N;
  const long long sz = g.s[2];
  const bool px = g.periodic[0], py = g.periodic[1], pz = g.periodic[2];
  auto xi_of = [&](int gi) { return px ? wrap(gi, nx) : min(max(gi, 0), nx - 1); };
  auto eta_of = [&](int gj) { return py ? wrap(gj, ny) : min(max(gj, 0), ny - 1); };
  auto zi = [&](int k) { return pz ? wrap(k, nz) : min(max(k, 0), nz - 1); };
  const long long colid = xi_of(i) + (long long)nx * eta_of(j);
  for (int r = threadIdx.x; r < NR; r += 256) {
    int at, gi, gj;
    if (r < NRX) {                      // xi patch: VH columns left and right of the tile
      const int row = r / (2 * VH), c = r % (2 * VH);
      const int xx = c < VH ? c : VT_X + c;
      at = row * (VT_X + 2 * VH) + xx;
      gi = tx * VT_X + xx - VH;
      gj = ty * VT_Y + row;
    } else {                            // eta patch: VH rows above and below
      const int r2 = r - NRX;
      const int row = r2 / VT_X, xx = r2 % VT_X;
      const int yy = row < VH ? row : row + VT_Y;
      at = 4 * SX + yy * VT_X + xx;
      gi = tx * VT_X + xx;
      gj = ty * VT_Y + yy - VH;
    }
    ring_at[r] = at;
    ring_pos[r] = xi_of(gi) + nx * eta_of(gj);
  }
  __syncthreads();
  // halo value s of this thread: v = thread + 256 s of the 4 NR (field-major);
  // xi-patch nodes read Fv[q], eta-patch nodes Fv[4 + q]
  auto ring_load = [&](double* ring, int k) {
#pragma unroll
    for (int s = 0; s < NH; ++s) {
      const int v = threadIdx.x + 256 * s;
      if (v < 4 * NR) {
        const int q = v / NR, r = v - q * NR;
        ring[s] = Fv[(r < NRX ? q : 4 + q) * N + ring_pos[r] + (long long)k * sz];
      }
    }
  };
  auto ring_store = [&](const double* ring) {
#pragma unroll
    for (int s = 0; s < NH; ++s) {
      const int v = threadIdx.x + 256 * s;
      if (v < 4 * NR) {
        const int q = v / NR, r = v - q * NR;
        pbuf[ring_at[r] + q * (r < NRX ? SX : SY)] = ring[s];
      }
    }
  };
  double zw[4][ZW];
#pragma unroll
  for (int o = -VH; o < VH; ++o) {
    const long long id = colid + (long long)zi(k0 + o) * sz;
#pragma unroll
    for (int q = 0; q < 4; ++q) zw[q][o + VH] = Fv[(8 + q) * N + id];
  }
  // this column's values of the next plane, read one plane ahead: the xi and
  // eta fluxes of plane k and the zeta fluxes of plane k + VH
  double nx_own[8], nx_z[4];
  auto own_load = [&](int k) {
    const long long id = colid + (long long)k * sz;
    const long long idz = colid + (long long)zi(k + VH) * sz;
#pragma unroll
    for (int q = 0; q < 8; ++q) nx_own[q] = Fv[q * N + id];
#pragma unroll
    for (int q = 0; q < 4; ++q) nx_z[q] = Fv[(8 + q) * N + idz];
  };
  own_load(k0);
  double ring[NH];
  ring_load(ring, k0);
  auto central = [&](auto val) {
    if constexpr (VH == 3)
      return 0.75 * (val(1) - val(-1)) - 0.15 * (val(2) - val(-2)) + (1.0 / 60.0) * (val(3) - val(-3));
    else
      return 0.8 * (val(1) - val(-1)) - 0.2 * (val(2) - val(-2)) + (4.0 / 105.0) * (val(3) - val(-3)) -
             (1.0 / 280.0) * (val(4) - val(-4));
  };
  for (int k = k0; k < k1; ++k) {
    const long long id = colid + (long long)k * sz;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      zw[q][ZW - 1] = nx_z[q];
      pbuf[q * SX + ly * (VT_X + 2 * VH) + VH + lx] = nx_own[q];
      pbuf[4 * SX + q * SY + (VH + ly) * VT_X + lx] = nx_own[4 + q];
    }
    ring_store(ring);
    __syncthreads();
    if (k + 1 < k1) {
      ring_load(ring, k + 1);
      own_load(k + 1);
    }
    if (own) {
      double r[5];
      r[0] = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double* fx = pbuf + q * SX + ly * (VT_X + 2 * VH) + VH + lx;
        const double* fy = pbuf + 4 * SX + q * SY + (VH + ly) * VT_X + lx;
        const double dx = px ? central([&](int m) { return fx[m]; })
                             : ((i == 0 || i == nx - 1) ? 0.0 : line_deriv([&](int m) { return fx[m]; }, i, nx, false, VH));
        const double dy = py ? central([&](int m) { return fy[m * VT_X]; })
                             : ((j == 0 || j == ny - 1) ? 0.0
                                                        : line_deriv([&](int m) { return fy[m * VT_X]; }, j, ny, false, VH));
        const double dz = pz ? central([&](int m) { return zw[q][VH + m]; })
                             : ((k == 0 || k == nz - 1) ? 0.0
                                                        : line_deriv([&](int m) { return zw[q][VH + m]; }, k, nz, false, VH));
        r[1 + q] = dx * ph.ih[0] + dy * ph.ih[1] + dz * ph.ih[2];
      }
#pragma unroll
      for (int q = 0; q < 5; ++q) __builtin_nontemporal_store(r[q], rhs + q * N + id);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int o = 0; o < ZW - 1; ++o) zw[q][o] = zw[q][o + 1];
  }
}

hipError_t launch_visc_div(const Geo& g, const Phys& ph, const double* Fv, double* rhs, hipStream_t st) {
  if (ph.vh == 4) {
    const TileGrid t = tile_grid(g, 32, 8, ph.vh);
    hipLaunchKernelGGL((k_visc_div<4, 32, 8>), dim3(t.nb), dim3(256), 0, st, g, ph, Fv, rhs, t.ntx, t.nty, t.nseg,
                       t.zseg);
  } else {
    const TileGrid t = tile_grid(g, 64, 4, ph.vh);
    hipLaunchKernelGGL((k_visc_div<3, 64, 4>), dim3(t.nb), dim3(256), 0, st, g, ph, Fv, rhs, t.ntx, t.nty, t.nseg,
                       t.zseg);
  }
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
// Characteristic nonreflecting faces (Thompson 1987, with the local
// one-dimensional relations of Poinsot & Lele 1992; the paper imposes
// nonreflecting conditions at the ramp's exit and upper boundary, Sec. 6.1,
// without formulas).  A node of such a face is advanced like an interior
// node: the sweeps give it the fluxes of the directions it is interior to,
// and this kernel adds, for its normal direction d, the time derivative
// carried by the characteristic waves that leave through the face (waves
// entering have amplitude zero):
//   s = |grad xi_d|, n = grad xi_d / s, q = (rho, u, v, w, p) and its
//   one-sided second-order difference dq along xi_d into the grid, u_n = u.n;
//   L1 = s (u_n - c)(dp - rho c du_n),  L5 = s (u_n + c)(dp + rho c du_n),
//   L2 = s u_n (c^2 drho - dp),         Lt = s u_n (du - n (n.du));
//   drho/dt = -(L2 + (L5 + L1)/2)/c^2, dp/dt = -(L5 + L1)/2,
//   du/dt = -(n (L5 - L1)/(2 rho c) + Lt), in conserved variables,
// plus the metric-derivative part of the normal flux derivative,
// -J sum_a d(xi_a/J)/dxi F_a (one-sided difference of the metrics; F_a the
// Cartesian inviscid flux), which keeps a uniform stream uniform on curved
// grids.  The result times coef (b dt in a Runge-Kutta stage, 1 for dU/dt)
// is added to out.  One thread per face node; nodes that also lie on a face
// whose kind sets them after the stage are skipped.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_nrbc(const Geo g, const Phys ph, const double* __restrict__ U,
                                              const double* __restrict__ met, double* __restrict__ out, int d,
                                              int side, double coef) {
  const int e0 = d == 0 ? 1 : 0, e1 = d == 2 ? 1 : 2;
  const long long nf = (long long)g.n[e0] * g.n[e1];
  const long long f = (long long)blockIdx.x * 256 + threadIdx.x;
  if (f >= nf) return;
  int c[3];
  c[e0] = (int)(f % g.n[e0]);
  c[e1] = (int)(f / g.n[e0]);
  c[d] = side ? g.n[d] - 1 : 0;
  for (int a = 0; a < 3; ++a)
    if ((c[a] == 0 && g.setface[2 * a]) || (c[a] == g.n[a] - 1 && g.setface[2 * a + 1])) return;
  const long long N = g.N;
  const long long id = c[0] + g.s[1] * c[1] + g.s[2] * c[2];
  const long long step = side ? -g.s[d] : g.s[d];   // toward the interior
  const double sgn = side ? -1.0 : 1.0;
  const double ih = ph.ih[d];
  double q[3][5], mt[3][3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const long long it = id + t * step;
    const double rho = U[it];
    const double ir = 1.0 / rho;
    const double u = U[N + it] * ir, v = U[2 * N + it] * ir, w = U[3 * N + it] * ir;
    q[t][0] = rho;
    q[t][1] = u;
    q[t][2] = v;
    q[t][3] = w;
    q[t][4] = ph.gm1 * (U[4 * N + it] - 0.5 * rho * (u * u + v * v + w * w));
#pragma unroll
    for (int a = 0; a < 3; ++a) mt[t][a] = met[(3 * d + a) * N + it];
  }
  double dq[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) dq[m] = sgn * 0.5 * (-3.0 * q[0][m] + 4.0 * q[1][m] - q[2][m]) * ih;
  const double jinv = met[9 * N + id];
  const double ij = 1.0 / jinv;
  const double gx = mt[0][0] * ij, gy = mt[0][1] * ij, gz = mt[0][2] * ij;
  const double sg = sqrt(gx * gx + gy * gy + gz * gz);
  const double n[3] = {gx / sg, gy / sg, gz / sg};
  const double rho = q[0][0], p = q[0][4];
  const double uv[3] = {q[0][1], q[0][2], q[0][3]};
  const double cs = sqrt(ph.gamma * p / rho);
  const double un = uv[0] * n[0] + uv[1] * n[1] + uv[2] * n[2];
  const double dun = dq[1] * n[0] + dq[2] * n[1] + dq[3] * n[2];
  const double lam1 = sg * (un - cs), lam2 = sg * un, lam5 = sg * (un + cs);
  auto outgoing = [&](double l) { return side ? l >= 0.0 : l <= 0.0; };
  const double L1 = outgoing(lam1) ? lam1 * (dq[4] - rho * cs * dun) : 0.0;
  const double L5 = outgoing(lam5) ? lam5 * (dq[4] + rho * cs * dun) : 0.0;
  const bool o2 = outgoing(lam2);
  const double L2 = o2 ? lam2 * (cs * cs * dq[0] - dq[4]) : 0.0;
  const double drho = -(L2 + 0.5 * (L5 + L1)) / (cs * cs);
  const double dp = -0.5 * (L5 + L1);
  double dv[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double Lt = o2 ? lam2 * (dq[1 + a] - n[a] * dun) : 0.0;
    dv[a] = -(n[a] * (L5 - L1) / (2.0 * rho * cs) + Lt);
  }
  double r[5];
  r[0] = drho;
#pragma unroll
  for (int a = 0; a < 3; ++a) r[1 + a] = uv[a] * drho + rho * dv[a];
  const double uu = uv[0] * uv[0] + uv[1] * uv[1] + uv[2] * uv[2];
  r[4] = dp / ph.gm1 + 0.5 * uu * drho + rho * (uv[0] * dv[0] + uv[1] * dv[1] + uv[2] * dv[2]);
  const double E = U[4 * N + id];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double dm = sgn * 0.5 * (-3.0 * mt[0][a] + 4.0 * mt[1][a] - mt[2][a]) * ih;
    const double Fa[5] = {rho * uv[a], rho * uv[0] * uv[a] + (a == 0 ? p : 0.0), rho * uv[1] * uv[a] + (a == 1 ? p : 0.0),
                          rho * uv[2] * uv[a] + (a == 2 ? p : 0.0), (E + p) * uv[a]};
#pragma unroll
    for (int m = 0; m < 5; ++m) r[m] -= dm * Fa[m] * ij;
  }
#pragma unroll
  for (int m = 0; m < 5; ++m) out[m * N + id] += coef * r[m];
}

hipError_t launch_nrbc(const Geo& g, const Phys& ph, const double* U, const double* met, double* out, int d, int side,
                       double coef, hipStream_t st) {
  const long long nf = (long long)g.n[d == 0 ? 1 : 0] * g.n[d == 2 ? 1 : 2];
  hipLaunchKernelGGL(k_nrbc, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, st, g, ph, U, met, out, d, side, coef);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Shock sensor (eq 42-43): theta = sum_d |-p_- + 2p - p_+| / (p_- + 2p + p_+)
// ---------------------------------------------------------------------------

// theta from the node pressures P[N].  Each thread marches one (xi, eta)
// column through a zeta segment with the pressures of planes k-1, k, k+1 in
// registers; xi and eta neighbours are read from the plane (cached).
__global__ __launch_bounds__(256) void k_sensor(const Geo g, const ZMarch zm, const double* __restrict__ P,
                                                double* __restrict__ theta) {
  int i, j, k0, k1;
  if (!zmarch_column(zm, g.n, &i, &j, &k0, &k1)) return;
  const int nz = g.n[2];
  const bool pz = g.periodic[2];
  const long long col = i + g.s[1] * j;
  auto plane = [&](int k) { return pz ? wrap(k, nz) : min(max(k, 0), nz - 1); };
  const long long xm = (long long)(wrap(i - 1, g.n[0]) - i), xp = (long long)(wrap(i + 1, g.n[0]) - i);
  const long long ym = (long long)(wrap(j - 1, g.n[1]) - j) * g.s[1], yp = (long long)(wrap(j + 1, g.n[1]) - j) * g.s[1];
  const bool xend = !g.periodic[0] && (i == 0 || i == g.n[0] - 1);
  const bool yend = !g.periodic[1] && (j == 0 || j == g.n[1] - 1);
  double pm = P[col + plane(k0 - 1) * g.s[2]];
  double p0 = P[col + (long long)k0 * g.s[2]];
  for (int k = k0; k < k1; ++k) {
    const long long id = col + (long long)k * g.s[2];
    const double pp = P[col + plane(k + 1) * g.s[2]];
    double th = 0.0;
    if (!xend) {
      const double a = P[id + xm], b = P[id + xp];
      th += fabs(-a + 2.0 * p0 - b) / (a + 2.0 * p0 + b);
    }
    if (!yend) {
      const double a = P[id + ym], b = P[id + yp];
      th += fabs(-a + 2.0 * p0 - b) / (a + 2.0 * p0 + b);
    }
    // a node at the end of a bounded line has no second difference there
    if (pz || (k != 0 && k != nz - 1)) th += fabs(-pm + 2.0 * p0 - pp) / (pm + 2.0 * p0 + pp);
    theta[id] = th;
    pm = p0;
    p0 = pp;
  }
}

hipError_t launch_sensor(const Geo& g, const double* P, double* theta, hipStream_t st) {
  const ZMarch zm = make_zmarch(g.n);
  hipLaunchKernelGGL(k_sensor, dim3(zm.blocks), dim3(256), 0, st, g, zm, P, theta);
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
  int pos[3];
  node_position(g, id, pos);
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
  int pos[3];
  node_position(g, id, pos);
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
constexpr int NRED = OCFD_RED_COUNT;

int reduce_blocks(const Geo& g) {
  long long b = (g.N + RED_T * 16 - 1) / (RED_T * 16);
  if (b < 1) b = 1;
  if (b > RED_MAX_BLOCKS) b = RED_MAX_BLOCKS;
  return (int)b;
}

// Combine two partial records (sums add; CFL max; p, rho min; counts add).
__device__ __forceinline__ void red_combine(double* a, const double* b) {
  for (int q = 0; q < 5; ++q) a[q] += b[q];
  a[5] = fmax(a[5], b[5]);
  a[6] = fmin(a[6], b[6]);
  a[7] = fmin(a[7], b[7]);
  a[8] += b[8];
  for (int d = 0; d < 3; ++d) a[9 + d] += b[9 + d];
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

// Entries 9..11 count the interfaces (node + 1/2 along d, where it exists)
// whose stencil was WENO: a nonzero flag or a bounded-end closure (flags null:
// no counts, the host fills in the fractions).
__global__ __launch_bounds__(RED_T) void k_reduce_partial(const Geo g, const Phys ph, const double* __restrict__ U,
                                                          const double* __restrict__ met, double dt,
                                                          const uint8_t* __restrict__ flags,
                                                          double* __restrict__ partial) {
  __shared__ double sh[NRED][RED_T];
  const long long N = g.N;
  double acc[NRED] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, INFINITY, INFINITY, 0.0, 0.0, 0.0, 0.0};
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
    if (flags) {
      int pq[3];
      node_position(g, id, pq);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int n = g.n[d];
        if (!g.periodic[d] && pq[d] == n - 1) continue;   // no interface at the last node
        const bool closure = !g.periodic[d] && (pq[d] < 3 || pq[d] > n - 5);
        acc[9 + d] += (closure || flags[d * N + id] != 0) ? 1.0 : 0.0;
      }
    }
  }
  block_reduce(sh, acc, partial + (long long)blockIdx.x * NRED);
}

__global__ __launch_bounds__(RED_T) void k_reduce_final(const double* __restrict__ partial, int nb,
                                                        double* __restrict__ out) {
  __shared__ double sh[NRED][RED_T];
  double acc[NRED] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, INFINITY, INFINITY, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += RED_T) red_combine(acc, partial + (long long)b * NRED);
  block_reduce(sh, acc, out);
}

hipError_t launch_reduce(const Geo& g, const Phys& ph, const double* U, const double* met, double dt,
                         const uint8_t* flags, double* partial, int nblocks, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partial, dim3(nblocks), dim3(RED_T), 0, st, g, ph, U, met, dt, flags, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_T), 0, st, partial, nblocks, out);
  return hipGetLastError();
}

}  // namespace ocfd
