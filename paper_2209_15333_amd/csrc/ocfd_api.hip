// C ABI of the ocfd library (declared in include/ocfd.h).  Host-side
// bookkeeping only: parameter checks, workspace carving, the order of kernel
// launches within a Runge-Kutta substep (eq 45) and optional event timing.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "ocfd_internal.h"

using namespace ocfd;

struct ocfd_solver {
  ocfd_params p;
  Geo g;
  Phys ph;
  hipStream_t st = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  double* met = nullptr;
  double* Ub[3] = {nullptr, nullptr, nullptr};  // [0] = U^n; [1], [2] = stage values
  double* rhs = nullptr;
  double* P = nullptr;            // [N] pressure (plain sensor)
  double* Fv = nullptr;
  double* theta = nullptr;
  double* partial = nullptr;
  double* red = nullptr;
  const uint8_t* flags = nullptr;
  // learned sensor
  uint16_t* feat = nullptr;       // [N][4] node features, bf16
  uint8_t* lflags = nullptr;      // [3][N] learned flags
  uint8_t* pflags = nullptr;      // [3][N] plain flags (audit, collection)
  const uint8_t* last_flags = nullptr;  // flags the last right-hand side read (hybrid)
  bool rhs_done = false;          // a right-hand side has been evaluated since creation or set_flags
  float* mlp = nullptr;           // [NPARAM] FP32 master weights
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  float* grad = nullptr;          // [NPARAM + 1]
  double* eloss = nullptr;        // running sum of the batch losses of a training epoch
  float* gpartial = nullptr;      // [GRAD_BLOCKS][NPARAM + 1]
  unsigned long long* cnt = nullptr;   // [COUNT_BLOCKS * 4]
  double* inflow = nullptr;       // [5][face] of the INFLOW face
  bool have_inflow = false;
  bool mlp_ready = false;
  double tau[3] = {0.5, 0.5, 0.5};   // learned-sensor threshold per direction
  int adam_t = 0;
  long long substep = 0;
  double audit[6] = {0, 0, 0, 0, 0, 0};
  char* smp = nullptr;            // caller-bound sample buffer
  long long smp_cap = 0, smp_n = 0;
  int stage = 0;
  bool have_grid = false;
  bool have_state = false;
  bool prof = false;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  std::string err;
};

namespace {

int fail(ocfd_solver* s, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(ocfd_solver* s, int code, const char* fmt, ...) {
  if (s) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    s->err = buf;
  }
  return code;
}

int hip_fail(ocfd_solver* s, hipError_t e, const char* what) {
  return fail(s, OCFD_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Field-region sizes of the workspace, in doubles per node.
constexpr int WS_MET = 10, WS_STATE = 5, WS_RHS = 5, WS_PRES = 1, WS_FV = 12, WS_THETA = 1;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

constexpr int GRAD_BLOCKS = 64;     // workgroups of one training step
constexpr int COUNT_BLOCKS = 1024;  // workgroups of the collection / flag-count passes

// Parameter check; *code receives the error code of a rejected set
// (BADARG, or UNSUPPORTED for a combination that is not built).
bool valid_params(const ocfd_params* p, std::string* why, int* code = nullptr) {
  char buf[256];
  if (code) *code = OCFD_ERR_BADARG;
  if (!p) { *why = "null params"; return false; }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1 || p->nx > 65535 || p->ny > 65535 || p->nz > 65535) {
    snprintf(buf, sizeof(buf), "grid %d x %d x %d outside [1, 65535]", p->nx, p->ny, p->nz);
    *why = buf;
    return false;
  }
  if ((long long)p->nx * p->ny * p->nz >= (1ll << 31)) { *why = "grid of 2^31 nodes or more"; return false; }
  for (int d = 0; d < 3; ++d)
    if (!(p->h[d] > 0.0) || !std::isfinite(p->h[d])) { *why = "h must be positive and finite"; return false; }
  if (!(p->gamma > 1.0)) { *why = "gamma must exceed 1"; return false; }
  if (!(p->Ma > 0.0)) { *why = "Ma must be positive"; return false; }
  if (p->viscous != 0 && p->viscous != 6 && p->viscous != 8) { *why = "viscous must be 0, 6 or 8"; return false; }
  if (p->viscous && !(p->Re > 0.0 && p->Pr > 0.0 && p->Tref > 0.0 && p->suth >= 0.0)) {
    *why = "Re, Pr, Tref must be positive and suth non-negative";
    return false;
  }
  if (p->scheme != OCFD_SCHEME_WENO7 && p->scheme != OCFD_SCHEME_HYBRID) { *why = "unknown scheme"; return false; }
  if (p->lowdiss != OCFD_LOWDISS_UD7 && p->lowdiss != OCFD_LOWDISS_C8) { *why = "unknown lowdiss"; return false; }
  if (!(p->weno_eps > 0.0)) { *why = "weno_eps must be positive"; return false; }
  if (p->precision != OCFD_PREC_FP64 && p->precision != OCFD_PREC_MIXED) { *why = "unknown precision"; return false; }
  if (p->sensor != OCFD_SENSOR_PLAIN && p->sensor != OCFD_SENSOR_LEARNED) { *why = "unknown sensor"; return false; }
  if (p->sensor_every < 0 || p->audit_every < 0) { *why = "sensor_every and audit_every must be >= 0"; return false; }
  if (p->three_way != 0 && p->three_way != 1) { *why = "three_way must be 0 or 1"; return false; }
  if (p->three_way && !(p->theta2 >= p->theta1)) { *why = "three_way needs theta2 >= theta1"; return false; }
  if (p->characteristic != 0 && p->characteristic != 1) { *why = "characteristic must be 0 or 1"; return false; }
  if (p->check_every < 0) { *why = "check_every must be >= 0"; return false; }
  if (p->flag_window != 0 && p->flag_window != 1) { *why = "flag_window must be 0 or 1"; return false; }
  if (!(p->cfl_max >= 0.0 && std::isfinite(p->cfl_max))) { *why = "cfl_max must be finite and >= 0"; return false; }
  if (p->sensor_inputs != OCFD_INPUTS_JUMP && p->sensor_inputs != OCFD_INPUTS_CURV) {
    *why = "unknown sensor_inputs";
    return false;
  }
  if (p->scheme == OCFD_SCHEME_HYBRID && p->sensor == OCFD_SENSOR_LEARNED && p->three_way) {
    // the network decides low-dissipation / WENO7 only; its audit fallback
    // could not tell the plain sensor's WENO5 tier apart
    *why = "the learned sensor decides two ways: three_way needs the plain sensor";
    if (code) *code = OCFD_ERR_UNSUPPORTED;
    return false;
  }
  int ninflow = 0;
  const int n[3] = {p->nx, p->ny, p->nz};
  for (int d = 0; d < 3; ++d) {
    if (p->periodic[d] != 0 && p->periodic[d] != 1) { *why = "periodic flags must be 0 or 1"; return false; }
    if (p->periodic[d]) continue;
    if (n[d] < 8) {
      snprintf(buf, sizeof(buf), "bounded direction %d has %d nodes; at least 8 needed", d, n[d]);
      *why = buf;
      return false;
    }
    for (int side = 0; side < 2; ++side) {
      const int k = p->bc[2 * d + side];
      if (k < OCFD_BC_NONE || k > OCFD_BC_NRBC) { *why = "unknown boundary kind"; return false; }
      if (k == OCFD_BC_INFLOW) ++ninflow;
      if (k == OCFD_BC_WALL && !(p->Tw > 0.0 && std::isfinite(p->Tw))) {
        *why = "a wall face needs Tw > 0";
        return false;
      }
    }
  }
  if (ninflow > 1) { *why = "at most one inflow face"; return false; }
  return true;
}

// Face index (0..5) of the INFLOW face, or -1.
int inflow_face(const ocfd_params& p) {
  for (int f = 0; f < 6; ++f)
    if (!p.periodic[f / 2] && p.bc[f] == OCFD_BC_INFLOW) return f;
  return -1;
}

// Nodes on a face normal to direction d.
long long face_nodes(const ocfd_params& p, int d) {
  const long long n[3] = {p.nx, p.ny, p.nz};
  return n[d == 0 ? 1 : 0] * n[d == 2 ? 1 : 2];
}

bool all_periodic(const ocfd_params& p) { return p.periodic[0] && p.periodic[1] && p.periodic[2]; }

// Interfaces whose scheme a sensor decides: all of a periodic line, and on a
// bounded line those whose 8-node window stays inside (n - 7 of them).
long long decided_interfaces(const Geo& g) {
  long long t = 0;
  for (int d = 0; d < 3; ++d) {
    const long long lines = g.N / g.n[d];
    t += lines * (g.periodic[d] ? g.n[d] : std::max(0, g.n[d] - 7));
  }
  return t;
}

void geo_phys_of(const ocfd_params& p, Geo* geo, Phys* phys) {
  Geo& g = *geo;
  g.n[0] = p.nx;
  g.n[1] = p.ny;
  g.n[2] = p.nz;
  g.s[0] = 1;
  g.s[1] = p.nx;
  g.s[2] = (long long)p.nx * p.ny;
  g.N = (long long)p.nx * p.ny * p.nz;
  for (int d = 0; d < 3; ++d) g.periodic[d] = p.periodic[d];
  for (int f = 0; f < 6; ++f) g.setface[f] = !p.periodic[f / 2] && p.bc[f] != OCFD_BC_NRBC;
  g.div[0] = make_fastdiv((uint32_t)p.nx);
  g.div[1] = make_fastdiv((uint32_t)p.ny);
  Phys& ph = *phys;
  ph.gamma = p.gamma;
  ph.gm1 = p.gamma - 1.0;
  ph.inv_gm1 = 1.0 / (p.gamma - 1.0);
  ph.inv_2g = 1.0 / (2.0 * p.gamma);
  ph.Ma2 = p.Ma * p.Ma;
  ph.inv_Re = p.viscous ? 1.0 / p.Re : 0.0;
  ph.kcoef = p.viscous ? 1.0 / ((p.gamma - 1.0) * p.Ma * p.Ma * p.Pr * p.Re) : 0.0;
  ph.suth = p.viscous ? p.suth / p.Tref : 0.0;
  ph.eps = p.weno_eps;
  ph.theta1 = p.theta1;
  ph.theta2 = p.theta2;
  ph.three_way = p.three_way;
  ph.flag_window = p.flag_window;
  ph.curv_inputs = p.sensor_inputs == OCFD_INPUTS_CURV;
  ph.vh = p.viscous == 8 ? 4 : 3;
  for (int d = 0; d < 3; ++d) {
    ph.h[d] = p.h[d];
    ph.ih[d] = 1.0 / p.h[d];
    ph.period[d] = p.period[d];
  }
}

void setup_geo_phys(ocfd_solver* s) { geo_phys_of(s->p, &s->g, &s->ph); }

size_t workspace_layout(const ocfd_params* p, long long N, int nred, ocfd_solver* s, char* base) {
  size_t off = 0;
  // Consecutive arrays are staggered by 64 KB + 2304 B: with power-of-two
  // field sizes every array would otherwise start at the same offset modulo
  // 1 GB; the stagger made the eta and zeta sweeps and the viscous fluxes
  // 3-5% faster on the 2048 x 256 x 256 ramp (measured).
  auto take = [&](size_t bytes) {
    char* ptr = base ? base + off : nullptr;
    off += align256(bytes) + 65536 + 2304;
    return (double*)ptr;
  };
  const size_t fb = (size_t)N * sizeof(double);
  double* met = take(WS_MET * fb);
  double* u0 = take(WS_STATE * fb);
  double* u1 = take(WS_STATE * fb);
  double* u2 = take(WS_STATE * fb);
  double* rhs = take(WS_RHS * fb);
  double* pres = take(WS_PRES * fb);
  double* Fv = take(WS_FV * fb);
  double* th = take(WS_THETA * fb);
  double* partial = take((size_t)nred * OCFD_RED_COUNT * sizeof(double));
  double* red = take(16 * sizeof(double));
  uint16_t* feat = (uint16_t*)take(4 * (size_t)N * sizeof(uint16_t));
  uint8_t* lflags = (uint8_t*)take(3 * (size_t)N);
  uint8_t* pflags = (uint8_t*)take(3 * (size_t)N);
  float* mlp = (float*)take(MLP_NPARAM * sizeof(float));
  float* am = (float*)take(MLP_NPARAM * sizeof(float));
  float* av = (float*)take(MLP_NPARAM * sizeof(float));
  float* grad = (float*)take((MLP_NPARAM + 1) * sizeof(float));
  double* eloss = take(sizeof(double));
  float* gpart = (float*)take((size_t)GRAD_BLOCKS * (MLP_NPARAM + 1) * sizeof(float));
  unsigned long long* cnt = (unsigned long long*)take((size_t)COUNT_BLOCKS * 4 * sizeof(unsigned long long));
  const int fin = inflow_face(*p);
  double* inflow = fin >= 0 ? take(5 * (size_t)face_nodes(*p, fin / 2) * sizeof(double)) : nullptr;
  if (s) {
    s->met = met;
    s->Ub[0] = u0;
    s->Ub[1] = u1;
    s->Ub[2] = u2;
    s->rhs = rhs;
    s->P = pres;
    s->Fv = Fv;
    s->theta = th;
    s->partial = partial;
    s->red = red;
    s->feat = feat;
    s->lflags = lflags;
    s->pflags = pflags;
    s->mlp = mlp;
    s->adam_m = am;
    s->adam_v = av;
    s->grad = grad;
    s->eloss = eloss;
    s->gpartial = gpart;
    s->cnt = cnt;
    s->inflow = inflow;
  }
  return off;
}

// Launch bracket for the optional timing.
struct Timed {
  ocfd_solver* s;
  int cls;
  hipEvent_t a = nullptr, b = nullptr;
  hipEvent_t get() {
    if (!s->pool.empty()) {
      hipEvent_t e = s->pool.back();
      s->pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  Timed(ocfd_solver* s_, int c) : s(s_), cls(c) {
    if (s->prof) {
      a = get();
      b = get();
      if (a) (void)hipEventRecord(a, s->st);
    }
  }
  ~Timed() {
    if (s->prof && a && b) {
      (void)hipEventRecord(b, s->st);
      s->recs.push_back({cls, a, b});
    }
  }
};

bool ready(ocfd_solver* s, int* rc) {
  if (!s) { *rc = OCFD_ERR_BADARG; return false; }
  if (!s->ws) { *rc = fail(s, OCFD_ERR_STATE, "no workspace bound"); return false; }
  return true;
}

Tau3 tau3(const ocfd_solver* s) {
  Tau3 t;
  for (int d = 0; d < 3; ++d) t.t[d] = (float)s->tau[d];
  return t;
}

// Node sensor theta of U into s->theta (the pressure of U into s->P first).
int plain_theta(ocfd_solver* s, const double* U) {
  hipError_t e;
  {
    Timed tm(s, OCFD_K_PRIM);
    e = launch_pressure(s->g, s->ph, U, s->P, s->st);
  }
  if (e == hipSuccess) {
    Timed tm(s, OCFD_K_OTHER);
    e = launch_sensor(s->g, s->P, s->theta, s->st);
  }
  return e == hipSuccess ? OCFD_OK : hip_fail(s, e, "sensor kernels");
}

// Evaluate the right-hand side of U_cur.  mode MODE_RK writes the next stage
// into out; MODE_DUDT writes dU/dt into out.
// Flags of the learned sensor for this substep: the network is re-evaluated
// every sensor_every substeps; every audit_every substeps the plain sensor is
// evaluated too, and interfaces it marks but the network missed fall back to
// WENO (the union of both flag fields is used).
int learned_flags(ocfd_solver* s, const double* Ucur, bool count_substep) {
  if (!s->mlp_ready) return fail(s, OCFD_ERR_STATE, "learned sensor selected but no network parameters set");
  hipError_t e = hipSuccess;
  const long long k = s->substep;
  const int every = s->p.sensor_every > 0 ? s->p.sensor_every : 1;
  if (!count_substep || k % every == 0) {
    Timed tm(s, OCFD_K_OTHER);
    e = launch_features(s->g, s->ph, Ucur, s->met, s->feat, s->st);
    if (e == hipSuccess) e = launch_mlp_flags(s->g, s->feat, s->mlp, tau3(s), s->lflags, s->st);
    if (e != hipSuccess) return hip_fail(s, e, "learned sensor kernels");
  }
  if (count_substep && s->p.audit_every > 0 && k % s->p.audit_every == 0) {
    int rc = plain_theta(s, Ucur);
    if (rc) return rc;
    e = launch_plain_flags(s->g, s->ph, s->theta, s->pflags, s->st);
    if (e == hipSuccess) e = launch_flag_stats(s->g, s->pflags, s->lflags, s->cnt, COUNT_BLOCKS, s->st);
    std::vector<unsigned long long> c(COUNT_BLOCKS * 4);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c.data(), s->cnt, c.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return hip_fail(s, e, "sensor audit");
    unsigned long long plain = 0, missed = 0, extra = 0, mism = 0;
    for (int b = 0; b < COUNT_BLOCKS; ++b) {
      plain += c[4 * b];
      missed += c[4 * b + 2];   // plain WENO, learned low
      extra += c[4 * b + 1];
      mism += c[4 * b + 3];
    }
    s->audit[0] += 1;
    s->audit[1] += (double)decided_interfaces(s->g);
    s->audit[2] += (double)plain;
    s->audit[3] += (double)(plain - missed + extra);
    s->audit[4] += (double)missed;
    s->audit[5] += (double)mism;
    if (missed) {
      e = launch_flags_or(s->lflags, s->pflags, 3 * s->g.N, s->st);
      if (e != hipSuccess) return hip_fail(s, e, "flag union");
    }
  }
  return OCFD_OK;
}

int run_rhs(ocfd_solver* s, const double* Ucur, int mode, double* out, const double* Un, double a, double b,
            double dt, int parts, bool count_substep = false) {
  hipError_t e;
  const bool visc = s->p.viscous && (parts & OCFD_PART_VISC);
  const bool hyb = s->p.scheme == OCFD_SCHEME_HYBRID;
  // Where the viscous derivative goes: the FP32 and hybrid sweeps stage the
  // viscous fluxes of their direction in an LDS ring and add the derivative
  // in their finishing step; the FP64 WENO7 sweep keeps its occupancy instead,
  // and a separate kernel writes the whole divergence first (the sweeps then
  // accumulate onto it).
  const bool vdiv = visc && !hyb && s->p.precision != OCFD_PREC_MIXED;
  if (visc) {
    {
      Timed tm(s, OCFD_K_VISC);
      e = launch_visc_flux(s->g, s->ph, Ucur, s->met, s->Fv, s->st);
      // the divergence of the viscous fluxes opens the sum the sweeps add to
      if (e == hipSuccess && vdiv) e = launch_visc_div(s->g, s->ph, s->Fv, s->rhs, s->st);
    }
    if (e != hipSuccess) return hip_fail(s, e, "viscous flux kernel");
  }
  const uint8_t* flags = s->flags;
  if (hyb && !flags && s->p.sensor == OCFD_SENSOR_LEARNED) {
    int rc = learned_flags(s, Ucur, count_substep);
    if (rc) return rc;
    flags = s->lflags;
  } else if (hyb && !flags) {
    int rc = plain_theta(s, Ucur);
    if (rc) return rc;
    {
      Timed tm(s, OCFD_K_OTHER);
      e = launch_plain_flags(s->g, s->ph, s->theta, s->pflags, s->st);
    }
    if (e != hipSuccess) return hip_fail(s, e, "sensor flags kernel");
    flags = s->pflags;
  }
  s->last_flags = hyb ? flags : nullptr;
  s->rhs_done = true;
  SweepArgs A;
  memset(&A, 0, sizeof(A));
  A.g = s->g;
  A.ph = s->ph;
  A.U = Ucur;
  A.met = s->met;
  A.Fv = visc && !vdiv ? s->Fv : nullptr;
  A.flags = flags;
  A.rhs = s->rhs;
  A.Un = Un;
  A.out = out;
  A.a = a;
  A.b = b;
  A.dt = dt;
  A.hybrid = hyb ? 1 : 0;
  A.lowdiss = s->p.lowdiss;
  A.mixed = s->p.precision == OCFD_PREC_MIXED ? 1 : 0;
  A.characteristic = s->p.characteristic;
  // zeta first (stores the sum, or adds to the viscous divergence), eta
  // accumulates, xi last: the last sweep reads and writes the most (sum, U^n,
  // 1/J, output), and along xi those accesses are contiguous.
  for (int step = 0; step < 3; ++step) {
    const int d = 2 - step;
    A.inviscid = (parts >> d) & 1;
    A.viscous = visc && !vdiv ? 1 : 0;
    const int m = step == 0 ? (vdiv ? MODE_ADD : MODE_SET) : (step == 1 ? MODE_ADD : mode);
    Timed tm(s, OCFD_K_SWEEP_XI + d);
    e = launch_sweep(d, m, A, s->st);
    if (e != hipSuccess) return hip_fail(s, e, "sweep kernel");
  }
  // normal-direction part of the nonreflecting faces, added to the stage
  // (b dt) or to dU/dt
  for (int f = 0; f < 6; ++f) {
    const int d = f / 2;
    if (s->p.periodic[d] || s->p.bc[f] != OCFD_BC_NRBC || !((parts >> d) & 1)) continue;
    Timed tm(s, OCFD_K_OTHER);
    e = launch_nrbc(s->g, s->ph, Ucur, s->met, out, d, f % 2, mode == MODE_RK ? b * dt : 1.0, s->st);
    if (e != hipSuccess) return hip_fail(s, e, "nonreflecting face kernel");
  }
  return OCFD_OK;
}

// Faces of the bounded directions of U, in the order xi-, xi+, eta-, eta+,
// zeta-, zeta+ (a corner node takes the value of the last face through it).
int apply_bc(ocfd_solver* s, double* U) {
  for (int f = 0; f < 6; ++f) {
    const int d = f / 2;
    if (s->p.periodic[d] || s->p.bc[f] == OCFD_BC_NONE || s->p.bc[f] == OCFD_BC_NRBC) continue;
    Timed tm(s, OCFD_K_OTHER);
    hipError_t e = launch_bc(s->g, s->ph, U, d, f % 2, s->p.bc[f], s->p.Tw, s->inflow, s->st);
    if (e != hipSuccess) return hip_fail(s, e, "boundary kernel");
  }
  return OCFD_OK;
}

// The state check of ocfd_advance: the reduction of the current state, then
// non-finite values or a non-positive density or pressure (NONFINITE) and the
// CFL number against cfl_max (CFL).  Synchronises.
int check_state(ocfd_solver* s, double dt) {
  hipError_t e = launch_reduce(s->g, s->ph, s->Ub[s->stage], s->met, dt, nullptr, s->partial, reduce_blocks(s->g),
                               s->red, s->st);
  double r[OCFD_RED_COUNT];
  if (e == hipSuccess) e = hipMemcpyAsync(r, s->red, sizeof(r), hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return hip_fail(s, e, "state check");
  if (r[OCFD_RED_NONFINITE] > 0.0 || !(r[OCFD_RED_RHOMIN] > 0.0) || !(r[OCFD_RED_PMIN] > 0.0))
    return fail(s, OCFD_ERR_NONFINITE,
                "state after substep %lld: %.0f non-finite conserved values, min density %g, min pressure %g",
                s->substep, r[OCFD_RED_NONFINITE], r[OCFD_RED_RHOMIN], r[OCFD_RED_PMIN]);
  if (s->p.cfl_max > 0.0 && !(r[OCFD_RED_CFL] <= s->p.cfl_max))
    return fail(s, OCFD_ERR_CFL, "state after substep %lld: CFL number %g above the limit %g", s->substep,
                r[OCFD_RED_CFL], s->p.cfl_max);
  return OCFD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Reduction without allocation (ocfd_reduce_static): the partial records live
// in a fixed array in device memory, one copy per GPU, held until the process
// ends.  Host code never passes the array's name to a kernel (in host code it
// is only a stand-in for the symbol): the device address of each GPU's copy is
// looked up once per device, with that device current, and kept here.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[RED_MAX_BLOCKS * OCFD_RED_COUNT];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_dev[MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch` (null on error).
double* scratch_of_current_device(hipError_t* err) {
  int dev = -1;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  if (dev < 0 || dev >= MAX_DEVICES) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* ptr = nullptr;
    *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    scratch_dev[dev] = (double*)ptr;
  }
  return scratch_dev[dev];
}

// The parameters the reduction reads, checked without allocating.
bool reduce_params_ok(const ocfd_params* p) {
  if (p->nx < 1 || p->ny < 1 || p->nz < 1 || p->nx > 65535 || p->ny > 65535 || p->nz > 65535) return false;
  if ((long long)p->nx * p->ny * p->nz >= (1ll << 31)) return false;
  for (int d = 0; d < 3; ++d) {
    if (!(p->h[d] > 0.0) || !std::isfinite(p->h[d])) return false;
    if (p->periodic[d] != 0 && p->periodic[d] != 1) return false;
  }
  return p->gamma > 1.0 && std::isfinite(p->gamma);
}

}  // namespace

extern "C" {

int ocfd_params_default(ocfd_params* p) {
  if (!p) return OCFD_ERR_BADARG;
  memset(p, 0, sizeof(*p));
  p->nx = p->ny = p->nz = 1;
  for (int d = 0; d < 3; ++d) {
    p->periodic[d] = 1;
    p->period[d] = 1.0;
    p->h[d] = 1.0;
  }
  p->Tw = 1.0;
  p->gamma = 1.4;
  p->Re = 1600.0;
  p->Ma = 0.1;
  p->Pr = 0.72;
  p->Tref = 288.15;
  p->suth = 110.4;
  p->theta1 = 0.02;
  p->theta2 = 0.1;
  p->weno_eps = 1e-6;
  p->viscous = 6;
  p->scheme = OCFD_SCHEME_WENO7;
  p->lowdiss = OCFD_LOWDISS_C8;
  p->sensor = OCFD_SENSOR_PLAIN;
  p->sensor_every = 1;
  p->audit_every = 0;
  return OCFD_OK;
}

size_t ocfd_workspace_bytes(const ocfd_params* p) {
  std::string why;
  if (!valid_params(p, &why)) return 0;
  ocfd_solver tmp;
  tmp.p = *p;
  setup_geo_phys(&tmp);
  return workspace_layout(p, tmp.g.N, reduce_blocks(tmp.g), nullptr, nullptr);
}

int ocfd_create(const ocfd_params* p, void* stream, ocfd_solver** out) {
  if (!out) return OCFD_ERR_BADARG;
  *out = nullptr;
  std::string why;
  int code = OCFD_ERR_BADARG;
  if (!valid_params(p, &why, &code)) {
    fprintf(stderr, "ocfd_create: %s\n", why.c_str());
    return code;
  }
  ocfd_solver* s = new (std::nothrow) ocfd_solver();
  if (!s) return OCFD_ERR_BADARG;
  s->p = *p;
  s->st = (hipStream_t)stream;
  setup_geo_phys(s);
  *out = s;
  return OCFD_OK;
}

int ocfd_bind_workspace(ocfd_solver* s, void* ws, size_t bytes) {
  if (!s) return OCFD_ERR_BADARG;
  if (!ws) return fail(s, OCFD_ERR_BADARG, "null workspace");
  if (((uintptr_t)ws) & 255) return fail(s, OCFD_ERR_BADARG, "workspace not 256-byte aligned");
  const size_t need = workspace_layout(&s->p, s->g.N, reduce_blocks(s->g), nullptr, nullptr);
  if (bytes < need) return fail(s, OCFD_ERR_BADSIZE, "workspace of %zu bytes, %zu needed", bytes, need);
  s->ws = (char*)ws;
  s->ws_bytes = bytes;
  workspace_layout(&s->p, s->g.N, reduce_blocks(s->g), s, s->ws);
  s->have_grid = false;
  s->have_state = false;
  s->have_inflow = false;
  return OCFD_OK;
}

int ocfd_set_inflow(ocfd_solver* s, const double* inflow) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!inflow) return fail(s, OCFD_ERR_BADARG, "null inflow");
  const int f = inflow_face(s->p);
  if (f < 0) return fail(s, OCFD_ERR_UNSUPPORTED, "no inflow face");
  hipError_t e = hipMemcpyAsync(s->inflow, inflow, 5 * face_nodes(s->p, f / 2) * sizeof(double),
                                hipMemcpyDeviceToDevice, s->st);
  if (e != hipSuccess) return hip_fail(s, e, "inflow copy");
  s->have_inflow = true;
  return OCFD_OK;
}

int ocfd_set_grid(ocfd_solver* s, const double* xyz) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!xyz) return fail(s, OCFD_ERR_BADARG, "null coordinates");
  // The viscous-flux region (12 N) is scratch for the 9 inner derivatives.
  Timed tm(s, OCFD_K_OTHER);
  hipError_t e = launch_metric_inner(s->g, s->ph, xyz, s->Fv, s->st);
  if (e == hipSuccess) e = launch_metric_outer(s->g, s->ph, xyz, s->Fv, s->met, s->st);
  if (e != hipSuccess) return hip_fail(s, e, "metric kernels");
  s->have_grid = true;
  return OCFD_OK;
}

int ocfd_set_metrics(ocfd_solver* s, const double* met) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!met) return fail(s, OCFD_ERR_BADARG, "null metrics");
  hipError_t e = hipMemcpyAsync(s->met, met, 10 * s->g.N * sizeof(double), hipMemcpyDeviceToDevice, s->st);
  if (e != hipSuccess) return hip_fail(s, e, "metrics copy");
  s->have_grid = true;
  return OCFD_OK;
}

int ocfd_get_metrics(ocfd_solver* s, double* met) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!met) return fail(s, OCFD_ERR_BADARG, "null metrics");
  if (!s->have_grid) return fail(s, OCFD_ERR_STATE, "no grid set");
  hipError_t e = hipMemcpyAsync(met, s->met, 10 * s->g.N * sizeof(double), hipMemcpyDeviceToDevice, s->st);
  return e == hipSuccess ? OCFD_OK : hip_fail(s, e, "metrics copy");
}

int ocfd_set_state(ocfd_solver* s, const double* U) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!U) return fail(s, OCFD_ERR_BADARG, "null state");
  hipError_t e = hipMemcpyAsync(s->Ub[0], U, 5 * s->g.N * sizeof(double), hipMemcpyDeviceToDevice, s->st);
  if (e != hipSuccess) return hip_fail(s, e, "state copy");
  s->stage = 0;
  s->substep = 0;
  s->have_state = true;
  return OCFD_OK;
}

int ocfd_get_state(ocfd_solver* s, double* U) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!U) return fail(s, OCFD_ERR_BADARG, "null state");
  if (!s->have_state) return fail(s, OCFD_ERR_STATE, "no state set");
  hipError_t e = hipMemcpyAsync(U, s->Ub[s->stage], 5 * s->g.N * sizeof(double), hipMemcpyDeviceToDevice, s->st);
  return e == hipSuccess ? OCFD_OK : hip_fail(s, e, "state copy");
}

int ocfd_get_step_state(ocfd_solver* s, double* Un, int32_t* stage) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!Un || !stage) return fail(s, OCFD_ERR_BADARG, "null argument");
  if (!s->have_state) return fail(s, OCFD_ERR_STATE, "no state set");
  hipError_t e = hipMemcpyAsync(Un, s->Ub[0], 5 * s->g.N * sizeof(double), hipMemcpyDeviceToDevice, s->st);
  *stage = s->stage;
  return e == hipSuccess ? OCFD_OK : hip_fail(s, e, "state copy");
}

int ocfd_set_step_state(ocfd_solver* s, const double* U, const double* Un, int32_t stage) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!U || !Un) return fail(s, OCFD_ERR_BADARG, "null state");
  if (stage < 0 || stage > 2) return fail(s, OCFD_ERR_BADARG, "stage %d not in 0..2", stage);
  const size_t b = 5 * s->g.N * sizeof(double);
  hipError_t e = hipMemcpyAsync(s->Ub[0], Un, b, hipMemcpyDeviceToDevice, s->st);
  if (e == hipSuccess && stage > 0) e = hipMemcpyAsync(s->Ub[stage], U, b, hipMemcpyDeviceToDevice, s->st);
  if (e != hipSuccess) return hip_fail(s, e, "state copy");
  s->stage = stage;
  s->substep = stage;
  s->have_state = true;
  return OCFD_OK;
}

int ocfd_advance(ocfd_solver* s, int32_t n, double dt) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (n < 0 || !std::isfinite(dt)) return fail(s, OCFD_ERR_BADARG, "bad substep count or dt");
  if (!s->have_grid || !s->have_state) return fail(s, OCFD_ERR_STATE, "grid and state must be set first");
  if (inflow_face(s->p) >= 0 && !s->have_inflow) return fail(s, OCFD_ERR_STATE, "inflow face without inflow state");
  static const double A[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
  static const double B[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};
  for (int i = 0; i < n; ++i) {
    const int k = s->stage;
    const double* cur = s->Ub[k];
    double* nxt = s->Ub[(k + 1) % 3];
    rc = run_rhs(s, cur, MODE_RK, nxt, s->Ub[0], A[k], B[k], dt, OCFD_PART_ALL, true);
    if (rc) return rc;
    if (!all_periodic(s->p)) {
      rc = apply_bc(s, nxt);
      if (rc) return rc;
    }
    s->stage = (k + 1) % 3;
    s->substep += 1;
    if (s->p.check_every > 0 && s->substep % s->p.check_every == 0) {
      rc = check_state(s, dt);
      if (rc) return rc;
    }
  }
  return OCFD_OK;
}

int64_t ocfd_substeps_done(const ocfd_solver* s) { return s ? (int64_t)s->substep : -1; }

int ocfd_dudt(ocfd_solver* s, const double* U, double* out, int32_t parts) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!U || !out) return fail(s, OCFD_ERR_BADARG, "null argument");
  if (U == out) return fail(s, OCFD_ERR_BADARG, "U and dudt alias");
  if (parts < 0 || parts > OCFD_PART_ALL) return fail(s, OCFD_ERR_BADARG, "bad parts mask");
  if (!s->have_grid) return fail(s, OCFD_ERR_STATE, "no grid set");
  return run_rhs(s, U, MODE_DUDT, out, nullptr, 0.0, 0.0, 0.0, parts);
}

int ocfd_reduce(ocfd_solver* s, double dt, double* out) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!out) return fail(s, OCFD_ERR_BADARG, "null output");
  if (!s->have_grid || !s->have_state) return fail(s, OCFD_ERR_STATE, "grid and state must be set first");
  const bool hyb = s->p.scheme == OCFD_SCHEME_HYBRID;
  const uint8_t* fl = hyb && s->rhs_done ? s->last_flags : nullptr;
  hipError_t e = launch_reduce(s->g, s->ph, s->Ub[s->stage], s->met, dt, fl, s->partial, reduce_blocks(s->g),
                               s->red, s->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, s->red, OCFD_RED_COUNT * sizeof(double), hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return hip_fail(s, e, "reduction");
  // WENO fractions: counts over the interfaces that exist along each direction
  const int n[3] = {s->p.nx, s->p.ny, s->p.nz};
  for (int d = 0; d < 3; ++d) {
    const double total = (double)s->g.N - (s->p.periodic[d] ? 0.0 : (double)(s->g.N / n[d]));
    double& f = out[OCFD_RED_WENO0 + d];
    if (!hyb)
      f = 1.0;
    else if (!fl)
      f = NAN;
    else
      f = total > 0.0 ? f / total : 0.0;
  }
  return OCFD_OK;
}

int ocfd_reduce_static(const ocfd_params* p, const double* U, const double* met, double dt, double* out,
                       void* stream) {
  if (!p || !U || !met || !out || !std::isfinite(dt)) return OCFD_ERR_BADARG;
  if (!reduce_params_ok(p)) {
    fprintf(stderr, "ocfd_reduce_static: invalid grid or gas parameters\n");
    return OCFD_ERR_BADARG;
  }
  Geo g;
  Phys ph;
  geo_phys_of(*p, &g, &ph);
  const int nb = reduce_blocks(g);
  if (nb > RED_MAX_BLOCKS) {
    fprintf(stderr, "ocfd_reduce_static: %d partial records needed, the fixed array holds %d\n", nb,
            RED_MAX_BLOCKS);
    return OCFD_ERR_BADSIZE;
  }
  hipError_t e;
  double* part = scratch_of_current_device(&e);
  if (!part) {
    fprintf(stderr, "ocfd_reduce_static: device address of the partial array: %s\n", hipGetErrorString(e));
    return OCFD_ERR_HIP;
  }
  // every partial record the final pass reads is written by the first pass
  // of this call, so nothing left by an earlier call is read
  e = launch_reduce(g, ph, U, met, dt, nullptr, part, nb, out, (hipStream_t)stream);
  if (e != hipSuccess) {
    fprintf(stderr, "ocfd_reduce_static: launch: %s\n", hipGetErrorString(e));
    return OCFD_ERR_HIP;
  }
  return OCFD_OK;
}

int ocfd_set_flags(ocfd_solver* s, const uint8_t* flags) {
  if (!s) return OCFD_ERR_BADARG;
  s->flags = flags;
  s->last_flags = nullptr;   // the previous evaluation's flags may belong to a buffer being released
  s->rhs_done = false;
  return OCFD_OK;
}

int ocfd_profile(ocfd_solver* s, int32_t enable) {
  if (!s) return OCFD_ERR_BADARG;
  hipError_t e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return hip_fail(s, e, "stream sync");
  for (auto& r : s->recs) {
    s->pool.push_back(r.a);
    s->pool.push_back(r.b);
  }
  s->recs.clear();
  s->prof = enable != 0;
  return OCFD_OK;
}

int ocfd_profile_read(ocfd_solver* s, double* ms, int64_t* count) {
  if (!s || !ms || !count) return OCFD_ERR_BADARG;
  hipError_t e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return hip_fail(s, e, "stream sync");
  for (int k = 0; k < OCFD_K_COUNT; ++k) {
    ms[k] = 0.0;
    count[k] = 0;
  }
  for (auto& r : s->recs) {
    float t = 0.f;
    e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) return hip_fail(s, e, "event timing");
    ms[r.cls] += t;
    count[r.cls] += 1;
  }
  return OCFD_OK;
}

// ---------------------------------------------------------------- learned sensor

int32_t ocfd_sensor_nparams(void) { return MLP_NPARAM; }

int ocfd_sensor_set_params(ocfd_solver* s, const float* P) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!P) return fail(s, OCFD_ERR_BADARG, "null parameters");
  for (int k = 0; k < MLP_NPARAM; ++k)
    if (!std::isfinite(P[k])) return fail(s, OCFD_ERR_BADARG, "non-finite parameter %d", k);
  hipError_t e = hipMemcpyAsync(s->mlp, P, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice, s->st);
  if (e == hipSuccess) e = hipMemsetAsync(s->adam_m, 0, MLP_NPARAM * sizeof(float), s->st);
  if (e == hipSuccess) e = hipMemsetAsync(s->adam_v, 0, MLP_NPARAM * sizeof(float), s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return hip_fail(s, e, "parameter upload");
  s->adam_t = 0;
  s->mlp_ready = true;
  return OCFD_OK;
}

int ocfd_sensor_get_params(ocfd_solver* s, float* P) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!P) return fail(s, OCFD_ERR_BADARG, "null parameters");
  if (!s->mlp_ready) return fail(s, OCFD_ERR_STATE, "no network parameters set");
  hipError_t e = hipMemcpyAsync(P, s->mlp, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  return e == hipSuccess ? OCFD_OK : hip_fail(s, e, "parameter download");
}

int ocfd_sensor_set_threshold(ocfd_solver* s, double tau) {
  if (!s) return OCFD_ERR_BADARG;
  if (!(tau >= 0.0 && tau <= 1.0)) return fail(s, OCFD_ERR_BADARG, "threshold %g not in [0, 1]", tau);
  for (int d = 0; d < 3; ++d) s->tau[d] = tau;
  return OCFD_OK;
}

int ocfd_sensor_set_thresholds(ocfd_solver* s, const double* tau_host) {
  if (!s) return OCFD_ERR_BADARG;
  if (!tau_host) return fail(s, OCFD_ERR_BADARG, "null thresholds");
  for (int d = 0; d < 3; ++d)
    if (!(tau_host[d] >= 0.0 && tau_host[d] <= 1.0))
      return fail(s, OCFD_ERR_BADARG, "threshold %g of direction %d not in [0, 1]", tau_host[d], d);
  for (int d = 0; d < 3; ++d) s->tau[d] = tau_host[d];
  return OCFD_OK;
}

int ocfd_sensor_get_thresholds(ocfd_solver* s, double* tau_host) {
  if (!s) return OCFD_ERR_BADARG;
  if (!tau_host) return fail(s, OCFD_ERR_BADARG, "null output");
  for (int d = 0; d < 3; ++d) tau_host[d] = s->tau[d];
  return OCFD_OK;
}

int ocfd_sensor_flags(ocfd_solver* s, const double* U, int32_t which, uint8_t* flags) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!U || !flags) return fail(s, OCFD_ERR_BADARG, "null argument");
  if (!s->have_grid) return fail(s, OCFD_ERR_STATE, "no grid set");
  hipError_t e;
  if (which == OCFD_SENSOR_PLAIN) {
    rc = plain_theta(s, U);
    if (rc) return rc;
    e = launch_plain_flags(s->g, s->ph, s->theta, flags, s->st);
  } else if (which == OCFD_SENSOR_LEARNED) {
    if (!s->mlp_ready) return fail(s, OCFD_ERR_STATE, "no network parameters set");
    e = launch_features(s->g, s->ph, U, s->met, s->feat, s->st);
    if (e == hipSuccess) e = launch_mlp_flags(s->g, s->feat, s->mlp, tau3(s), flags, s->st);
  } else {
    return fail(s, OCFD_ERR_BADARG, "unknown sensor %d", which);
  }
  return e == hipSuccess ? OCFD_OK : hip_fail(s, e, "sensor kernels");
}

// Sample buffer layout for capacity C: X [C][32] bf16 | w [C] f32 | idx [C] i32 | prob [C] f32 | y [C] u8.
static size_t smp_off_w(long long C) { return (size_t)C * 64; }
static size_t smp_off_idx(long long C) { return smp_off_w(C) + (size_t)C * 4; }
static size_t smp_off_prob(long long C) { return smp_off_idx(C) + (size_t)C * 4; }
static size_t smp_off_y(long long C) { return smp_off_prob(C) + (size_t)C * 4; }

size_t ocfd_sensor_sample_bytes(int64_t capacity) { return capacity > 0 ? smp_off_y(capacity) + (size_t)capacity : 0; }

int ocfd_sensor_bind_samples(ocfd_solver* s, void* dev, size_t bytes) {
  if (!s) return OCFD_ERR_BADARG;
  if (!dev) return fail(s, OCFD_ERR_BADARG, "null sample buffer");
  if (((uintptr_t)dev) & 255) return fail(s, OCFD_ERR_BADARG, "sample buffer not 256-byte aligned");
  long long cap = (long long)(bytes / 77);
  while (cap > 0 && ocfd_sensor_sample_bytes(cap) > bytes) --cap;
  if (cap < 16) return fail(s, OCFD_ERR_BADSIZE, "sample buffer of %zu bytes holds fewer than 16 samples", bytes);
  s->smp = (char*)dev;
  s->smp_cap = cap;
  s->smp_n = 0;
  return OCFD_OK;
}

int ocfd_sensor_collect(ocfd_solver* s, uint64_t seed, double keep_weno, double keep_low, int64_t* total) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!total) return fail(s, OCFD_ERR_BADARG, "null output");
  if (!s->smp) return fail(s, OCFD_ERR_STATE, "no sample buffer bound");
  if (!s->have_grid || !s->have_state) return fail(s, OCFD_ERR_STATE, "grid and state must be set first");
  if (!(keep_weno >= 0 && keep_weno <= 1 && keep_low >= 0 && keep_low <= 1))
    return fail(s, OCFD_ERR_BADARG, "keep probabilities must be in [0, 1]");
  const uint32_t tp = (uint32_t)std::min(4294967295.0, keep_weno * 4294967296.0);
  const uint32_t tl = (uint32_t)std::min(4294967295.0, keep_low * 4294967296.0);
  const double* U = s->Ub[s->stage];
  rc = plain_theta(s, U);
  if (rc) return rc;
  hipError_t e = launch_plain_flags(s->g, s->ph, s->theta, s->pflags, s->st);
  if (e == hipSuccess) e = launch_features(s->g, s->ph, U, s->met, s->feat, s->st);
  if (e == hipSuccess) e = launch_collect_count(s->g, s->pflags, seed, tp, tl, s->cnt, COUNT_BLOCKS, s->st);
  std::vector<unsigned long long> c(COUNT_BLOCKS);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c.data(), s->cnt, COUNT_BLOCKS * sizeof(unsigned long long), hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return hip_fail(s, e, "sample count");
  unsigned long long acc = (unsigned long long)s->smp_n;
  for (int b = 0; b < COUNT_BLOCKS; ++b) {
    const unsigned long long v = c[b];
    c[b] = acc;
    acc += v;
  }
  e = hipMemcpyAsync(s->cnt, c.data(), COUNT_BLOCKS * sizeof(unsigned long long), hipMemcpyHostToDevice, s->st);
  const long long C = s->smp_cap;
  if (e == hipSuccess)
    e = launch_collect_write(s->g, s->pflags, s->feat, seed, tp, tl, s->cnt, C, (uint16_t*)s->smp,
                             (uint8_t*)(s->smp + smp_off_y(C)), (float*)(s->smp + smp_off_w(C)), COUNT_BLOCKS, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return hip_fail(s, e, "sample write");
  s->smp_n = (long long)std::min<unsigned long long>(acc, (unsigned long long)C);
  *total = s->smp_n;
  return OCFD_OK;
}

// One gradient evaluation (and Adam step when lr > 0) over nb samples listed in idx_dev.
static int grad_step(ocfd_solver* s, const uint16_t* X, const uint8_t* y, const float* w, const int* idx, long long nb,
                     float Wsum, float lr) {
  if (lr > 0.f) s->adam_t += 1;
  hipError_t e = launch_mlp_grad(X, y, w, idx, nb, Wsum, s->mlp, s->gpartial, GRAD_BLOCKS, s->grad, s->mlp,
                                 s->adam_m, s->adam_v, lr, s->adam_t, s->eloss, s->st);
  return e == hipSuccess ? OCFD_OK : hip_fail(s, e, "training kernels");
}

int ocfd_sensor_train(ocfd_solver* s, int32_t epochs, int32_t batch, float lr, uint64_t seed, double holdout,
                      double* stats) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!stats) return fail(s, OCFD_ERR_BADARG, "null output");
  if (!s->mlp_ready) return fail(s, OCFD_ERR_STATE, "set initial network parameters first");
  if (epochs < 1 || batch < 16 || !(lr > 0.f) || !(holdout >= 0.0 && holdout < 1.0))
    return fail(s, OCFD_ERR_BADARG, "bad training arguments");
  const long long C = s->smp_cap;
  const long long ntrain = (long long)((1.0 - holdout) * (double)s->smp_n);
  if (ntrain < batch) return fail(s, OCFD_ERR_STATE, "%lld training samples, fewer than one batch", ntrain);
  // Class balance: WENO samples are rare (a fraction of a percent of the
  // interfaces of a resolved flow), so each class gets the same total weight
  // (WENO samples weigh n_low / n_weno, at most 1000; low-dissipation ones 1).
  std::vector<uint8_t> hy(ntrain);
  hipError_t e = hipMemcpyAsync(hy.data(), s->smp + smp_off_y(C), ntrain, hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return hip_fail(s, e, "label download");
  long long npos = 0;
  for (long long k = 0; k < ntrain; ++k) npos += hy[k] & 1;
  const long long nneg = ntrain - npos;
  const float wpos = (npos > 0 && nneg > 0) ? (float)std::min(1000.0, (double)nneg / (double)npos) : 1.f;
  std::vector<float> hw(ntrain);
  for (long long k = 0; k < ntrain; ++k) hw[k] = (hy[k] & 1) ? wpos : 1.f;
  e = hipMemcpyAsync(s->smp + smp_off_w(C), hw.data(), ntrain * sizeof(float), hipMemcpyHostToDevice, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return hip_fail(s, e, "weight upload");
  std::vector<int> perm(ntrain);
  std::mt19937_64 rng(seed);
  int* didx = (int*)(s->smp + smp_off_idx(C));
  const uint16_t* X = (const uint16_t*)s->smp;
  const uint8_t* y = (const uint8_t*)(s->smp + smp_off_y(C));
  const float* w = (const float*)(s->smp + smp_off_w(C));
  double first = 0, last = 0;
  long long steps = 0;
  for (int ep = 0; ep < epochs; ++ep) {
    for (long long k = 0; k < ntrain; ++k) perm[k] = (int)k;
    std::shuffle(perm.begin(), perm.end(), rng);
    e = hipMemcpyAsync(didx, perm.data(), ntrain * sizeof(int), hipMemcpyHostToDevice, s->st);
    // the batch losses are summed on the device and read once per epoch
    if (e == hipSuccess) e = hipMemsetAsync(s->eloss, 0, sizeof(double), s->st);
    if (e != hipSuccess) return hip_fail(s, e, "index upload");
    long long nbatch = 0;
    for (long long b0 = 0; b0 + batch <= ntrain; b0 += batch) {
      double W = 0.0;
      for (long long k = b0; k < b0 + batch; ++k) W += hw[perm[k]];
      rc = grad_step(s, X, y, w, didx + b0, batch, (float)W, lr);
      if (rc) return rc;
      nbatch += 1;
      steps += 1;
    }
    double eloss = 0.0;
    e = hipMemcpyAsync(&eloss, s->eloss, sizeof(double), hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return hip_fail(s, e, "loss download");
    eloss /= (double)(nbatch > 0 ? nbatch : 1);
    if (ep == 0) first = eloss;
    last = eloss;
  }
  stats[0] = first;
  stats[1] = last;
  stats[2] = (double)steps;
  stats[3] = (double)ntrain;
  return OCFD_OK;
}

int ocfd_sensor_calibrate(ocfd_solver* s, double holdout, double margin, double miss, double* out) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!out) return fail(s, OCFD_ERR_BADARG, "null output");
  if (!s->mlp_ready) return fail(s, OCFD_ERR_STATE, "no network parameters set");
  if (!(holdout > 0.0 && holdout < 1.0) || !(margin > 0.0 && margin <= 1.0) || !(miss >= 0.0 && miss < 0.5))
    return fail(s, OCFD_ERR_BADARG, "holdout in (0,1), margin in (0,1] and miss in [0,0.5) required");
  const long long C = s->smp_cap;
  const long long a = (long long)((1.0 - holdout) * (double)s->smp_n);
  const long long nh = s->smp_n - a;
  if (nh < 1) return fail(s, OCFD_ERR_STATE, "no held-out samples");
  float* prob = (float*)(s->smp + smp_off_prob(C));
  hipError_t e = launch_mlp_prob((const uint16_t*)s->smp + a * 32, nh, s->mlp, prob, s->st);
  std::vector<float> p(nh);
  std::vector<uint8_t> y(nh);
  if (e == hipSuccess) e = hipMemcpyAsync(p.data(), prob, nh * sizeof(float), hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipMemcpyAsync(y.data(), s->smp + smp_off_y(C) + a, nh, hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return hip_fail(s, e, "calibration");
  // per direction (bits 1-2 of the label byte): tau_d = margin * the k-th
  // least probability of the held-out WENO samples of direction d,
  // k = floor(miss * their count); a direction with none takes the value
  // over all directions
  std::vector<float> pw[4];
  long long npos = 0, nneg = 0;
  for (long long k = 0; k < nh; ++k) {
    const int d = std::min(2, (int)(y[k] >> 1));
    if (y[k] & 1) {
      pw[d].push_back(p[k]);
      pw[3].push_back(p[k]);
      ++npos;
    } else {
      ++nneg;
    }
  }
  auto kth = [&](std::vector<float>& v) {
    const size_t k = std::min(v.size() - 1, (size_t)(miss * (double)v.size()));
    std::nth_element(v.begin(), v.begin() + k, v.end());
    return (double)v[k];
  };
  const double pall = npos ? kth(pw[3]) : 0.0;
  for (int d = 0; d < 3; ++d) s->tau[d] = npos ? margin * (pw[d].empty() ? pall : kth(pw[d])) : 0.5;
  long long fp = 0, tp = 0;
  for (long long k = 0; k < nh; ++k) {
    const int d = std::min(2, (int)(y[k] >> 1));
    const bool on = p[k] >= (float)s->tau[d];
    if ((y[k] & 1) && on) ++tp;
    if (!(y[k] & 1) && on) ++fp;
  }
  out[0] = std::min(s->tau[0], std::min(s->tau[1], s->tau[2]));
  out[1] = npos ? (double)tp / (double)npos : 1.0;
  out[2] = nneg ? (double)fp / (double)nneg : 0.0;
  out[3] = (double)nh;
  return OCFD_OK;
}

int ocfd_sensor_grad(ocfd_solver* s, const uint16_t* X, const uint8_t* y, const float* w, int64_t n, float* grad) {
  int rc;
  if (!ready(s, &rc)) return rc;
  if (!X || !y || !w || !grad || n < 1) return fail(s, OCFD_ERR_BADARG, "bad argument");
  if (!s->mlp_ready) return fail(s, OCFD_ERR_STATE, "no network parameters set");
  if (!s->smp || s->smp_cap < n) return fail(s, OCFD_ERR_STATE, "bind a sample buffer of at least n samples");
  std::vector<int> idx(n);
  std::vector<float> hw(n);
  double W = 0.0;
  hipError_t e = hipMemcpyAsync(hw.data(), w, n * sizeof(float), hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return hip_fail(s, e, "weight download");
  for (long long k = 0; k < n; ++k) {
    idx[k] = (int)k;
    W += hw[k];
  }
  int* didx = (int*)(s->smp + smp_off_idx(s->smp_cap));
  e = hipMemcpyAsync(didx, idx.data(), n * sizeof(int), hipMemcpyHostToDevice, s->st);
  if (e != hipSuccess) return hip_fail(s, e, "index upload");
  rc = grad_step(s, X, y, w, didx, n, (float)W, 0.f);
  if (rc) return rc;
  e = hipMemcpyAsync(grad, s->grad, (MLP_NPARAM + 1) * sizeof(float), hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  return e == hipSuccess ? OCFD_OK : hip_fail(s, e, "gradient download");
}

int ocfd_sensor_audit(ocfd_solver* s, double* out) {
  if (!s || !out) return OCFD_ERR_BADARG;
  for (int k = 0; k < 6; ++k) out[k] = s->audit[k];
  return OCFD_OK;
}

const char* ocfd_kernel_name(int32_t k) {
  static const char* names[OCFD_K_COUNT] = {"sweep_xi", "sweep_eta", "sweep_zeta", "viscous_flux", "primitives",
                                            "other"};
  return (k >= 0 && k < OCFD_K_COUNT) ? names[k] : "unknown";
}

const char* ocfd_last_error(const ocfd_solver* s) { return s ? s->err.c_str() : "null solver"; }

void ocfd_destroy(ocfd_solver* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->st);
  for (auto& r : s->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : s->pool) (void)hipEventDestroy(e);
  delete s;
}

}  // extern "C"
