"""Seeded synthetic inputs shared by the GPU library's callers and the oracle.

This module holds grids, initial states and run parameters only: node
coordinates, primitive fields turned into conserved variables, and the numbers
a run needs (sizes, Reynolds and Mach numbers, time step).  It contains none of
the numerical method, so both the GPU path and the CPU oracle can take their
inputs from it without sharing any of the scheme.

Workloads (paper: Dang et al., arXiv:2209.15333; the problems stand in for the
paper's own flows, whose data are not public):
  * Taylor-Green vortex on a uniform or sinusoidally distorted periodic grid;
  * isentropic vortex advection (exact translated solution);
  * Sod shock tube laid along any of the three directions;
  * uniform flow on a distorted grid (free-stream preservation).
Random numbers come from numpy's PCG64 with the stated seeds.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclasses.dataclass
class Case:
    """One run: grid, initial state and the physical / scheme parameters."""
    name: str
    nx: int
    ny: int
    nz: int
    xyz: np.ndarray                      # [3, nz, ny, nx] node coordinates
    U0: np.ndarray                       # [5, nz, ny, nx] conserved rho, rho u, rho v, rho w, E
    period: Tuple[float, float, float]   # coordinate d shifts by period[d] across the seam of direction d
    h: Tuple[float, float, float]        # computational spacing per direction
    dt: float
    nsteps: int
    periodic: Tuple[int, int, int] = (1, 1, 1)
    bc: Tuple[int, int, int, int, int, int] = (0, 0, 0, 0, 0, 0)
    gamma: float = 1.4
    Re: float = 1600.0
    Ma: float = 0.1
    Pr: float = 0.72
    Tref: float = 288.15
    suth: float = 110.4
    Tw: float = 1.0
    theta1: float = 0.02
    theta2: float = 0.1
    eps: float = 1e-6
    viscous: int = 6
    scheme: str = "weno7"                # "weno7" | "hybrid"
    lowdiss: str = "c8"                  # "ud7" | "c8"
    three_way: bool = False
    characteristic: bool = False         # reconstruct in characteristic variables (Sec. 2.2.2)
    flag_window: int = 0                 # plain sensor window: 0 nodes j-3..j+4, 1 nodes j, j+1
    inflow: Optional[np.ndarray] = None
    precision: str = "fp64"              # "fp64" | "mixed" (GPU only)
    sensor: str = "plain"                # hybrid: "plain" (pressure sensor) | "learned" (GPU only)
    sensor_every: int = 1
    audit_every: int = 0
    sensor_inputs: str = "jump"          # learned sensor: "jump" (first differences) | "curv" (eq 42's)

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz


def conserved(gamma: float, rho, u, v, w, p) -> np.ndarray:
    """Conserved variables from primitive fields (rho, velocity, pressure)."""
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.ascontiguousarray(np.stack([rho, rho * u, rho * v, rho * w, E]).astype(np.float64))


def _lattice(n: Tuple[int, int, int], L: Tuple[float, float, float]):
    nx, ny, nz = n
    X = np.arange(nx) * (L[0] / nx)
    Y = np.arange(ny) * (L[1] / ny)
    Z = np.arange(nz) * (L[2] / nz)
    Zg, Yg, Xg = np.meshgrid(Z, Y, X, indexing="ij")
    return Xg, Yg, Zg


def distortion_phases(seed: int) -> np.ndarray:
    """The nine phases of the sinusoidal grid distortion, uniform on [0, 2 pi)."""
    return np.random.Generator(np.random.PCG64(seed)).uniform(0.0, TWO_PI, size=9)


def periodic_grid(n: Tuple[int, int, int], L: Tuple[float, float, float],
                  amplitude: float = 0.0, seed: int = 0) -> np.ndarray:
    """Nodes of a periodic box, optionally with a smooth sinusoidal distortion.

    x = X + A sin(2 pi X/Lx + p1) sin(2 pi Y/Ly + p2) sin(2 pi Z/Lz + p3), and
    likewise for y (phases p4..p6) and z (p7..p9), with the nine phases drawn
    uniformly from [0, 2 pi) by PCG64(seed).  The distortion is periodic, so
    coordinate d still grows by exactly L[d] across the seam of direction d.
    """
    Xg, Yg, Zg = _lattice(n, L)
    xyz = np.stack([Xg, Yg, Zg]).astype(np.float64)
    if amplitude != 0.0:
        ph = distortion_phases(seed)
        sx = TWO_PI * Xg / L[0]
        sy = TWO_PI * Yg / L[1]
        sz = TWO_PI * Zg / L[2]
        for c in range(3):
            xyz[c] += amplitude * np.sin(sx + ph[3 * c]) * np.sin(sy + ph[3 * c + 1]) * np.sin(sz + ph[3 * c + 2])
    return np.ascontiguousarray(xyz)


def taylor_green(n: int = 32, distorted: bool = False, seed: int = 22092, Ma: float = 0.1,
                 Re: float = 1600.0, dt: Optional[float] = None, nsteps: int = 20,
                 shape: Optional[Tuple[int, int, int]] = None) -> Case:
    """Taylor-Green vortex on [0, 2 pi)^3 (rho = 1, M = 0.1, Re = 1600, Pr = 0.72).

    u = sin x cos y cos z, v = -cos x sin y cos z, w = 0,
    p = 1/(gamma M^2) + (cos 2x + cos 2y)(cos 2z + 2)/16, evaluated at the
    (possibly distorted) node positions.  Distortion amplitude 0.1 h.
    """
    nx, ny, nz = shape if shape is not None else (n, n, n)
    L = (TWO_PI, TWO_PI, TWO_PI)
    h = (L[0] / nx, L[1] / ny, L[2] / nz)
    xyz = periodic_grid((nx, ny, nz), L, 0.1 * h[0] if distorted else 0.0, seed)
    x, y, z = xyz
    g = 1.4
    rho = np.ones_like(x)
    u = np.sin(x) * np.cos(y) * np.cos(z)
    v = -np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(x)
    p = 1.0 / (g * Ma * Ma) + (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0) / 16.0
    if dt is None:
        dt = 1e-3 if nx <= 32 else 2.5e-4 * 256.0 / max(nx, ny, nz)
    return Case(name=f"tgv{nx}x{ny}x{nz}{'-distorted' if distorted else ''}", nx=nx, ny=ny, nz=nz,
                xyz=xyz, U0=conserved(g, rho, u, v, w, p), period=L, h=h, dt=dt, nsteps=nsteps,
                gamma=g, Re=Re, Ma=Ma, viscous=6)


def vortex_primitive(x, y, t: float, L: float = 20.0, strength: float = 5.0, Ma: float = 0.5,
                     gamma: float = 1.4, center=(10.0, 10.0), advect=(1.0, 1.0)):
    """Isentropic vortex in the paper's units (rho_inf = T_inf = 1, p_inf = 1/(gamma Ma^2)),
    translated by advect*t, nearest periodic image of the centre."""
    dx = x - center[0] - advect[0] * t
    dy = y - center[1] - advect[1] * t
    dx = dx - L * np.round(dx / L)
    dy = dy - L * np.round(dy / L)
    r2 = dx * dx + dy * dy
    e = strength / TWO_PI * np.exp(0.5 * (1.0 - r2))
    u = advect[0] - e * dy
    v = advect[1] + e * dx
    th_inf = 1.0 / (gamma * Ma * Ma)
    th = th_inf - (gamma - 1.0) * strength ** 2 / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    rho = (th / th_inf) ** (1.0 / (gamma - 1.0))
    p = rho * th
    return rho, u, v, np.zeros_like(u), p


def isentropic_vortex(n: int = 256, distorted: bool = True, seed: int = 22091, nsteps: int = 200,
                      shape: Optional[Tuple[int, int, int]] = None, dt: Optional[float] = None) -> Case:
    """Isentropic vortex (strength 5, advection (1,1,0), Ma 0.5) on [0,20)^3, Euler.

    Distortion amplitude 0.1 h with seeded phases.  The box is 20 wide so the
    Gaussian tail at the periodic images is far below roundoff."""
    nx, ny, nz = shape if shape is not None else (n, n, n)
    Lb = 20.0
    L = (Lb, Lb, Lb)
    h = (Lb / nx, Lb / ny, Lb / nz)
    xyz = periodic_grid((nx, ny, nz), L, 0.1 * h[0] if distorted else 0.0, seed)
    g = 1.4
    rho, u, v, w, p = vortex_primitive(xyz[0], xyz[1], 0.0, L=Lb, gamma=g)
    if dt is None:
        dt = 2e-3 * 256.0 / max(nx, ny)
    return Case(name=f"vortex{nx}x{ny}x{nz}{'-distorted' if distorted else ''}", nx=nx, ny=ny, nz=nz,
                xyz=xyz, U0=conserved(g, rho, u, v, w, p), period=L, h=h, dt=dt, nsteps=nsteps,
                gamma=g, Re=1.0, Ma=0.5, viscous=0)


def uniform_flow(n: Tuple[int, int, int] = (16, 16, 16), amplitude_frac: float = 0.1, seed: int = 7,
                 vel=(0.5, 0.3, 0.2), Ma: float = 0.5, viscous: int = 6, L: float = 2 * math.pi) -> Case:
    """Uniform flow (rho = 1, T = 1) on a distorted periodic grid."""
    nx, ny, nz = n
    Ls = (L, L, L)
    h = (L / nx, L / ny, L / nz)
    xyz = periodic_grid(n, Ls, amplitude_frac * h[0], seed)
    g = 1.4
    shp = xyz[0].shape
    rho = np.ones(shp)
    p = np.full(shp, 1.0 / (g * Ma * Ma))
    U0 = conserved(g, rho, np.full(shp, vel[0]), np.full(shp, vel[1]), np.full(shp, vel[2]), p)
    return Case(name="uniform-flow", nx=nx, ny=ny, nz=nz, xyz=xyz, U0=U0, period=Ls, h=h, dt=1e-3,
                nsteps=3, gamma=g, Re=100.0, Ma=Ma, viscous=viscous)


def sod(n: int = 200, axis: int = 0, width: int = 4) -> Case:
    """Sod tube (rho, u, p) = (1, 0, 1) | (0.125, 0, 0.1) on a periodic box [0, 2)
    along `axis`: the high state fills 0.5 < x < 1.5, so the box holds two
    mirrored tubes whose waves do not meet before t = 0.2.  Nodes sit at cell
    centres (i + 1/2) h so no node lies on a discontinuity.  The other two
    directions carry `width` identical nodes.  Euler, gamma = 1.4; time step
    0.4/n, 0.2/dt steps of three substeps each."""
    shape = [width, width, width]
    shape[axis] = n
    nx, ny, nz = shape
    Ls = [0.1 * width, 0.1 * width, 0.1 * width]
    Ls[axis] = 2.0
    xyz = periodic_grid((nx, ny, nz), tuple(Ls))
    h = tuple(Ls[d] / shape[d] for d in range(3))
    xyz[axis] += 0.5 * h[axis]
    s = xyz[axis]
    inside = (s > 0.5) & (s < 1.5)
    rho = np.where(inside, 1.0, 0.125)
    p = np.where(inside, 1.0, 0.1)
    zero = np.zeros_like(rho)
    g = 1.4
    dt = 0.4 / n
    steps = int(round(0.2 / dt))
    return Case(name=f"sod{n}-axis{axis}", nx=nx, ny=ny, nz=nz, xyz=xyz, U0=conserved(g, rho, zero, zero, zero, p),
                period=tuple(Ls), h=h, dt=dt, nsteps=3 * steps, gamma=g, Re=1.0, Ma=1.0 / math.sqrt(1.4), viscous=0)


def lax(n: int = 200, width: int = 2) -> Case:
    """Lax tube on the periodic box [0, 2) along x: (rho, u, p) = (0.445, 0.698,
    3.528) for 0.5 < x < 1.5, (0.5, 0, 0.571) outside.  The discontinuity at
    x = 1.5 is the Lax problem; on 1 <= x < 2 its waves are the only ones up to
    t = 0.13 (the faster left state pushes the waves of x = 0.5 no further
    than x = 1.03).  Cell-centred nodes, Euler, gamma = 1.4, time step 0.2/n,
    0.13/dt steps of three substeps each."""
    case = sod(n, axis=0, width=width)
    s = case.xyz[0]
    inside = (s > 0.5) & (s < 1.5)
    g = case.gamma
    rho = np.where(inside, 0.445, 0.5)
    u = np.where(inside, 0.698, 0.0)
    p = np.where(inside, 3.528, 0.571)
    zero = np.zeros_like(rho)
    dt = 0.2 / n
    return dataclasses.replace(case, name=f"lax{n}", U0=conserved(g, rho, u, zero, zero, p), dt=dt,
                               nsteps=3 * int(round(0.13 / dt)))


def acoustic_pulse(n: int = 201, width: int = 4, u0: float = 0.3, amplitude: float = 1e-3, sigma: float = 0.05,
                   x0: float = 0.5, direction: int = 1, bc: int = 4) -> Case:
    """A plane acoustic pulse in a uniform stream on x in [0, 1] (n nodes,
    bounded, faces of kind `bc` at both ends) with `width` identical nodes in
    the two periodic directions.  Free stream rho = 1, u = u0, Ma = 1 (sound
    speed 1, p = 1/gamma); the pulse p' = amplitude p exp(-((x-x0)/sigma)^2)
    with u' = direction p'/(rho c), rho' = p'/c^2 runs in +x (direction 1) or
    -x (direction -1).  Euler; time step 0.4 h."""
    nx, ny, nz = n, width, width
    h = 1.0 / (n - 1)
    Ls = (1.0, 0.1 * width, 0.1 * width)
    X = np.arange(nx) * h
    Y = np.arange(ny) * (Ls[1] / ny)
    Z = np.arange(nz) * (Ls[2] / nz)
    Zg, Yg, Xg = np.meshgrid(Z, Y, X, indexing="ij")
    xyz = np.ascontiguousarray(np.stack([Xg, Yg, Zg]).astype(np.float64))
    g = 1.4
    p0 = 1.0 / g
    pp = amplitude * p0 * np.exp(-((Xg - x0) / sigma) ** 2)
    rho = 1.0 + pp
    u = u0 + direction * pp
    zero = np.zeros_like(rho)
    return Case(name=f"pulse{n}", nx=nx, ny=ny, nz=nz, xyz=xyz, U0=conserved(g, rho, u, zero, zero, p0 + pp),
                period=(0.0, Ls[1], Ls[2]), h=(h, Ls[1] / ny, Ls[2] / nz), dt=0.4 * h, nsteps=0,
                periodic=(0, 1, 1), bc=(bc, bc, 0, 0, 0, 0), gamma=g, Re=1.0, Ma=1.0, viscous=0)


def isotropic_turbulence(n: int = 512, seed: int = 22093, k0: float = 4.0, Mt: float = 0.6,
                         Re_lambda: float = 100.0, dt: Optional[float] = None, nsteps: int = 500) -> Case:
    """Decaying compressible isotropic turbulence on [0, 2 pi)^3.

    Solenoidal velocity with energy spectrum E(k) ~ k^4 exp(-2 k^2 / k0^2):
    each Fourier mode gets a complex Gaussian amplitude (PCG64(seed)) scaled
    to the spectrum, the k = 0 mode is removed and the field projected onto
    its divergence-free part.  Scaled to u_rms = 1 per component, so the
    turbulent Mach number sqrt(<u.u>)/c = Mt fixes c and Ma = 1/c.  Uniform
    rho = T = 1.  Re = Re_lambda / (u_rms lambda) with the Taylor microscale
    lambda = u_rms / rms(du/dx) measured on the field (spectrally).  Pr 0.72.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    kz, ky, kx = np.meshgrid(k1, k1, np.fft.rfftfreq(n, d=1.0 / n), indexing="ij")
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    spec = np.where(kk > 0, kk ** 4 * np.exp(-2.0 * kk * kk / (k0 * k0)), 0.0)
    # amplitude per mode so that the shell sum follows E(k): |u_k|^2 ~ E(k) / (4 pi k^2)
    amp = np.where(kk > 0, np.sqrt(spec / (4.0 * math.pi * np.maximum(kk, 1e-30) ** 2)), 0.0)
    uh = []
    for _ in range(3):
        re = rng.standard_normal(kk.shape)
        im = rng.standard_normal(kk.shape)
        uh.append(amp * (re + 1j * im))
    # project out the compressive part: u <- u - k (k.u) / |k|^2
    kdotu = kx * uh[0] + ky * uh[1] + kz * uh[2]
    k2 = np.where(kk > 0, kk * kk, 1.0)
    uh[0] = uh[0] - kx * kdotu / k2
    uh[1] = uh[1] - ky * kdotu / k2
    uh[2] = uh[2] - kz * kdotu / k2
    vel = [np.fft.irfftn(c, s=(n, n, n), axes=(0, 1, 2)) for c in uh]
    dudx = np.fft.irfftn(1j * kx * uh[0], s=(n, n, n), axes=(0, 1, 2))
    del uh, kdotu
    urms = math.sqrt(sum(float(np.mean(v * v)) for v in vel) / 3.0)
    vel = [v / urms for v in vel]
    lam = 1.0 / math.sqrt(float(np.mean((dudx / urms) ** 2)))   # u_rms = 1 after scaling
    c = math.sqrt(3.0) / Mt
    Ma = 1.0 / c
    g = 1.4
    L = (TWO_PI, TWO_PI, TWO_PI)
    h = (TWO_PI / n,) * 3
    xyz = periodic_grid((n, n, n), L)
    rho = np.ones((n, n, n))
    p = rho / (g * Ma * Ma)
    if dt is None:
        dt = 0.3 * h[0] / (3.0 * (4.0 + c))
    case = Case(name=f"hit{n}", nx=n, ny=n, nz=n, xyz=xyz, U0=conserved(g, rho, vel[0], vel[1], vel[2], p),
                period=L, h=h, dt=dt, nsteps=nsteps, gamma=g, Re=Re_lambda / lam, Ma=Ma, viscous=6,
                scheme="hybrid", lowdiss="c8")
    case.taylor_microscale = lam
    return case


def _smooth_noise(rng, shape, sigma_cells: float = 2.0):
    """Gaussian-smoothed white noise (periodic smoothing by FFT), unit rms.
    Real-to-complex transforms on all host cores (the filter is real and
    even, so the result is the real part of the full complex product)."""
    import os
    import scipy.fft
    w = rng.standard_normal(shape)
    k = [np.fft.fftfreq(n) for n in shape[:-1]] + [np.fft.rfftfreq(shape[-1])]
    filt = np.exp(-2.0 * (math.pi * sigma_cells) ** 2 * (k[0][:, None, None] ** 2 + k[1][None, :, None] ** 2 +
                                                         k[2][None, None, :] ** 2))
    nw = os.cpu_count() or 1
    out = scipy.fft.irfftn(scipy.fft.rfftn(w, workers=nw) * filt, s=shape, workers=nw)
    return out / np.sqrt(np.mean(out * out))


def compression_ramp(shape: Tuple[int, int, int] = (1024, 160, 128), seed: int = 22094, Ma: float = 2.9,
                     angle_deg: float = 24.0, Re: float = 5e4, Tw: float = 2.84, dt: Optional[float] = None,
                     nsteps: int = 100, noise: float = 0.05, viscous: int = 8, exit_bc: int = 4) -> Case:
    """Supersonic flow over a compression ramp on a body-fitted grid (lengths in
    units of the inflow boundary-layer thickness delta).

    x in [-20, 12] uniform; wall y_w(x) = tan(angle) r ln(1 + exp(x/r)),
    r = 0.25 (a smoothed corner at x = 0); y = y_w(x) + H s_j with H = 10 and
    tanh clustering s_j = 1 - tanh(b (1 - j/(ny-1))) / tanh(b), b chosen so the
    first cell is 0.002 high; z in [0, 4) periodic.  Initial state: the
    wall-parallel velocity tanh(3 y_n) (y_n the height above the wall),
    temperature from the Crocco-Busemann relation with wall temperature Tw
    and recovery factor Pr^(1/2), uniform pressure 1/(gamma Ma^2), plus
    noise * u_bar * (Gaussian-smoothed white noise, 2 cells, unit rms) on u,
    v, w (PCG64(seed)).  Boundaries: inflow (the initial profile) at x = -20,
    isothermal wall at y_w, and at the outlet and the top faces of kind
    exit_bc: 4 characteristic nonreflecting (the paper's Sec. 6.1), 2
    extrapolation.  Viscous terms of eighth order, as the paper's ramp runs
    (Sec. 5.1, 6.1)."""
    nx, ny, nz = shape
    g, Pr = 1.4, 0.72
    r, H, Lz = 0.25, 10.0, 4.0
    tan_a = math.tan(math.radians(angle_deg))
    X = -20.0 + 32.0 * np.arange(nx) / (nx - 1)
    # stretching parameter: H (1 - tanh(b (1 - 1/(ny-1)))/tanh(b)) = 0.002
    lo, hi = 1e-3, 20.0
    for _ in range(200):
        b = 0.5 * (lo + hi)
        first = H * (1.0 - math.tanh(b * (1.0 - 1.0 / (ny - 1))) / math.tanh(b))
        lo, hi = (b, hi) if first > 0.002 else (lo, b)
    s = 1.0 - np.tanh(b * (1.0 - np.arange(ny) / (ny - 1))) / math.tanh(b)
    yw = tan_a * r * np.log1p(np.exp(X / r))
    slope = tan_a / (1.0 + np.exp(-X / r))
    Z = np.arange(nz) * (Lz / nz)
    Zg, Sg, Xg = np.meshgrid(Z, s, X, indexing="ij")
    Yw = np.broadcast_to(yw[None, None, :], Xg.shape)
    xyz = np.ascontiguousarray(np.stack([Xg, Yw + H * Sg, Zg]).astype(np.float64))
    yn = H * Sg
    ub = np.tanh(3.0 * yn)
    rf = math.sqrt(Pr)
    Taw = 1.0 + rf * 0.5 * (g - 1.0) * Ma * Ma
    T = Tw + (Taw - Tw) * ub - rf * 0.5 * (g - 1.0) * Ma * Ma * ub * ub
    p = np.full_like(T, 1.0 / (g * Ma * Ma))
    rho = g * Ma * Ma * p / T
    phi = np.arctan(np.broadcast_to(slope[None, None, :], Xg.shape))
    rng = np.random.Generator(np.random.PCG64(seed))
    u = ub * np.cos(phi) + noise * ub * _smooth_noise(rng, Xg.shape)
    v = ub * np.sin(phi) + noise * ub * _smooth_noise(rng, Xg.shape)
    w = noise * ub * _smooth_noise(rng, Xg.shape)
    U0 = conserved(g, rho, u, v, w, p)
    # inflow face (i = 0), [5][nz][ny] with eta fastest
    inflow = np.ascontiguousarray(U0[:, :, :, 0])
    if dt is None:
        dt = 8e-4   # set by the 0.002-high wall cell (acoustic CFL ~0.33)
    h = (32.0 / (nx - 1), H / (ny - 1), Lz / nz)
    return Case(name=f"ramp{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, xyz=xyz, U0=U0, period=(0.0, 0.0, Lz), h=h,
                dt=dt, nsteps=nsteps, periodic=(0, 0, 1), bc=(1, exit_bc, 3, exit_bc, 0, 0), gamma=g, Re=Re, Ma=Ma, Pr=Pr,
                Tref=108.1, Tw=Tw, inflow=inflow, viscous=viscous)


def bounded_box(shape: Tuple[int, int, int] = (36, 20, 18), seed: int = 22095, Ma: float = 0.5, Re: float = 500.0,
                amplitude: float = 0.04, noise: float = 0.02) -> Case:
    """A box bounded in all three directions on a distorted grid: unit spacing
    nodes moved by amplitude * sin products (phases from PCG64(seed)); a smooth
    shear flow u = 1 + 0.3 tanh(2 (y - y_mid)), v = 0.1 sin(x/2), w = 0.05 cos(z/2)
    at Mach Ma with uniform pressure and temperature 1, plus relative noise on
    the velocities.  Faces: inflow (the initial face) at xi-, characteristic
    nonreflecting at xi+ and zeta+ (their common edge takes both normal
    parts), isothermal wall (Tw = 1) at eta-, extrapolation at eta+ and
    zeta-."""
    nx, ny, nz = shape
    rng = np.random.Generator(np.random.PCG64(seed))
    ph = rng.uniform(0.0, 2.0 * math.pi, 9)
    K, J, I = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    a = amplitude
    x = I + a * np.sin(0.3 * J + ph[0]) * np.sin(0.2 * K + ph[1])
    y = J + a * np.sin(0.25 * I + ph[2]) * np.sin(0.3 * K + ph[3])
    z = K + a * np.sin(0.2 * I + ph[4]) * np.sin(0.25 * J + ph[5])
    xyz = np.ascontiguousarray(np.stack([x, y, z]))
    g = 1.4
    u = 1.0 + 0.3 * np.tanh(2.0 * (y - 0.5 * (ny - 1)))
    v = 0.1 * np.sin(0.5 * x)
    w = 0.05 * np.cos(0.5 * z)
    u = u * (1.0 + noise * rng.standard_normal(u.shape))
    v = v + noise * rng.standard_normal(v.shape)
    w = w + noise * rng.standard_normal(w.shape)
    p = np.full_like(u, 1.0 / (g * Ma * Ma))
    rho = np.ones_like(u)
    U0 = conserved(g, rho, u, v, w, p)
    inflow = np.ascontiguousarray(U0[:, :, :, 0])
    return Case(name=f"box{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, xyz=xyz, U0=U0, period=(0.0, 0.0, 0.0),
                h=(1.0, 1.0, 1.0), dt=0.05, nsteps=10, periodic=(0, 0, 0), bc=(1, 4, 3, 2, 2, 4), gamma=g, Re=Re,
                Ma=Ma, Pr=0.72, Tw=1.0, inflow=inflow)


def sensor_initial_weights(seed: int = 0) -> np.ndarray:
    """Initial weights of the 32-64-64-64-1 shock-sensor perceptron as one
    flat array W1 [32 in][64 out], b1, W2 [64][64], b2, W3 [64][64], b3,
    w4 [64], b4: He-uniform hidden layers, an output layer ten times smaller,
    zero biases (PCG64(seed) draws in that order)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.uniform(-1, 1, (32, 64)) * math.sqrt(6.0 / 32)
    W2 = rng.uniform(-1, 1, (64, 64)) * math.sqrt(6.0 / 64)
    W3 = rng.uniform(-1, 1, (64, 64)) * math.sqrt(6.0 / 64)
    w4 = rng.uniform(-1, 1, 64) * math.sqrt(6.0 / 64) * 0.1
    return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), W3.ravel(), np.zeros(64), w4,
                           np.zeros(1)])


def projection_weights(n_nodes: int, count: int = 4, seed: int = 22096):
    """`count` seeded standard-normal vectors over the nodes (PCG64(seed),
    drawn in order), for comparing two whole fields through a few random
    projections: for a difference d the projection r.d has the spread of the
    L2 norm |d|, so the projections of two fields agree only if the fields
    do."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.standard_normal(n_nodes) for _ in range(count)]


def sample_nodes(n_nodes: int, count: int = 1024, seed: int = 22097) -> np.ndarray:
    """`count` distinct node indices in increasing order (PCG64(seed))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(n_nodes, size=count, replace=False)).astype(np.int64)
