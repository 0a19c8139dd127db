"""CPU oracle of the learned shock sensor (test infrastructure only).

The learned sensor replaces the pressure sensor of the hybrid scheme
(Sec. 2.2.3, eq 42-43) by a small multilayer perceptron that maps a local
stencil of flow features to the probability that an interface needs the
WENO stencil.  This module holds, in plain numpy:

* the node features: Delta * div(u) / c, Delta * |curl u| / c (Delta = (1/J)^(1/3),
  the cell size), and the pressure and density jumps: normalised first
  differences |q+ - q-| / (q+ + q-) across the node, summed over the three
  grid directions, in units of the sensor threshold theta1 (not the plain
  sensor's second difference, so the label is not among the inputs), or
  those second differences themselves (the "curv" inputs);
  velocity derivatives are second-order central differences mapped to
  x, y, z with the node metrics;
* the interface input: the four features of the 8 nodes j-3 .. j+4 of the
  interface j+1/2, node-major;
* the network 32 -> 64 -> 64 -> 64 -> 1 (ReLU hidden layers, sigmoid
  output), its weighted binary cross-entropy loss and the exact backward pass
  in FP64;
* the same forward/backward with values rounded to bfloat16 at the points
  where the GPU kernels feed its matrix cores (inputs, weights of the three
  hidden layers, the hidden activations entering layers 2 and 3, the
  back-propagated pre-activation gradients), so the two can be compared on
  identical operands;
* the Adam update of the training loop.

Parameters are one flat float array: W1 [32 in x 64 out] (row = input),
b1 [64], W2 [64 x 64], b2 [64], W3 [64 x 64], b3 [64], w4 [64], b4 [1].
"""
from __future__ import annotations

import numpy as np

NIN, NH = 32, 64
SIZES = [("W1", (NIN, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH, NH)), ("b3", (NH,)),
         ("w4", (NH,)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def init_params(seed: int = 0):
    """He-uniform hidden layers, small output layer (numpy PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = {"W1": rng.uniform(-1, 1, (NIN, NH)) * np.sqrt(6.0 / NIN), "b1": np.zeros(NH),
         "W2": rng.uniform(-1, 1, (NH, NH)) * np.sqrt(6.0 / NH), "b2": np.zeros(NH),
         "W3": rng.uniform(-1, 1, (NH, NH)) * np.sqrt(6.0 / NH), "b3": np.zeros(NH),
         "w4": rng.uniform(-1, 1, NH) * np.sqrt(6.0 / NH) * 0.1, "b4": np.zeros(1)}
    return pack(d)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(theta, X, round_bf16: bool = False):
    """Probabilities for inputs X [n, 32]; returns (p, cache)."""
    P = unpack(theta)
    r = bf16 if round_bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    x = r(X)
    a1 = x @ r(P["W1"]) + P["b1"]
    h1 = r(np.maximum(a1, 0.0))
    a2 = h1 @ r(P["W2"]) + P["b2"]
    h2 = r(np.maximum(a2, 0.0))
    a3 = h2 @ r(P["W3"]) + P["b3"]
    h3 = np.maximum(a3, 0.0)
    z = h3 @ P["w4"] + P["b4"][0]
    return _sigmoid(z), (x, a1, h1, a2, h2, a3, h3, z)


def loss_and_grad(theta, X, y, w, round_bf16: bool = False):
    """Weighted binary cross-entropy  L = -sum_i w_i [y_i log p_i + (1-y_i) log(1-p_i)] / sum_i w_i
    and its gradient with respect to the flat parameters."""
    P = unpack(theta)
    r = bf16 if round_bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    p, (x, a1, h1, a2, h2, a3, h3, z) = forward(theta, X, round_bf16)
    y = np.asarray(y, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    W = w.sum()
    eps = 1e-12
    L = -np.sum(w * (y * np.log(p + eps) + (1 - y) * np.log(1 - p + eps))) / W
    dz = w * (p - y) / W                          # dL/dz
    g = {"w4": h3.T @ dz, "b4": np.array([dz.sum()])}
    da3 = np.outer(dz, P["w4"]) * (a3 > 0)       # dL/da3
    g["W3"] = h2.T @ r(da3)
    g["b3"] = da3.sum(axis=0)
    da2 = (r(da3) @ r(P["W3"]).T) * (a2 > 0)
    g["W2"] = h1.T @ r(da2)
    g["b2"] = da2.sum(axis=0)
    da1 = (r(da2) @ r(P["W2"]).T) * (a1 > 0)
    g["W1"] = x.T @ r(da1)
    g["b1"] = da1.sum(axis=0)
    return L, pack(g)


def adam_step(theta, m, v, g, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba, "Adam: a method for stochastic
    optimization", ICLR 2015, Algorithm 1) of the flat parameters theta with
    gradient g at step t >= 1: biased moments m, v, their bias corrections
    m / (1 - b1^t), v / (1 - b2^t), and the step lr * mhat / (sqrt(vhat) + eps).
    Returns new (theta, m, v)."""
    g = np.asarray(g, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return np.asarray(theta, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ------------------------------------------------------------------ features

def node_features(gamma: float, h, met: np.ndarray, U: np.ndarray, periodic=(1, 1, 1),
                  theta1: float = 0.02, inputs: str = "jump") -> np.ndarray:
    """Node features [4, nz, ny, nx]: Delta div/c, Delta |curl|/c, and the
    pressure and density jumps sum_d |q+ - q-| / (q+ + q-) divided by theta1
    (q+, q- the next and previous node along d); with inputs="curv" the
    normalised second differences sum_d |q- - 2q + q+| / (q- + 2q + q+)
    divided by theta1 instead (the plain sensor's node value, eq 42).  Along
    a bounded direction an end node takes a one-sided velocity difference
    over one spacing and adds no jump term."""
    rho = U[0]
    vel = [U[1] / rho, U[2] / rho, U[3] / rho]
    p = (gamma - 1.0) * (U[4] - 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2))
    c = np.sqrt(gamma * p / rho)
    jinv = met[9]
    axis = {0: 2, 1: 1, 2: 0}

    def plus_minus(q, d):
        """q at the next and previous node along d, the spacing between them,
        and a mask of the end nodes of a bounded line."""
        ax = axis[d]
        n = q.shape[ax]
        if periodic[d]:
            return np.roll(q, -1, ax), np.roll(q, 1, ax), np.full(q.shape, 2.0 * h[d]), np.zeros(q.shape, bool)
        idx = np.arange(n)
        ip, im = np.minimum(idx + 1, n - 1), np.maximum(idx - 1, 0)
        shape = [1, 1, 1]
        shape[ax] = n
        span = np.broadcast_to(((ip - im) * h[d]).astype(np.float64).reshape(shape), q.shape)
        end = np.broadcast_to(((idx == 0) | (idx == n - 1)).reshape(shape), q.shape)
        return np.take(q, ip, axis=ax), np.take(q, im, axis=ax), span, end

    dvd = [[None] * 3 for _ in range(3)]      # d(vel_a)/d(xi_d)
    jp = np.zeros(rho.shape)
    jr = np.zeros(rho.shape)
    for d in range(3):
        for a in range(3):
            vp, vm, span, _ = plus_minus(vel[a], d)
            dvd[a][d] = (vp - vm) / span
        for q, acc in ((p, jp), (rho, jr)):
            qp, qm, _, end = plus_minus(q, d)
            if inputs == "curv":
                acc += np.where(end, 0.0, np.abs(-qm + 2.0 * q - qp) / (qm + 2.0 * q + qp))
            else:
                acc += np.where(end, 0.0, np.abs(qp - qm) / (qp + qm))
    grad = [[sum((met[3 * d + col] / jinv) * dvd[a][d] for d in range(3)) for col in range(3)] for a in range(3)]
    div = grad[0][0] + grad[1][1] + grad[2][2]
    wx = grad[2][1] - grad[1][2]
    wy = grad[0][2] - grad[2][0]
    wz = grad[1][0] - grad[0][1]
    vort = np.sqrt(wx * wx + wy * wy + wz * wz)
    delta = np.cbrt(np.abs(jinv))
    return np.stack([delta * div / c, delta * vort / c, jp / theta1, jr / theta1])


def interface_inputs(F: np.ndarray, d: int, nodes: np.ndarray, periodic: bool = True) -> np.ndarray:
    """Inputs [n, 32] of the interfaces (node + 1/2 along direction d) at the
    given linear node indices: x[4t + f] = feature f of node j - 3 + t (on a
    bounded line, positions outside are clamped to the ends; such interfaces
    are not decided by a sensor)."""
    nz, ny, nx = F.shape[1:]
    n = (nx, ny, nz)[d]
    k, j, i = np.unravel_index(nodes, (nz, ny, nx))
    pos = (i, j, k)[d]
    X = np.zeros((len(nodes), 32))
    for t in range(8):
        q = (pos + t - 3) % n if periodic else np.clip(pos + t - 3, 0, n - 1)
        ii, jj, kk = (q if d == 0 else i), (q if d == 1 else j), (q if d == 2 else k)
        for f in range(4):
            X[:, 4 * t + f] = F[f][kk, jj, ii]
    return X


def window_inside(n: int, pos, periodic: bool):
    """Interfaces whose 8-node window stays inside the grid."""
    pos = np.asarray(pos)
    return np.ones(pos.shape, bool) if periodic else (pos >= 3) & (pos <= n - 5)
