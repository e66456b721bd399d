"""FP64 numpy oracle of the Ewald-surrogate network.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  The network is not
part of the paper; it replaces the paper's Ewald evaluation (Sec. 3.1) by a
learned function of the folded offset, and this module is the plain
reference its GPU forward/backward/Adam kernels are checked against.

Network: 3 -> 128 -> 128 -> 128 -> 4, SiLU after the three hidden layers,
linear output.  Parameters are one flat float vector in the order
W1[128,3], b1[128], W2[128,128], b2[128], W3[128,128], b3[128], W4[4,128],
b4[4] (row-major, out x in), 34052 values.

``bf16=True`` reproduces where the GPU rounds to bfloat16 (round to nearest
even): the weights of every layer and the inputs of the two 128x128 layers
(the operands of its matrix-core products).  Everything else is float64.
"""
from __future__ import annotations

import numpy as np

H = 128
SHAPES = [("W1", (H, 3)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)),
          ("b3", (H,)), ("W4", (4, H)), ("b4", (4,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(theta: np.ndarray) -> dict:
    out, off = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = theta[off:off + k].reshape(shp)
        off += k
    return out


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned as
    float64.  bfloat16 keeps the top 16 bits of a float32."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta: np.ndarray, x: np.ndarray, bf16: bool = False):
    """y [n,4] and the cache needed by ``backward``."""
    p = unflatten(np.asarray(theta, dtype=np.float64))
    r = round_bf16 if bf16 else (lambda a: a)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ r(p["W1"]).T + p["b1"]
    h1 = silu(z1)
    a1 = r(h1)
    z2 = a1 @ r(p["W2"]).T + p["b2"]
    h2 = silu(z2)
    a2 = r(h2)
    z3 = a2 @ r(p["W3"]).T + p["b3"]
    h3 = silu(z3)
    y = h3 @ r(p["W4"]).T + p["b4"]
    return y, dict(x=x, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, h3=h3, p=p, bf16=bf16)


def loss(y: np.ndarray, t: np.ndarray, w: np.ndarray) -> float:
    """Weighted mean squared error: mean over samples of sum_k w_k (y-t)^2."""
    return float(np.mean(np.sum(w * (y - t) ** 2, axis=1)))


def backward(cache: dict, dy: np.ndarray) -> np.ndarray:
    """Gradient (flat, same layout as theta) of sum(dy * y)."""
    p = cache["p"]
    r = round_bf16 if cache["bf16"] else (lambda a: a)
    g = {}
    g["W4"] = dy.T @ cache["h3"]
    g["b4"] = dy.sum(0)
    dh3 = dy @ r(p["W4"])
    dz3 = dh3 * dsilu(cache["z3"])
    g["W3"] = dz3.T @ cache["a2"]
    g["b3"] = dz3.sum(0)
    dh2 = dz3 @ r(p["W3"])
    dz2 = dh2 * dsilu(cache["z2"])
    g["W2"] = dz2.T @ cache["a1"]
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ r(p["W2"])
    dz1 = dh1 * dsilu(cache["z1"])
    g["W1"] = dz1.T @ cache["x"]
    g["b1"] = dz1.sum(0)
    return flatten(g)


def loss_grad(theta, x, t, w, bf16=False):
    """Weighted MSE and its gradient."""
    y, cache = forward(theta, x, bf16)
    n = x.shape[0]
    dy = 2.0 * w * (y - t) / n
    return loss(y, t, w), backward(cache, dy)


def adam_step(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; step >= 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# --------------------------------------------------------------------------
# The learned Ewald correction applied to particles (FP64).
#
# The network stands for the Ewald kernel psi of Sec. 3.1 (the periodic
# field of a unit mass minus its 27 nearest images), as a function of the
# folded offset u = |r| / L per axis in the positive octant; its four
# outputs are residuals of the quadratic background term:
#   psi(u)       = y0(u) - (2 pi / 3) |u|^2 + psi(0),
#   d psi / d u_a = y_a(u) - (4 pi / 3) u_a.
# psi is even in every coordinate of r, so d psi / d r_a = sign(r_a) times
# d psi / d u_a (r_a = 0 is taken with the + sign; there the exact
# derivative is zero).  The correction at particle x from the monopoles
# (M_c, X_c) of a set of cells is
#   phi(x) = sum_c M_c psi((x - X_c) / L) / L,
#   acc(x) = -sum_c M_c grad psi((x - X_c) / L) / L^2,
# summed in double.  The network reads its input as float, so u is rounded
# to float32 before the (double) forward pass; the weights and the two
# inner layers' inputs are rounded to bfloat16 as on the device.
# --------------------------------------------------------------------------

def top_cells(child: np.ndarray, ncell: int) -> list:
    """Cells at depth log2(ncell) below the root (cell 0), breadth first,
    each parent's lower child before its upper one; a leaf reached above
    that depth stands for its own branch.  ncell is 1, 8 or 64."""
    depth = {1: 0, 8: 3, 64: 6}[ncell]
    frontier = [0]
    for _ in range(depth):
        nxt = []
        for c in frontier:
            lo, hi = int(child[c][0]), int(child[c][1])
            nxt.extend([lo, hi] if lo >= 0 else [c])
        frontier = nxt
    return frontier


def surrogate_correction(theta: np.ndarray, pos: np.ndarray, cell_mass: np.ndarray,
                         cell_com: np.ndarray, L: float, psi0: float, chunk: int = 4096):
    """Accelerations [n,3] and potentials [n] of the learned correction at
    positions pos [n,3] from cells (masses [k], centres of mass [k,3])."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    acc = np.zeros((n, 3))
    pot = np.zeros(n)
    for c in range(len(cell_mass)):
        M = float(cell_mass[c])
        for s in range(0, n, chunk):
            r = (pos[s:s + chunk] - cell_com[c]) / L
            u = np.abs(r).astype(np.float32).astype(np.float64)
            y, _ = forward(theta, u, bf16=True)
            psi = y[:, 0] - (2.0 * np.pi / 3.0) * np.sum(u * u, axis=1) + psi0
            dpsi_du = y[:, 1:] - (4.0 * np.pi / 3.0) * u
            grad = np.where(r < 0.0, -dpsi_du, dpsi_du)
            pot[s:s + chunk] += M * psi / L
            acc[s:s + chunk] -= M * grad / (L * L)
    return acc, pot
