"""FP64 CPU oracle of the learned coarse correction (the paper fixes none of
it; the readings are stated with each function).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and ``bench.py``'s CPU
leg.  The GPU library never imports it and it never imports the GPU library.

Conventions
-----------
* Patches are NHWC arrays ``x[n, y, x, c]``; a 16 x 16 output tile takes a
  24 x 24 input patch (4 nodes of halo per side, periodic wrap) and four
  valid 3 x 3 convolutions shrink it to 22, 20, 18 and 16.
* Layer l has weights ``W[l][dy, dx, ci, co]`` and bias ``b[l][co]``:
  z[p, co] = b[co] + sum_{dy, dx, ci} a[p + (dy, dx), ci] W[dy, dx, ci, co].
  ReLU follows layers 1-3, none follows layer 4.
* Network channels 4 -> 32 -> 32 -> 32 -> 9.
* Input channels: rho - 1, u_x, u_y (u = sum_i e_i f_i, the moments the
  method itself uses) and the signed distance to the marker polygon,
  positive outside, clipped to [-8, 8].
* Band: nodes with |sd| <= 4.  Target: the change of the equilibrium part
  that brings the coarse velocity to the fine one at unchanged density,
  df_i = f_i^eq(rho_c, u_hat) - f_i^eq(rho_c, u_c),
  with u_hat = 2 u_f at fine node (2x, 2y) (diffusive scaling: lattice
  velocities halve on the twice finer grid).
"""
from __future__ import annotations

import numpy as np

import oracle as O

CHANNELS = (4, 32, 32, 32, 9)
HALO = 4
TILE = 16
PATCH = TILE + 2 * HALO
BAND = 4.0
SD_CLIP = 8.0


# ---------------------------------------------------------------------------
# Network
# ---------------------------------------------------------------------------
def init_params(seed: int = 0, channels=CHANNELS):
    """He-normal weights, zero biases (FP64)."""
    rng = np.random.default_rng(seed)
    W, b = [], []
    for ci, co in zip(channels[:-1], channels[1:]):
        W.append(rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), size=(3, 3, ci, co)))
        b.append(np.zeros(co))
    return W, b


def conv3x3_valid(a: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """z[n, y, x, co] = b[co] + sum_{dy,dx,ci} a[n, y+dy, x+dx, ci] W[dy, dx, ci, co]
    (the nine shifted products summed in (dy, dx) order)."""
    n, h, w, _ = a.shape
    z = np.broadcast_to(b, (n, h - 2, w - 2, W.shape[3])).copy()
    for dy in range(3):
        for dx in range(3):
            z += np.tensordot(a[:, dy:dy + h - 2, dx:dx + w - 2, :], W[dy, dx], axes=([3], [0]))
    return z


def forward(W, b, x: np.ndarray):
    """Activations a_0 = x, a_1..a_3 (after ReLU) and the output z_4."""
    acts = [x]
    for l in range(4):
        z = conv3x3_valid(acts[-1], W[l], b[l])
        acts.append(np.maximum(z, 0.0) if l < 3 else z)
    return acts


def loss(out: np.ndarray, target: np.ndarray, mask: np.ndarray) -> float:
    """Mean squared error over the masked output pixels and all 9 channels."""
    m = mask[..., None].astype(np.float64)
    return float((m * (out - target) ** 2).sum() / (9.0 * max(mask.sum(), 1)))


def backward(W, b, acts, target: np.ndarray, mask: np.ndarray):
    """Gradients of `loss` with respect to every W[l] and b[l], by the chain
    rule through the four layers."""
    m = mask[..., None].astype(np.float64)
    dz = 2.0 * m * (acts[4] - target) / (9.0 * max(mask.sum(), 1))
    gW = [None] * 4
    gb = [None] * 4
    for l in range(3, -1, -1):
        a = acts[l]
        n, ho, wo, _ = dz.shape
        gb[l] = dz.sum(axis=(0, 1, 2))
        g = np.zeros_like(W[l])
        for dy in range(3):
            for dx in range(3):
                g[dy, dx] = np.tensordot(a[:, dy:dy + ho, dx:dx + wo, :], dz,
                                         axes=([0, 1, 2], [0, 1, 2]))
        gW[l] = g
        if l == 0:
            break
        da = np.zeros_like(a)
        for dy in range(3):
            for dx in range(3):
                da[:, dy:dy + ho, dx:dx + wo, :] += np.tensordot(dz, W[l][dy, dx], axes=([3], [1]))
        dz = da * (a > 0.0)
    return gW, gb


class Adam:
    """Adam (Kingma & Ba): first and second moment estimates with bias
    correction; FP64 master parameters."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for p, g, m, v in zip(params, grads, self.m, self.v):
            m *= self.b1
            m += (1.0 - self.b1) * g
            v *= self.b2
            v += (1.0 - self.b2) * g * g
            p -= self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps)


# ---------------------------------------------------------------------------
# Features, band, targets, correction
# ---------------------------------------------------------------------------
def _seg_dist(px, py, ax, ay, bx, by):
    """Distance from (px, py) to segment A-B: clamp the projection to [0, 1]."""
    dx, dy = bx - ax, by - ay
    ll = dx * dx + dy * dy
    t = np.clip(((px - ax) * dx + (py - ay) * dy) / ll, 0.0, 1.0)
    qx, qy = ax + t * dx - px, ay + t * dy - py
    return np.sqrt(qx * qx + qy * qy)


def inside_polygon(X: np.ndarray, px, py) -> np.ndarray:
    """Even-odd rule: a ray from the point towards +x crosses the closed
    polygon an odd number of times iff the point is inside (half-open test
    on the edge's y-range so that a vertex is counted once)."""
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    inside = np.zeros(px.shape, dtype=bool)
    N = len(X)
    for k in range(N):
        ax, ay = X[k]
        bx, by = X[(k + 1) % N]
        straddle = (ay > py) != (by > py)
        with np.errstate(divide="ignore", invalid="ignore"):
            xc = ax + (py - ay) * (bx - ax) / (by - ay)
        inside ^= straddle & (px < xc)
    return inside


def signed_distance(X: np.ndarray, px, py) -> np.ndarray:
    """Distance to the closed polygon through the markers, negative inside
    (brute force over all chords)."""
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    d = np.full(px.shape, np.inf)
    N = len(X)
    for k in range(N):
        ax, ay = X[k]
        bx, by = X[(k + 1) % N]
        d = np.minimum(d, _seg_dist(px, py, ax, ay, bx, by))
    return np.where(inside_polygon(X, px, py), -d, d)


def node_features(f: np.ndarray, X: np.ndarray):
    """Per-node channels (rho - 1, u_x, u_y, clipped sd) of a full field
    f[9][ny][nx] (pre-collision) and the unclipped sd."""
    _, ny, nx = f.shape
    ex, ey, _ = O.d2q9()
    rho = f.sum(axis=0)
    ux = np.tensordot(ex.astype(np.float64), f, axes=1)
    uy = np.tensordot(ey.astype(np.float64), f, axes=1)
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    sd = signed_distance(X, xx, yy)
    feat = np.stack([rho - 1.0, ux, uy, np.clip(sd, -SD_CLIP, SD_CLIP)], axis=-1)
    return feat, sd


def patch_amplitude(feat_patch: np.ndarray, in_scale) -> float:
    """s = max(rms over the patch nodes of |(rho - 1, u_x, u_y) * in_scale|, 1e-6):
    the network sees the flow channels divided by s and its output is
    multiplied back by s."""
    v = feat_patch[..., :3] * np.asarray(in_scale[:3], dtype=np.float64)
    return max(float(np.sqrt((v * v).sum(axis=-1).mean())), 1e-6)


def band_tiles(sd: np.ndarray):
    """Tiles (tx, ty) of 16 x 16 nodes holding a band node (|sd| <= 4), in
    row-major tile order."""
    ny, nx = sd.shape
    out = []
    for ty in range(ny // TILE):
        for tx in range(nx // TILE):
            if (np.abs(sd[ty * TILE:(ty + 1) * TILE, tx * TILE:(tx + 1) * TILE]) <= BAND).any():
                out.append((tx, ty))
    return out


def extract_patch(field: np.ndarray, tx: int, ty: int, halo: int = HALO) -> np.ndarray:
    """The (16 + 2 halo)^2 window of a periodic [ny][nx][...] field around
    tile (tx, ty)."""
    ny, nx = field.shape[:2]
    ys = (ty * TILE - halo + np.arange(TILE + 2 * halo)) % ny
    xs = (tx * TILE - halo + np.arange(TILE + 2 * halo)) % nx
    return field[np.ix_(ys, xs)]


def feq(rho, ux, uy) -> np.ndarray:
    """He-Luo incompressible equilibrium w_i [rho + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u]
    over arrays of nodes, shape (9,) + rho.shape."""
    ex, ey, w = O.d2q9()
    rho, ux, uy = (np.asarray(a, dtype=np.float64) for a in (rho, ux, uy))
    out = np.empty((9,) + rho.shape)
    for i in range(9):
        eu = ex[i] * ux + ey[i] * uy
        out[i] = w[i] * (rho + 3.0 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy))
    return out


def targets(f_coarse: np.ndarray, f_fine: np.ndarray) -> np.ndarray:
    """df[ny][nx][9] = f^eq(rho_c, u_hat) - f^eq(rho_c, u_c) at every coarse
    node, with u_hat twice the fine velocity at (2x, 2y)."""
    ex, ey, _ = O.d2q9()
    rc = f_coarse.sum(axis=0)
    uc = np.tensordot(ex.astype(np.float64), f_coarse, axes=1)
    vc = np.tensordot(ey.astype(np.float64), f_coarse, axes=1)
    ff = f_fine[:, ::2, ::2]
    uf = 2.0 * np.tensordot(ex.astype(np.float64), ff, axes=1)
    vf = 2.0 * np.tensordot(ey.astype(np.float64), ff, axes=1)
    d = feq(rc, uf, vf) - feq(rc, uc, vc)
    return np.moveaxis(d, 0, -1)


def apply_correction(f: np.ndarray, df: np.ndarray, sd: np.ndarray) -> None:
    """f_i(x) += df_i(x) at band nodes x (|sd(x)| <= 4), except on links
    (x - e_i -> x) whose ends lie on different sides of the polygon (sd < 0
    is inside); f is the pre-collision full field, changed in place."""
    ex, ey, _ = O.d2q9()
    ny, nx = sd.shape
    band = np.abs(sd) <= BAND
    ins = sd < 0.0
    for i in range(9):
        src = np.roll(np.roll(ins, int(ey[i]), axis=0), int(ex[i]), axis=1)  # inside(x - e_i)
        ok = band & ((src == ins) | (i == 0))
        f[i][ok] += df[..., i][ok]
