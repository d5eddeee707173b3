"""FP64 NumPy oracle of the neural field (test infrastructure only).

A Fourier-feature multilayer perceptron stands in for the gridded field:
  x~ = ((r - r_min)/(r_max - r_min), th/pi),  psi_j = 2 pi (a_j r~ + b_j th~) + n_j ph   (n_j integer:
        periodic in ph),  j = 0..63
  h0 = [sin psi_0, cos psi_0, sin psi_1, cos psi_1, ...]                 (128 features)
  h_l = silu(W_l h_{l-1} + c_l),  l = 1..6,  W_l 128x128,  silu(z) = z / (1 + e^-z)
  y^ = W_o h_6 + c_o                                                   (6 outputs)
  B_i = S_i (r_ref/r)^p_i y^_i (i = 0..2),  E_i = S_{i+3} (r_ref/r)^p_{i+3} y^_{i+3}
grad|B| and (b.grad)b follow from the derivatives of B with respect to
(r, th, ph), obtained by forward-mode propagation of three tangents through the
network, with the metric factors and connection terms of the local spherical
basis:
  grad|B| = (d_r |B|, d_th |B| / r, d_ph |B| / (r sin th)),
  ((b.grad) b)_r  = D b_r - (b_th^2 + b_ph^2)/r
  ((b.grad) b)_th = D b_th + b_r b_th / r - b_ph^2 cot(th)/r
  ((b.grad) b)_ph = D b_ph + b_r b_ph / r + b_th b_ph cot(th)/r
  with D f = b_r d_r f + (b_th/r) d_th f + (b_ph/(r sin th)) d_ph f.
Training loss (per batch of N points, weights w_c on the 6 normalized outputs):
  L = (1/N) sum_n sum_c w_c (y^_c(x_n) - t_c(x_n))^2
    + (beta/N) sum_n sum_c w_c ((y^_c(x'_n) - y^_c(x_n)) - (t_c(x'_n) - t_c(x_n)))^2
where t = target / envelope and x'_n a nearby point: the second term fits the
differences of the field between paired points, i.e. its derivatives.
"""
from __future__ import annotations

import math
import numpy as np

from synthetic.mlp_setup import N_FREQ, WIDTH, DEPTH, N_OUT, MLPSpec, init_params, make_spec  # noqa: F401


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def _phases(spec: MLPSpec, r, th, ph):
    rt = (r - spec.r_min) / (spec.r_max - spec.r_min)
    tt = th / math.pi
    a, b, n = spec.freq[:, 0], spec.freq[:, 1], spec.freq[:, 2]
    psi = 2 * math.pi * (np.outer(rt, a) + np.outer(tt, b)) + np.outer(ph, n)
    dpsi = np.stack([np.broadcast_to(2 * math.pi * a / (spec.r_max - spec.r_min), psi.shape),
                     np.broadcast_to(2 * b, psi.shape),          # d/dth of 2 pi b th / pi
                     np.broadcast_to(n, psi.shape)])
    return psi, dpsi


def features(spec: MLPSpec, r, th, ph):
    """h0 [N,128] and its derivatives with respect to (r, th, ph): [3, N, 128]."""
    psi, dpsi = _phases(spec, r, th, ph)
    N = psi.shape[0]
    h0 = np.empty((N, 2 * N_FREQ))
    h0[:, 0::2] = np.sin(psi)
    h0[:, 1::2] = np.cos(psi)
    dh0 = np.empty((3, N, 2 * N_FREQ))
    for d in range(3):
        dh0[d][:, 0::2] = np.cos(psi) * dpsi[d]
        dh0[d][:, 1::2] = -np.sin(psi) * dpsi[d]
    return h0, dh0


def forward(params, h0, keep=False):
    """Normalized outputs y^ [N,6]; with keep, the pre-activations and activations."""
    hs, zs = [h0], []
    h = h0
    for l in range(1, DEPTH + 1):
        z = h @ params[f"W{l}"].T + params[f"c{l}"]
        h = silu(z)
        zs.append(z)
        hs.append(h)
    y = h @ params["Wo"].T + params["co"]
    return (y, zs, hs) if keep else y


def forward_jvp(params, h0, dh0):
    """y^ [N,6] and dy^/d(r,th,ph) [3,N,6] by forward-mode propagation."""
    h, dh = h0, dh0
    for l in range(1, DEPTH + 1):
        W = params[f"W{l}"]
        z = h @ W.T + params[f"c{l}"]
        dz = dh @ W.T
        h, dh = silu(z), dsilu(z)[None] * dz
    return h @ params["Wo"].T + params["co"], dh @ params["Wo"].T


def envelope(spec: MLPSpec, r):
    """env [N,6] and d env / dr [N,6]."""
    env = spec.scale[None, :] * (spec.r_ref / r[:, None]) ** spec.power[None, :]
    return env, -spec.power[None, :] * env / r[:, None]


def field(spec: MLPSpec, params, r, th, ph):
    """The 12 field components (local basis) at the points: [N, 12]."""
    r, th, ph = (np.asarray(v, dtype=np.float64) for v in (r, th, ph))
    h0, dh0 = features(spec, r, th, ph)
    y, dy = forward_jvp(params, h0, dh0)
    env, denv = envelope(spec, r)
    B = env[:, 0:3] * y[:, 0:3]
    E = env[:, 3:6] * y[:, 3:6]
    dB = np.stack([denv[:, 0:3] * y[:, 0:3] + env[:, 0:3] * dy[0][:, 0:3],
                   env[:, 0:3] * dy[1][:, 0:3], env[:, 0:3] * dy[2][:, 0:3]])   # [3 (d/dr,dth,dph), N, 3]
    Bm = np.linalg.norm(B, axis=1)
    b = B / Bm[:, None]
    dBm = np.einsum("dni,ni->dn", dB, b)                                      # d|B|
    st, ct = np.sin(th), np.cos(th)
    G = np.stack([dBm[0], dBm[1] / r, dBm[2] / (r * st)], axis=1)
    db = (dB - b[None] * dBm[:, :, None]) / Bm[None, :, None]                  # d b_i
    D = b[:, 0][:, None] * db[0] + (b[:, 1] / r)[:, None] * db[1] + (b[:, 2] / (r * st))[:, None] * db[2]
    K = np.empty_like(B)
    K[:, 0] = D[:, 0] - (b[:, 1] ** 2 + b[:, 2] ** 2) / r
    K[:, 1] = D[:, 1] + b[:, 0] * b[:, 1] / r - b[:, 2] ** 2 * ct / (st * r)
    K[:, 2] = D[:, 2] + b[:, 0] * b[:, 2] / r + b[:, 1] * b[:, 2] * ct / (st * r)
    return np.concatenate([B, E, G, K], axis=1)


def loss_and_grad(spec: MLPSpec, params, pts, tgt, pts2, tgt2, wc, beta):
    """Training loss of the module docstring and its gradient (hand-written
    reverse mode).  pts/pts2: [N,3] paired points; tgt/tgt2: [N,6] field targets
    (physical B, E); wc: [6] output weights."""
    env1, _ = envelope(spec, pts[:, 0])
    env2, _ = envelope(spec, pts2[:, 0])
    t1, t2 = tgt / env1, tgt2 / env2
    h01, _ = features(spec, pts[:, 0], pts[:, 1], pts[:, 2])
    h02, _ = features(spec, pts2[:, 0], pts2[:, 1], pts2[:, 2])
    y1, z1, hs1 = forward(params, h01, keep=True)
    y2, z2, hs2 = forward(params, h02, keep=True)
    N = pts.shape[0]
    e1 = y1 - t1
    e12 = (y2 - y1) - (t2 - t1)
    L = (np.sum(wc * e1 ** 2) + beta * np.sum(wc * e12 ** 2)) / N
    gy1 = (2 * wc * e1 - 2 * beta * wc * e12) / N
    gy2 = (2 * beta * wc * e12) / N
    grads = {k: np.zeros_like(v) for k, v in params.items()}
    for gy, zs, hs in ((gy1, z1, hs1), (gy2, z2, hs2)):
        grads["Wo"] += gy.T @ hs[-1]
        grads["co"] += gy.sum(0)
        gh = gy @ params["Wo"]
        for l in range(DEPTH, 0, -1):
            gz = gh * dsilu(zs[l - 1])
            grads[f"W{l}"] += gz.T @ hs[l - 1]
            grads[f"c{l}"] += gz.sum(0)
            gh = gz @ params[f"W{l}"]
    return L, grads
