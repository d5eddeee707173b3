"""Arithmetic model of the device's network (test infrastructure): the FP64
oracle network of oracle/mlp_oracle.py with every operand of a matrix product
rounded to BF16 where the device's kernels round it.  The parity tolerances
of the network tests are derived from it, on the CPU, before any device
output is seen: the model's error against the exact FP64 network is the
error that BF16 operands with FP32 accumulation imply.

Where the device rounds (and the model with it):
* evaluation (and the push): the 128 features and their three tangents, and
  after each hidden layer the activation and its three tangents, enter the
  next product as BF16, in log2 units (times log2(e)); the weights are BF16
  (the test networks are BF16-representable, so they are exact); products
  accumulate in FP32;
* training: the stored activations H_0..H_6 and the pre-activation
  gradients dZ are BF16, the pre-activations Z, the output gradients and the
  output layer's backward product are FP32.

Each rounding to BF16 (8 significant bits) moves a value by at most 2^-8
of itself.  FP32 accumulation of 128 terms adds at most 128 x 2^-24
relative, 1/500 of one BF16 rounding, and the model keeps FP64 there.  The
device computes the values it rounds in FP32 (features, exp2 and reciprocal
in hardware, sums in another order), so a value within about 1e-7 of a
rounding midpoint can round the other way; the training kernels' partial
sums differ in order.  The tests therefore bound the device by a small
multiple of the model's error (MAX_OVER_MODEL, RMS_OVER_MODEL), not by the
model's error itself.
"""
from __future__ import annotations

import numpy as np

from oracle import mlp_oracle as M

# Bars: the device's maximum errors within 3x the model's maximum over a
# large sample of points, its RMS errors within 2x the model's RMS: the same
# error distribution realised by different roundings (see above).
MAX_OVER_MODEL = 3.0
RMS_OVER_MODEL = 2.0


def bf16(a):
    """Nearest BF16-representable values (round half to even), as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


LOG2E, LN2 = 1.4426950408889634, 0.6931471805599453


def forward_jvp(params, h0, dh0, rnd=bf16):
    """oracle.mlp_oracle.forward_jvp with the operands of every product rounded
    where the evaluation kernels round them: they carry activations and
    tangents in log2 units (h log2(e), biases scaled by log2(e), the output
    product by ln 2), so the values rounded are log2(e) times the activations."""
    h, dh = rnd(LOG2E * h0), rnd(LOG2E * dh0)
    for l in range(1, M.DEPTH + 1):
        W = params[f"W{l}"]
        z = h @ W.T + LOG2E * params[f"c{l}"]          # log2(e) times the pre-activation
        dz = dh @ W.T
        h, dh = rnd(LOG2E * M.silu(LN2 * z)), rnd(M.dsilu(LN2 * z)[None] * dz)
    return LN2 * (h @ params["Wo"].T) + params["co"], LN2 * (dh @ params["Wo"].T)


def field(spec, params, r, th, ph, rnd=bf16):
    """oracle.mlp_oracle.field through the rounded network."""
    saved = M.forward_jvp
    try:
        M.forward_jvp = lambda p, h0, dh0: forward_jvp(p, h0, dh0, rnd)
        return M.field(spec, params, r, th, ph)
    finally:
        M.forward_jvp = saved


def loss_and_grad(spec, params, pts, tgt, pts2, tgt2, wc, beta, rnd=bf16):
    """oracle.mlp_oracle.loss_and_grad with the training kernels' roundings:
    BF16 activations (forward and weight-gradient products) and BF16
    pre-activation gradients; FP64 elsewhere."""
    env1, _ = M.envelope(spec, pts[:, 0])
    env2, _ = M.envelope(spec, pts2[:, 0])
    t1, t2 = tgt / env1, tgt2 / env2

    def fwd(p):
        h0, _ = M.features(spec, p[:, 0], p[:, 1], p[:, 2])
        hs, zs = [rnd(h0)], []
        for l in range(1, M.DEPTH + 1):
            z = hs[-1] @ params[f"W{l}"].T + params[f"c{l}"]
            zs.append(z)
            hs.append(rnd(M.silu(z)))
        return hs[-1] @ params["Wo"].T + params["co"], zs, hs

    y1, z1, hs1 = fwd(pts)
    y2, z2, hs2 = fwd(pts2)
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
        for l in range(M.DEPTH, 0, -1):
            gz = rnd(gh * M.dsilu(zs[l - 1]))
            grads[f"W{l}"] += gz.T @ hs[l - 1]
            grads[f"c{l}"] += gz.sum(0)
            gh = gz @ params[f"W{l}"]
    return L, grads


def field_scales(spec, params, pts, exact):
    """Per-point scales of the four vectors: |B|, |E|, the Jacobian norm of B
    in the local basis (grad|B| is a projection of it) and that norm over
    |B| plus 1/r (the scale of the field-line curvature (b.grad)b)."""
    r, th = pts[0], pts[1]
    h0, dh0 = M.features(spec, pts[0], pts[1], pts[2])
    y, dy = M.forward_jvp(params, h0, dh0)
    env, denv = M.envelope(spec, r)
    J = np.stack([denv[:, :3] * y[:, :3] + env[:, :3] * dy[0][:, :3], env[:, :3] * dy[1][:, :3] / r[:, None],
                  env[:, :3] * dy[2][:, :3] / (r * np.sin(th))[:, None]])
    jn = np.sqrt(np.sum(J ** 2, axis=(0, 2)))
    bn = np.linalg.norm(exact[:, 0:3], axis=1)
    return {"B": bn, "E": np.linalg.norm(exact[:, 3:6], axis=1), "G": jn, "K": jn / bn + 1.0 / r}


VECTORS = (("B", slice(0, 3)), ("E", slice(3, 6)), ("G", slice(6, 9)), ("K", slice(9, 12)))


def field_errors(got, exact, scales):
    """Per-point relative errors of the four vectors."""
    return {name: np.linalg.norm(got[:, sl] - exact[:, sl], axis=1) / scales[name] for name, sl in VECTORS}


def eval_bars(spec, params, pts):
    """(max, rms) bars of the evaluation test per vector, from the model's
    errors at the points pts [3, n]."""
    exact = M.field(spec, params, pts[0], pts[1], pts[2])
    model = field(spec, params, pts[0], pts[1], pts[2])
    errs = field_errors(model, exact, field_scales(spec, params, pts, exact))
    return {k: (MAX_OVER_MODEL * float(e.max()), RMS_OVER_MODEL * float(np.sqrt(np.mean(e ** 2))))
            for k, e in errs.items()}
