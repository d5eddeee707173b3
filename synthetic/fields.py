"""Gridded steady fields: node values of B, E, grad|B| and (b.grad)b.

The paper drives its electrons with a steady MHD wind (Sect. 2.1) that is not
available here; these seeded analytic winds stand in for it.

* ``parker``: the Parker spiral with radial wind V and rotation Omega,
  B_r = a0 / r^2, B_ph = -B_r * Omega r sin(th) / V, with ideal Ohm's law
  E = -u x B (Sect. 2.2) for u = V r^.
* ``perturbed_parker``: the same plus a sum of divergence-free Fourier modes
  with amplitude eps * |B_parker| (a synthetic stand-in for the structure of a
  simulated wind).
* ``affine``: every component affine in (r, th) and constant in ph, so that
  trilinear interpolation reproduces it exactly (smooth right-hand side on a
  grid, used for order-of-accuracy tests).
* ``mirror`` and ``straight``: textbook fields (radial B growing with r; radial
  uniform B with no E and no gradients).

B is built in Cartesian coordinates; its Jacobian comes from forward-mode
automatic differentiation (torch.autograd.forward_ad), and
  grad|B|   = J^T b,
  (b.grad)b = (J b - b (b . J b)) / |B|,
before all vectors are projected on the local basis (r^, th^, ph^) at the node.
Everything is float64.  The builder runs on any torch device.

For the full guiding-centre equations (the terms of Eqs. 1-2 with derivatives
of b and v_E) a second node array holds, in the same local basis,
  A = (v_E.grad) b,   C = (b.grad) v_E,   D = (v_E.grad) v_E,
with v_E = E x B / B^2, each a directional derivative taken by forward-mode
automatic differentiation along v_E or b at the node (``*_extra`` builders,
[nr][nth][nph][9]).
"""
from __future__ import annotations

import math
from typing import Callable

import numpy as np
import torch
import torch.autograd.forward_ad as fwAD

from .constants import AU, OMEGA_SUN, V_WIND, B0_1AU
from .grid import SphericalGrid, N_COMP, N_EXTRA


# ----------------------------------------------------------------------------
# Cartesian magnetic fields (torch, differentiable)
# ----------------------------------------------------------------------------
def parker_B(x, y, z, a0=B0_1AU * AU * AU, omega=OMEGA_SUN, v=V_WIND):
    """Parker spiral in Cartesian components.  B_ph ph^ = -(omega/v) B_r (-y, x, 0)."""
    r2 = x * x + y * y + z * z
    r = torch.sqrt(r2)
    br = a0 / r2
    w = omega / v
    bx = br * x / r + w * br * y
    by = br * y / r - w * br * x
    bz = br * z / r
    return bx, by, bz


def parker_Bmag(x, y, z, a0=B0_1AU * AU * AU, omega=OMEGA_SUN, v=V_WIND):
    r2 = x * x + y * y + z * z
    w = omega / v
    return (a0 / r2) * torch.sqrt(1.0 + w * w * (x * x + y * y))


def draw_modes(seed: int, n_modes: int = 16, k_lo: float = 2.0 / AU, k_hi: float = 20.0 / AU):
    """Seeded Fourier modes: |k| ~ U[k_lo, k_hi], k^ isotropic, xi perpendicular
    to k (each mode divergence-free), phase ~ U[0, 2pi), equal amplitudes with
    unit rms of the sum."""
    rng = np.random.default_rng(seed)
    kmag = rng.uniform(k_lo, k_hi, n_modes)
    cos_t = rng.uniform(-1.0, 1.0, n_modes)
    phk = rng.uniform(0.0, 2.0 * math.pi, n_modes)
    chi = rng.uniform(0.0, 2.0 * math.pi, n_modes)
    psi = rng.uniform(0.0, 2.0 * math.pi, n_modes)
    sin_t = np.sqrt(1.0 - cos_t ** 2)
    khat = np.stack([sin_t * np.cos(phk), sin_t * np.sin(phk), cos_t], axis=1)
    # orthonormal pair perpendicular to khat
    ref = np.where(np.abs(khat[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    e1 = np.cross(khat, ref)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(khat, e1)
    xi = np.cos(chi)[:, None] * e1 + np.sin(chi)[:, None] * e2
    amp = np.full(n_modes, math.sqrt(2.0 / n_modes))
    return {"k": khat * kmag[:, None], "xi": xi, "psi": psi, "amp": amp}


def perturbed_parker_B(modes, eps=0.1):
    k = modes["k"]
    xi = modes["xi"]
    psi = modes["psi"]
    amp = modes["amp"]

    def fn(x, y, z):
        bx, by, bz = parker_B(x, y, z)
        env = eps * parker_Bmag(x, y, z)
        sx = torch.zeros_like(x)
        sy = torch.zeros_like(x)
        sz = torch.zeros_like(x)
        for i in range(len(psi)):
            c = amp[i] * torch.cos(k[i, 0] * x + k[i, 1] * y + k[i, 2] * z + psi[i])
            sx = sx + xi[i, 0] * c
            sy = sy + xi[i, 1] * c
            sz = sz + xi[i, 2] * c
        return bx + env * sx, by + env * sy, bz + env * sz

    return fn


# ----------------------------------------------------------------------------
# node evaluation
# ----------------------------------------------------------------------------
def _node_coords(grid: SphericalGrid, i0: int, i1: int, device):
    r = torch.as_tensor(grid.r_nodes()[i0:i1], dtype=torch.float64, device=device)
    th = torch.as_tensor(grid.th_nodes(), dtype=torch.float64, device=device)
    ph = torch.as_tensor(grid.ph_nodes(), dtype=torch.float64, device=device)
    R, TH, PH = torch.meshgrid(r, th, ph, indexing="ij")
    return R.reshape(-1), TH.reshape(-1), PH.reshape(-1)


def _local_from_cartesian(bfun: Callable, r, th, ph, v_wind: float):
    st, ct = torch.sin(th), torch.cos(th)
    sp, cp = torch.sin(ph), torch.cos(ph)
    x, y, z = r * st * cp, r * st * sp, r * ct
    pos = torch.stack([x, y, z])
    jac = []
    with fwAD.dual_level():
        for j in range(3):
            tan = torch.zeros_like(pos)
            tan[j] = 1.0
            dual = fwAD.make_dual(pos, tan)
            comps = bfun(dual[0], dual[1], dual[2])
            prim, tang = [], []
            for c in comps:
                p, t = fwAD.unpack_dual(c)
                prim.append(p)
                tang.append(t)
            jac.append(torch.stack(tang))          # column j: dB_i/dx_j
            B = torch.stack(prim)
    J = torch.stack(jac, dim=1)                    # [i][j][n]
    Bmag = torch.sqrt((B * B).sum(0))
    b = B / Bmag
    G = (J * b[:, None, :]).sum(0)                 # G_j = sum_i b_i J_ij
    Jb = (J * b[None, :, :]).sum(1)                # (J b)_i
    K = (Jb - b * (b * Jb).sum(0)) / Bmag
    rhat = torch.stack([st * cp, st * sp, ct])
    E = -v_wind * torch.linalg.cross(rhat, B, dim=0)
    thhat = torch.stack([ct * cp, ct * sp, -st])
    phhat = torch.stack([-sp, cp, torch.zeros_like(sp)])
    out = []
    for vec in (B, E, G, K):
        out.append((vec * rhat).sum(0))
        out.append((vec * thhat).sum(0))
        out.append((vec * phhat).sum(0))
    return torch.stack(out, dim=1)                 # [n][12]


def _cross(a, b):
    return torch.stack([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def _extra_from_cartesian(bfun: Callable, r, th, ph, v_wind: float):
    """A = (v_E.grad) b, C = (b.grad) v_E, D = (v_E.grad) v_E at the nodes, [n][9]."""
    st, ct = torch.sin(th), torch.cos(th)
    sp, cp = torch.sin(ph), torch.cos(ph)
    pos = torch.stack([r * st * cp, r * st * sp, r * ct])

    def b_and_vE(q):
        B = torch.stack(bfun(q[0], q[1], q[2]))
        rhat = q / torch.sqrt((q * q).sum(0))
        E = -v_wind * _cross(rhat, B)
        B2 = (B * B).sum(0)
        return B / torch.sqrt(B2), _cross(E, B) / B2

    b0, vE0 = b_and_vE(pos)
    with fwAD.dual_level():
        b1, vE1 = b_and_vE(fwAD.make_dual(pos, vE0))
        A = torch.stack([fwAD.unpack_dual(c).tangent for c in b1])
        D = torch.stack([fwAD.unpack_dual(c).tangent for c in vE1])
    with fwAD.dual_level():
        _, vE2 = b_and_vE(fwAD.make_dual(pos, b0))
        C = torch.stack([fwAD.unpack_dual(c).tangent for c in vE2])
    rhat = torch.stack([st * cp, st * sp, ct])
    thhat = torch.stack([ct * cp, ct * sp, -st])
    phhat = torch.stack([-sp, cp, torch.zeros_like(sp)])
    out = []
    for vec in (A, C, D):
        out.append((vec * rhat).sum(0))
        out.append((vec * thhat).sum(0))
        out.append((vec * phhat).sum(0))
    return torch.stack(out, dim=1)                 # [n][9]


def _build(grid: SphericalGrid, bfun: Callable, v_wind: float, device=None, slab: int = 0,
           extra: bool = False) -> np.ndarray:
    device = torch.device("cpu") if device is None else torch.device(device)
    if slab <= 0:   # r-slices per batch: ~4M nodes on a GPU, ~0.25M on the host
        per = grid.nth * grid.nph
        slab = max(1, (4_000_000 if device.type == "cuda" else 250_000) // per)
    nc = N_EXTRA if extra else N_COMP
    out = np.empty(grid.shape()[:3] + (nc,), dtype=np.float64)
    for i0 in range(0, grid.nr, slab):
        i1 = min(grid.nr, i0 + slab)
        r, th, ph = _node_coords(grid, i0, i1, device)
        vals = (_extra_from_cartesian if extra else _local_from_cartesian)(bfun, r, th, ph, v_wind)
        out[i0:i1] = vals.reshape(i1 - i0, grid.nth, grid.nph, nc).cpu().numpy()
    return out


def parker(grid: SphericalGrid, device=None) -> np.ndarray:
    """Parker spiral node values, float64 [nr][nth][nph][12]."""
    return _build(grid, parker_B, V_WIND, device)


def perturbed_parker(grid: SphericalGrid, seed: int = 1, eps: float = 0.1,
                     n_modes: int = 16, device=None) -> np.ndarray:
    """Parker spiral plus seeded Fourier perturbation, float64 [nr][nth][nph][12]."""
    modes = draw_modes(seed, n_modes)
    return _build(grid, perturbed_parker_B(modes, eps), V_WIND, device)


def parker_extra(grid: SphericalGrid, device=None) -> np.ndarray:
    """(v_E.grad) b, (b.grad) v_E, (v_E.grad) v_E of the Parker spiral, [nr][nth][nph][9]."""
    return _build(grid, parker_B, V_WIND, device, extra=True)


def perturbed_parker_extra(grid: SphericalGrid, seed: int = 1, eps: float = 0.1,
                           n_modes: int = 16, device=None) -> np.ndarray:
    """The same terms for the perturbed spiral, [nr][nth][nph][9]."""
    modes = draw_modes(seed, n_modes)
    return _build(grid, perturbed_parker_B(modes, eps), V_WIND, device, extra=True)


# Affine test field: value = a + b * (r - r_ref) / AU + c * (th - pi/2), per component.
AFFINE_COEFFS = np.array([
    # a           b (per AU)   c (per rad)
    [2.0e-8,     -1.0e-8,      2.0e-9],     # Br
    [0.0,         1.0e-10,     5.0e-10],    # Bth
    [-8.0e-9,     3.0e-9,     -1.0e-9],     # Bph
    [0.0,         1.0e-5,      0.0],        # Er
    [-3.3e-3,     1.0e-3,      2.0e-4],     # Eth
    [0.0,         0.0,         1.0e-4],     # Eph
    [-5.8e-19,    2.0e-19,     1.0e-20],    # Gr
    [1.0e-20,     0.0,         2.0e-20],    # Gth
    [0.0,         1.0e-21,     0.0],        # Gph
    [-2.0e-12,    5.0e-13,     1.0e-13],    # Kr
    [-1.0e-12,    2.0e-13,     0.0],        # Kth
    [-3.0e-12,    1.0e-12,     2.0e-13],    # Kph
], dtype=np.float64)


def affine(grid: SphericalGrid, r_ref: float = 0.5 * AU, coeffs: np.ndarray = AFFINE_COEFFS) -> np.ndarray:
    r = grid.r_nodes()[:, None, None, None]
    th = grid.th_nodes()[None, :, None, None]
    out = (coeffs[:, 0] + coeffs[:, 1] * (r - r_ref) / AU + coeffs[:, 2] * (th - 0.5 * math.pi))
    return np.ascontiguousarray(np.broadcast_to(out, grid.shape()), dtype=np.float64)


def affine_at(r: float, th: float, r_ref: float = 0.5 * AU, coeffs: np.ndarray = AFFINE_COEFFS) -> np.ndarray:
    return coeffs[:, 0] + coeffs[:, 1] * (r - r_ref) / AU + coeffs[:, 2] * (th - 0.5 * math.pi)


def mirror(grid: SphericalGrid, b1: float = 1.0e-8, r_a: float = 0.3 * AU, length: float = 0.5 * AU) -> np.ndarray:
    """Radial field B_r = b1 (1 + (r - r_a)/L), no E, straight field lines:
    grad|B| = (b1/L, 0, 0) and (b.grad)b = 0."""
    out = np.zeros(grid.shape(), dtype=np.float64)
    r = grid.r_nodes()
    out[..., 0] = (b1 * (1.0 + (r - r_a) / length))[:, None, None]
    out[..., 6] = b1 / length
    return out


def straight(grid: SphericalGrid, b1: float = 1.0e-8) -> np.ndarray:
    """Radial B of constant local magnitude, no E, no gradient, no curvature."""
    out = np.zeros(grid.shape(), dtype=np.float64)
    out[..., 0] = b1
    return out
