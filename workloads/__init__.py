"""Seeded synthetic inputs for the ghost-FEM multigrid solver.

This module only *generates inputs*: nodal level-set values, manufactured
solutions and right-hand sides, and the seeded draws of the batched workload.
It holds none of the method's arithmetic (no geometry, no quadrature, no
multigrid), so both the CPU oracle and the HIP path can be fed from it without
sharing any of the solver's code.

Grid convention: a uniform grid of N x N cells over the box
[x_lo, x_hi] x [y_lo, y_hi]; node (i, j) sits at (x_lo + i h, y_lo + j h) with
h = (x_hi - x_lo) / N, and its flat index is k = i + j (N + 1) (the single
index of the paper's two-dimensional transfer-operator section).
Arrays are returned as float64 numpy arrays of length (N + 1)**2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BOX = (-1.0, -1.0, 1.0, 1.0)
UNIT_BOX = (0.0, 0.0, 1.0, 1.0)


def grid_xy(N: int, box=BOX):
    """Node coordinates (x, y), each of shape ((N+1)**2,), x-index fastest."""
    x_lo, y_lo, x_hi, y_hi = box
    xs = x_lo + (x_hi - x_lo) * np.arange(N + 1, dtype=np.float64) / N
    ys = y_lo + (y_hi - y_lo) * np.arange(N + 1, dtype=np.float64) / N
    X, Y = np.meshgrid(xs, ys, indexing="xy")  # X[j, i] = xs[i]
    return X.ravel(), Y.ravel()


# ----------------------------------------------------------------------------
# Level sets (Omega = {psi < 0})
# ----------------------------------------------------------------------------

def circle(N, radius=0.5, center=(0.0, 0.0), box=BOX):
    """Signed distance to a circle: sqrt((x-cx)^2 + (y-cy)^2) - r."""
    x, y = grid_xy(N, box)
    return np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2) - radius


def circle_quadratic(N, radius=0.4, center=(0.5, 0.5), box=UNIT_BOX):
    """The disk of the paper's 2D tests, as a quadratic level set
    (x-xc)^2 + (y-yc)^2 - r^2 on [0,1]^2 (section 5.3, circular domain)."""
    x, y = grid_xy(N, box)
    return (x - center[0]) ** 2 + (y - center[1]) ** 2 - radius ** 2


def flower(N, center=(0.02, 0.03), r0=0.5, amp=0.1, petals=5, box=BOX):
    """Five-petal flower r - 0.5 - 0.1 sin(5 theta) about (0.02, 0.03)."""
    x, y = grid_xy(N, box)
    X = x - center[0]
    Y = y - center[1]
    r = np.sqrt(X * X + Y * Y)
    th = np.arctan2(Y, X)
    return r - r0 - amp * np.sin(petals * th)


def paper_flower(N, box=BOX):
    """The flower of the paper's 2D tests (section 5.3, flower-shaped domain):
    R - 0.52 - (Y^5 + 5 X^4 Y - 10 X^2 Y^3) / (5 R^5) about (0.03 sqrt 3, 0.04 sqrt 2)."""
    x, y = grid_xy(N, box)
    X = x - 0.03 * math.sqrt(3.0)
    Y = y - 0.04 * math.sqrt(2.0)
    R = np.sqrt(X * X + Y * Y)
    Rs = np.where(R == 0.0, 1.0, R)
    return R - 0.52 - (Y ** 5 + 5 * X ** 4 * Y - 10 * X ** 2 * Y ** 3) / (5 * Rs ** 5)


def hourglass(N, box=BOX):
    """The hourglass of the paper's 2D tests (section 5.3):
    256 Y^4 - 16 X^4 - 128 Y^2 + 36 X^2 about (0.03 sqrt 3, 0.04 sqrt 2)."""
    x, y = grid_xy(N, box)
    X = x - 0.03 * math.sqrt(3.0)
    Y = y - 0.04 * math.sqrt(2.0)
    return 256 * Y ** 4 - 16 * X ** 4 - 128 * Y ** 2 + 36 * X ** 2


def ellipse(N, a=0.7, b=0.35, phi=0.3, center=(0.0, 0.0), box=BOX):
    """Rotated ellipse b (sqrt((x'/a)^2 + (y'/b)^2) - 1), with
    x' = cos(phi)(x-cx) + sin(phi)(y-cy), y' = -sin(phi)(x-cx) + cos(phi)(y-cy)."""
    x, y = grid_xy(N, box)
    dx = x - center[0]
    dy = y - center[1]
    xp = math.cos(phi) * dx + math.sin(phi) * dy
    yp = -math.sin(phi) * dx + math.cos(phi) * dy
    return b * (np.sqrt((xp / a) ** 2 + (yp / b) ** 2) - 1.0)


def annulus(N, r1=0.5, r2=0.8, box=BOX):
    """The annulus of the paper's 2D tests (section 5.3): max(psi1, psi2) with
    psi1 = r1^2 - r^2 (inner circle) and psi2 = r^2 - r2^2 (outer circle),
    centred at the origin.  Returns (psi, chi) with the Neumann indicator
    chi = psi2 - psi1, positive on the outer circle (Neumann) and negative on
    the inner one (Dirichlet)."""
    x, y = grid_xy(N, box)
    r2s = x * x + y * y
    p1 = r1 * r1 - r2s
    p2 = r2s - r2 * r2
    return np.maximum(p1, p2), p2 - p1


LEAF_X1 = -0.25 * math.cos(math.pi / 4.0)
LEAF_X2 = 0.25 * math.sin(math.pi / 4.0)


def leaf(N, radius=0.7, box=BOX):
    """The leaf of the paper's 2D tests (section 5.3): max(R1, R2) - 0.7 with
    R_m the distance to (x_m, 0), x1 = -0.25 cos(pi/4), x2 = 0.25 sin(pi/4).
    Returns (psi, chi) with chi = -x: Neumann where x < 0, Dirichlet where
    x >= 0."""
    x, y = grid_xy(N, box)
    R1 = np.sqrt((x - LEAF_X1) ** 2 + y * y)
    R2 = np.sqrt((x - LEAF_X2) ** 2 + y * y)
    return np.maximum(R1 - radius, R2 - radius), -x


def vertical_line(N, theta, box=UNIT_BOX):
    """x - 1 + (1 - theta) h: the rectangle cut by a vertical line (section 5.3)."""
    x, _ = grid_xy(N, box)
    h = (box[2] - box[0]) / N
    return x - 1.0 + (1.0 - theta) * h


# ----------------------------------------------------------------------------
# Manufactured solutions: (u, f = -lap u) evaluated at the nodes
# ----------------------------------------------------------------------------

def mms_exp_sin(N, box=BOX):
    """u = exp(x) sin(y); harmonic, so f = 0."""
    x, y = grid_xy(N, box)
    u = np.exp(x) * np.sin(y)
    return u, np.zeros_like(u)


def mms_flower(N, box=BOX):
    """u = sin(pi x) cos(pi y) + x^2; f = -lap u = 2 pi^2 sin(pi x) cos(pi y) - 2."""
    x, y = grid_xy(N, box)
    s = np.sin(np.pi * x) * np.cos(np.pi * y)
    return s + x * x, 2.0 * np.pi ** 2 * s - 2.0


def mms_flower_grad(N, box=BOX):
    """Gradient (u_x, u_y) of the flower's manufactured solution."""
    x, y = grid_xy(N, box)
    ux = np.pi * np.cos(np.pi * x) * np.cos(np.pi * y) + 2.0 * x
    uy = -np.pi * np.sin(np.pi * x) * np.sin(np.pi * y)
    return ux, uy


def adjoint_target(N, box=BOX):
    """u_t = cos(2 pi x) sin(pi y) (the misfit target of the adjoint workload)."""
    x, y = grid_xy(N, box)
    return np.cos(2 * np.pi * x) * np.sin(np.pi * y)


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    name: str
    N: int
    psi: np.ndarray
    f: np.ndarray
    g: np.ndarray
    u_exact: np.ndarray | None = None
    box: tuple = BOX
    meta: dict = field(default_factory=dict)
    chi: np.ndarray | None = None   # Neumann indicator (None: Dirichlet everywhere)
    gN: np.ndarray | None = None    # nodal Neumann data


def circle_mms(N=64):
    """Circle r = 0.5, u = exp(x) sin(y), g = u at the nodes."""
    u, f = mms_exp_sin(N)
    return Problem("circle_mms", N, circle(N), f, u.copy(), u)


def flower_mms(N=1024):
    """Flower r - 0.5 - 0.1 sin(5 theta) about (0.02, 0.03), u = sin(pi x) cos(pi y) + x^2."""
    u, f = mms_flower(N)
    return Problem("flower_mms", N, flower(N), f, u.copy(), u)


def ellipse_mms(N=4096):
    """Ellipse (0.7, 0.35) rotated 0.3 rad, the flower's manufactured solution."""
    u, f = mms_flower(N)
    return Problem("ellipse_mms", N, ellipse(N), f, u.copy(), u)


def annulus_mms(N=256):
    """Annulus r1 = 0.5 (Dirichlet), r2 = 0.8 (Neumann); the flower's
    manufactured solution, g_D = u and g_N = (x, y)/r . grad u at the nodes
    (the outer circle's normal extended off the circle)."""
    u, f = mms_flower(N)
    ux, uy = mms_flower_grad(N)
    x, y = grid_xy(N)
    r = np.sqrt(x * x + y * y)
    gN = np.where(r > 0.0, (x * ux + y * uy) / np.where(r > 0.0, r, 1.0), 0.0)
    psi, chi = annulus(N)
    return Problem("annulus_mms", N, psi, f, u.copy(), u, chi=chi, gN=gN)


def leaf_mms(N=256):
    """Leaf, Neumann where x < 0; the flower's manufactured solution, g_D = u
    and g_N = the normal derivative of u on the circle about (x2, 0), which
    bounds the leaf on that side."""
    u, f = mms_flower(N)
    ux, uy = mms_flower_grad(N)
    x, y = grid_xy(N)
    R2 = np.sqrt((x - LEAF_X2) ** 2 + y * y)
    gN = ((x - LEAF_X2) * ux + y * uy) / np.where(R2 > 0.0, R2, 1.0)
    psi, chi = leaf(N)
    return Problem("leaf_mms", N, psi, f, u.copy(), u, chi=chi, gN=gN)


def linear_strip(N, axis=0, a=-0.61, b=0.57, c0=0.3, c1=1.7, box=BOX):
    """Strip a < x_axis < b across the box, Dirichlet on the side x_axis = a,
    Neumann on x_axis = b (chi = x_axis), u = c0 + c1 x_axis, f = 0, g_N = c1.
    g_D is u plus 5 where x_axis > 0, so that data read on the wrong side
    shows.  The box edges bound the strip with the natural condition, which
    u meets (its gradient is parallel to them)."""
    X = grid_xy(N, box)[axis]
    psi = np.maximum(a - X, X - b)
    u = c0 + c1 * X
    g = u + 5.0 * (X > 0.0)
    return Problem("linear_strip", N, psi, np.zeros_like(u), g, u, box=box, chi=X.copy(),
                   gN=np.full_like(u, c1), meta=dict(axis=axis))


def linear_rectangle(N, cx=0.03, cy=-0.02, half_t=0.7, half_n=0.35,
                     c0=0.2, c1=-1.3, neu_t=0.2, box=BOX):
    """Rectangle |s_t| < half_t, |s_n| < half_n tilted by phi = atan(1/2), with
    s_n = n . (x - c), s_t = t . (x - c), n = (-sin phi, cos phi),
    t = (cos phi, sin phi), inside the box.  u = c0 + c1 s_n, f = 0.

    Neumann (g_N = c1) on the middle part of the side s_n = half_n:
    chi = +1 at the nodes with s_n > 0.1 and |s_t| < neu_t, else -1.
    g_D = u, plus 5 deep inside the chi = +1 region (s_n > 0.2,
    |s_t| < neu_t - 3h), where only Neumann cells read it.

    The side s_n = half_n is the line y = x/2 + b; b is moved (through the
    centre's y) to an odd multiple of h/4, so that every node is at least
    h/4 cos(phi) from that line and none near it is snapped: the Neumann
    side stays straight after snapping, which the exact reproduction of u
    needs."""
    h = (box[2] - box[0]) / N
    phi = math.atan(0.5)
    b0 = cy - 0.5 * cx + half_n / math.cos(phi)
    lat = 0.5 * h                     # y - x/2 at the nodes: -0.5 + multiples of h/2
    b = -0.5 + (math.floor((b0 + 0.5) / lat) + 0.5) * lat
    cy = b + 0.5 * cx - half_n / math.cos(phi)
    x, y = grid_xy(N, box)
    dx, dy = x - cx, y - cy
    sn = -math.sin(phi) * dx + math.cos(phi) * dy
    st = math.cos(phi) * dx + math.sin(phi) * dy
    psi = np.maximum(np.abs(sn) - half_n, np.abs(st) - half_t)
    chi = np.where((sn > 0.1) & (np.abs(st) < neu_t), 1.0, -1.0)
    u = c0 + c1 * sn
    g = u + 5.0 * ((sn > 0.2) & (np.abs(st) < neu_t - 3 * h))
    return Problem("linear_rectangle", N, psi, np.zeros_like(u), g, u, box=box, chi=chi,
                   gN=np.full_like(u, c1), meta=dict(cx=cx, cy=cy, phi=phi))


def batched_draws(count=256, seed=0, sizes=(64, 128, 256, 512)):
    """Seeded random-ellipse problems of the batched workload.

    Draw order per problem (numpy default_rng(seed)): N from `sizes`,
    semi-axes a, b ~ U[0.2, 0.8], rotation ~ U[0, pi], centre ~ U[-0.1, 0.1]^2,
    then f ~ U[-1, 1] per node; g = 0.
    """
    rng = np.random.default_rng(seed)
    out = []
    for p in range(count):
        N = int(rng.choice(np.asarray(sizes)))
        a = float(rng.uniform(0.2, 0.8))
        b = float(rng.uniform(0.2, 0.8))
        phi = float(rng.uniform(0.0, math.pi))
        cx, cy = (float(v) for v in rng.uniform(-0.1, 0.1, size=2))
        psi = ellipse(N, a=a, b=b, phi=phi, center=(cx, cy))
        f = rng.uniform(-1.0, 1.0, size=(N + 1) ** 2)
        out.append(Problem(f"ellipse_{p}", N, psi, f, np.zeros_like(f), None,
                           meta=dict(a=a, b=b, phi=phi, cx=cx, cy=cy)))
    return out


def random_directions(n, count, seed=1):
    """Seeded standard-normal directions (count x n) for finite-difference checks."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((count, n))


def flower_mms_device(N, device, box=BOX):
    """flower_mms with the same formulas evaluated by torch on `device`
    (float64): (psi, f, g) as device tensors, for grids too large to build
    with numpy in reasonable time (N = 16384: 268M nodes per array).  Values
    agree with flower_mms up to the last bits of sin/cos/atan2."""
    import torch
    x_lo, y_lo, x_hi, y_hi = box
    xs = x_lo + (x_hi - x_lo) * torch.arange(N + 1, dtype=torch.float64, device=device) / N
    ys = y_lo + (y_hi - y_lo) * torch.arange(N + 1, dtype=torch.float64, device=device) / N
    y = ys.view(-1, 1).expand(N + 1, N + 1)
    x = xs.view(1, -1).expand(N + 1, N + 1)
    X, Y = x - 0.02, y - 0.03
    psi = (torch.sqrt(X * X + Y * Y) - 0.5 - 0.1 * torch.sin(5 * torch.atan2(Y, X))).reshape(-1)
    del X, Y
    s = torch.sin(math.pi * x) * torch.cos(math.pi * y)
    g = (s + x * x).reshape(-1)
    f = (2.0 * math.pi ** 2 * s - 2.0).reshape(-1)
    return psi, f, g
