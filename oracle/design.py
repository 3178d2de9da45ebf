"""FP64 CPU oracle of the design-space steps of the optimization loop.

This module is test infrastructure only: the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; it shares no code with the
HIP library and does not import it.  It follows Zhang et al., arXiv
2301.08911:

* Sec. 6.1 "Symmetry": the density is averaged over the orbits of one of
  three symmetry groups of the cube: reflect3 (mirror planes x, y, z = 0.5),
  reflect6 (those and the three diagonal planes x = y, y = z, z = x) and
  rotate3 (quarter turns about the three axes through the centre, and their
  compositions).
* Sec. 6.2 "Density initializations": a random combination of trigonometric
  basis functions of rotated coordinates and of their pairwise products,
  projected into [rho_min, 1] by a steep sigmoid whose shift meets the volume
  constraint.
* Sec. 5.3 (material interpolation without density filtering) and the OC
  optimizer's sensitivity filter: the sensitivity is smoothed with the
  density-weighted cone filter before the OC update.
* Sec. 5.2 / 5.3: the objectives F(C^H) (bulk, shear, relaxed Poisson,
  logarithmic Poisson) and their gradients W = dF/dC^H, which the element
  sensitivities contract (sum_ij W_ij dC_ij / drho_e).
* Sec. 6 (experiment parameters): the stopping rule.

Readings where the paper is silent or garbled (each also in the design
notes): the diagonal mirror planes, printed as "x+y=0" etc., are x = y,
y = z, z = x through the cube's centre; the products of Q_n run over unordered
pairs with repetition (squares included); the sigmoid shift is found by
bisection; the sensitivity filter is Sigmund's density-weighted form with the
floor 1e-3 in the denominator; the objective's relative change is measured
against the previous value.

Layout: element index e = x + nx (y + ny z), arrays of n values.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

# ---------------------------------------------------------------------------
# Symmetry (Sec. 6.1)
# ---------------------------------------------------------------------------

SYMMETRIES = ("reflect3", "reflect6", "rotate3")


def _perm_sign(perm) -> int:
    """Sign of a permutation of (0, 1, 2)."""
    s = 1
    p = list(perm)
    for i in range(3):
        for j in range(i + 1, 3):
            if p[i] > p[j]:
                s = -s
    return s


def symmetry_group(kind: str):
    """The group as a list of signed axis permutations (perm, flips).

    The image of element coordinates c = (c0, c1, c2) (c0 = x) is
    c'_a = N - 1 - c_{perm[a]} if flips[a] else c_{perm[a]}: output axis a
    takes input axis perm[a], mirrored about the centre if flips[a].  The
    linear part is a signed permutation matrix; reflect3 keeps the identity
    permutation, reflect6 is every signed permutation (the full symmetry
    group of the cube, 48 elements), rotate3 those of determinant +1 (24).
    """
    out = []
    for perm in itertools.permutations(range(3)):
        for flips in itertools.product((0, 1), repeat=3):
            det = _perm_sign(perm) * (-1) ** sum(flips)
            if kind == "reflect3" and perm != (0, 1, 2):
                continue
            if kind == "rotate3" and det != 1:
                continue
            if kind not in SYMMETRIES:
                raise ValueError(kind)
            out.append((perm, flips))
    return out


def symmetrize(x, shape, kind: str) -> np.ndarray:
    """Average of x over the group: x_s(e) = (1/|G|) sum_g x(g e).

    reflect3 works on any box; reflect6 and rotate3 need a cube."""
    nx, ny, nz = shape
    if kind != "reflect3" and not (nx == ny == nz):
        raise ValueError("reflect6 and rotate3 need a cubic grid")
    a = np.asarray(x, dtype=np.float64).reshape(nz, ny, nx)
    dims = (nx, ny, nz)
    cz, cy, cx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coords = (cx, cy, cz)
    acc = np.zeros_like(a)
    G = symmetry_group(kind)
    for perm, flips in G:
        img = []
        for ax in range(3):
            c = coords[perm[ax]]
            img.append(dims[ax] - 1 - c if flips[ax] else c)
        acc += a[img[2], img[1], img[0]]
    return (acc / len(G)).ravel()


def orbit_count(n: int, kind: str) -> int:
    """Number of orbits of the group on the n^3 cells (Burnside's lemma:
    the mean number of cells each group element leaves fixed)."""
    total = 0
    G = symmetry_group(kind)
    for perm, flips in G:
        # cell c is fixed iff c_a = image_a(c) for every axis a
        fixed = 0
        for c in itertools.product(range(n), repeat=3):
            ok = True
            for ax in range(3):
                v = c[perm[ax]]
                if flips[ax]:
                    v = n - 1 - v
                if v != c[ax]:
                    ok = False
                    break
            fixed += ok
        total += fixed
    assert total % len(G) == 0
    return total // len(G)


# ---------------------------------------------------------------------------
# Trigonometric initialization (Sec. 6.2)
# ---------------------------------------------------------------------------

def quaternion_rotation(q) -> np.ndarray:
    """Rotation matrix of the normalized quaternion q = (w, x, y, z)."""
    w, x, y, z = np.asarray(q, dtype=np.float64) / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def trig_basis_count(nfreq: int) -> int:
    """|Q_n| = |T_n| + |T_n| (|T_n| + 1) / 2 with |T_n| = 6 n."""
    t = 6 * nfreq
    return t + t * (t + 1) // 2


def trig_basis(shape, nfreq: int, q) -> np.ndarray:
    """Values of Q_n at the element centres, shape (|Q_n|, n).

    T_n in the order (axis i, frequency k, cos then sin):
    cos(2 pi k xb_i), sin(2 pi k xb_i), k = 1..n, i = 0..2, with
    xb = R_q (x - (0.5, 0.5, 0.5)) and x the element centre in [0, 1]^3;
    then the products T_a T_b for a <= b in row-major order of (a, b)."""
    nx, ny, nz = shape
    cz, cy, cx = np.meshgrid((np.arange(nz) + 0.5) / nz, (np.arange(ny) + 0.5) / ny,
                             (np.arange(nx) + 0.5) / nx, indexing="ij")
    X = np.stack([cx.ravel(), cy.ravel(), cz.ravel()]) - 0.5
    xb = quaternion_rotation(q) @ X
    T = []
    for i in range(3):
        for k in range(1, nfreq + 1):
            T.append(np.cos(2 * math.pi * k * xb[i]))
            T.append(np.sin(2 * math.pi * k * xb[i]))
    Q = list(T)
    for a in range(len(T)):
        for b in range(a, len(T)):
            Q.append(T[a] * T[b])
    return np.array(Q)


def sigmoid_projection(y, volfrac: float, rho_min: float = 1e-3, k: float = 15.0,
                       steps: int = 200):
    """S(y) = rho_min + Vh / (1 + exp(-k (y - mu))), Vh = min(1.5 V, 1), with mu
    such that mean S(y) = V (bisection; mean S falls as mu grows).
    Returns (rho, mu)."""
    y = np.asarray(y, dtype=np.float64)
    vh = min(1.5 * volfrac, 1.0)

    def S(mu):
        return rho_min + vh / (1.0 + np.exp(-k * (y - mu)))

    lo, hi = float(y.min()) - 40.0 / k, float(y.max()) + 40.0 / k
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        if S(mid).mean() > volfrac:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 1e-14 * max(1.0, abs(mid)):
            break
    mu = 0.5 * (lo + hi)
    return S(mu), mu


def trig_init(shape, nfreq: int, q, weights, volfrac: float, rho_min: float = 1e-3,
              k: float = 15.0):
    """Initial density (Sec. 6.2): y = sum_m w_m Q_m(x), rho = S(y).
    Returns (rho, mu)."""
    Q = trig_basis(shape, nfreq, q)
    w = np.asarray(weights, dtype=np.float64)
    if w.size != Q.shape[0]:
        raise ValueError("need one weight per basis function")
    return sigmoid_projection(w @ Q, volfrac, rho_min, k)


# ---------------------------------------------------------------------------
# Sensitivity filter (Sec. 5.3; the OC optimizer's filterSens)
# ---------------------------------------------------------------------------

def filter_sensitivity(x, g, shape, radius: float = 2.0, floor: float = 1e-3) -> np.ndarray:
    """g~_e = sum_f w_ef x_f g_f / (max(floor, x_e) sum_f w_ef), w the periodic
    cone max(0, R - |d|) over integer offsets."""
    nx, ny, nz = shape
    xv = np.asarray(x, dtype=np.float64).reshape(nz, ny, nx)
    gv = np.asarray(g, dtype=np.float64).reshape(nz, ny, nx)
    h = int(math.ceil(radius)) - 1
    num = np.zeros_like(xv)
    wsum = 0.0
    for dz in range(-h, h + 1):
        for dy in range(-h, h + 1):
            for dx in range(-h, h + 1):
                wt = radius - math.sqrt(dx * dx + dy * dy + dz * dz)
                if wt <= 0:
                    continue
                num += wt * np.roll(xv * gv, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
                wsum += wt
    return (num / (np.maximum(floor, xv) * wsum)).ravel()


# ---------------------------------------------------------------------------
# Objectives and their gradients (Sec. 5.2 Eq. bulk-obj, Sec. 5.3 Eq. shear-obj,
# poisson-relx, poisson-new)
# ---------------------------------------------------------------------------

OBJECTIVES = ("bulk", "shear", "poisson_relaxed", "poisson_log")


def objective(kind: str, C, iteration: int = 0, beta: float = 0.8, eta: float = 0.6,
              tau: float | None = None, gamma: float = 0.5, E0: float = 1.0):
    """F(C^H) and W = dF/dC^H (6x6, entry by entry as written in the formula).

    bulk:            F = -(1/9) sum_{i,j < 3} C_ij
    shear:           F = -(C33 + C44 + C55) / 3
    poisson_relaxed: F = C01 + C02 + C12 - beta^l (C00 + C11 + C22), l = iteration
    poisson_log:     F = log(1 + eta A / B) + tau B^gamma, A = C01 + C12 + C20,
                     B = C00 + C11 + C22, tau = -1 / E0^gamma by default."""
    C = np.asarray(C, dtype=np.float64).reshape(6, 6)
    W = np.zeros((6, 6))
    if kind == "bulk":
        W[:3, :3] = -1.0 / 9.0
        return float((W * C).sum()), W
    if kind == "shear":
        for i in (3, 4, 5):
            W[i, i] = -1.0 / 3.0
        return float((W * C).sum()), W
    if kind == "poisson_relaxed":
        b = beta ** iteration
        W[0, 1] = W[0, 2] = W[1, 2] = 1.0
        for i in range(3):
            W[i, i] = -b
        return float((W * C).sum()), W
    if kind == "poisson_log":
        if tau is None:
            tau = -1.0 / E0 ** gamma
        A = C[0, 1] + C[1, 2] + C[2, 0]
        B = C[0, 0] + C[1, 1] + C[2, 2]
        F = math.log(1.0 + eta * A / B) + tau * B ** gamma
        dA = eta / (B + eta * A)
        dB = -eta * A / (B * (B + eta * A)) + tau * gamma * B ** (gamma - 1.0)
        W[0, 1] = W[1, 2] = W[2, 0] = dA
        for i in range(3):
            W[i, i] = dB
        return F, W
    raise ValueError(kind)


# ---------------------------------------------------------------------------
# Stopping rule (Sec. 6 parameters)
# ---------------------------------------------------------------------------

def should_stop(history, rel: float = 5e-4, window: int = 3, max_iter: int = 300) -> bool:
    """True once the objective's relative change |F_k - F_{k-1}| / |F_{k-1}| has
    stayed below `rel` for `window` consecutive iterations, or the history
    holds `max_iter` values."""
    f = [float(v) for v in history]
    if len(f) >= max_iter:
        return True
    if len(f) < window + 1:
        return False
    for k in range(len(f) - window, len(f)):
        if not abs(f[k] - f[k - 1]) < rel * abs(f[k - 1]):
            return False
    return True
