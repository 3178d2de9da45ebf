"""FP64 CPU oracle for periodic 3D inverse homogenization (test infrastructure).

This module is test infrastructure only.  It is the plain, slow, obviously
correct reference that the GPU path is checked against; only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it.  It shares
no code with the HIP library and does not import it.

What it computes follows Zhang et al., "An Optimized, Easy-to-use, Open-source
GPU Solver for Large-scale Inverse Homogenization Problems" (arXiv 2301.08911):

* Sec. 3.1, Eq. (opt-prob): SIMP densities on a periodic unit cell of M voxels.
* Sec. 3.2, Eq. (el-force), (fem), (elasttensor): element stiffness K0 of the
  8-node trilinear brick, macro-strain loads, the six periodic FE solves and the
  homogenized tensor C^H in the engineering order 11,22,33,12,23,13.
* Sec. 3.2, Eq. (obj-grad), (ch-sens): element sensitivities of C^H.
* Sec. 4.2, Eq. (macro-strain): the unit-strain nodal displacements chi^i in
  element-relative coordinates.
* Sec. 3.3 (multigrid): trilinear interpolation P and its transpose as the
  restriction, used here only to build the Galerkin reference P^T K P.
* Sec. 5.2 / Sec. 6: density filter of radius 2 and the optimality-criteria
  update with move limit 0.05 and damping 0.5.

Readings taken where the paper is silent (each is also listed in the design
notes): the SIMP scale is s = Emin + rho^p (E0 - Emin); |Omega| equals the
number of elements (unit elements, element-relative chi); the translation null
space is removed by zero-mean projection rather than by fixing corners; the
filter kernel is the linear cone w(d) = max(0, R - |d|) with periodic wrap; OC
uses a lambda bisection that makes the mean density equal the target.

Layout conventions: vertex/element index ``v = x + nx*(y + ny*z)``; nodal
vectors are ``(n, 3)`` arrays (dof ``3v + k``); the six load cases stack as
``(6, n, 3)``.  Local node ``a = a0 + 2 a1 + 4 a2`` of the element with origin
``(x, y, z)`` sits at ``(x + a0, y + a1, z + a2)`` modulo the grid.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp

NCASES = 6


# ---------------------------------------------------------------------------
# Material and element (Sec. 3.2; Sec. 6: E0 = 1, nu = 0.3, 8-node brick)
# ---------------------------------------------------------------------------

def lame(E: float, nu: float):
    """Lame constants (lambda, mu) of an isotropic material."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def constitutive_matrix(E: float = 1.0, nu: float = 0.3) -> np.ndarray:
    """6x6 isotropic elasticity matrix, engineering shear, order 11,22,33,12,23,13."""
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    for i in range(3):
        D[i, i] = lam + 2.0 * mu
        D[3 + i, 3 + i] = mu
    return D


def _node_bits(a: int):
    return (a & 1, (a >> 1) & 1, (a >> 2) & 1)


def strain_displacement(xi) -> np.ndarray:
    """6x24 B matrix of the unit trilinear brick at local point xi in [0,1]^3.

    Rows are strains 11,22,33,12,23,13 with engineering shear; columns are dofs
    ``3a + k`` (node-major).
    """
    B = np.zeros((6, 24))
    for a in range(8):
        bits = _node_bits(a)
        N = [xi[k] if bits[k] else 1.0 - xi[k] for k in range(3)]
        dN = [1.0 if bits[k] else -1.0 for k in range(3)]
        g = (dN[0] * N[1] * N[2], N[0] * dN[1] * N[2], N[0] * N[1] * dN[2])
        B[0, 3 * a + 0] = g[0]
        B[1, 3 * a + 1] = g[1]
        B[2, 3 * a + 2] = g[2]
        B[3, 3 * a + 0] = g[1]
        B[3, 3 * a + 1] = g[0]
        B[4, 3 * a + 1] = g[2]
        B[4, 3 * a + 2] = g[1]
        B[5, 3 * a + 0] = g[2]
        B[5, 3 * a + 2] = g[0]
    return B


def element_stiffness(E: float = 1.0, nu: float = 0.3) -> np.ndarray:
    """K0 = integral over the unit cube of B^T D B by 2x2x2 Gauss quadrature.

    The integrand is at most quadratic in each coordinate, so the rule is exact.
    """
    D = constitutive_matrix(E, nu)
    g = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))
    K0 = np.zeros((24, 24))
    for xi in itertools.product(g, g, g):
        B = strain_displacement(xi)
        K0 += 0.125 * (B.T @ D @ B)
    return 0.5 * (K0 + K0.T)


def unit_strain_displacements() -> np.ndarray:
    """chi^i (6 x 24): nodal displacements of the six unit macro strains.

    Element-relative node coordinates (b0, b1, b2) in {0,1}^3, Sec. 4.2
    Eq. (macro-strain): chi^0 = (x0,0,0), chi^1 = (0,x1,0), chi^2 = (0,0,x2),
    chi^3 = (x1/2, x0/2, 0), chi^4 = (0, x2/2, x1/2), chi^5 = (x2/2, 0, x0/2).
    """
    chi = np.zeros((6, 24))
    for b in range(8):
        x0, x1, x2 = _node_bits(b)
        chi[0, 3 * b:3 * b + 3] = (x0, 0, 0)
        chi[1, 3 * b:3 * b + 3] = (0, x1, 0)
        chi[2, 3 * b:3 * b + 3] = (0, 0, x2)
        chi[3, 3 * b:3 * b + 3] = (x1 / 2, x0 / 2, 0)
        chi[4, 3 * b:3 * b + 3] = (0, x2 / 2, x1 / 2)
        chi[5, 3 * b:3 * b + 3] = (x2 / 2, 0, x0 / 2)
    return chi


def simp_scale(rho, E0: float = 1.0, Emin: float = 1e-9, penal: float = 3.0) -> np.ndarray:
    """Element stiffness scale s_e = Emin + rho_e^p (E0 - Emin) (Sec. 3.2, SIMP)."""
    rho = np.asarray(rho, dtype=np.float64).ravel()
    return Emin + rho ** penal * (E0 - Emin)


# ---------------------------------------------------------------------------
# Periodic grid, assembly, loads (Sec. 3.2, Eq. el-force and fem)
# ---------------------------------------------------------------------------

def element_nodes(shape) -> np.ndarray:
    """(8, n) global vertex index of local node a of every element (periodic)."""
    nx, ny, nz = shape
    x = np.arange(nx)
    y = np.arange(ny)
    z = np.arange(nz)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    out = np.empty((8, nx * ny * nz), dtype=np.int64)
    for a in range(8):
        a0, a1, a2 = _node_bits(a)
        out[a] = (((X + a0) % nx) + nx * (((Y + a1) % ny) + ny * ((Z + a2) % nz))).ravel()
    return out


def element_dofs(shape) -> np.ndarray:
    """(24, n) global dof index of local dof 3a+k of every element."""
    nodes = element_nodes(shape)
    return (3 * nodes[:, None, :] + np.arange(3)[None, :, None]).reshape(24, -1)


def assemble_stiffness(s, shape, K0) -> sp.csr_matrix:
    """Global periodic stiffness K = sum_e s_e Q_e^T K0 Q_e as CSR (3n x 3n)."""
    s = np.asarray(s, dtype=np.float64).ravel()
    n = s.size
    dofs = element_dofs(shape)
    rows = np.broadcast_to(dofs[:, None, :], (24, 24, n)).ravel()
    cols = np.broadcast_to(dofs[None, :, :], (24, 24, n)).ravel()
    vals = (K0[:, :, None] * s[None, None, :]).ravel()
    K = sp.coo_matrix((vals, (rows, cols)), shape=(3 * n, 3 * n)).tocsr()
    K.sum_duplicates()
    return K


def apply_elementwise(s, shape, K0, u) -> np.ndarray:
    """Matrix-free K u by looping the element formula; u is (n, 3) or (c, n, 3)."""
    s = np.asarray(s, dtype=np.float64).ravel()
    u = np.asarray(u, dtype=np.float64)
    squeeze = u.ndim == 2
    if squeeze:
        u = u[None]
    nodes = element_nodes(shape)
    out = np.zeros_like(u)
    for c in range(u.shape[0]):
        ue = u[c][nodes].transpose(1, 0, 2).reshape(-1, 24)      # (n, 24)
        ye = (ue @ K0.T) * s[:, None]
        ye = ye.reshape(-1, 8, 3)
        for a in range(8):
            np.add.at(out[c], nodes[a], ye[:, a, :])
    return out[0] if squeeze else out


def vertex_neighbourhood(shape, verts):
    """Index data of [K u]_v at the given vertices (Sec. 4.2, Eq. st-assemb).

    Vertex v is local node a of the element whose origin is v - bits(a), for
    a = 0..7.  Returns ``elems`` (m, 8): that element for each a, and ``nodes``
    (m, 8, 8): global vertex of local node b of element ``elems[:, a]``."""
    nx, ny, nz = shape
    verts = np.asarray(verts, dtype=np.int64)
    vx, vy, vz = verts % nx, (verts // nx) % ny, verts // (nx * ny)
    elems = np.empty((verts.size, 8), dtype=np.int64)
    nodes = np.empty((verts.size, 8, 8), dtype=np.int64)
    for a in range(8):
        a0, a1, a2 = _node_bits(a)
        ox, oy, oz = (vx - a0) % nx, (vy - a1) % ny, (vz - a2) % nz
        elems[:, a] = ox + nx * (oy + ny * oz)
        for b in range(8):
            b0, b1, b2 = _node_bits(b)
            nodes[:, a, b] = ((ox + b0) % nx) + nx * (((oy + b1) % ny) + ny * ((oz + b2) % nz))
    return elems, nodes


def apply_at_vertices(K0, s_elems, u_nodes) -> np.ndarray:
    """[K u]_v = sum_a s_{e_a} sum_b K0[3a:3a+3, 3b:3b+3] u[node_b(e_a)] at m vertices.

    s_elems (m, 8) are the scales of the incident elements of
    ``vertex_neighbourhood``; u_nodes (c, m, 8, 8, 3) the displacements at their
    nodes.  Returns (c, m, 3)."""
    s_elems = np.asarray(s_elems, dtype=np.float64)
    u_nodes = np.asarray(u_nodes, dtype=np.float64)
    out = np.zeros(u_nodes.shape[:2] + (3,))
    for a in range(8):
        ue = u_nodes[:, :, a].reshape(u_nodes.shape[0], -1, 24)          # (c, m, 24)
        out += s_elems[None, :, a, None] * (ue @ K0[3 * a:3 * a + 3, :].T)
    return out


def load_vectors(s, shape, K0, chi) -> np.ndarray:
    """f^i = sum_e s_e Q_e^T K0 chi^i for the six cases, shape (6, n, 3)."""
    s = np.asarray(s, dtype=np.float64).ravel()
    n = s.size
    nodes = element_nodes(shape)
    f = np.zeros((NCASES, n, 3))
    for i in range(NCASES):
        fe = np.outer(s, K0 @ chi[i]).reshape(n, 8, 3)
        for a in range(8):
            np.add.at(f[i], nodes[a], fe[:, a, :])
    return f


def translation_projection(v: np.ndarray) -> np.ndarray:
    """Remove the per-component mean of an (n,3) or (c,n,3) nodal field."""
    return v - v.mean(axis=-2, keepdims=True)


# ---------------------------------------------------------------------------
# Solve (Sec. 3.2 Eq. fem; spec oracle: CG to 1e-10)
# ---------------------------------------------------------------------------

def block_jacobi_inverse(K: sp.csr_matrix) -> np.ndarray:
    """Inverse of every 3x3 diagonal block of K, shape (n, 3, 3)."""
    n = K.shape[0] // 3
    blocks = np.zeros((n, 3, 3))
    for i in range(3):
        for j in range(3):
            blocks[:, i, j] = K[np.arange(n) * 3 + i, np.arange(n) * 3 + j].A1
    return np.linalg.inv(blocks)


def absolute_floor(s, E: float = 1.0, nu: float = 0.3) -> float:
    """Residual floor eps_abs = 1e-12 sqrt(n) (lambda + 2 mu) mean(s).

    Cases whose load is below it (e.g. a uniform cell) have f = 0 up to
    rounding and are returned with zero iterations.
    """
    lam, mu = lame(E, nu)
    s = np.asarray(s).ravel()
    return 1e-12 * math.sqrt(s.size) * (lam + 2 * mu) * float(s.mean())


def pcg_solve(K: sp.csr_matrix, f: np.ndarray, tol: float = 1e-10, max_iter: int = 20000,
              x0: np.ndarray | None = None, eps_abs: float = 0.0, prec=None):
    """Preconditioned CG on the projected singular periodic system.

    ``f`` is (c, n, 3).  Each case runs its own CG.  A case is converged when
    the recomputed residual satisfies ||f - K x|| <= max(tol ||f||, eps_abs); a
    case with ||f|| <= eps_abs is solved by x = 0 with zero iterations.
    ``prec`` maps a (c, n, 3) residual to the preconditioned one; the default is
    3x3 block Jacobi.  The preconditioner only changes how fast the iteration
    gets there: the stopping test is on the recomputed residual.
    Returns the zero-mean solution (c, n, 3), iteration counts and the final
    relative residuals ||f - K x|| / ||f|| (reported as 0 for trivial cases).
    """
    f = translation_projection(np.asarray(f, dtype=np.float64))
    c, n, _ = f.shape
    if prec is None:
        Minv = block_jacobi_inverse(K)

        def prec(r):
            return np.einsum("nij,cnj->cni", Minv, r)

    def matvec(v):
        return (K @ v.reshape(c, 3 * n).T).T.reshape(c, n, 3)

    def norms(v):
        return np.sqrt((v ** 2).sum(axis=(1, 2)))

    fnorm = norms(f)
    trivial = fnorm <= eps_abs
    thresh = np.maximum(tol * fnorm, eps_abs)
    x = np.zeros_like(f) if x0 is None else translation_projection(np.array(x0, dtype=np.float64))
    x[trivial] = 0.0
    iters = np.zeros(c, dtype=np.int64)
    r = f - matvec(x)
    active = ~trivial & (norms(r) > thresh)
    z = prec(r)
    p = z.copy()
    rz = (r * z).sum(axis=(1, 2))
    for _ in range(max_iter):
        if not active.any():
            break
        q = matvec(p)
        pq = (p * q).sum(axis=(1, 2))
        alpha = np.where(active, rz / np.where(pq != 0, pq, 1.0), 0.0)
        x += alpha[:, None, None] * p
        r -= alpha[:, None, None] * q
        iters += active
        check = active & (norms(r) <= thresh)
        if check.any():
            # confirm on the recomputed residual before stopping a case
            rtrue = f - matvec(x)
            done = check & (norms(rtrue) <= thresh)
            r = np.where(check[:, None, None], rtrue, r)
            active &= ~done
        z = prec(r)
        rz_new = (r * z).sum(axis=(1, 2))
        beta = np.where(active, rz_new / np.where(rz != 0, rz, 1.0), 0.0)
        p = z + beta[:, None, None] * p
        rz = rz_new
    relres = np.where(trivial, 0.0, norms(f - matvec(x)) / np.where(trivial, 1.0, fnorm))
    return translation_projection(x), iters, relres


def solve_cases(s, shape, E: float = 1.0, nu: float = 0.3, tol: float = 1e-10,
                max_iter: int = 20000, x0=None, multigrid: bool = False):
    """Assemble K and the six loads for scale ``s`` and solve them (6, n, 3).

    ``multigrid`` preconditions CG with ``multigrid_preconditioner`` instead of
    block Jacobi (same stopping test, so the same answer to the tolerance)."""
    K0 = element_stiffness(E, nu)
    chi = unit_strain_displacements()
    K = assemble_stiffness(s, shape, K0)
    f = load_vectors(s, shape, K0, chi)
    prec = multigrid_preconditioner(K, shape) if multigrid else None
    return pcg_solve(K, f, tol=tol, max_iter=max_iter, x0=x0,
                     eps_abs=absolute_floor(s, E, nu), prec=prec)


def vertex_colours(shape) -> np.ndarray:
    """Colour (x mod 2) + 2 (y mod 2) + 4 (z mod 2) of every vertex (Sec. 4.1,
    the eight independent vertex subsets of the Gauss-Seidel relaxation)."""
    nx, ny, nz = shape
    v = np.arange(nx * ny * nz)
    return (v % nx) % 2 + 2 * (((v // nx) % ny) % 2) + 4 * ((v // (nx * ny)) % 2)


def gs_colour_step(K_rows: sp.csr_matrix, Dinv_rows: np.ndarray, r: np.ndarray, z: np.ndarray,
                   verts: np.ndarray) -> np.ndarray:
    """One colour of block Gauss-Seidel (Sec. 4.2, Eq. st-gs-relx), in place.

    At the vertices ``verts`` of one colour, S_v u_v = f_v - M_v with M_v the
    row sum without the diagonal block S_v, i.e. u_v += S_v^-1 (f - K u)_v.
    ``K_rows`` holds the rows of K at those vertices (3 per vertex),
    ``Dinv_rows`` the inverse diagonal blocks S_v^-1 there, r and z are
    (c, n, 3).  Returns z."""
    c, m, _ = z.shape
    kz = (K_rows @ z.reshape(c, 3 * m).T).T.reshape(c, verts.size, 3)
    z[:, verts] += np.einsum("nij,cnj->cni", Dinv_rows, r[:, verts] - kz)
    return z


def multigrid_preconditioner(K: sp.csr_matrix, shape, min_dim: int = 4, sweeps: int = 1,
                             smoother: str = "gs", omega_scale: float = 1.0 / 1.1,
                             first_factor: int = 2):
    """One symmetric multigrid V-cycle (Sec. 3.3, Alg. 1) as a CG preconditioner.

    Levels: K_{l+1} = P_l^T K_l P_l with the periodic trilinear P of
    ``prolongation`` (restriction = P^T), halving while every axis stays even
    and the coarse grid keeps at least ``min_dim`` cells per axis.  With
    ``first_factor`` 4 the first step divides every axis by 4 instead
    (non-dyadic coarsening, Sec. 4.2), the later ones halve.  Coarsest
    level: the dense solve of the vertex-0-pinned matrix.  Every residual is
    projected to zero mean per component before it is smoothed or solved (the
    translation null space); the cycle starts from zero on every level.

    Smoothers (``sweeps`` before and after the coarse correction):
      "gs": eight-colour block Gauss-Seidel (Sec. 4.2, Eq. st-gs-relx): for each
            colour in turn, u_v += S_v^-1 (f - K u)_v at the vertices of that
            colour, S_v the 3x3 diagonal block; colours 0..7 before the coarse
            correction and 7..0 after it, so the cycle is symmetric.
      "jacobi": damped 3x3 block Jacobi with damping omega_scale / lambda_l,
            lambda_l the largest eigenvalue of D_l^-1 K_l estimated by 30
            power iterations.
    Both make the cycle symmetric positive definite on zero-mean fields.
    Returns a function of a (c, n, 3) residual."""
    Ks, shapes, Ps = [K.tocsr()], [tuple(shape)], []
    while True:
        nx, ny, nz = shapes[-1]
        F = first_factor if len(shapes) == 1 else 2
        if nx % F or ny % F or nz % F or min(nx, ny, nz) // F < min_dim:
            break
        P = prolongation(shapes[-1], F)
        Ps.append(P)
        Ks.append((P.T @ Ks[-1] @ P).tocsr())
        shapes.append((nx // F, ny // F, nz // F))
    L = len(Ks) - 1
    Dinv, omegas, colour_rows = [], [], []
    rng = np.random.default_rng(12345)
    for l in range(L):
        Kl = Ks[l]
        Di = block_jacobi_inverse(Kl)
        Dinv.append(Di)
        if smoother == "jacobi":
            m = Kl.shape[0] // 3
            v = translation_projection(rng.standard_normal((m, 3)))
            lam = 1.0
            for _ in range(30):
                w = np.einsum("nij,nj->ni", Di, (Kl @ v.ravel()).reshape(m, 3))
                lam = float(np.linalg.norm(w) / np.linalg.norm(v))
                v = translation_projection(w / np.linalg.norm(w))
            omegas.append(omega_scale / lam)
        elif smoother == "gs":
            col = vertex_colours(shapes[l])
            rows = []
            for c in range(8):
                verts = np.flatnonzero(col == c)
                dofs = (3 * verts[:, None] + np.arange(3)[None, :]).ravel()
                rows.append((verts, Kl[dofs, :].tocsr()))
            colour_rows.append(rows)
        else:
            raise ValueError(smoother)
    Kc = Ks[-1].toarray()
    Kc[0:3, :] = 0.0
    Kc[:, 0:3] = 0.0
    Kc[0:3, 0:3] = np.eye(3)
    Kc_inv = np.linalg.inv(Kc)

    def apply(Kl, v):
        c, m, _ = v.shape
        return (Kl @ v.reshape(c, 3 * m).T).T.reshape(c, m, 3)

    def smooth(l, r, z, order):
        if smoother == "jacobi":
            return z + omegas[l] * np.einsum("nij,cnj->cni", Dinv[l], r - apply(Ks[l], z))
        for col in order:
            verts, Kcol = colour_rows[l][col]
            z = gs_colour_step(Kcol, Dinv[l][verts], r, z, verts)
        return z

    def cycle(l, r):
        r = translation_projection(r)
        if l == L:
            c, m, _ = r.shape
            rhs = r.reshape(c, 3 * m).T.copy()
            rhs[0:3, :] = 0.0
            return translation_projection((Kc_inv @ rhs).T.reshape(c, m, 3))
        z = np.zeros_like(r)
        for _ in range(sweeps):
            z = smooth(l, r, z, range(8))
        P = Ps[l]
        t = r - apply(Ks[l], z)
        c, m, _ = t.shape
        rc = (P.T @ t.reshape(c, 3 * m).T).T.reshape(c, -1, 3)
        ec = cycle(l + 1, rc)
        z = z + (P @ ec.reshape(c, -1).T).T.reshape(c, m, 3)
        for _ in range(sweeps):
            z = smooth(l, r, z, range(7, -1, -1))
        return z

    def prec(r):
        return cycle(0, np.asarray(r, dtype=np.float64))

    prec.levels = L + 1
    return prec


def dense_pinned_solve(K: sp.spmatrix, f: np.ndarray) -> np.ndarray:
    """Brute force for tiny grids: dense solve with vertex 0 fixed, then zero mean.

    ``f`` is (c, n, 3) and must have zero mean per component.
    """
    A = K.toarray()
    c, n, _ = f.shape
    A[0:3, :] = 0.0
    A[:, 0:3] = 0.0
    A[0:3, 0:3] = np.eye(3)
    rhs = f.reshape(c, 3 * n).T.copy()
    rhs[0:3, :] = 0.0
    u = np.linalg.solve(A, rhs).T.reshape(c, n, 3)
    return translation_projection(u)


# ---------------------------------------------------------------------------
# Homogenized tensor and sensitivities (Eq. elasttensor, obj-grad, ch-sens)
# ---------------------------------------------------------------------------

def element_energies(u, shape, K0, chi) -> np.ndarray:
    """E[e, i, j] = (chi^i - u^i_e)^T K0 (chi^j - u^j_e), shape (n, 6, 6)."""
    u = np.asarray(u, dtype=np.float64)
    nodes = element_nodes(shape)
    ue = u[:, nodes, :].transpose(0, 2, 1, 3).reshape(NCASES, -1, 24)   # (6, n, 24)
    d = chi[:, None, :] - ue
    Kd = np.einsum("ab,cnb->cna", K0, d)
    return np.einsum("ina,jna->nij", d, Kd)


def elastic_tensor(s, u, shape, K0, chi) -> np.ndarray:
    """C^H_ij = (1/n) sum_e s_e (chi^i - u^i_e)^T K0 (chi^j - u^j_e), 6x6."""
    s = np.asarray(s, dtype=np.float64).ravel()
    Ee = element_energies(u, shape, K0, chi)
    return np.einsum("n,nij->ij", s, Ee) / s.size


def sensitivity(rho, u, shape, K0, chi, W, E0: float = 1.0, Emin: float = 1e-9,
                penal: float = 3.0) -> np.ndarray:
    """sum_ij W_ij dC_ij/drho_e, with dC_ij/drho_e = (1/n) p rho^(p-1) (E0-Emin) d^i K0 d^j.

    Eq. (ch-sens) read per element (no sum over e; see the design notes).
    """
    rho = np.asarray(rho, dtype=np.float64).ravel()
    Ee = element_energies(u, shape, K0, chi)
    ds = penal * rho ** (penal - 1.0) * (E0 - Emin)
    return ds * np.einsum("ij,nij->n", np.asarray(W, dtype=np.float64), Ee) / rho.size


def bulk_weights() -> np.ndarray:
    """dF/dC for F = -(C00+C11+C22 + 2(C01+C02+C12))/9 (Sec. 5.2, Eq. bulk-obj)."""
    W = np.zeros((6, 6))
    W[:3, :3] = -1.0 / 9.0
    return W


def shear_weights() -> np.ndarray:
    """dF/dC for F = -(C33+C44+C55)/3 (Sec. 5.3, Eq. shear-obj)."""
    W = np.zeros((6, 6))
    for i in (3, 4, 5):
        W[i, i] = -1.0 / 3.0
    return W


# ---------------------------------------------------------------------------
# Density filter and OC update (Sec. 5.2; Sec. 6 parameters)
# ---------------------------------------------------------------------------

def filter_weights(radius: float = 2.0):
    """Offsets and unnormalized weights max(0, R - |d|) of the periodic cone filter."""
    h = int(math.ceil(radius)) - 1
    offs, w = [], []
    for dz in range(-h, h + 1):
        for dy in range(-h, h + 1):
            for dx in range(-h, h + 1):
                wt = radius - math.sqrt(dx * dx + dy * dy + dz * dz)
                if wt > 0:
                    offs.append((dx, dy, dz))
                    w.append(wt)
    return offs, np.array(w)


def density_filter(x, shape, radius: float = 2.0) -> np.ndarray:
    """rho~ = H x: periodic normalized cone convolution (H is symmetric, H^T = H)."""
    nx, ny, nz = shape
    v = np.asarray(x, dtype=np.float64).reshape(nz, ny, nx)
    offs, w = filter_weights(radius)
    out = np.zeros_like(v)
    for (dx, dy, dz), wt in zip(offs, w):
        out += wt * np.roll(v, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
    return (out / w.sum()).ravel()


def oc_candidate(x, g, lam, move, damp, xmin):
    """x_new(lambda) = clamp(x * (max(0,-g)/lambda)^damp, max(xmin, x-move), min(1, x+move))."""
    B = np.maximum(0.0, -g) / lam
    lo = np.maximum(xmin, x - move)
    hi = np.minimum(1.0, x + move)
    return np.clip(x * B ** damp, lo, hi)


def oc_update(x, g, volfrac: float, move: float = 0.05, damp: float = 0.5,
              xmin: float = 1e-3, steps: int = 200):
    """Optimality-criteria update; lambda by bisection of log(lambda) on mean(x_new) = V.

    The bracket [1e-40, 1e40] is halved ``steps`` times (it stops early once the
    relative width is below 1e-15).  Returns (x_new, lambda).
    """
    x = np.asarray(x, dtype=np.float64).ravel()
    g = np.asarray(g, dtype=np.float64).ravel()
    lo, hi = math.log(1e-40), math.log(1e40)
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        if oc_candidate(x, g, math.exp(mid), move, damp, xmin).mean() > volfrac:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-15:
            break
    lam = math.exp(0.5 * (lo + hi))
    return oc_candidate(x, g, lam, move, damp, xmin), lam


# ---------------------------------------------------------------------------
# Multigrid reference (Sec. 3.3): periodic trilinear prolongation and Galerkin
# ---------------------------------------------------------------------------

def prolongation(shape, factor: int = 2) -> sp.csr_matrix:
    """Periodic trilinear interpolation P from the grid coarser by ``factor`` per
    axis, as (3 n_f) x (3 n_c).  Factor 2 is the dyadic hierarchy of Sec. 3.3;
    factor 4 is the non-dyadic first step of Sec. 4.2 (the second level skipped),
    with the weights (d - |x_v - x_f|) / d of Eq. st-assemb-w, d = 4 fine cells:
    fine coordinate f = 4 X + r takes coarse X with weight (4 - r) / 4 and
    X + 1 with r / 4."""
    nx, ny, nz = shape
    F = int(factor)
    cx, cy, cz = nx // F, ny // F, nz // F
    rows, cols, vals = [], [], []

    def taps(f, nc):
        X, r = divmod(f, F)
        if r == 0:
            return [(X, 1.0)]
        if F == 2:
            return [((f - 1) // 2, 0.5), (((f + 1) // 2) % nc, 0.5)]
        return [(X, (F - r) / F), ((X + 1) % nc, r / F)]

    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                v = x + nx * (y + ny * z)
                for (X, wx) in taps(x, cx):
                    for (Y, wy) in taps(y, cy):
                        for (Z, wz) in taps(z, cz):
                            V = X + cx * (Y + cy * Z)
                            for k in range(3):
                                rows.append(3 * v + k)
                                cols.append(3 * V + k)
                                vals.append(wx * wy * wz)
    return sp.csr_matrix((vals, (rows, cols)), shape=(3 * nx * ny * nz, 3 * cx * cy * cz))


def prolongate(uc: np.ndarray, shape) -> np.ndarray:
    """P uc without forming P: periodic trilinear interpolation of a (c, n_c, 3)
    coarse field on the (n/2)^3 grid to the fine grid ``shape`` (x fastest).

    Fine vertex 2X along an axis takes coarse X; fine 2X + 1 takes the mean of
    coarse X and X + 1 (periodic), one axis after the other."""
    nx, ny, nz = shape
    c = uc.shape[0]
    U = np.asarray(uc, dtype=np.float64).reshape(c, nz // 2, ny // 2, nx // 2, 3)
    for axis, nf in ((3, nx), (2, ny), (1, nz)):
        odd = 0.5 * (U + np.roll(U, -1, axis=axis))
        shp = list(U.shape)
        shp[axis] = nf
        out = np.empty(shp)
        sl_even = [slice(None)] * 5
        sl_odd = [slice(None)] * 5
        sl_even[axis] = slice(0, nf, 2)
        sl_odd[axis] = slice(1, nf, 2)
        out[tuple(sl_even)] = U
        out[tuple(sl_odd)] = odd
        U = out
    return U.reshape(c, nx * ny * nz, 3)


def stencil_blocks(A: sp.spmatrix, shape) -> np.ndarray:
    """27-point 3x3 stencil of a periodic operator: out[d, i, j, v] = A[3v+i, 3(v+d)+j].

    Offset index d = (dx+1) + 3 (dy+1) + 9 (dz+1).
    """
    nx, ny, nz = shape
    n = nx * ny * nz
    A = A.tocsr()
    out = np.zeros((27, 3, 3, n))
    v = np.arange(n)
    x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                d = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)
                w = ((x + dx) % nx) + nx * (((y + dy) % ny) + ny * ((z + dz) % nz))
                for i in range(3):
                    for j in range(3):
                        out[d, i, j] = A[3 * v + i, 3 * w + j].A1
    return out


# ---------------------------------------------------------------------------
# Bounds used as pins (Voigt/Reuss and two-phase Hashin-Shtrikman bulk)
# ---------------------------------------------------------------------------

def voigt_bound(s, E: float = 1.0, nu: float = 0.3) -> np.ndarray:
    return float(np.mean(s)) * constitutive_matrix(E, nu)


def reuss_bound(s, E: float = 1.0, nu: float = 0.3) -> np.ndarray:
    return constitutive_matrix(E, nu) / float(np.mean(1.0 / np.asarray(s)))


def hs_bulk_upper(f1: float, K1: float, G1: float, K2: float) -> float:
    """Two-phase Hashin-Shtrikman upper bound on the bulk modulus (phase 1 stiffer)."""
    f2 = 1.0 - f1
    if f2 == 0.0:
        return K1
    return K1 + f2 / (1.0 / (K2 - K1) + 3.0 * f1 / (3.0 * K1 + 4.0 * G1))


def bulk_modulus(C: np.ndarray) -> float:
    """B = (1/9) sum_{i,j<3} C_ij."""
    return float(C[:3, :3].sum()) / 9.0
