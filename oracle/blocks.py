"""FP64 oracle of the block coupling between the DD boxes and the continuum
mesh -- TEST INFRASTRUCTURE ONLY (imported by tests/, the smoke check and the
benchmark's CPU baseline, never by the product library).

Geometry (Sec. "DD-MFDM coupling"): the domain is n x n square blocks of side
B and thickness h (one block through the thickness: plane stress); each block
is meshed by m x m x 1 trilinear hexahedra for the continuum calculation,
with 2 x 2 x 2 Gauss points per element.  Numbering: element e = ey * (n m) +
ex; Gauss point g = 4 gz + 2 gy + gx at isoparametric coordinates
(+-1/sqrt(3))^3 (minus first); block r = by * n + bx.  Fields at Gauss points
are arrays [n_elements * 8][c], at blocks [n * n][c].

What it computes:
  * block_average: <f>_r = int_{Omega_r} f dv / |Omega_r|, by the elements'
    Gauss rule (Sec. "DD-MFDM coupling", the block stress average);
  * block_to_gauss: the L2 projection of the blockwise-constant field onto the
    continuous trilinear finite-element space of the block mesh (assembled
    consistent mass matrix and load vector, dense solve), then its value at
    the Gauss points by the two-level isoparametric interpolation of Sec.
    "Obtaining L^p, V at Gauss point of element": first at the element's
    nodes with the block's shape functions, then at the Gauss point with the
    element's;
  * dissipation_fix: Eq. Lp_gauss and Eq. V_gauss (Sec. "Ensuring
    non-negative dissipation").
"""
from __future__ import annotations

import numpy as np

GP = 1.0 / np.sqrt(3.0)


def _shape(xi, eta, zeta):
    """Trilinear shape functions of the 8-node brick, node k = 4 kz + 2 ky + kx
    at (-1)^(kx+1), ..."""
    N = np.empty(8)
    for kz in range(2):
        for ky in range(2):
            for kx in range(2):
                sx = 2 * kx - 1
                sy = 2 * ky - 1
                sz = 2 * kz - 1
                N[4 * kz + 2 * ky + kx] = (1 + sx * xi) * (1 + sy * eta) * (1 + sz * zeta) / 8.0
    return N


def gauss_points(n, m, B, h):
    """Physical coordinates [n_el * 8][3] of every Gauss point."""
    ne = n * m
    de = B / m
    out = np.empty((ne * ne * 8, 3))
    for ey in range(ne):
        for ex in range(ne):
            e = ey * ne + ex
            for gz in range(2):
                for gy in range(2):
                    for gx in range(2):
                        g = 4 * gz + 2 * gy + gx
                        xi = (2 * gx - 1) * GP
                        et = (2 * gy - 1) * GP
                        ze = (2 * gz - 1) * GP
                        out[8 * e + g] = ((ex + 0.5 * (1 + xi)) * de, (ey + 0.5 * (1 + et)) * de,
                                          0.5 * (1 + ze) * h)
    return out


def block_average(f_gp, n, m, B, h):
    """<f>_r over each block: sum over its Gauss points of f w detJ, over |Omega_r|."""
    f_gp = np.asarray(f_gp, float)
    c = f_gp.shape[1]
    ne = n * m
    de = B / m
    w_detJ = (de / 2) * (de / 2) * (h / 2)   # unit Gauss weights, affine element
    out = np.zeros((n * n, c))
    for ey in range(ne):
        for ex in range(ne):
            r = (ey // m) * n + ex // m
            e = ey * ne + ex
            for g in range(8):
                out[r] += w_detJ * f_gp[8 * e + g]
    return out / (B * B * h)


def _block_mesh(n, B, h):
    """Nodes of the block mesh: node (i, j, k) at (i B, j B, k h), index
    (k (n+1) + j)(n+1) + i; brick r has corner nodes in shape-function order."""
    nn = (n + 1) * (n + 1) * 2
    conn = np.empty((n * n, 8), int)
    for by in range(n):
        for bx in range(n):
            r = by * n + bx
            for kz in range(2):
                for ky in range(2):
                    for kx in range(2):
                        conn[r, 4 * kz + 2 * ky + kx] = (kz * (n + 1) + by + ky) * (n + 1) + bx + kx
    return nn, conn


def l2_projection(f_block, n, B, h):
    """Nodal values [nn][c] of the L2 projection of the blockwise-constant field
    onto the trilinear space of the block mesh: M A = b with
    M_RQ = int N^R N^Q dv and b_R = int N^R f dv, both by 2x2x2 Gauss per brick."""
    f_block = np.asarray(f_block, float)
    c = f_block.shape[1]
    nn, conn = _block_mesh(n, B, h)
    M = np.zeros((nn, nn))
    b = np.zeros((nn, c))
    w_detJ = (B / 2) * (B / 2) * (h / 2)
    for r in range(n * n):
        for gz in range(2):
            for gy in range(2):
                for gx in range(2):
                    N = _shape((2 * gx - 1) * GP, (2 * gy - 1) * GP, (2 * gz - 1) * GP)
                    M[np.ix_(conn[r], conn[r])] += w_detJ * np.outer(N, N)
                    b[conn[r]] += w_detJ * np.outer(N, f_block[r])
    return np.linalg.solve(M, b)


def block_to_gauss(f_block, n, m, B, h):
    """L2 projection, then the two-level interpolation to every Gauss point."""
    return interpolate(l2_projection(f_block, n, B, h), n, m, B, h)


def interpolate(A, n, m, B, h, elements=None):
    """Two-level isoparametric interpolation of nodal values A [nn][c] of the
    block mesh to the Gauss points of the element mesh: all of them
    ([n_el * 8][c]), or those of the listed elements ([len * 8][c])."""
    A = np.asarray(A, float)
    _, conn = _block_mesh(n, B, h)
    c = A.shape[1]
    ne = n * m
    els = range(ne * ne) if elements is None else elements
    out = np.empty((len(els) * 8, c))
    for slot, e_id in enumerate(els):
        ey, ex = divmod(int(e_id), ne)
        bx, by = ex // m, ey // m
        r = by * n + bx
        # the element's nodes in the block's isoparametric coordinates
        A_el = np.empty((8, c))
        for kz in range(2):
            for ky in range(2):
                for kx in range(2):
                    xi_b = -1 + 2 * ((ex - bx * m) + kx) / m
                    et_b = -1 + 2 * ((ey - by * m) + ky) / m
                    ze_b = 2 * kz - 1
                    A_el[4 * kz + 2 * ky + kx] = _shape(xi_b, et_b, ze_b) @ A[conn[r]]
        for gz in range(2):
            for gy in range(2):
                for gx in range(2):
                    N = _shape((2 * gx - 1) * GP, (2 * gy - 1) * GP, (2 * gz - 1) * GP)
                    out[8 * slot + 4 * gz + 2 * gy + gx] = N @ A_el
    return out


def _x_t_alpha(T, alpha):
    """(X T alpha)_i = eps_ijk (T alpha)_jk."""
    P = T @ alpha
    return np.array([P[1, 2] - P[2, 1], P[2, 0] - P[0, 2], P[0, 1] - P[1, 0]])


def dissipation_fix(T, alpha, Lp, V):
    """Eq. Lp_gauss and Eq. V_gauss at every Gauss point (arrays [n][9], [n][9],
    [n][9], [n][3]; Lp or V may be None).  Returns new copies."""
    T = np.asarray(T, float).reshape(-1, 3, 3)
    Lp_o = None if Lp is None else np.array(Lp, float).reshape(-1, 3, 3)
    V_o = None if V is None else np.array(V, float).reshape(-1, 3)
    for g in range(T.shape[0]):
        if Lp_o is not None:
            d = float(np.sum(T[g] * Lp_o[g]))
            t2 = float(np.sum(T[g] * T[g]))
            if d < 0 and t2 > 0:
                Lp_o[g] = Lp_o[g] - d * T[g] / t2
        if V_o is not None:
            w = _x_t_alpha(T[g], np.asarray(alpha, float).reshape(-1, 3, 3)[g])
            beta = float(V_o[g] @ w)
            w2 = float(w @ w)
            if beta < 0 and w2 > 0:
                V_o[g] = V_o[g] - beta * w / w2
    return (None if Lp_o is None else Lp_o.reshape(-1, 9)), V_o
