"""Closed-form and brute-force references used to pin the oracle.

Nothing here calls the oracle or the GPU library.  Every dense matrix is
built from its mathematical definition in a form different from the oracle's
per-vertex loops (sums of rank-1 link contributions, Kronecker products,
matrix polynomials), so a slip in either one shows up as a mismatch.
"""
from __future__ import annotations

import numpy as np


def grid(n):
    return np.linspace(0.0, 1.0, n)


def interior_mask(n):
    m = np.zeros((n, n, n), dtype=bool)
    m[1:-1, 1:-1, 1:-1] = True
    return m


def interior(v):
    return np.ascontiguousarray(v[1:-1, 1:-1, 1:-1]).ravel()


def embed(vi, n):
    v = np.zeros((n, n, n))
    v[1:-1, 1:-1, 1:-1] = vi.reshape(n - 2, n - 2, n - 2)
    return v


# --------------------------------------------------------------------------
# dense operator from link contributions: A = sum_f k_f h^-2 (e_p - e_q)(e_p - e_q)^T
# restricted to interior unknowns (boundary end points carry no unknown)
# --------------------------------------------------------------------------
def link_list(n):
    """All links with at least one interior end point, as (axis, face index tuple, p, q)
    where p, q are vertex (k, j, i) tuples."""
    out = []
    for k in range(n):
        for j in range(n):
            for i in range(n - 1):
                p, q = (k, j, i), (k, j, i + 1)
                out.append((0, (k, j, i), p, q))
    for k in range(n):
        for j in range(n - 1):
            for i in range(n):
                out.append((1, (k, j, i), (k, j, i), (k, j + 1, i)))
    for k in range(n - 1):
        for j in range(n):
            for i in range(n):
                out.append((2, (k, j, i), (k, j, i), (k + 1, j, i)))

    def inner(v):
        return all(1 <= c <= n - 2 for c in v)

    return [l for l in out if inner(l[2]) or inner(l[3])]


def unknown_index(n, v):
    k, j, i = v
    if not (1 <= i <= n - 2 and 1 <= j <= n - 2 and 1 <= k <= n - 2):
        return None
    return ((k - 1) * (n - 2) + (j - 1)) * (n - 2) + (i - 1)


def dense_from_links(kx, ky, kz):
    n = kx.shape[0]
    m = (n - 2) ** 3
    A = np.zeros((m, m))
    s = float(n - 1) ** 2
    ks = (kx, ky, kz)
    for ax, fidx, p, q in link_list(n):
        c = s * ks[ax][fidx]
        ip, iq = unknown_index(n, p), unknown_index(n, q)
        vec = {}
        if ip is not None:
            vec[ip] = 1.0
        if iq is not None:
            vec[iq] = -1.0
        for a, va in vec.items():
            for b, vb in vec.items():
                A[a, b] += c * va * vb
    return A


def link_gradient_matrix(kx, ky, kz):
    """Dense list of (dA/dtheta_f) as (index arrays) for the brute-force adjoint."""
    n = kx.shape[0]
    s = float(n - 1) ** 2
    ks = (kx, ky, kz)
    out = []
    for ax, fidx, p, q in link_list(n):
        ip, iq = unknown_index(n, p), unknown_index(n, q)
        out.append((ax, fidx, s * ks[ax][fidx], ip, iq))
    return out


# --------------------------------------------------------------------------
# 1D trilinear interpolation as a matrix; 3D by Kronecker products
# --------------------------------------------------------------------------
def interp_1d_matrix(n):
    """(n-2) x (nc-2) interior interpolation matrix, nc = (n-1)/2 + 1."""
    nc = (n - 1) // 2 + 1
    P = np.zeros((n - 2, nc - 2))
    for i in range(1, n - 1):
        for I in range(1, nc - 1):
            if i == 2 * I:
                P[i - 1, I - 1] = 1.0
            elif abs(i - 2 * I) == 1:
                P[i - 1, I - 1] = 0.5
    return P


def prolongation_matrix(n):
    P1 = interp_1d_matrix(n)
    return np.kron(P1, np.kron(P1, P1))


# --------------------------------------------------------------------------
# Chebyshev error polynomial p(lambda) = T_m((theta - lambda)/delta) / T_m(theta/delta)
# --------------------------------------------------------------------------
def cheb_T(m, t):
    return np.cos(m * np.arccos(t)) if abs(t) <= 1 else np.cosh(m * np.arccosh(abs(t))) * (np.sign(t) ** m)


def cheb_poly_scalar(lam, m, lo, hi):
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    return cheb_T(m, (theta - lam) / delta) / cheb_T(m, theta / delta)


def cheb_poly_matrix(K, m, lo, hi):
    """p(K) by the Chebyshev three-term recurrence on matrices T_{j+1} = 2 X T_j - T_{j-1}."""
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    I = np.eye(K.shape[0])
    X = (theta * I - K) / delta
    T0, T1 = I, X
    if m == 0:
        Tm = T0
    else:
        for _ in range(m - 1):
            T0, T1 = T1, 2.0 * X @ T1 - T0
        Tm = T1
    return Tm / cheb_T(m, theta / delta)


# --------------------------------------------------------------------------
# exact quadratic solution with linear k (the 7-point scheme is exact)
# --------------------------------------------------------------------------
def linear_k_faces(n, c):
    """k = c0 + c1 x + c2 y + c3 z sampled at link midpoints."""
    x = grid(n)
    xm = 0.5 * (x[:-1] + x[1:])
    c0, c1, c2, c3 = c
    kx = c0 + c1 * xm[None, None, :] + c2 * x[None, :, None] + c3 * x[:, None, None]
    ky = c0 + c1 * x[None, None, :] + c2 * xm[None, :, None] + c3 * x[:, None, None]
    kz = c0 + c1 * x[None, None, :] + c2 * x[None, :, None] + c3 * xm[:, None, None]
    return (np.ascontiguousarray(np.broadcast_to(kx, (n, n, n - 1))),
            np.ascontiguousarray(np.broadcast_to(ky, (n, n - 1, n))),
            np.ascontiguousarray(np.broadcast_to(kz, (n - 1, n, n))))


def quadratic_solution(n):
    x = grid(n)
    X = x * (1 - x)
    return X[:, None, None] * X[None, :, None] * X[None, None, :]


def quadratic_rhs(n, c):
    """f = -div(k grad phi) for phi = X(x)Y(y)Z(z), X = x(1-x), k linear."""
    x = grid(n)
    c0, c1, c2, c3 = c
    Z, Y, Xg = np.meshgrid(x, x, x, indexing="ij")
    X = Xg * (1 - Xg)
    Yq = Y * (1 - Y)
    Zq = Z * (1 - Z)
    k = c0 + c1 * Xg + c2 * Y + c3 * Z
    f = (2.0 * k * (Yq * Zq + X * Zq + X * Yq)
         - c1 * (1 - 2 * Xg) * Yq * Zq - c2 * (1 - 2 * Y) * X * Zq - c3 * (1 - 2 * Z) * X * Yq)
    f[0, :, :] = f[-1, :, :] = 0
    f[:, 0, :] = f[:, -1, :] = 0
    f[:, :, 0] = f[:, :, -1] = 0
    return f


def sine_mode(n, m):
    x = grid(n)
    s = [np.sin(mm * np.pi * x) for mm in m]  # m = (mx, my, mz)
    u = s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :]
    u[0, :, :] = u[-1, :, :] = 0
    u[:, 0, :] = u[:, -1, :] = 0
    u[:, :, 0] = u[:, :, -1] = 0
    return u
