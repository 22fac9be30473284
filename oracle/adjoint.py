"""Gradient of L = 0.5 ||p - p*||^2 with p = A(kappa)^{-1} f for the
two-point-flux finite-volume matrix (a differentiable form of the solve; the
paper's operator of Sec. 2 with a per-cell coefficient).

  lambda = A^{-1} (p - p*)            (A symmetric: the same solve)
  dL/df = lambda
  dL/dkappa_i = - lambda^T (dA/dkappa_i) p = sum_f g_f dT_f/dkappa_i
  g_f = -(lambda_u - lambda_v)(p_u - p_v) for a face between cells u, v,
        -lambda_u p_u for a wall face of cell u.
  interior T = S/(d_a/k_a + d_b/k_b): dT/dk_a = T^2 d_a / (S k_a^2)
  wall     T = S k_a / d_a:           dT/dk_a = S / d_a
  mirror   T = S k_a / (2 d_a) (both sides carry the same base kappa):
                                      dT/dk_a = S / (2 d_a)
kappa is one value per base cell, mirrored to every image, so the gradient
sums over the images.  This module assembles A itself from the faces.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

INTERIOR, WALL, MIRROR = 0, 1, 2


def face_T(faces, kappa):
    ka = kappa[faces.cell_a]
    T = np.zeros(faces.area.size)
    dT_a = np.zeros_like(T)
    dT_b = np.zeros_like(T)
    it = faces.kind == INTERIOR
    kb = kappa[faces.cell_b[it]]
    den = faces.dist_a[it] / ka[it] + faces.dist_b[it] / kb
    T[it] = faces.area[it] / den
    dT_a[it] = T[it] ** 2 * faces.dist_a[it] / (faces.area[it] * ka[it] ** 2)
    dT_b[it] = T[it] ** 2 * faces.dist_b[it] / (faces.area[it] * kb ** 2)
    w = faces.kind == WALL
    T[w] = faces.area[w] * ka[w] / faces.dist_a[w]
    dT_a[w] = faces.area[w] / faces.dist_a[w]
    mi = faces.kind == MIRROR
    T[mi] = faces.area[mi] * ka[mi] / (2.0 * faces.dist_a[mi])
    dT_a[mi] = faces.area[mi] / (2.0 * faces.dist_a[mi])
    return T, dT_a, dT_b


def assemble(faces, kappa, img) -> sp.csr_matrix:
    """Full matrix in the ordering of img (n_b x 2^s)."""
    n_b, S = img.shape
    n = n_b * S
    T, _, _ = face_T(faces, kappa)
    rows, cols, vals = [], [], []
    diag = np.zeros(n_b)
    np.add.at(diag, faces.cell_a, T)
    it = faces.kind == INTERIOR
    np.add.at(diag, faces.cell_b[it], T[it])
    for a in range(S):
        rows.append(img[:, a]); cols.append(img[:, a]); vals.append(diag)
        u, v = img[faces.cell_a[it], a], img[faces.cell_b[it], a]
        rows += [u, v]; cols += [v, u]; vals += [-T[it], -T[it]]
        mi = faces.kind == MIRROR
        for t in np.unique(faces.axis[mi]):
            sel = mi & (faces.axis == t)
            u = img[faces.cell_a[sel], a]
            v = img[faces.cell_a[sel], a ^ (1 << int(t))]
            rows.append(u); cols.append(v); vals.append(-T[sel])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    A.sort_indices()
    return A


def kappa_gradient(faces, img, kappa, lam, p):
    """sum over faces, images and right-hand sides of g_f dT_f/dkappa."""
    n_b, S = img.shape
    lam = lam.reshape(lam.shape[0], -1)
    p = p.reshape(p.shape[0], -1)
    _, dT_a, dT_b = face_T(faces, kappa)
    grad = np.zeros(n_b)
    it = faces.kind == INTERIOR
    w = faces.kind == WALL
    mi = faces.kind == MIRROR
    for a in range(S):
        u, v = img[faces.cell_a[it], a], img[faces.cell_b[it], a]
        g = -np.sum((lam[u] - lam[v]) * (p[u] - p[v]), axis=1)
        np.add.at(grad, faces.cell_a[it], g * dT_a[it])
        np.add.at(grad, faces.cell_b[it], g * dT_b[it])
        u = img[faces.cell_a[w], a]
        g = -np.sum(lam[u] * p[u], axis=1)
        np.add.at(grad, faces.cell_a[w], g * dT_a[w])
        for t in np.unique(faces.axis[mi]):
            bit = 1 << int(t)
            if a & bit:
                continue
            sel = mi & (faces.axis == t)
            u = img[faces.cell_a[sel], a]
            v = img[faces.cell_a[sel], a ^ bit]
            g = -np.sum((lam[u] - lam[v]) * (p[u] - p[v]), axis=1)
            np.add.at(grad, faces.cell_a[sel], g * dT_a[sel])
    return grad


def loss_and_gradients(faces, img, kappa, f, p_star):
    """Direct sparse solves (splu): returns L, dL/df, dL/dkappa, p."""
    A = assemble(faces, kappa, img).tocsc()
    lu = spla.splu(A)
    f2 = f.reshape(f.shape[0], -1)
    p = lu.solve(f2)
    r = p - p_star.reshape(p.shape)
    lam = lu.solve(r)
    L = 0.5 * float(np.sum(r * r))
    return L, lam, kappa_gradient(faces, img, kappa, lam, p), p
