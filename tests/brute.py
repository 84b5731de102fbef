"""Brute-force transfers for tiny grids: every (node, particle) pair is visited
with the 1-D quadratic B-spline N(t) evaluated from its closed form, no stencil,
no base-node arithmetic.  Test-only; written independently of the oracle."""
import numpy as np


def N(t):
    a = np.abs(t)
    return np.where(a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


def node_positions(params):
    nx, ny, nz = params.nodes
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    # flattened in (k, j, i) order: index = (k*ny + j)*nx + i
    X = np.stack([(i - params.pad_lateral), (j - params.pad_lateral), (k - params.pad_bottom)], -1)
    X = X.transpose(2, 1, 0, 3).reshape(-1, 3).astype(np.float64) * params.dx
    return X


def weights(params, X, x):
    """w[i, p] for all nodes i and particles p."""
    t = (X[:, None, :] - x[None, :, :]) / params.dx
    return N(t[..., 0]) * N(t[..., 1]) * N(t[..., 2])


def polar_svd(F):
    U, _, Vt = np.linalg.svd(F)
    R = U @ Vt
    return R


def kirchhoff_svd(F, mu, lam):
    R = polar_svd(F)
    J = np.linalg.det(F)
    return 2 * mu * (F - R) @ F.T + lam * J * (J - 1) * np.eye(3)


def p2g(params, x, v, Cm, F, h, with_stress=True):
    X = node_positions(params)
    w = weights(params, X, x)
    mu = params.E / (2 * (1 + params.nu))
    lam = params.E * params.nu / ((1 + params.nu) * (1 - 2 * params.nu))
    Vp = params.dx ** 3 / params.ppc
    mp = params.rho * Vp
    M = w.sum(1) * mp
    MG = np.zeros((X.shape[0], 3))
    for p in range(x.shape[0]):
        A = mp * Cm[p]
        if with_stress:
            A = A - 4 * h / params.dx ** 2 * Vp * kirchhoff_svd(F[p], mu, lam)
        d = X - x[p]
        MG += w[:, p:p + 1] * (mp * v[p] + d @ A.T)
    return M, MG


def g2p(params, x, V):
    X = node_positions(params)
    w = weights(params, X, x)
    v = w.T @ V
    Cm = np.zeros((x.shape[0], 3, 3))
    for p in range(x.shape[0]):
        d = X - x[p]
        Cm[p] = 4 / params.dx ** 2 * (w[:, p:p + 1] * V).T @ d
    return v, Cm
