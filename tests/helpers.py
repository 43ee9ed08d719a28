"""Shared test utilities (no method arithmetic beyond evaluating a modal field)."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def duffy_rule(n1: int):
    """Collapsed Gauss-Legendre rule on the reference triangle built with numpy."""
    t, w = np.polynomial.legendre.leggauss(n1)
    t = 0.5 * (t + 1.0)
    w = 0.5 * w
    X, Y, W = [], [], []
    for i in range(n1):
        for j in range(n1):
            X.append(t[i])
            Y.append(t[j] * (1.0 - t[i]))
            W.append(w[i] * w[j] * (1.0 - t[i]))
    return np.array(X), np.array(Y), np.array(W)


def basis_table(K: int, xr: np.ndarray, yr: np.ndarray) -> np.ndarray:
    """[npts, K] values of the oracle's reference basis."""
    return np.array([O.basis(K, float(x), float(y))[0] for x, y in zip(xr, yr)])


def point_values(c: np.ndarray, mesh, xr: np.ndarray, yr: np.ndarray) -> np.ndarray:
    """[ne, npts, ncomp] values of modal fields c[e][comp][mode] at reference points."""
    K = c.shape[2]
    phi = basis_table(K, xr, yr)
    s = np.sqrt(2.0 * mesh.areas())
    return np.einsum("pk,eck->epc", phi, c) / s[:, None, None]


def physical_points(mesh, xr, yr):
    P = mesh.vxy[mesh.tri]
    x = P[:, 0, 0][:, None] + xr[None, :] * (P[:, 1, 0] - P[:, 0, 0])[:, None] + yr[None, :] * (P[:, 2, 0] - P[:, 0, 0])[:, None]
    y = P[:, 0, 1][:, None] + xr[None, :] * (P[:, 1, 1] - P[:, 0, 1])[:, None] + yr[None, :] * (P[:, 2, 1] - P[:, 0, 1])[:, None]
    return x, y


def l2_norm(c: np.ndarray) -> float:
    """L2 norm of a modal field in an orthonormal basis (Parseval)."""
    return float(np.sqrt(np.sum(c * c)))
