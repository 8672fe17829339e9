"""Closed forms and independent re-derivations used to pin the oracle (no import of the HIP path).

Each function states the passage of the paper, or the mathematics, it follows.
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import expm

R_GAS = 8.3145
FARADAY = 96485.0


def stefan_continuum(D: np.ndarray, T: float, p: float, X_in, N, xs) -> np.ndarray:
    """Steady 1D Stefan tube straight from the Maxwell-Stefan equations (Eq. 19, ideal gas):

        -C_t dX_i/dx = sum_{j != i} (X_j N_i - X_i N_j) / D_ij ,   i = 1, 2,

    with constant fluxes N (Eq. 39 at the electrode, conserved along the tube) and X_3 = 1 - X_1 -
    X_2.  The right side is affine in (X_1, X_2); for N_1 = -N_2, N_3 = 0 its matrix is singular,
    so the solution uses the augmented exponential [X(x); 1] = expm(x [[Phi, phi], [0, 0]]) [X0; 1].
    Returns X [3, len(xs)].
    """
    Ct = p / (R_GAS * T)

    def dXdx(X12):
        X = np.array([X12[0], X12[1], 1.0 - X12[0] - X12[1]])
        out = np.zeros(2)
        for i in range(2):
            acc = 0.0
            for j in range(3):
                if j != i:
                    acc += (X[j] * N[i] - X[i] * N[j]) / D[i, j]
            out[i] = -acc / Ct
        return out

    phi = dXdx(np.zeros(2))
    Phi = np.column_stack([dXdx(np.array([1.0, 0.0])) - phi, dXdx(np.array([0.0, 1.0])) - phi])
    A = np.zeros((3, 3))
    A[:2, :2] = Phi
    A[:2, 2] = phi
    v0 = np.array([X_in[0], X_in[1], 1.0])
    out = np.zeros((3, len(xs)))
    for k, x in enumerate(xs):
        v = expm(A * x) @ v0
        out[0, k], out[1, k], out[2, k] = v[0], v[1], 1.0 - v[0] - v[1]
    return out


def eq19_residual(Dl: np.ndarray, X: np.ndarray, g: np.ndarray, J: np.ndarray) -> np.ndarray:
    """Maxwell-Stefan relation (Eq. 19 with Eq. 30, Gamma = I) in lattice units (C_t = 1):
    -g_i = sum_{j != i} (X_j J_i - X_i J_j) / D*_ij  for i = 1, 2, with J_3 = -J_1 - J_2.
    Returns the residual of both equations (shape [2, ...])."""
    J3 = -J[0] - J[1]
    Jf = [J[0], J[1], J3]
    res = []
    for i in range(2):
        acc = 0.0
        for j in range(3):
            if j != i:
                acc = acc + (X[j] * Jf[i] - X[i] * Jf[j]) / Dl[i, j]
        res.append(acc + g[i])
    return np.array(res)


def stoich_D(Dl: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Eq. 24 at stoichiometric fluxes (N_2 = -N_1, N_3 = 0 as Eq. 38-39 fix them):
    1/D_1 = (X_1 + X_2)/D_12 + X_3/D_13,  1/D_2 = (X_1 + X_2)/D_12 + X_3/D_23."""
    X3 = 1.0 - X[0] - X[1]
    inv1 = (X[0] + X[1]) / Dl[0, 1] + X3 / Dl[0, 2]
    inv2 = (X[0] + X[1]) / Dl[0, 1] + X3 / Dl[1, 2]
    return np.array([1.0 / inv1, 1.0 / inv2])


def discrete_chain_stoich(Dl: np.ndarray, X_in, Q, n: int, tol: float = 1e-15) -> np.ndarray:
    """Exact steady state of the D1Q3-reduced scheme with node-wise tau.  At steady state every
    link carries the outlet flux: Phi = f*_+(k) - f*_-(k+1) = Q.  A node's first moment relaxes
    as J* = (1 - 1/tau) J, and the node's post-stream J is set by the neighbours' equilibria, so
    the step across a link is the flux times the half-sum of the two nodes' resistances 1/D*
    (D* = (tau - 1/2)/3):

        X_s(k) - X_s(k+1) = Q_s * (1/D*_s(k) + 1/D*_s(k+1)) / 2,   X_s(0) = X_in,s,

    marched link by link with Newton's method for X(k+1).  Returns X [2, n]."""
    X = np.zeros((2, n))
    X[:, 0] = X_in[:2]
    Q = np.asarray(Q, dtype=float)
    for k in range(n - 1):
        a = X[:, k]
        Da = stoich_D(Dl, a)
        b = a - Q / Da  # explicit first guess
        for _ in range(60):
            Db = stoich_D(Dl, b)
            F = a - b - 0.5 * Q * (1.0 / Da + 1.0 / Db)
            # Jacobian by central differences (2x2)
            Jm = np.zeros((2, 2))
            for c in range(2):
                h = 1e-7
                bp = b.copy(); bp[c] += h
                bm = b.copy(); bm[c] -= h
                Fp = a - bp - 0.5 * Q * (1.0 / Da + 1.0 / stoich_D(Dl, bp))
                Fm = a - bm - 0.5 * Q * (1.0 / Da + 1.0 / stoich_D(Dl, bm))
                Jm[:, c] = (Fp - Fm) / (2 * h)
            step = np.linalg.solve(Jm, -F)
            b = b + step
            if np.max(np.abs(step)) < tol:
                break
        X[:, k + 1] = b
    return X


def exact_variance(sigma0_sq: float, tau: float, t: int) -> float:
    """Second moment of a pulse under the D1Q3 marginal of BGK diffusion with constant tau,
    started from equilibrium on an unbounded lattice:

        sigma^2(t) = sigma0^2 + 2 D* t - (2/3) tau (tau - 1) (1 - (1 - 1/tau)^t),

    with D* = (tau - 1/2) / 3.  Tracking the moments sum x^2 X and sum x J (J the first
    velocity moment) through stream and collide gives this form: the variance grows at the BGK
    diffusivity, and the position-flux correlation starts at zero (equilibrium start) and
    approaches its steady value geometrically with the factor (1 - 1/tau) per step, which is
    the transient term."""
    D = (tau - 0.5) / 3.0
    q = 1.0 - 1.0 / tau
    return sigma0_sq + 2.0 * D * t - (2.0 / 3.0) * tau * (tau - 1.0) * (1.0 - q ** t)


def overpotential(T, n_e, X_in, X_out):
    """Eq. 43."""
    return (R_GAS * T / (n_e * FARADAY)) * np.log(X_in[0] * X_out[1] / (X_out[0] * X_in[1]))
