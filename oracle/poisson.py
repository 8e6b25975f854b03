"""TEST INFRASTRUCTURE -- double-precision CPU oracle of the modified Poisson equation.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline leg of
``bench.py`` may use it.  Plain numpy, independent of the GPU library.

The equation is eq. discrete_poisson (Sec. IV) in code units (box side 1, h = 1/N):

    (1/h^2) [sum of the 6 neighbours of phi - 6 phi] = S,
    S = 2 Om a (rho~ - 1) - (1/6) Om a^4 [ (n a^2 xi)^(1/(n+1)) exp(-u/(n+1))
                                          - 3 (a^-3 + 4 OL/Om) ],

the Newtonian potential phi sourced by the density and by delta R of the scalaron
f~_R = -exp(u) (Sec. II, Sec. III.B).  On the periodic grid the system is solvable only for a
source of zero mean and fixes phi up to a constant; reading (the paper is silent): the mean of
S is removed and phi has zero mean.  The solution is then unique, and ``solve`` gives it
exactly up to rounding: the periodic 7-point Laplacian is diagonal in the discrete Fourier
basis (an FFT is the library primitive used as a step).
"""
from __future__ import annotations

import numpy as np

from . import Model, constants


def omega_lambda(model: Model) -> float:
    return model.omega_l if model.omega_l >= 0.0 else 1.0 - model.omega_m


def source(rho, u, model: Model) -> np.ndarray:
    """Right-hand side S of eq. discrete_poisson at every cell (rho~ and u of the same shape)."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    om, a, n = model.omega_m, model.a, model.n
    K = constants(model, rho.shape[0])["K"]          # (n a^2 xi)^(1/(n+1))
    dR = K * np.exp(-u / (n + 1.0)) - 3.0 * (a ** -3 + 4.0 * omega_lambda(model) / om)
    return 2.0 * om * a * (rho - 1.0) - om * a ** 4 * dR / 6.0


def laplacian(phi) -> np.ndarray:
    """(1/h^2) [sum of the 6 periodic neighbours - 6 phi], h = 1/N."""
    phi = np.asarray(phi, dtype=np.float64)
    N = phi.shape[0]
    s = -6.0 * phi
    for ax in range(3):
        s = s + np.roll(phi, 1, axis=ax) + np.roll(phi, -1, axis=ax)
    return s * (N * N)


def solve(S) -> np.ndarray:
    """phi with laplacian(phi) = S - mean(S) and mean(phi) = 0 on the periodic N^3 grid."""
    S = np.asarray(S, dtype=np.float64)
    N = S.shape[0]
    F = np.fft.rfftn(S - S.mean())
    k = np.arange(N)
    lam_full = (2.0 * np.cos(2.0 * np.pi * k / N) - 2.0) * (N * N)      # per axis
    lam_half = lam_full[: N // 2 + 1]
    lam = lam_full[:, None, None] + lam_full[None, :, None] + lam_half[None, None, :]
    lam[0, 0, 0] = 1.0
    P = F / lam
    P[0, 0, 0] = 0.0
    return np.fft.irfftn(P, s=S.shape, axes=(0, 1, 2))
