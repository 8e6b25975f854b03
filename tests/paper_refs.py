"""Reference quantities written from the paper's physics, independent of the oracle's code.

Used by the oracle pins.  Each function states the passage it follows.  Where the oracle
evaluates (n a^2 xi)^(1/(n+1)) exp(-u/(n+1)), these helpers go through the background
value instead (f_R0 is by definition the present background f_R, Sec. II), so a wrong
constant in the oracle cannot cancel against the same constant here.
"""
from __future__ import annotations

import json
import os

import numpy as np

C_KMS = 299792.458
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden_background():
    with open(os.path.join(GOLDEN, "background.json")) as f:
        return json.load(f)


def omega_l(model):
    return 1.0 - model.omega_m if model.omega_l < 0 else model.omega_l


def ctilde(model):
    """Sec. III.A: c~ = c/(B H0), with H0 = 100 h km/s/Mpc and B in Mpc/h."""
    return C_KMS / (100.0 * model.box_mpc_h)


def curvature_bg(model, a=None):
    """-Rbar/m^2 = 3 (a^-3 + 4 OL/Om) (Sec. II / Sec. III.B)."""
    a = model.a if a is None else a
    return 3.0 * (a ** -3 + 4.0 * omega_l(model) / model.omega_m)


def ubar(model):
    """Background u.  Sec. II: f_R ~ -n xi (m^2/-R)^(n+1), so the background f_R scales as
    Rbar^-(n+1) and equals -|f_R0| at a = 1; the code variable is f~_R = a^2 f_R = -e^u
    (Sec. III.A, III.C)."""
    a, n = model.a, model.n
    return np.log(a * a * model.fr0_abs) + (n + 1.0) * np.log(curvature_bg(model, 1.0) / curvature_bg(model, a))


def u_uniform(model, c):
    """Uniform density rho~ = c: the Laplacian term vanishes, so delta R = 8 pi G delta rho
    (Sec. II, the GR-restored limit), i.e. R/m^2 = 3 (a^-3 c + 4 OL/Om); with f_R ~ R^-(n+1)
    this gives u - u_bar = (n+1) ln(Rbar / R)."""
    a, n = model.a, model.n
    R = 3.0 * (a ** -3 * c + 4.0 * omega_l(model) / model.omega_m)
    return ubar(model) + (n + 1.0) * np.log(curvature_bg(model) / R)


def m_eff2_code(model):
    """Squared scalaron mass in code units (box side = 1).  Sec. VI.A.2 gives
    m_eff^2 = [3(1+4 OL/Om)]^(n+2) Om H0^2 / (3 n (n+1) xi) (the printed formula lacks the
    square), at a = 1, with c = 1 and lengths in 1/H0; with the box side as the length unit
    (c~ = c/(B H0), Sec. III.A) it is divided by c~^2.
    Rewritten with n xi = |f_R0| [3(1+4 OL/Om)]^(n+1) (Sec. II)."""
    assert model.a == 1.0
    n = model.n
    three_q = curvature_bg(model, 1.0)
    return three_q * model.omega_m / (3.0 * (n + 1.0) * model.fr0_abs) / ctilde(model) ** 2


def source_S(model, u):
    """Curvature term of the code-unit f(R) equation, written through the background:
    (1/3) Om a^4 R(u)/m^2 with R/m^2 = (-Rbar/m^2) exp(-(u - u_bar)/(n+1)) (Sec. II, III.C)."""
    a = model.a
    return model.omega_m * a ** 4 / 3.0 * curvature_bg(model) * np.exp(-(u - ubar(model)) / (model.n + 1.0))


def sbar(model):
    return model.omega_m * model.a ** 4 * curvature_bg(model) / 3.0


def laplacian_symbol(N):
    """Eigenvalues (times -h^2) of the periodic 7-point Laplacian: 4 sum_d sin^2(pi k_d / N)."""
    s = 4.0 * np.sin(np.pi * np.fft.fftfreq(N) * 1.0) ** 2
    return s[:, None, None] + s[None, :, None] + s[None, None, :]


def linear_response(model, delta):
    """Linearised discrete solution v with u = u_bar + v for rho~ = 1 + delta, delta small:
    c~^2 b_bar (Lap_h - m_eff^2) v = Om a delta (screened Poisson / Yukawa, Sec. VI.A.2)."""
    N = delta.shape[0]
    h = 1.0 / N
    bbar = np.exp(ubar(model))
    lam = laplacian_symbol(N) / h ** 2
    dk = np.fft.fftn(delta)
    vk = -model.omega_m * model.a * dk / (ctilde(model) ** 2 * bbar * (lam + m_eff2_code(model)))
    return np.real(np.fft.ifftn(vk))


def sine_density(model, x):
    """Sec. VI.A.3, eq. sine_dens: density contrast of the sine test (x in [0,1])."""
    a, n = model.a, model.n
    fbar = np.exp(ubar(model))           # = n a^2 xi / [3(a^-3 + 4 OL/Om)]^(n+1)
    s = np.sin(2 * np.pi * x)
    return (ctilde(model) ** 2 / (model.omega_m * a) * (2 * np.pi) ** 2 * fbar * s
            + (1.0 + 4.0 * a ** 3 * omega_l(model) / model.omega_m) * ((2.0 - s) ** (-1.0 / (n + 1.0)) - 1.0))


def sine_u(model, x):
    """Sec. VI.A.3: f~_R = fbar (sin 2 pi x - 2), i.e. u = u_bar + ln(2 - sin 2 pi x)."""
    return ubar(model) + np.log(2.0 - np.sin(2 * np.pi * x))


def gaussian_density(model, x, alpha, W):
    """Sec. VI.A.4, eq. gaussian_dens, with c -> c~ and A = |background f~_R| (the exponent of
    the bracket in the definition of A is n+1, so that f_R -> background at the edges)."""
    a, n = model.a, model.n
    A = np.exp(ubar(model))
    X2 = (x - 0.5) ** 2
    g = np.exp(-X2 / W ** 2)
    nxi_a2 = A * curvature_bg(model) ** (n + 1.0)      # n a^2 xi
    return (ctilde(model) ** 2 / (model.omega_m * a) * 2 * A * alpha / W ** 2 * g * (1 - 2 * X2 / W ** 2)
            + a ** 3 / 3.0 * (nxi_a2 / (A * (1 - alpha * g))) ** (1.0 / (n + 1.0))
            - (1.0 + 4.0 * omega_l(model) / model.omega_m * a ** 3))


def gaussian_u(model, x, alpha, W):
    """Sec. VI.A.4, eq. fR_gaussian_dens: f_R = -A [1 - alpha exp(-(x-0.5)^2/W^2)]."""
    A = np.exp(ubar(model))
    return np.log(A * (1 - alpha * np.exp(-(x - 0.5) ** 2 / W ** 2)))


def operator_1d(model, u, rho, h):
    """x-only form of the discrete equation (eq. discrete_fR times c~^2): periodic 1-D
    conservative flux with face b = arithmetic mean; y,z neighbours carry no flux."""
    C = ctilde(model) ** 2 / (2 * h * h)
    b = np.exp(u)
    up, um = np.roll(u, -1), np.roll(u, 1)
    bp, bm = np.roll(b, -1), np.roll(b, 1)
    return (C * ((bp + b) * (up - u) + (bm + b) * (um - u)) + source_S(model, u)
            - model.omega_m * model.a * (rho - 1.0) - sbar(model))


def newton_1d(model, rho, h, u0, iters=60):
    """Brute-force Newton on the 1-D periodic system with a dense (cyclic tridiagonal)
    Jacobian from centred finite differences of operator_1d (column by column)."""
    u = np.array(u0, dtype=float)
    N = u.shape[0]
    for _ in range(iters):
        F = operator_1d(model, u, rho, h)
        J = np.zeros((N, N))
        for j in range(N):
            e = np.zeros(N)
            eps = 1e-6 * max(1.0, abs(u[j]))
            e[j] = eps
            J[:, j] = (operator_1d(model, u + e, rho, h) - operator_1d(model, u - e, rho, h)) / (2 * eps)
        du = np.linalg.solve(J, -F)
        u = u + du
        if np.max(np.abs(du)) < 1e-14 * np.max(np.abs(u)):
            break
    return u
