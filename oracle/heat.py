"""Nonlinear heat transfer with weighted quadrature (Section 5): plain FP64 reference.

TEST INFRASTRUCTURE ONLY (see package docstring).

Problem (Section 5.1, weak residual): R_A = int Tdot N_A + int k(T) grad T . grad N_A
- int f N_A = 0. Time: generalised trapezoidal rule (Section 5.2), predictor-corrector
Newton with the symmetric tangent of Eq. (35), discretised by WQ as in Eq. (36).

READING (load vector): the paper does not say how F is integrated; F_i is formed with
the mass-family weights of row i, F_i = sum_q w0_iq f(x_q), which is the WQ rule for
int f N_i and is exact for constant f.
READING (residual): R is formed with the same weights at the same points,
R_i = sum_q [w0_iq (Tdot(x_q) - f(x_q)) + k(T(x_q)) (wx_iq dT/dx(x_q) + wy_iq dT/dy(x_q))],
which equals M Tdot + K[k(T_q)] T - F exactly, since T(x_q) = sum_j T_j N_j(x_q).
READING (Eq. 36): the sum over the points covers both the mass and the conductivity
terms (a line break in the printed equation).
READING (Eq. 34): the non-symmetric term of the exact tangent is taken as
k'(T) N_B grad T . grad N_A (the derivative of the residual); it is dropped by Eq. (35)
and used here only to check the tangent against finite differences.
READING (stop): Newton stops when the 2-norm of R over the free DOFs is <= tol
(absolute, 1e-10 by default), at most max_iter iterations.
Dirichlet DOFs are eliminated: they carry prescribed values, their rows and columns
are dropped from the Newton system.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .wq import point_values

# thermal conductivity kinds: k(u) and k'(u) with parameters (a, b)
K_LINEAR, K_QUADRATIC, K_EXP, K_SIN = 0, 1, 2, 3


def conductivity(kind, a, b):
    """k(u) = a + b u | a + b u^2 | a exp(b u) | a sin(b u), and k'(u). Section 6.3 uses
    k = 1, e^{-T}, sin(pi T) and 200 - 0.05 T; the default workload uses 1 + u^2."""
    if kind == K_LINEAR:
        return (lambda u: a + b * u), (lambda u: b + 0.0 * u)
    if kind == K_QUADRATIC:
        return (lambda u: a + b * u * u), (lambda u: 2.0 * b * u)
    if kind == K_EXP:
        return (lambda u: a * np.exp(b * u)), (lambda u: a * b * np.exp(b * u))
    if kind == K_SIN:
        return (lambda u: a * np.sin(b * u)), (lambda u: a * b * np.cos(b * u))
    raise ValueError(kind)


def point_field(data, vec):
    """u(x_q), du/dx(x_q), du/dy(x_q) at every WQ point (global point order) of the
    spline field u = sum_j vec_j N_j, from the basis values at the points."""
    u, ux, uy = [], [], []
    for d in data:
        coef = vec[d["fn"]]
        u.append(d["N"] @ coef)
        ux.append(d["Nx"] @ coef)
        uy.append(d["Ny"] @ coef)
    return np.concatenate(u), np.concatenate(ux), np.concatenate(uy)


def tangent_residual(fx, pat, data, W, T, Tdot, inv_theta_dt, kfun, f_pts=None, dkfun=None):
    """Eq. (36) row by row: S_il = sum_q [inv_theta_dt w0_iq N_l(x_q)
    + k(T_q) (wx_iq dN_l/dx(x_q) + wy_iq dN_l/dy(x_q))] on the CSR pattern, and the
    residual R (module READINGS). With dkfun = k' given, S also carries the non-symmetric
    term of the exact tangent (Eq. 34, module READING):
    + sum_q k'(T_q) N_l(x_q) (wx_iq dT/dx(x_q) + wy_iq dT/dy(x_q)).
    Returns (S values aligned with pat['col'], R)."""
    n = fx["n_fn"]
    Tq, Tx, Ty = point_field(data, T)
    Dq, _, _ = point_field(data, Tdot)
    kq = kfun(Tq)
    fq = np.zeros_like(Tq) if f_pts is None else f_pts
    dq = None if dkfun is None else dkfun(Tq)
    from .wq import local_matrix
    S = np.zeros(len(pat["col"]))
    R = np.zeros(n)
    for i in range(n):
        q0, q1 = pat["qptr"][i], pat["qptr"][i + 1]
        Q = pat["qidx"][q0:q1]
        w0, wx, wy = W["mass"][q0:q1], W["x"][q0:q1], W["y"][q0:q1]
        A0 = local_matrix(fx, pat, data, i, "N")
        Ax = local_matrix(fx, pat, data, i, "Nx")
        Ay = local_matrix(fx, pat, data, i, "Ny")
        S[pat["row_ptr"][i]:pat["row_ptr"][i + 1]] = (A0 @ (inv_theta_dt * w0)
                                                      + Ax @ (kq[Q] * wx) + Ay @ (kq[Q] * wy))
        if dq is not None:
            S[pat["row_ptr"][i]:pat["row_ptr"][i + 1]] += A0 @ (dq[Q] * (wx * Tx[Q] + wy * Ty[Q]))
        R[i] = np.sum(w0 * (Dq[Q] - fq[Q]) + kq[Q] * (wx * Tx[Q] + wy * Ty[Q]))
    return S, R


def load_vector(pat, W, f_pts, n):
    """F_i = sum_q w0_iq f(x_q) (module READING on the load vector)."""
    F = np.zeros(n)
    for i in range(n):
        q0, q1 = pat["qptr"][i], pat["qptr"][i + 1]
        F[i] = np.sum(W["mass"][q0:q1] * f_pts[pat["qidx"][q0:q1]])
    return F


def heat_step(fx, pat, data, W, T_n, Tdot_n, dt, theta, kfun, f_pts, dirichlet, g_next, tol=1e-10,
              max_iter=50, dkfun=None):
    """One time step t_n -> t_{n+1} (Section 5.2): predictor T = T_n + (1-theta) dt Tdot_n
    with the Dirichlet values g_next imposed; corrector iterations
    Tdot = (T - T_n - (1-theta) dt Tdot_n) / (theta dt), S and R at (T, Tdot) by Eq. (36),
    solve -S_ff dT_f = R_f (Eq. 33 with the tangent of Eq. 35, or with the exact tangent
    of Eq. 34 when dkfun = k' is given), T_f += dT_f, until ||R_f||_2 <= tol.
    Returns (T, Tdot, iterations, [||R_f|| per iteration])."""
    n = fx["n_fn"]
    free = ~dirichlet.astype(bool)
    T = T_n + (1.0 - theta) * dt * Tdot_n
    T[~free] = g_next[~free]
    norms = []
    it = 0
    while True:
        Tdot = (T - T_n - (1.0 - theta) * dt * Tdot_n) / (theta * dt)
        Sv, R = tangent_residual(fx, pat, data, W, T, Tdot, 1.0 / (theta * dt), kfun, f_pts, dkfun)
        nr = float(np.linalg.norm(R[free]))
        norms.append(nr)
        if nr <= tol or it >= max_iter:
            break
        S = sp.csr_matrix((Sv, pat["col"], pat["row_ptr"]), shape=(n, n))
        Sff = S[free][:, free].tocsc()
        dT = spla.spsolve(Sff, -R[free])
        T = T.copy()
        T[free] += dT
        it += 1
    return T, Tdot, it, norms


def manufactured(kind, a, b, lam=5.0):
    """T*(x, y, t) = (1 - e^{-lam t}) sin(pi x) sin(pi y) (the planar analogue of the
    paper's (1 - e^{-5t}) xyz) and the source f = dT*/dt - div(k(T*) grad T*) for the
    conductivity (kind, a, b). Returns callables T*(x, t), f(x, t) of x (npts x 2)."""
    k, dk = conductivity(kind, a, b)

    def Ts(x, t):
        return (1.0 - math.exp(-lam * t)) * np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1])

    def f(x, t):
        s = 1.0 - math.exp(-lam * t)
        sx, sy = np.sin(np.pi * x[:, 0]), np.sin(np.pi * x[:, 1])
        cx, cy = np.cos(np.pi * x[:, 0]), np.cos(np.pi * x[:, 1])
        u = s * sx * sy
        ux, uy = s * np.pi * cx * sy, s * np.pi * sx * cy
        lap = -2.0 * np.pi ** 2 * u
        ut = lam * math.exp(-lam * t) * sx * sy
        # div(k(u) grad u) = k'(u) |grad u|^2 + k(u) lap u
        return ut - (dk(u) * (ux * ux + uy * uy) + k(u) * lap)

    return Ts, f


def points_x(data):
    return point_values(data, "x")
