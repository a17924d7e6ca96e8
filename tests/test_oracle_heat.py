"""Pins of the nonlinear heat-transfer oracle (Section 5, Eqs. 30-36) on the CPU.

Each check ties the oracle to a fact that does not come from re-running its own
formula: the residual against an independent matrix form (M Tdot + K[k] T - F),
the tangent against a finite-difference Jacobian of the residual (with and without
the non-symmetric term that Eq. (35) drops), the linear case converging in one Newton
iteration (k constant: the tangent is exact), and a manufactured solution.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import fixtures as fxm
import oracle as O
from oracle import heat as H


@pytest.fixture(scope="module")
def setup():
    F = fxm.fixture_grid(8, displace=0.05, seed=11)
    S = O.setup(F, families=("mass", "x", "y"))
    return F, S


def _fields(F, seed=3):
    rng = np.random.default_rng(seed)
    n = F["n_fn"]
    return rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)


def test_residual_equals_matrix_form(setup):
    F, S = setup
    pat, data, W = S["pat"], S["data"], S["W"]
    n = F["n_fn"]
    T, Td = _fields(F)
    k, _ = H.conductivity(H.K_QUADRATIC, 1.0, 1.0)
    x = H.points_x(data)
    f = 1.0 + x[:, 0] * x[:, 1]
    Sv, R = H.tangent_residual(F, pat, data, W, T, Td, 7.0, k, f)
    Tq, _, _ = H.point_field(data, T)
    M = O.csr(pat, O.wq_assemble(F, pat, data, W, "mass"), n)
    K = O.csr(pat, O.wq_assemble(F, pat, data, W, "stiffness", coef_pts=k(Tq)), n)
    Fv = H.load_vector(pat, W, f, n)
    R2 = M @ Td + K @ T - Fv
    scale = max(np.abs(M @ Td).max(), np.abs(K @ T).max(), np.abs(Fv).max())
    assert np.abs(R - R2).max() <= 1e-12 * scale
    # tangent = M / (theta dt) + K[k(T_q)] on the pattern
    S2 = 7.0 * M + K
    assert np.abs(O.csr(pat, Sv, n) - S2).max() <= 1e-12 * abs(S2).max()


def _residual_of_T(F, S, T, T_n, inv_tdt, k, f):
    Td = (T - T_n) * inv_tdt  # theta = 1
    return H.tangent_residual(F, S["pat"], S["data"], S["W"], T, Td, inv_tdt, k, f)


@pytest.mark.parametrize("kind,a,b", [(H.K_QUADRATIC, 1.0, 1.0), (H.K_EXP, 1.0, -1.0), (H.K_LINEAR, 1.0, 0.0)])
def test_tangent_against_finite_differences(setup, kind, a, b):
    F, S = setup
    pat, data, W = S["pat"], S["data"], S["W"]
    n = F["n_fn"]
    T, T_n = _fields(F, seed=5)
    k, dk = H.conductivity(kind, a, b)
    inv = 10.0
    x = H.points_x(data)
    f = np.sin(3 * x[:, 0])
    Sv, _ = _residual_of_T(F, S, T, T_n, inv, k, f)
    Sm = O.csr(pat, Sv, n).toarray()
    # exact tangent of the oracle (Eq. 34, READING): S + the non-symmetric term
    # sum_q k'(T_q) N_B(x_q) (wx_Aq Tx_q + wy_Aq Ty_q)
    Se, _ = H.tangent_residual(F, pat, data, W, T, (T - T_n) * inv, inv, k, f, dk)
    Nm = O.csr(pat, Se, n).toarray() - Sm
    h = 1e-6
    rng = np.random.default_rng(9)
    for B in rng.choice(n, 6, replace=False):
        e = np.zeros(n)
        e[B] = h
        Rp = _residual_of_T(F, S, T + e, T_n, inv, k, f)[1]
        Rm = _residual_of_T(F, S, T - e, T_n, inv, k, f)[1]
        col = (Rp - Rm) / (2 * h)
        full = Sm[:, B] + Nm[:, B]
        assert np.abs(col - full).max() <= 1e-7 * np.abs(full).max()
        if b != 0.0:
            # the dropped term is really there: S alone is not the Jacobian
            assert np.abs(col - Sm[:, B]).max() > 1e-4 * np.abs(full).max()


def test_linear_problem_converges_in_one_iteration(setup):
    """k constant: R is linear in T and S is its exact Jacobian, so one corrector
    iteration reaches the tolerance (Eq. 35 with k' = 0)."""
    F, S = setup
    pat, data, W = S["pat"], S["data"], S["W"]
    n = F["n_fn"]
    k, _ = H.conductivity(H.K_LINEAR, 1.0, 0.0)
    Ts, f = H.manufactured(H.K_LINEAR, 1.0, 0.0)
    x = H.points_x(data)
    T = np.zeros(n)
    Td = np.zeros(n)
    dirichlet = F["dir1"].astype(bool)
    for step in range(2):
        t1 = 0.1 * (step + 1)
        T, Td, it, norms = H.heat_step(F, pat, data, W, T, Td, 0.1, 1.0, k, f(x, t1), dirichlet, np.zeros(n))
        assert it == 1 and norms[-1] <= 1e-10, norms


def test_nonlinear_newton_and_manufactured_solution():
    """k = 1 + u^2 with the manufactured source: Newton with the symmetric tangent
    converges to 1e-10 (linearly: the dropped term makes it a fixed-point iteration, so
    the count can exceed the paper's cap of 7 on large steps), the residual norm falls
    every iteration, and the discrete solution approaches T* under mesh refinement."""
    errs = []
    for N in (8, 12):
        F = fxm.fixture_grid(N, displace=0.05, seed=11)
        S = O.setup(F, families=("mass", "x", "y"))
        pat, data, W = S["pat"], S["data"], S["W"]
        n = F["n_fn"]
        k, _ = H.conductivity(H.K_QUADRATIC, 1.0, 1.0)
        Ts, f = H.manufactured(H.K_QUADRATIC, 1.0, 1.0)
        x = H.points_x(data)
        dirichlet = F["dir1"].astype(bool)
        T = np.zeros(n)
        Td = np.zeros(n)
        dt = 0.5
        for step in range(4):
            t1 = dt * (step + 1)
            T, Td, it, norms = H.heat_step(F, pat, data, W, T, Td, dt, 1.0, k, f(x, t1), dirichlet, np.zeros(n))
            assert norms[-1] <= 1e-10 and it < 50, norms
            assert all(b < a for a, b in zip(norms, norms[1:])), norms
        # nodal error at t = 2 (T* nearly steady: backward-Euler error ~ lam e^{-lam t})
        Tq, _, _ = H.point_field(data, T)
        M = O.csr(pat, O.wq_assemble(F, pat, data, W, "mass"), n)
        e = Tq - Ts(x, 2.0)
        # discrete L2 error with the mass-family weights of all rows (sum_i w0_iq = |detJ| w_q by PU)
        wq = np.zeros(len(x))
        np.add.at(wq, pat["qidx"], W["mass"])
        errs.append(np.sqrt(np.sum(wq * e * e)))
        assert abs(M.sum() - 1.0) < 1e-12
    assert errs[1] < 0.5 * errs[0], errs


def test_exact_tangent_newton_converges_quadratically():
    """With the exact tangent (Eq. 34, the non-symmetric term k'(T) N_B grad T . grad N_A
    kept), Newton converges quadratically: each step needs at most the paper's 7
    corrector solves (Section 6.3) where the symmetric tangent of Eq. (35) needs more,
    and once the residual is small it is roughly squared per iteration."""
    F = fxm.fixture_grid(8, displace=0.05, seed=11)
    S = O.setup(F, families=("mass", "x", "y"))
    pat, data, W = S["pat"], S["data"], S["W"]
    n = F["n_fn"]
    k, dk = H.conductivity(H.K_QUADRATIC, 1.0, 1.0)
    _, f = H.manufactured(H.K_QUADRATIC, 1.0, 1.0)
    x = H.points_x(data)
    dirichlet = F["dir1"].astype(bool)
    runs = {}
    for name, d in (("symmetric", None), ("exact", dk)):
        T, Td = np.zeros(n), np.zeros(n)
        its, last = [], None
        for step in range(3):
            t1 = 0.5 * (step + 1)
            T, Td, it, norms = H.heat_step(F, pat, data, W, T, Td, 0.5, 1.0, k, f(x, t1), dirichlet, np.zeros(n),
                                           dkfun=d)
            assert norms[-1] <= 1e-10, norms
            its.append(it)
            last = norms
        runs[name] = (its, T, last)
    assert max(runs["exact"][0]) <= 7 and sum(runs["exact"][0]) < sum(runs["symmetric"][0]), runs
    # both iterations solve the same discrete problem
    assert np.abs(runs["exact"][1] - runs["symmetric"][1]).max() < 1e-8
    nm = runs["exact"][2]
    small = [(a, b) for a, b in zip(nm, nm[1:]) if a < 1e-3]
    assert small and all(b <= 10.0 * a * a + 1e-12 for a, b in small), nm
