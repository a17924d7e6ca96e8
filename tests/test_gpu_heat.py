"""Nonlinear heat transfer on the GPU (assemble_tangent, wq_heat_step) against the oracle.

The tangent and residual kernels are compared with the oracle's Eq. (36) evaluated
with the GPU's own weights (so only the contraction is under test): 1e-12 normwise,
the residual scaled by its largest term (R = M Tdot + K T - F cancels). The time step is
compared with the oracle's predictor-corrector Newton (direct sparse solves) on the
same weights: both stop at ||R_free|| <= 1e-10, so the fields agree to the solver
tolerance over the smallest eigenvalue of S.
"""
import numpy as np
import pytest

import fixtures as fx
import oracle as O
from oracle import heat as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _wq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_29334_amd.wq as W
    return W


def _np(t):
    return t.detach().cpu().numpy()


def _case(F):
    W = _wq()
    R = O.setup(F, families=("mass", "x", "y"))
    mesh = W.Mesh(F)
    pts = W.Points(mesh)
    wts = W.Weights(mesh, pts, 1 | 2 | 4, tau=1e-12)
    Wg = {f: _np(wts.weights(b)) for f, b in (("mass", 1), ("x", 2), ("y", 4))}
    return {"F": F, "R": R, "W": W, "mesh": mesh, "pts": pts, "wts": wts, "Wg": Wg}


@pytest.fixture(scope="module")
def grid8():
    print("[gpu] heat case grid8", flush=True)
    return _case(fx.fixture_grid(8, displace=0.05, seed=11))


@pytest.fixture(scope="module")
def hs():
    print("[gpu] heat case half_strip", flush=True)
    return _case(fx.fixture_half_strip())


@pytest.mark.parametrize("case", ["grid8", "hs"])
@pytest.mark.parametrize("kind,a,b", [(H.K_QUADRATIC, 1.0, 1.0), (H.K_EXP, 1.0, -1.0), (H.K_SIN, 1.0, np.pi)])
def test_tangent_and_residual_parity(case, kind, a, b, request):
    c = request.getfixturevalue(case)
    F, R, W, pts, wts, Wg = c["F"], c["R"], c["W"], c["pts"], c["wts"], c["Wg"]
    pat, data = R["pat"], R["data"]
    n = F["n_fn"]
    rng = np.random.default_rng(21)
    T, Td = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    x = H.points_x(data)
    f = 1.0 + np.sin(2 * x[:, 0]) * x[:, 1]
    k, _ = H.conductivity(kind, a, b)
    Sg, Rg = W.assemble_tangent(pts, wts, torch.tensor(T, device="cuda"), torch.tensor(Td, device="cuda"), 7.0,
                                (kind, a, b), torch.tensor(f, device="cuda"))
    So, Ro = H.tangent_residual(F, pat, data, Wg, T, Td, 7.0, k, f)
    Tq, _, _ = H.point_field(data, T)
    M = O.csr(pat, O.wq_assemble(F, pat, data, Wg, "mass"), n)
    K = O.csr(pat, O.wq_assemble(F, pat, data, Wg, "stiffness", coef_pts=k(Tq)), n)
    scale = max(np.abs(M @ Td).max(), np.abs(K @ T).max(), np.abs(H.load_vector(pat, Wg, f, n)).max())
    es = np.abs(_np(Sg) - So).max() / np.abs(So).max()
    er = np.abs(_np(Rg) - Ro).max() / scale
    print(f"[gpu] {case} k={kind}: tangent rel err {es:.2e}, residual rel err {er:.2e}")
    assert es < 1e-12 and er < 1e-12


def _run_steps(c, kind, a, b, dt, steps, **kw):
    W, F, pts, wts = c["W"], c["F"], c["pts"], c["wts"]
    n = F["n_fn"]
    x = H.points_x(c["R"]["data"])
    _, f = H.manufactured(kind, a, b)
    dirichlet = torch.tensor(F["dir1"].astype(np.uint8), device="cuda")
    T = torch.zeros(n, dtype=torch.float64, device="cuda")
    Td = torch.zeros(n, dtype=torch.float64, device="cuda")
    out = []
    for s in range(steps):
        ft = torch.tensor(f(x, dt * (s + 1)), device="cuda")
        rep = W.heat_step(pts, wts, dirichlet, T, Td, dt, 1.0, (kind, a, b), ft, **kw)
        out.append((_np(T).copy(), _np(Td).copy(), rep))
    return out


def test_heat_step_matches_oracle_newton(grid8):
    c = grid8
    F, R, Wg = c["F"], c["R"], c["Wg"]
    pat, data = R["pat"], R["data"]
    n = F["n_fn"]
    x = H.points_x(data)
    kind, a, b = H.K_QUADRATIC, 1.0, 1.0
    k, _ = H.conductivity(kind, a, b)
    _, f = H.manufactured(kind, a, b)
    dirichlet = F["dir1"].astype(bool)
    gpu = _run_steps(c, kind, a, b, 0.5, 3, cg_rtol=1e-12)
    T, Td = np.zeros(n), np.zeros(n)
    for s in range(3):
        T, Td, it, norms = H.heat_step(F, pat, data, Wg, T, Td, 0.5, 1.0, k, f(x, 0.5 * (s + 1)), dirichlet, np.zeros(n))
        Tg, Tdg, rep = gpu[s]
        dT = np.abs(Tg - T).max() / np.abs(T).max()
        print(f"[gpu] step {s}: newton gpu {rep['newton_iters']} oracle {it}, cg {rep['cg_iters']}, "
              f"|R| {rep['residual']:.2e}, T rel diff {dT:.2e}")
        assert rep["residual"] <= 1e-10
        assert abs(rep["newton_iters"] - it) <= 1
        assert dT < 1e-8
        assert np.abs(Tdg - Td).max() / np.abs(Td).max() < 1e-7


def test_linear_conductivity_one_iteration(grid8):
    """k constant: with the linear solve taken to the Newton tolerance, one corrector
    iteration converges (the tangent is the exact Jacobian)."""
    out = _run_steps(grid8, H.K_LINEAR, 1.0, 0.0, 0.1, 2, cg_rtol=1e-14)
    for _, _, rep in out:
        assert rep["newton_iters"] == 1 and rep["residual"] <= 1e-10, rep


def test_heat_step_deterministic(grid8):
    a = _run_steps(grid8, H.K_QUADRATIC, 1.0, 1.0, 0.5, 2)
    b = _run_steps(grid8, H.K_QUADRATIC, 1.0, 1.0, 0.5, 2)
    for (ta, da, ra), (tb, db, rb) in zip(a, b):
        assert np.array_equal(ta, tb) and np.array_equal(da, db) and ra == rb


def test_heat_step_rejects_bad_parameters(grid8):
    W = grid8["W"]
    with pytest.raises(W.WQError) as e:
        _run_steps(grid8, H.K_QUADRATIC, 1.0, 1.0, -0.5, 1)
    assert e.value.status == -1


def test_newton_cap_reports_no_convergence(grid8):
    """A cap of zero corrector solves cannot reach 1e-10 from the predictor: WQ_ENOCONV."""
    W = grid8["W"]
    with pytest.raises(W.WQError) as e:
        _run_steps(grid8, H.K_QUADRATIC, 1.0, 1.0, 0.5, 1, max_newton=0)
    assert e.value.status == -5


@pytest.mark.parametrize("case", ["grid8", "hs"])
@pytest.mark.parametrize("kind,a,b", [(H.K_QUADRATIC, 1.0, 1.0), (H.K_EXP, 1.0, -1.0), (H.K_SIN, 1.0, np.pi)])
def test_exact_tangent_parity(case, kind, a, b, request):
    """assemble_tangent_exact (Eq. 34 with the non-symmetric term k'(T) N_j grad T . grad N_i,
    the reading the oracle's finite-difference test pins) against the oracle's exact
    tangent with the GPU's own weights: 1e-12 normwise; the residual is unchanged."""
    c = request.getfixturevalue(case)
    F, R, W, pts, wts, Wg = c["F"], c["R"], c["W"], c["pts"], c["wts"], c["Wg"]
    pat, data = R["pat"], R["data"]
    n = F["n_fn"]
    rng = np.random.default_rng(23)
    T, Td = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    x = H.points_x(data)
    f = 1.0 + np.sin(2 * x[:, 0]) * x[:, 1]
    k, dk = H.conductivity(kind, a, b)
    args = (torch.tensor(T, device="cuda"), torch.tensor(Td, device="cuda"), 7.0, (kind, a, b),
            torch.tensor(f, device="cuda"))
    Se, Re = W.assemble_tangent(pts, wts, *args, exact=True)
    Ss, Rs = W.assemble_tangent(pts, wts, *args)
    So, _ = H.tangent_residual(F, pat, data, Wg, T, Td, 7.0, k, f, dk)
    es = np.abs(_np(Se) - So).max() / np.abs(So).max()
    print(f"[gpu] {case} k={kind}: exact tangent rel err {es:.2e}")
    assert es < 1e-12
    assert torch.equal(Re, Rs)


def test_exact_tangent_heat_steps(grid8):
    """Newton with the exact tangent: the same states as the oracle's direct-solve Newton
    with its exact tangent (1e-8), at most the paper's 7 corrector solves per step, and
    fewer than the symmetric tangent needs."""
    c = grid8
    F, R, Wg, W = c["F"], c["R"], c["Wg"], c["W"]
    pat, data = R["pat"], R["data"]
    n = F["n_fn"]
    x = H.points_x(data)
    kind, a, b = H.K_QUADRATIC, 1.0, 1.0
    k, dk = H.conductivity(kind, a, b)
    _, f = H.manufactured(kind, a, b)
    dirichlet = F["dir1"].astype(bool)
    exact = _run_steps(c, kind, a, b, 0.5, 3, cg_rtol=1e-12, tangent=W.TANGENT_EXACT)
    sym = _run_steps(c, kind, a, b, 0.5, 3, cg_rtol=1e-12)
    T, Td = np.zeros(n), np.zeros(n)
    for s in range(3):
        T, Td, it, norms = H.heat_step(F, pat, data, Wg, T, Td, 0.5, 1.0, k, f(x, 0.5 * (s + 1)), dirichlet,
                                       np.zeros(n), dkfun=dk)
        Tg, _, rep = exact[s]
        dT = np.abs(Tg - T).max() / np.abs(T).max()
        print(f"[gpu] step {s}: exact-tangent newton gpu {rep['newton_iters']} oracle {it} "
              f"(symmetric {sym[s][2]['newton_iters']}), |R| {rep['residual']:.2e}, T rel diff {dT:.2e}")
        assert rep["residual"] <= 1e-10 and dT < 1e-8
        assert abs(rep["newton_iters"] - it) <= 1 and rep["newton_iters"] <= 7
        assert rep["newton_iters"] < sym[s][2]["newton_iters"]
