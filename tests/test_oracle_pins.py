"""Pins of the FP64 oracle against facts fixed by the paper and by the mathematics.

Each test checks the oracle against something other than itself: exact rational
arithmetic for the B-spline case of Section 2, closed-form Gram integrals, exactness
(Eqs. 4, 9-12), partition of unity, the divergence theorem, rank identities, counts of
Table 2, an independent min-norm solver, and convergence rates of Section 6.1.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import fixtures as fx
import oracle as O


# ----------------------------------------------------------------- exact 1D B-splines
class Poly:
    """Exact polynomial with Fraction coefficients (c[k] * u^k)."""

    def __init__(self, c):
        self.c = [Fr(x) for x in c]

    def __call__(self, u):
        return sum(ck * Fr(u) ** k for k, ck in enumerate(self.c))

    def __mul__(self, o):
        out = [Fr(0)] * (len(self.c) + len(o.c) - 1)
        for i, a in enumerate(self.c):
            for j, b in enumerate(o.c):
                out[i + j] += a * b
        return Poly(out)

    def deriv(self):
        return Poly([k * self.c[k] for k in range(1, len(self.c))] or [0])

    def integral(self, a, b):
        return sum(ck * (Fr(b) ** (k + 1) - Fr(a) ** (k + 1)) / (k + 1) for k, ck in enumerate(self.c))

    def shift(self, s):
        """p(u - s) as a polynomial in u."""
        from math import comb
        out = [Fr(0)] * len(self.c)
        for k, ck in enumerate(self.c):
            for j in range(k + 1):
                out[j] += ck * comb(k, j) * (-Fr(s)) ** (k - j)
        return Poly(out)


# uniform cubic B-spline on [0, 4], one polynomial per unit interval
_B = [Poly([0, 0, 0, Fr(1, 6)]),
      Poly([Fr(4, 6), -2, 2, Fr(-3, 6)]),
      Poly([Fr(-44, 6), 10, -4, Fr(3, 6)]),
      Poly([Fr(64, 6), -8, 2, Fr(-1, 6)])]


def bspline_piece(shift, interval, d=0):
    """Polynomial of B(u - shift) (or its d-th derivative) on [interval, interval+1]."""
    k = interval - shift
    if k < 0 or k > 3:
        return Poly([0])
    p = _B[k].shift(shift)
    for _ in range(d):
        p = p.deriv()
    return p


def exact_1d():
    """Section 2 for the interior test function B_0 on [0,4]: two cell-centred points
    per knot interval, trial functions B_k, k = -3..3. Returns exact mass weights w
    (Eq. (6)) and derivative weights w' (same formula on the independent rows; the
    derivative system loses one rank to partition of unity)."""
    pts = [Fr(2 * q + 1, 4) for q in range(8)]
    ks = list(range(-3, 4))

    def val(k, u, d=0):
        iv = int(u)  # u is never an integer here
        return bspline_piece(k, iv, d)(u)

    def integ(k, d):
        return sum((bspline_piece(0, iv, d) * bspline_piece(k, iv, d)).integral(iv, iv + 1)
                   for iv in range(-3, 7))

    z = [val(0, u) for u in pts]

    def solve(rows, rhs):
        # w = Z^2 A^T (A Z^2 A^T)^{-1} b in exact arithmetic
        n = len(rows)
        G = [[sum(rows[a][q] * z[q] ** 2 * rows[b][q] for q in range(8)) for b in range(n)] for a in range(n)]
        y = gauss_solve(G, rhs)
        return [z[q] ** 2 * sum(rows[a][q] * y[a] for a in range(n)) for q in range(8)]

    A = [[val(k, u) for u in pts] for k in ks]
    b = [integ(k, 0) for k in ks]
    w = solve(A, b)
    Ad = [[val(k, u, 1) for u in pts] for k in ks]
    bd = [integ(k, 1) for k in ks]
    assert sum(bd) == 0 and all(sum(Ad[r][q] for r in range(7)) == 0 for q in range(8))
    wd = solve(Ad[:6], bd[:6])
    return w, wd, b, bd


def gauss_solve(G, rhs):
    n = len(G)
    M = [row[:] + [rhs[i]] for i, row in enumerate(G)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


# ----------------------------------------------------------------- shared setups
@pytest.fixture(scope="module")
def grid14():
    F = fx.fixture_grid(14)
    return F, O.setup(F, families=("mass", "x", "y", "lap"))


@pytest.fixture(scope="module")
def hs():
    F = fx.fixture_half_strip()
    return F, O.setup(F, families=("mass", "x", "y", "lap"))


def _row_of_vertex(F, ix, iy, N):
    v = ix + (N + 1) * iy
    return int(np.nonzero(F["fn_vertex"] == v)[0][0])


# ----------------------------------------------------------------- P1, P2
def test_p1_weights_are_kronecker_of_exact_1d(grid14):
    F, R = grid14
    N = 14
    w, wd, _, _ = exact_1d()
    w = np.array([float(x) for x in w])
    wd = np.array([float(x) for x in wd])
    # the 1D rule reproduces its own integrals: sum of mass weights = int B = 1
    assert abs(w.sum() - 1.0) < 1e-15
    i = _row_of_vertex(F, 7, 7, N)
    pat, cl = R["pat"], R["cells"]
    q0, q1 = pat["qptr"][i], pat["qptr"][i + 1]
    assert q1 - q0 == 64
    # element (ex, ey) holds 2x2 points (a, b); 1D index = 2 (e - e0) + a
    ex0, ey0 = 7 - 2, 7 - 2
    h = 1.0 / (N - 2)
    exp_m, exp_x, exp_y = [], [], []
    for c in pat["supp"][i]:
        f = int(cl["elem"][c])
        ex, ey = f % N, f // N
        for b in range(2):
            for a in range(2):
                px, py = 2 * (ex - ex0) + a, 2 * (ey - ey0) + b
                # physical coordinates x = h u: b scales by h^2 (mass) or 1 (gradient),
                # A by 1 (values) or 1/h (derivatives), hence w by h^2 or h
                exp_m.append(h * h * w[px] * w[py])
                exp_x.append(h * wd[px] * w[py])
                exp_y.append(h * w[px] * wd[py])
    # the weights are a forward quantity: their error is ~ kappa(A) kappa(Z V_t) eps
    # relative to the largest weight (~1e4 x 1e4 here), while the exactness residual
    # stays at round-off
    np.testing.assert_allclose(R["W"]["mass"][q0:q1], exp_m, rtol=0, atol=1e-9 * np.abs(exp_m).max())
    tol = 1e-9 * np.abs(exp_x).max()
    np.testing.assert_allclose(R["W"]["x"][q0:q1], exp_x, rtol=0, atol=tol)
    np.testing.assert_allclose(R["W"]["y"][q0:q1], exp_y, rtol=0, atol=tol)


def test_p2_gauss_rows_equal_exact_gram_products(grid14):
    F, R = grid14
    N = 14
    h = 1.0 / (N - 2)
    ks = range(-3, 4)

    def gram(d1, d2, k):
        return float(sum((bspline_piece(0, iv, d1) * bspline_piece(k, iv, d2)).integral(iv, iv + 1)
                         for iv in range(-3, 7)))
    G = {(d1, d2, k): gram(d1, d2, k) for d1 in range(3) for d2 in range(3) for k in ks}
    # the 1D closed forms quoted for uniform cubic B-splines
    assert abs(G[(0, 0, 0)] - 151 / 315) < 1e-15 and abs(G[(0, 0, 3)] - 1 / 5040) < 1e-15
    assert abs(G[(1, 1, 0)] - 2 / 3) < 1e-15 and abs(G[(1, 1, 1)] + 1 / 8) < 1e-15
    i = _row_of_vertex(F, 7, 7, N)
    gq = R["gq"]
    worst = 0.0
    for dy in ks:
        for dx in ks:
            j = _row_of_vertex(F, 7 + dx, 7 + dy, N)
            # area element h^2; each x-derivative brings 1/h
            m = G[(0, 0, dx)] * G[(0, 0, dy)] * h * h
            kx = G[(1, 1, dx)] * G[(0, 0, dy)]
            ky = G[(0, 0, dx)] * G[(1, 1, dy)]
            bb = (G[(2, 2, dx)] * G[(0, 0, dy)] + G[(2, 0, dx)] * G[(0, 2, dy)]
                  + G[(0, 2, dx)] * G[(2, 0, dy)] + G[(0, 0, dx)] * G[(2, 2, dy)]) / (h * h)
            for key, ref in (("M", m), ("Kx", kx), ("Ky", ky), ("B", bb)):
                worst = max(worst, abs(gq[key][i, j] - ref) / max(abs(ref), 1e-3))
    assert worst < 1e-12


# ----------------------------------------------------------------- P3 .. P10
@pytest.mark.parametrize("which", ["grid14", "hs"])
def test_p3_exactness_residual(which, request):
    F, R = request.getfixturevalue(which)
    for fam, r in R["resid"].items():
        assert r.max() < 2e-12, (fam, r.max())


@pytest.mark.parametrize("which", ["grid14", "hs"])
def test_p4_constant_coefficient_wq_equals_gq(which, request):
    F, R = request.getfixturevalue(which)
    n = F["n_fn"]
    pat, data, W, gq = R["pat"], R["data"], R["W"], R["gq"]
    M = O.csr(pat, O.wq_assemble(F, pat, data, W, "mass"), n)
    K = O.csr(pat, O.wq_assemble(F, pat, data, W, "stiffness"), n)
    B = O.csr(pat, O.wq_assemble(F, pat, data, W, "biharmonic"), n)
    for X, Y in ((M, gq["M"]), (K, gq["Kx"] + gq["Ky"]), (B, gq["B"])):
        assert abs(X - Y).max() / abs(Y).max() < 1e-12


def test_p5_partition_of_unity_row_sums(hs):
    F, R = hs
    n = F["n_fn"]
    pat, data, W = R["pat"], R["data"], R["W"]
    M = O.csr(pat, O.wq_assemble(F, pat, data, W, "mass"), n)
    rows = np.asarray(M.sum(axis=1)).ravel()
    # int N_i dx by an independent route: Gauss on every cell of the support
    gp, gw = O.gauss4()
    cl = R["cells"]
    ref = np.zeros(n)
    for c in range(len(cl["elem"])):
        for b in range(4):
            for a in range(4):
                fn, N, _, _, _, _, dJ = O.eval_cell(F, int(cl["elem"][c]), int(cl["sub"][c]), (gp[a], gp[b]))
                ref[fn] += gw[a] * gw[b] * abs(dJ) * N
    assert np.abs(rows - ref).max() < 1e-14
    assert abs(rows.sum() - 1.0) < 1e-13  # the domain is the unit square


def test_p6_derivative_rows_sum_to_zero_for_any_coefficient(hs):
    F, R = hs
    n = F["n_fn"]
    pat, data, W = R["pat"], R["data"], R["W"]
    x = O.point_values(data, "x")
    k = 1.0 + 0.5 * np.cos(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1])
    K = O.csr(pat, O.wq_assemble(F, pat, data, W, "stiffness", k), n)
    B = O.csr(pat, O.wq_assemble(F, pat, data, W, "biharmonic", k), n)
    assert np.abs(np.asarray(K.sum(axis=1))).max() < 1e-12 * abs(K).max()
    assert np.abs(np.asarray(B.sum(axis=1))).max() < 1e-12 * abs(B).max()


def test_p7_stiffness_annihilates_linear_fields(hs):
    F, R = hs
    n = F["n_fn"]
    pat, data, W = R["pat"], R["data"], R["W"]
    K = O.csr(pat, O.wq_assemble(F, pat, data, W, "stiffness"), n)
    interior = F["dir1"] == 0
    for d in range(2):
        r = K @ F["ctrl"][:, d]
        assert np.abs(r[interior]).max() < 1e-12 * abs(K).max()


def test_p8_rank_deficiency(grid14, hs):
    F, R = grid14
    N = 14
    i = _row_of_vertex(F, 7, 7, N)
    n_i = R["pat"]["row_ptr"][i + 1] - R["pat"]["row_ptr"][i]
    assert n_i - R["rank"]["mass"][i] == 0
    # identity geometry: the x system is a Kronecker product with one null direction
    # of the 1D derivative matrix times 7 y-functions
    assert n_i - R["rank"]["x"][i] == 7 and n_i - R["rank"]["y"][i] == 7
    for FF, RR in (grid14, hs):
        ni = np.diff(RR["pat"]["row_ptr"])
        assert (ni - RR["rank"]["x"]).min() >= 2  # partition of unity + linear precision
        assert (ni - RR["rank"]["y"]).min() >= 2
        assert (ni - RR["rank"]["lap"]).min() >= 3  # 1, x, y are harmonic


def test_p10_constant_coefficient_symmetry(hs):
    F, R = hs
    n = F["n_fn"]
    pat, data, W = R["pat"], R["data"], R["W"]
    for kind in ("mass", "stiffness", "biharmonic"):
        A = O.csr(pat, O.wq_assemble(F, pat, data, W, kind), n)
        assert abs(A - A.T).max() < 1e-12 * abs(A).max()


def test_tsvd_is_weighted_min_norm_solution(hs):
    """Independent route: rank-revealing pivoted QR of (A Z)^T gives the minimiser of
    ||Z^{-1} w|| subject to A w = b (Eq. (5)), which Eq. (22) must reproduce when the
    truncated singular values are exact zeros."""
    F, R = hs
    pat, data, gq = R["pat"], R["data"], R["gq"]
    nvf = int((F["fn_vertex"] >= 0).sum())
    rows = [0, 200, nvf - 1, nvf, F["n_fn"] - 1] + list(range(nvf, F["n_fn"], 7))
    for i in rows:
        z = O.z_diag(F, pat, data, i)
        S = pat["S"][i]
        for key, g in (("N", "M"), ("Nx", "Kx"), ("Lap", "B")):
            A = O.local_matrix(F, pat, data, i, key)
            b = np.asarray(gq[g][i, S].todense()).ravel()
            w, t, _ = O.tsvd_solve(A, z, b, 1e-12)
            Qf, Rf, piv = sla.qr((A * z[None, :]).T, mode="economic", pivoting=True)
            r = int(np.sum(np.abs(np.diag(Rf)) > 1e-10 * abs(Rf[0, 0])))
            assert r == t
            y = sla.solve_triangular(Rf[:r, :r].T, b[piv[:r]], lower=True)
            w2 = z * (Qf[:, :r] @ y)
            # two factorisations of the same constrained minimiser: both feasible, equal
            # objective ||Z^-1 w||^2 (flat at the minimum, so it agrees to round-off);
            # the weights themselves agree to their forward error (kappa up to ~1e8 on
            # Laplacian rows next to EPs)
            nb = np.abs(b).max()
            assert np.abs(A @ w - b).max() < 1e-12 * nb
            assert np.abs(A @ w2 - b).max() < 1e-12 * nb
            o1, o2 = np.sum((w / z) ** 2), np.sum((w2 / z) ** 2)
            assert abs(o1 - o2) < 1e-8 * o2
            assert np.abs(w - w2).max() < 1e-6 * np.abs(w).max()


# ----------------------------------------------------------------- P13 counts
def test_p13_point_counts_ep_free():
    for N in (8, 11, 14):
        F = fx.fixture_grid(N)
        cls = O.classify(F)
        s = O.points_per_element(F, cls)
        cl = O.cells(F, s)
        assert cl["pt_off"][-1] == 64 * (N - 3) + 4 * (N - 4) ** 2
        assert 16 * len(cl["elem"]) == 16 * (N - 2) ** 2  # GQ: 4x4 per Bezier cell


def test_table2_points_by_type(hs):
    F, R = hs
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")) as fh:
        tab = json.load(fh)
    t2 = tab["table2_wq_points_per_direction"]
    et, s = R["cls"]["etype"], R["s"]
    names = {O.ET_REGULAR: "regular", O.ET_BOUNDARY: "boundary", O.ET_IRREGULAR: "irregular",
             O.ET_TRANSITION: "non_enriched_transition"}
    for code, name in names.items():
        sel = et == code
        if sel.any():
            assert set(s[sel].tolist()) <= set(t2[name]), name
    # GQ: 4x4 per Bezier cell, i.e. 4x4x4 on an irregular (split) element
    ncell = len(R["cells"]["elem"])
    assert 16 * ncell == sum(tab["table2_gq_points"][names.get(int(e), "regular")] for e in et if e != O.ET_PASSIVE)


# ----------------------------------------------------------------- P11 convergence
def _poisson_l2(F):
    R = O.setup(F, families=("mass", "x", "y"))
    n = F["n_fn"]
    pat, data, W, cl = R["pat"], R["data"], R["W"], R["cells"]
    K = O.csr(pat, O.wq_assemble(F, pat, data, W, "stiffness"), n)
    x = O.point_values(data, "x")
    f = 2 * np.pi ** 2 * np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1])
    # load F_i = sum_q w0_iq f(x_q) (READING X12)
    rhs = np.array([W["mass"][pat["qptr"][i]:pat["qptr"][i + 1]] @ f[pat["qidx"][pat["qptr"][i]:pat["qptr"][i + 1]]]
                    for i in range(n)])
    free = np.nonzero(F["dir1"] == 0)[0]
    u = np.zeros(n)
    Kf = K[free][:, free]
    u[free] = sp.linalg.spsolve(Kf.tocsc(), rhs[free])
    gp, gw = O.gauss4()
    err = 0.0
    for c in range(len(cl["elem"])):
        for b in range(4):
            for a in range(4):
                fn, N, _, _, _, xx, dJ = O.eval_cell(F, int(cl["elem"][c]), int(cl["sub"][c]), (gp[a], gp[b]))
                ex = np.sin(np.pi * xx[0]) * np.sin(np.pi * xx[1])
                err += gw[a] * gw[b] * abs(dJ) * (N @ u[fn] - ex) ** 2
    return np.sqrt(err)


@pytest.mark.slow
def test_p11_poisson_l2_rate_four():
    Ns = (8, 12, 20)
    errs = [_poisson_l2(fx.fixture_grid(N)) for N in Ns]
    hs_ = [1.0 / (N - 2) for N in Ns]
    rate = np.polyfit(np.log(hs_), np.log(errs), 1)[0]
    assert rate > 3.6, (errs, rate)


def test_gq_assemble_with_given_basis_matches_gq_matrices(hs):
    """The element-wise Gauss assembly with the basis computed ahead (used to time Gauss
    formation against WQ formation, Section 6.1) equals gq_matrices term by term."""
    F, R = hs
    cl = R["cells"]
    gd = O.gauss_data(F, cl)
    coef = lambda x: 1.0 + 0.5 * np.sin(2 * np.pi * x[..., 0]) * np.sin(2 * np.pi * x[..., 1])  # noqa: E731
    ref = O.gq_matrices(F, cl, coef=coef)
    M = O.gq_assemble(F, gd, "mass", coef)
    K = O.gq_assemble(F, gd, "stiffness", coef)
    assert abs(M - ref["M"]).max() <= 1e-15 * abs(ref["M"]).max()
    assert abs(K - (ref["Kx"] + ref["Ky"])).max() <= 1e-14 * abs(ref["Kx"] + ref["Ky"]).max()
