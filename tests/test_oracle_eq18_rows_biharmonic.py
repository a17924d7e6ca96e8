"""Further pins of the FP64 oracle: the min-max allocation of Eq. (18) against numbers
worked out by hand and against Table 2, the row-by-row path (sample_rows) against the
whole-mesh setup, and the biharmonic manufactured solution of Section 6.1."""
import numpy as np
import pytest
import scipy.sparse as sp

import fixtures as fx
import oracle as O

REG, BND, IRR, TRN = O.ET_REGULAR, O.ET_BOUNDARY, O.ET_IRREGULAR, O.ET_TRANSITION


# ----------------------------------------------------------------- Eq. (18) by hand
def test_eq18_hand_worked_requirements():
    """Eq. (18) with every term active. Row with n_i = 87 and a support of 3 regular
    (m = 16), 2 boundary (m = 16) and 3 other elements with m = 21, 18, 16:
      n_i - 4 e^r - 16 e^b = 87 - 12 - 32 = 43,   sum of m over supp minus R = 55,
      r = 21*43/55 = 16.42 -> 17,  18*43/55 = 14.07 -> 15,  16*43/55 = 12.51 -> 13."""
    elems = [(REG, 16), (IRR, 21), (BND, 16), (REG, 16), (TRN, 18), (BND, 16), (TRN, 16), (REG, 16)]
    assert O.minmax_row_requirement(87, elems) == [None, 17, None, None, 15, None, 13, None]
    # an exact quotient is not rounded up: 60 - 16 - 16 = 28, 22 * 28 / 44 = 14
    elems = [(REG, 16)] * 4 + [(BND, 16), (TRN, 22), (TRN, 22)]
    assert O.minmax_row_requirement(60, elems)[-2:] == [14, 14]
    # regular and boundary counts alone exceed n_i: nothing is required of the others
    assert O.minmax_row_requirement(30, [(REG, 16), (REG, 16), (BND, 16), (BND, 16), (TRN, 17)])[-1] <= 0


def test_eq18_points_per_direction():
    """s_k = smallest s >= 2 with s^2 >= r_k; even on split (irregular) elements."""
    cases = [(0, False, 2), (4, False, 2), (5, False, 3), (9, False, 3), (10, False, 4),
             (13, False, 4), (15, False, 4), (17, False, 5), (17, True, 6), (5, True, 4), (16, True, 4)]
    for r, split, s in cases:
        assert O.minmax_points_per_direction(r, split) == s, (r, split)


@pytest.mark.parametrize("name", ["hs", "eps32"])
def test_minmax_from_2x2_reproduces_table2(name):
    """Section 4.2: running the min-max strategy gives the counts of Table 2 (regular 2x2
    and boundary 4x4 kept; irregular 4x4; non-enriched transition 3x3 when no EP is of
    valence >= 7 or clustered). Start every other element at 2x2 and let Eq. (18) raise
    them until every row is well posed."""
    F = fx.fixture_half_strip() if name == "hs" else fx.fixture_eps(32, 0.02, (3, 5, 6), seed=5)
    cls = O.classify(F)
    et = cls["etype"]
    s0 = np.where(et == REG, 2, np.where(et == BND, 4, np.where(et == O.ET_PASSIVE, 0, 2)))
    s = O.points_per_element(F, cls, s0)
    assert (s[et == REG] == 2).all() and (s[et == BND] == 4).all()
    assert (et == IRR).any() and (s[et == IRR] == 4).all()
    assert (et == TRN).any() and (s[et == TRN] == 3).all()
    assert np.array_equal(s, O.points_per_element(F, cls))


# ----------------------------------------------------------------- sampled rows
@pytest.mark.parametrize("name,step", [("hs", 1), ("eps32", 3)])
def test_sample_rows_reproduce_whole_mesh_setup(name, step, fixture_cache):
    """The row-by-row path (used to check large meshes) against the whole-mesh setup:
    S_i and Q_i bit for bit, A and z bit for bit (same evaluation), b to round-off of the
    Gauss sums (Section 2, Section 4.2), weights within their forward error, and the
    assembled rows of Eqs. (9) and (11) with variable coefficients to 1e-12."""
    F = fx.fixture_half_strip() if name == "hs" else fx.fixture_eps(32, 0.02, (3, 5, 6), seed=5)
    R = O.setup(F, families=("mass", "x", "y"))
    pat, data = R["pat"], R["data"]
    cm = lambda x: 1.0 + 0.5 * np.sin(2 * np.pi * x[:, 0]) * np.sin(2 * np.pi * x[:, 1])  # noqa: E731
    ck = lambda x: 1.0 + 0.5 * np.cos(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1])  # noqa: E731
    xq = O.point_values(data, "x")
    M = O.wq_assemble(F, pat, data, R["W"], "mass", cm(xq))
    K = O.wq_assemble(F, pat, data, R["W"], "stiffness", ck(xq))
    rows = list(range(0, F["n_fn"], step))
    out, _ = O.sample_rows(F, rows, coef={"mass": cm, "stiffness": ck})
    sm, sk = np.abs(M).max(), np.abs(K).max()
    for i in rows:
        r = out[i]
        a, b = pat["row_ptr"][i], pat["row_ptr"][i + 1]
        q0, q1 = pat["qptr"][i], pat["qptr"][i + 1]
        assert np.array_equal(r["S"], pat["col"][a:b])
        assert np.array_equal(r["Q"], pat["qidx"][q0:q1])
        assert np.array_equal(r["z"], O.z_diag(F, pat, data, i))
        for fam, key, g in (("mass", "N", "M"), ("x", "Nx", "Kx"), ("y", "Ny", "Ky")):
            assert np.array_equal(r["A_" + fam], O.local_matrix(F, pat, data, i, key))
            bw = np.asarray(R["gq"][g][i, r["S"]].todense()).ravel()
            assert np.abs(r["b_" + fam] - bw).max() <= 1e-14 * np.abs(bw).max()
            w, ww = r["W"][fam], R["W"][fam][q0:q1]
            assert np.abs(w - ww).max() <= 1e-6 * np.abs(ww).max()
        assert np.abs(r["M"] - M[a:b]).max() <= 1e-12 * sm
        # a variable coefficient also weighs the weights' components along the (near-)null
        # space of A, where the two b's rounding differences are amplified: the stiffness
        # rows agree to 1e-12 plus that forward error, mapped through |A| diag(k)
        k_i = ck(r["x"])
        fwd = sum(np.abs(r["A_" + f]) @ (k_i * np.abs(r["W"][f] - R["W"][f][q0:q1])) for f in ("x", "y"))
        assert (np.abs(r["K"] - K[a:b]) <= 1e-12 * sk + 2 * fwd).all()
    # with coefficient 1 the rows are A w = b itself: 1e-12 with no allowance
    out1, _ = O.sample_rows(F, rows[:: max(1, len(rows) // 40)])
    M1 = O.wq_assemble(F, pat, data, R["W"], "mass")
    K1 = O.wq_assemble(F, pat, data, R["W"], "stiffness")
    for i, r in out1.items():
        a, b = pat["row_ptr"][i], pat["row_ptr"][i + 1]
        assert np.abs(r["M"] - M1[a:b]).max() <= 1e-12 * np.abs(M1).max()
        assert np.abs(r["K"] - K1[a:b]).max() <= 1e-12 * np.abs(K1).max()


# ----------------------------------------------------------------- biharmonic P11
def _u_star(x):
    return (1 - np.cos(2 * np.pi * x[..., 0])) * (1 - np.cos(2 * np.pi * x[..., 1]))


def _bilaplacian_u_star(x):
    """Delta^2 of (1 - cos 2 pi x)(1 - cos 2 pi y), written out term by term:
    u_xxxx = -(2pi)^4 cos2pix (1 - cos2piy), u_xxyy = (2pi)^4 cos2pix cos2piy, u_yyyy by symmetry."""
    k4 = (2 * np.pi) ** 4
    cx, cy = np.cos(2 * np.pi * x[..., 0]), np.cos(2 * np.pi * x[..., 1])
    return -k4 * cx * (1 - cy) + 2 * k4 * cx * cy - k4 * cy * (1 - cx)


def _biharmonic_errors(N):
    F = fx.fixture_grid(N, displace=0.05, seed=11)
    R = O.setup(F, families=("mass", "lap"))
    n = F["n_fn"]
    pat, data, W, cl, gq = R["pat"], R["data"], R["W"], R["cells"], R["gq"]
    B = O.csr(pat, O.wq_assemble(F, pat, data, W, "biharmonic"), n)
    g = _bilaplacian_u_star(O.point_values(data, "x"))
    # WQ load with the mass-family weights (READING X12); GQ load for the GQ solution
    rhs_wq = np.array([W["mass"][pat["qptr"][i]:pat["qptr"][i + 1]] @ g[pat["qidx"][pat["qptr"][i]:pat["qptr"][i + 1]]]
                       for i in range(n)])
    gp, gw = O.gauss4()
    rhs_gq = np.zeros(n)
    evals = []
    for c in range(len(cl["elem"])):
        for b in range(4):
            for a in range(4):
                fn, Nv, _, _, _, xx, dJ = O.eval_cell(F, int(cl["elem"][c]), int(cl["sub"][c]), (gp[a], gp[b]))
                wgt = gw[a] * gw[b] * abs(dJ)
                rhs_gq[fn] += wgt * Nv * _bilaplacian_u_star(xx)
                evals.append((fn, Nv, xx, wgt))
    free = np.nonzero(F["dir2"] == 0)[0]  # clamped: the outer two function layers are 0

    def solve(A, r):
        u = np.zeros(n)
        u[free] = sp.linalg.spsolve(A[free][:, free].tocsc(), r[free])
        return u

    def l2(u):
        return np.sqrt(sum(wgt * (Nv @ u[fn] - _u_star(xx)) ** 2 for fn, Nv, xx, wgt in evals))

    return l2(solve(B, rhs_wq)), l2(solve(gq["B"], rhs_gq)), abs(B - gq["B"]).max() / abs(gq["B"]).max()


@pytest.mark.slow
def test_p11_biharmonic_wq_matches_gq_at_rate_four():
    """Section 6.1 biharmonic test, clamped, u = (1 - cos 2 pi x)(1 - cos 2 pi y): the WQ
    error curve lies on the GQ curve and both converge at the optimal L2 rate p + 1 = 4
    under refinement of a fixed smooth geometry map (EP-free: with EPs the rate depends
    on the spline space near them)."""
    Ns = (8, 12, 20)
    res = [_biharmonic_errors(N) for N in Ns]
    h = [1.0 / (N - 2) for N in Ns]
    for ew, eg, db in res:
        assert db < 1e-12  # constant coefficient: WQ B equals GQ B (P4)
        assert abs(ew / eg - 1.0) < 0.05
    for k in range(2):
        rate = np.polyfit(np.log(h), np.log([r[k] for r in res]), 1)[0]
        assert 3.7 < rate < 5.0, (k, rate, res)
