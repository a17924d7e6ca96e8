"""Surfaces on the GPU (Section 4.1 on 2-manifolds: surface gradient with three
components, the d/dz weight family, Laplace-Beltrami operator) against the oracle, through
the C ABI, on a curved 2-EP cap (the half strip lifted onto a sphere) and on a plane placed
in 3-D by a rotation. The same bars as the planar parity tests: integers bit-exact,
geometry and right-hand sides 1e-13, weights through their exactness residual, the row
contraction with the GPU's weights 1e-12, constant-coefficient matrices equal to the Gauss
ones to 1e-12, and the Gauss comparison system 1e-12.
"""
import numpy as np
import pytest

import fixtures as fx
import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FAM = {"mass": 1, "x": 2, "y": 4, "lap": 8, "z": 16}
FAMS = ("mass", "x", "y", "z", "lap")


def _wq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_29334_amd.wq as W
    return W


def _run(F):
    W = _wq()
    R = O.setup(F, families=FAMS)
    mesh = W.Mesh(F)
    pts = W.Points(mesh, want_laplacian=True)
    wts = W.Weights(mesh, pts, sum(FAM[f] for f in FAMS), tau=1e-12)
    return {"F": F, "R": R, "W": W, "mesh": mesh, "pts": pts, "wts": wts}


@pytest.fixture(scope="module")
def dome():
    print("[gpu] surface case dome (half strip on a sphere)", flush=True)
    return _run(fx.fixture_dome(fx.fixture_half_strip(), radius=1.5))


@pytest.fixture(scope="module")
def plane3():
    print("[gpu] surface case rotated grid 8", flush=True)
    return _run(fx.rotate_to_3d(fx.fixture_grid(8, displace=0.05, seed=11)))


CASES = ["dome", "plane3"]


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("case", CASES)
def test_surface_points_and_pattern(case, request):
    c = request.getfixturevalue(case)
    W, R, pts = c["W"], c["R"], c["pts"]
    pat = R["pat"]
    assert np.array_equal(_np(pts.get(W.ARR_ROW_PTR)), pat["row_ptr"])
    assert np.array_equal(_np(pts.get(W.ARR_COL)), pat["col"])
    assert np.array_equal(_np(pts.get(W.ARR_QPTR)), pat["qptr"])
    assert np.array_equal(_np(pts.get(W.ARR_QIDX)), pat["qidx"])
    x = _np(pts.get(W.ARR_X)).reshape(-1, 3)
    xo = O.point_values(R["data"], "x")
    dj = _np(pts.get(W.ARR_DETJ))
    djo = O.point_values(R["data"], "detJ")
    print(f"[gpu] {case}: x {_rel(x, xo):.2e}, sqrt(det g) {_rel(dj, djo):.2e}")
    assert _rel(x, xo) < 1e-13 and _rel(dj, djo) < 1e-13


@pytest.mark.parametrize("case", CASES)
def test_surface_gauss_rhs(case, request):
    c = request.getfixturevalue(case)
    F, R, wts = c["F"], c["R"], c["wts"]
    for fam in FAMS:
        ref = R["gq"][O.wq._FAM_GQ[fam]]
        got = O.csr(R["pat"], _np(wts.rhs(FAM[fam])), F["n_fn"])
        err = abs(got - ref).max() / abs(ref).max()
        print(f"[gpu] {case} rhs {fam}: {err:.2e}")
        assert err < 1e-13, fam


@pytest.mark.parametrize("case", CASES)
def test_surface_weights_exactness(case, request):
    """As for the planar systems: the residual of the GPU weights on the oracle's system,
    against the backward-error bound of the kept singular subspace."""
    c = request.getfixturevalue(case)
    F, R, wts = c["F"], c["R"], c["wts"]
    pat, data, gq = R["pat"], R["data"], R["gq"]
    eps = np.finfo(np.float64).eps
    for fam in FAMS:
        wg = _np(wts.weights(FAM[fam]))
        wo = R["W"][fam]
        bg = _np(wts.rhs(FAM[fam]))
        rp = pat["row_ptr"]
        worst_res, worst_ratio, worst_diff = 0.0, 0.0, 0.0
        for i in range(F["n_fn"]):
            q0, q1 = pat["qptr"][i], pat["qptr"][i + 1]
            A = O.local_matrix(F, pat, data, i, O.wq._FAM_KEY[fam])
            b = np.asarray(gq[O.wq._FAM_GQ[fam]][i, pat["S"][i]].todense()).ravel()
            w = wg[q0:q1]
            bi = bg[rp[i]:rp[i + 1]]
            U, sg, Vt = np.linalg.svd(A, full_matrices=False)
            kept = sg > 1e-12 * sg[0]
            Ut = U[:, kept]
            dropped = np.linalg.norm(bi - Ut @ (Ut.T @ bi))
            res = np.abs(A @ w - bi).max()
            bound = 8 * eps * (sg[0] / sg[kept][-1] * np.linalg.norm(bi) + sg[0] * np.linalg.norm(w)) + 2 * dropped
            worst_res = max(worst_res, np.abs(A @ w - b).max() / np.abs(b).max())
            worst_ratio = max(worst_ratio, res / bound)
            # agreement with the oracle's weights: 1e-4, or the weights' first-order
            # sensitivity to rounding, (sigma_1 / sigma_t) kappa(Z V_t), where that is larger
            # (the Laplace-Beltrami systems of the curved cap reach it)
            diff = np.abs(w - wo[q0:q1]).max() / np.abs(wo[q0:q1]).max()
            if diff > 1e-4:
                z = O.z_diag(F, pat, data, i)
                cond = sg[0] / sg[kept][-1] * np.linalg.cond(z[:, None] * Vt[kept].T)
                diff = 1e-4 * diff / max(1e-4, 8 * eps * cond)
            worst_diff = max(worst_diff, diff)
        print(f"[gpu] {case} weights {fam}: exactness {worst_res:.2e}, residual/bound {worst_ratio:.2f}, "
              f"diff (scaled to 1e-4 at the conditioning bound) {worst_diff:.2e}")
        assert worst_ratio <= 1.0 and worst_res < 1e-10 and worst_diff < 1e-4, fam


@pytest.mark.parametrize("case", CASES)
def test_surface_assembly_with_same_weights(case, request):
    """Mass, stiffness (three surface-gradient families) and Laplace-Beltrami matrices:
    the oracle's row contraction with the GPU's weights equals the GPU assembly."""
    c = request.getfixturevalue(case)
    F, R, W, pts, wts = c["F"], c["R"], c["W"], c["pts"], c["wts"]
    pat, data = R["pat"], R["data"]
    Wg = {f: _np(wts.weights(FAM[f])) for f in FAMS}
    x = O.point_values(data, "x")
    cc = 1.0 + 0.5 * np.sin(2 * np.pi * x[:, 0]) * np.sin(2 * np.pi * x[:, 1])
    kk = 1.0 + 0.3 * x[:, 2]
    tc, tk = torch.tensor(cc, device="cuda"), torch.tensor(kk, device="cuda")
    mg, kg = W.assemble_mass_stiffness(pts, wts, tc, tk)
    errs = {
        "Mc": _rel(_np(mg), O.wq_assemble(F, pat, data, Wg, "mass", cc)),
        "Kk": _rel(_np(kg), O.wq_assemble(F, pat, data, Wg, "stiffness", kk)),
        "Kk_single": _rel(_np(W.assemble_stiffness(pts, wts, tk)), O.wq_assemble(F, pat, data, Wg, "stiffness", kk)),
        "Bk": _rel(_np(W.assemble_biharmonic(pts, wts, tk)), O.wq_assemble(F, pat, data, Wg, "biharmonic", kk)),
    }
    print(f"[gpu] {case} surface kernel-only rel err {errs}")
    for k, v in errs.items():
        assert v < 1e-12, (k, v)


@pytest.mark.parametrize("case", CASES)
def test_surface_constant_coefficient_matches_gauss(case, request):
    c = request.getfixturevalue(case)
    F, R, W, pts, wts = c["F"], c["R"], c["W"], c["pts"], c["wts"]
    n = F["n_fn"]
    pat, gq = R["pat"], R["gq"]
    M = O.csr(pat, _np(W.assemble_mass(pts, wts)), n)
    K = O.csr(pat, _np(W.assemble_stiffness(pts, wts)), n)
    Kg = gq["Kx"] + gq["Ky"] + gq["Kz"]
    em = abs(M - gq["M"]).max() / abs(gq["M"]).max()
    ek = abs(K - Kg).max() / abs(Kg).max()
    print(f"[gpu] {case} WQ vs Gauss, coefficient 1: M {em:.2e}, K {ek:.2e}")
    assert em < 1e-12 and ek < 1e-12


@pytest.mark.parametrize("case", CASES)
def test_surface_gauss_assembly(case, request):
    c = request.getfixturevalue(case)
    F, R, W = c["F"], c["R"], c["W"]
    G = W.Gauss(c["mesh"], c["pts"], want_laplacian=True)
    xg = _np(G.x()).reshape(-1, 3)
    coef = lambda x: 1.0 + 0.3 * x[..., 2]  # noqa: E731
    cg = torch.tensor(coef(xg), device="cuda")
    ref = O.gq_matrices(F, R["cells"], coef=coef)
    for kind, Rm in ((W.GQ_MASS, ref["M"]), (W.GQ_STIFFNESS, ref["Kx"] + ref["Ky"] + ref["Kz"]),
                     (W.GQ_BIHARMONIC, ref["B"])):
        got = O.csr(R["pat"], _np(G.assemble(kind, cg)), F["n_fn"])
        err = abs(got - Rm).max() / abs(Rm).max()
        print(f"[gpu] {case} surface gauss kind {kind}: {err:.2e}")
        assert err < 1e-12, kind


def test_surface_rejections(dome):
    W, pts, wts = dome["W"], dome["pts"], dome["wts"]
    n = dome["F"]["n_fn"]
    T = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(W.WQError):
        W.assemble_tangent(pts, wts, T, T, 1.0)
    with pytest.raises(W.WQError):
        W.assemble_stiffness(pts, wts, prec=W.WQ_SPLIT_BF16)
    # without the d/dz weights a surface stiffness is refused; a plane has no d/dz family
    w3 = W.Weights(dome["mesh"], pts, W.WQ_FAM_MASS | W.WQ_FAM_DX | W.WQ_FAM_DY, tau=1e-12)
    with pytest.raises(W.WQError):
        W.assemble_stiffness(pts, w3)
    F2 = fx.fixture_grid(6, displace=0.05, seed=2)
    m2 = W.Mesh(F2)
    p2 = W.Points(m2)
    with pytest.raises(W.WQError):
        W.Weights(m2, p2, W.WQ_FAM_DZ, tau=1e-12)
