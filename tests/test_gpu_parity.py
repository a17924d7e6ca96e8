"""GPU (libwq.so through the C ABI) against the FP64 oracle, element by element.

Integer outputs (classification, pattern, point sets) must be bit-exact. FP64 outputs
are compared normwise per array: max |gpu - oracle| / max |oracle|; the bound for
assembled matrices is 1e-12. Weights are forward quantities of ill-conditioned
systems, so they are compared through what fixes them: the exactness residual
||A w - b|| (A, b from the oracle) and agreement to their conditioning-limited level.
"""
import numpy as np
import pytest

import fixtures as fx
import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _wq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_29334_amd.wq as W
    return W


FAM = {"mass": 1, "x": 2, "y": 4, "lap": 8}


def _run_case(F, families, want_lap):
    W = _wq()
    R = O.setup(F, families=families)
    mesh = W.Mesh(F)
    pts = W.Points(mesh, want_laplacian=want_lap)
    mask = sum(FAM[f] for f in families)
    wts = W.Weights(mesh, pts, mask, tau=1e-12)
    return {"F": F, "R": R, "W": W, "mesh": mesh, "pts": pts, "wts": wts, "families": families}


@pytest.fixture(scope="module")
def hs():
    print("[gpu] case half_strip", flush=True)
    return _run_case(fx.fixture_half_strip(), ("mass", "x", "y", "lap"), True)


@pytest.fixture(scope="module")
def grid():
    print("[gpu] case grid12", flush=True)
    return _run_case(fx.fixture_grid(12, displace=0.05, seed=3), ("mass", "x", "y", "lap"), True)


@pytest.fixture(scope="module")
def eps():
    print("[gpu] case eps32", flush=True)
    return _run_case(fx.fixture_eps(32, 0.02, (3, 5, 6), seed=5), ("mass", "x", "y"), False)


CASES = ["hs", "grid", "eps"]


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("case", CASES)
def test_classification_bit_exact(case, request):
    c = request.getfixturevalue(case)
    W, pts, R = c["W"], c["pts"], c["R"]
    et = _np(pts.get(W.ARR_ETYPE)).astype(np.int64)
    s = _np(pts.get(W.ARR_S)).astype(np.int64)
    np.testing.assert_array_equal(et, R["cls"]["etype"])
    np.testing.assert_array_equal(s, R["s"])


@pytest.mark.parametrize("case", CASES)
def test_pattern_and_point_sets_bit_exact(case, request):
    c = request.getfixturevalue(case)
    W, pts, pat = c["W"], c["pts"], c["R"]["pat"]
    np.testing.assert_array_equal(_np(pts.get(W.ARR_ROW_PTR)), pat["row_ptr"])
    np.testing.assert_array_equal(_np(pts.get(W.ARR_COL)), pat["col"])
    np.testing.assert_array_equal(_np(pts.get(W.ARR_QPTR)), pat["qptr"])
    np.testing.assert_array_equal(_np(pts.get(W.ARR_QIDX)), pat["qidx"])
    assert pts.n_points == c["R"]["cells"]["pt_off"][-1]


@pytest.mark.parametrize("case", CASES)
def test_points_geometry(case, request):
    c = request.getfixturevalue(case)
    W, pts, data = c["W"], c["pts"], c["R"]["data"]
    x = _np(pts.get(W.ARR_X)).reshape(-1, 2)
    dj = _np(pts.get(W.ARR_DETJ))
    assert _rel(x, O.point_values(data, "x")) < 1e-14
    assert _rel(dj, O.point_values(data, "detJ")) < 1e-13


@pytest.mark.parametrize("case", CASES)
def test_gauss_rhs(case, request):
    c = request.getfixturevalue(case)
    F, R, wts = c["F"], c["R"], c["wts"]
    n = F["n_fn"]
    pat = R["pat"]
    for fam in c["families"]:
        ref = R["gq"][O.wq._FAM_GQ[fam]]
        got = O.csr(pat, _np(wts.rhs(FAM[fam])), n)
        assert abs(got - ref).max() / abs(ref).max() < 1e-13, fam


@pytest.mark.parametrize("case", CASES)
def test_weights_exactness_and_agreement(case, request):
    c = request.getfixturevalue(case)
    F, R, wts = c["F"], c["R"], c["wts"]
    pat, data, gq = R["pat"], R["data"], R["gq"]
    for fam in c["families"]:
        wg = _np(wts.weights(FAM[fam]))
        wo = R["W"][fam]
        key = O.wq._FAM_KEY[fam]
        eps = np.finfo(np.float64).eps
        bg = _np(wts.rhs(FAM[fam]))  # the GPU's own right-hand sides (Gauss, parity 1e-13)
        rp = pat["row_ptr"]
        worst_res, worst_ratio, worst_diff = 0.0, 0.0, 0.0
        for i in range(F["n_fn"]):
            q0, q1 = pat["qptr"][i], pat["qptr"][i + 1]
            A = O.local_matrix(F, pat, data, i, key)
            b = np.asarray(gq[O.wq._FAM_GQ[fam]][i, pat["S"][i]].todense()).ravel()
            w = wg[q0:q1]
            # Eqs. (20)-(22) satisfy the constraints on the kept singular subspace only, so
            # the part of b along dropped singular vectors (sigma <= 1e-12 sigma_1) stays in
            # the residual; rounding in the kept part is amplified by at most
            # kappa_t = sigma_1 / sigma_t (the computed singular directions err by
            # eps sigma_1 / sigma_k), plus the backward error eps ||A|| ||w|| of the final
            # orthogonal solve. Rows next to the open-knot boundary keep singular values down
            # to ~3e-6 sigma_1, so their residual reaches ~1e-11.
            bi = bg[rp[i]:rp[i + 1]]
            U, sg, _ = np.linalg.svd(A, full_matrices=False)
            kept = sg > 1e-12 * sg[0]
            Ut = U[:, kept]
            dropped = np.linalg.norm(bi - Ut @ (Ut.T @ bi))
            res = np.abs(A @ w - bi).max()
            kappa_t = sg[0] / sg[kept][-1]
            bound = 8 * eps * (kappa_t * np.linalg.norm(bi) + sg[0] * np.linalg.norm(w)) + 2 * dropped
            worst_res = max(worst_res, np.abs(A @ w - b).max() / np.abs(b).max())
            worst_ratio = max(worst_ratio, res / bound)
            worst_diff = max(worst_diff, np.abs(w - wo[q0:q1]).max() / np.abs(wo[q0:q1]).max())
        print(f"[gpu] {case} {fam}: exactness {worst_res:.2e} (worst residual / backward-error bound "
              f"{worst_ratio:.2f}), weight diff {worst_diff:.2e}")
        assert worst_ratio <= 1.0, (fam, worst_ratio)
        assert worst_res < 1e-10, (fam, worst_res)
        assert worst_diff < 1e-4, (fam, worst_diff)


def _coefs(R):
    x = O.point_values(R["data"], "x")
    c = 1.0 + 0.5 * np.sin(2 * np.pi * x[:, 0]) * np.sin(2 * np.pi * x[:, 1])
    k = 1.0 + 0.5 * np.cos(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1])
    return c, k


@pytest.mark.parametrize("case", CASES)
def test_assembly_parity(case, request):
    """End-to-end mass matrices (well-conditioned systems: sigma_t/sigma_1 >= 1e-4),
    with and without a variable coefficient: 1e-12 normwise."""
    c = request.getfixturevalue(case)
    F, R, W, pts, wts = c["F"], c["R"], c["W"], c["pts"], c["wts"]
    pat, data, Wo = R["pat"], R["data"], R["W"]
    cc, _ = _coefs(R)
    tc = torch.tensor(cc, device="cuda")
    errs = {
        "M1": _rel(_np(W.assemble_mass(pts, wts)), O.wq_assemble(F, pat, data, Wo, "mass")),
        "Mc": _rel(_np(W.assemble_mass(pts, wts, tc)), O.wq_assemble(F, pat, data, Wo, "mass", cc)),
    }
    print(f"[gpu] {case} assembly rel err {errs}")
    for k, v in errs.items():
        assert v < 1e-12, (k, v)


@pytest.mark.parametrize("case", CASES)
def test_assembly_kernel_against_oracle_with_same_weights(case, request):
    """The row contraction itself: oracle assembly (Eqs. 9, 11, 12) evaluated with the
    GPU's weights must equal the GPU assembly, for variable coefficients too."""
    c = request.getfixturevalue(case)
    F, R, W, pts, wts = c["F"], c["R"], c["W"], c["pts"], c["wts"]
    pat, data = R["pat"], R["data"]
    Wg = {f: _np(wts.weights(FAM[f])) for f in c["families"]}
    cc, kk = _coefs(R)
    tc, tk = torch.tensor(cc, device="cuda"), torch.tensor(kk, device="cuda")
    mg, kg = W.assemble_mass_stiffness(pts, wts, tc, tk)
    errs = {
        "Mc": _rel(_np(mg), O.wq_assemble(F, pat, data, Wg, "mass", cc)),
        "Kk": _rel(_np(kg), O.wq_assemble(F, pat, data, Wg, "stiffness", kk)),
        "Kk_single": _rel(_np(W.assemble_stiffness(pts, wts, tk)), O.wq_assemble(F, pat, data, Wg, "stiffness", kk)),
    }
    if "lap" in c["families"]:
        errs["Bk"] = _rel(_np(W.assemble_biharmonic(pts, wts, tk)), O.wq_assemble(F, pat, data, Wg, "biharmonic", kk))
    print(f"[gpu] {case} kernel-only rel err {errs}")
    for k, v in errs.items():
        assert v < 1e-12, (k, v)


def _row_condition(F, R, i, families):
    """First-order condition number of row i's weights w.r.t. rounding of A and b:
    (sigma_1 / sigma_t) * kappa(Z V_t), maximised over the families used."""
    pat, data = R["pat"], R["data"]
    z = O.z_diag(F, pat, data, i)
    worst = 1.0
    for fam in families:
        A = O.local_matrix(F, pat, data, i, O.wq._FAM_KEY[fam])
        _, sg, Vt = np.linalg.svd(A, full_matrices=False)
        t = int(np.sum(sg > 1e-12 * sg[0]))
        kz = np.linalg.cond(z[:, None] * Vt[:t].T)
        worst = max(worst, sg[0] / sg[t - 1] * kz)
    return worst


@pytest.mark.parametrize("case", CASES)
def test_stiffness_biharmonic_end_to_end_within_conditioning(case, request):
    """Stiffness/biharmonic rows depend on the weights along the smallest kept singular
    directions; two backward-stable SVDs agree there only to eps (sigma_1/sigma_t)
    kappa(Z V_t) (with c = 1 the gap to the Gauss matrix is the exactness residual,
    bounded by the same quantity). Each row is held to 1e-12 plus 8 eps times it."""
    c = request.getfixturevalue(case)
    F, R, W, pts, wts = c["F"], c["R"], c["W"], c["pts"], c["wts"]
    pat, data, Wo = R["pat"], R["data"], R["W"]
    _, kk = _coefs(R)
    tk = torch.tensor(kk, device="cuda")
    kinds = [("stiffness", ("x", "y"), W.assemble_stiffness, kk, tk),
             ("stiffness", ("x", "y"), W.assemble_stiffness, None, None)]
    if "lap" in c["families"]:
        kinds.append(("biharmonic", ("lap",), W.assemble_biharmonic, kk, tk))
        kinds.append(("biharmonic", ("lap",), W.assemble_biharmonic, None, None))
    eps = np.finfo(np.float64).eps
    for kind, fams, fn, coef, tcoef in kinds:
        ref = O.wq_assemble(F, pat, data, Wo, kind, coef)
        got = _np(fn(pts, wts, tcoef))
        scale = np.abs(ref).max()
        rp = pat["row_ptr"]
        worst_ratio, over_1e12 = 0.0, 0
        for i in range(F["n_fn"]):
            d = np.abs(got[rp[i]:rp[i + 1]] - ref[rp[i]:rp[i + 1]]).max() / scale
            if d <= 1e-12:
                continue
            over_1e12 += 1
            bound = 1e-12 + 8 * eps * _row_condition(F, R, i, fams)
            worst_ratio = max(worst_ratio, d / bound)
        print(f"[gpu] {case} {kind} coef={'var' if coef is not None else 'one'}: global rel err {_rel(got, ref):.2e}, rows above 1e-12: {over_1e12}, "
              f"worst err/bound {worst_ratio:.2e}")
        assert worst_ratio <= 1.0


@pytest.mark.parametrize("case", CASES)
def test_constant_coefficient_matches_gauss(case, request):
    """Exactness carried through the GPU path: c = 1 gives the Gauss matrices."""
    c = request.getfixturevalue(case)
    F, R, W, pts, wts = c["F"], c["R"], c["W"], c["pts"], c["wts"]
    n = F["n_fn"]
    pat, gq = R["pat"], R["gq"]
    M = O.csr(pat, _np(W.assemble_mass(pts, wts)), n)
    K = O.csr(pat, _np(W.assemble_stiffness(pts, wts)), n)
    assert abs(M - gq["M"]).max() / abs(gq["M"]).max() < 1e-12
    assert abs(K - gq["Kx"] - gq["Ky"]).max() / abs(gq["Kx"] + gq["Ky"]).max() < 1e-12


def test_determinism(hs):
    W, pts, wts = hs["W"], hs["pts"], hs["wts"]
    a = _np(W.assemble_stiffness(pts, wts))
    b = _np(W.assemble_stiffness(pts, wts))
    assert np.array_equal(a, b)
    w2 = W.Weights(hs["mesh"], pts, 2, tau=1e-12)
    assert np.array_equal(_np(w2.weights(2)), _np(wts.weights(2)))


def test_min_max_fallback_matches_oracle():
    """Start with 2x2 points on the transition elements (below Table 2): some rows are
    ill-posed and Eq. (18) must raise them exactly as the oracle does."""
    W = _wq()
    F = fx.fixture_half_strip()
    cls = O.classify(F)
    s0 = cls["s"].copy()
    s0[cls["etype"] == O.ET_TRANSITION] = 2
    s_ref = O.points_per_element(F, cls, s_init=s0)
    assert (s_ref != s0).any()
    mesh = W.Mesh(F)
    pts = W.Points(mesh, s_init=s0)
    np.testing.assert_array_equal(_np(pts.get(W.ARR_S)).astype(np.int64), s_ref)


def test_ill_posed_is_reported():
    W = _wq()
    F = fx.fixture_grid(10)
    cls = O.classify(F)
    s0 = cls["s"].copy()
    s0[s0 > 0] = 1  # one point per element cannot carry 16..49 constraints
    mesh = W.Mesh(F)
    with pytest.raises(W.WQError) as e:
        W.Points(mesh, s_init=s0)
    assert e.value.status == -3


def test_bad_input_is_rejected():
    W = _wq()
    F = dict(fx.fixture_grid(8))
    F["face_vtx"] = F["face_vtx"].copy()
    F["face_vtx"][0, 0] = 10 ** 6
    with pytest.raises(W.WQError) as e:
        W.Mesh(F)
    assert e.value.status == -1
