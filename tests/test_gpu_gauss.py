"""Element-wise Gauss assembly on the GPU (the comparison system; gauss_setup and
assemble_gauss through the C ABI) against the oracle's element-wise Gauss matrices.

The oracle evaluates the basis at the 4 x 4 Gauss points of every Bezier cell and sums
the weighted outer products cell by cell (Section 1, Section 6.1); the GPU forms each
cell's local matrix on FP64 MFMA and adds it into the CSR values with atomics, so only
the order of additions differs: held normwise to 1e-12, with a variable coefficient
given at the Gauss points (the GPU's own points, the oracle evaluates the same function
at its points). With coefficient 1 the Gauss matrices are the right-hand sides of the
weight systems, which solve_weights computes row by row.
"""
import numpy as np
import pytest

import fixtures as fx
import oracle as O
from oracle import wq as OW

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _wq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_29334_amd.wq as W
    return W


def coef(x):
    return 1.0 + 0.5 * np.sin(2 * np.pi * x[..., 0]) * np.sin(2 * np.pi * x[..., 1])


def _case(F, want_lap):
    W = _wq()
    cls = OW.classify(F)
    cl = OW.cells(F, OW.points_per_element(F, cls))
    mesh = W.Mesh(F)
    pts = W.Points(mesh, want_laplacian=want_lap)
    G = W.Gauss(mesh, pts, want_laplacian=want_lap)
    return {"F": F, "cl": cl, "W": W, "mesh": mesh, "pts": pts, "G": G, "lap": want_lap}


@pytest.fixture(scope="module")
def hs():
    print("[gpu] gauss case half_strip", flush=True)
    return _case(fx.fixture_half_strip(), True)


@pytest.fixture(scope="module")
def eps():
    print("[gpu] gauss case eps32", flush=True)
    return _case(fx.fixture_eps(32, 0.02, (3, 5, 6), seed=5), False)


@pytest.fixture(scope="module")
def grid():
    print("[gpu] gauss case grid12", flush=True)
    return _case(fx.fixture_grid(12, displace=0.05, seed=3), True)


def _csr(c, vals):
    W = c["W"]
    row_ptr = c["pts"].get(W.ARR_ROW_PTR).cpu().numpy()
    col = c["pts"].get(W.ARR_COL).cpu().numpy()
    n = c["F"]["n_fn"]
    import scipy.sparse as sp
    return sp.csr_matrix((vals.cpu().numpy(), col, row_ptr), shape=(n, n))


def _rel(a, b):
    return float(abs(a - b).max() / abs(b).max())


@pytest.mark.parametrize("case", ["hs", "eps", "grid"])
def test_gauss_assembly_matches_oracle(case, request):
    c = request.getfixturevalue(case)
    W, G = c["W"], c["G"]
    x = G.x().reshape(-1, 2).cpu().numpy()
    cg = torch.tensor(coef(x), dtype=torch.float64, device="cuda")
    ref = O.gq_matrices(c["F"], c["cl"], coef=coef)
    kinds = [(W.GQ_MASS, ref["M"]), (W.GQ_STIFFNESS, ref["Kx"] + ref["Ky"])]
    if c["lap"]:
        kinds.append((W.GQ_BIHARMONIC, ref["B"]))
    for kind, R in kinds:
        got = _csr(c, G.assemble(kind, cg))
        err = _rel(got, R)
        print(f"[gpu] {case} gauss kind {kind}: normwise error {err:.2e}")
        assert err < 1e-12, (kind, err)
        # nothing outside the pattern: the oracle's matrix has no entry the CSR lacks
        assert abs(R).sum() <= abs(got).sum() * (1 + 1e-12) + 1e-300


@pytest.mark.parametrize("case", ["hs", "eps"])
def test_gauss_constant_coefficient_is_the_weight_rhs(case, request):
    """Coefficient 1: the element-wise matrices equal the right-hand sides of the weight
    systems (the same integrals summed row by row), to rounding."""
    c = request.getfixturevalue(case)
    W, G = c["W"], c["G"]
    wts = W.Weights(c["mesh"], c["pts"], W.WQ_FAM_MASS | W.WQ_FAM_DX | W.WQ_FAM_DY, tau=1e-12)
    M = G.assemble(W.GQ_MASS)
    K = G.assemble(W.GQ_STIFFNESS)
    bm = wts.rhs(W.WQ_FAM_MASS)
    bk = wts.rhs(W.WQ_FAM_DX) + wts.rhs(W.WQ_FAM_DY)
    assert float((M - bm).abs().max() / bm.abs().max()) < 1e-13
    assert float((K - bk).abs().max() / bk.abs().max()) < 1e-13


def test_gauss_points_and_rejections(hs):
    W, G = hs["W"], hs["G"]
    F = hs["F"]
    assert G.size == 16 * hs["pts"].info()["cells"]
    x = G.x().reshape(-1, 2).cpu().numpy()
    # the points lie in the control points' bounding box (the geometry is in their convex
    # hull) and every cell's 16 points are distinct
    ctrl = np.asarray(F["ctrl"]).reshape(-1, 2)
    assert np.all(x >= ctrl.min(axis=0) - 1e-12) and np.all(x <= ctrl.max(axis=0) + 1e-12)
    assert all(len(np.unique(x[16 * k:16 * k + 16].round(14), axis=0)) == 16 for k in range(len(x) // 16))
    # the biharmonic kind needs the Laplacians
    G2 = W.Gauss(hs["mesh"], hs["pts"], want_laplacian=False)
    with pytest.raises(W.WQError):
        G2.assemble(W.GQ_BIHARMONIC)
    with pytest.raises(W.WQError):
        G2.assemble(7)
