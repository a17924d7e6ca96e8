"""The entry point that allocates nothing (assemble_tangent_noalloc) against
assemble_tangent: same kernels, so the tangent S and the residual R must be identical bit
for bit. Two calls in a row through the no-allocation entry point, the second on a
smaller mesh, so the second reuses the fixed per-GPU array the first one filled."""
import numpy as np
import pytest

import fixtures as fx

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _setup(F):
    import paper_2605_29334_amd.wq as W
    mesh = W.Mesh(F)
    pts = W.Points(mesh)
    wts = W.Weights(mesh, pts, W.WQ_FAM_MASS | W.WQ_FAM_DX | W.WQ_FAM_DY, tau=1e-12)
    return W, mesh, pts, wts


def _fields(pts, seed):
    g = np.random.default_rng(seed)
    T = torch.tensor(g.uniform(-1.0, 1.0, pts.n_rows), dtype=torch.float64, device="cuda")
    Td = torch.tensor(g.uniform(-1.0, 1.0, pts.n_rows), dtype=torch.float64, device="cuda")
    f = torch.tensor(g.uniform(-1.0, 1.0, pts.n_points), dtype=torch.float64, device="cuda")
    return T, Td, f


def test_noalloc_tangent_matches_assemble_tangent_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    cases = [(fx.fixture_half_strip(), 31), (fx.fixture_grid(8, displace=0.05, seed=7), 32)]
    assert cases[1][0]["n_fn"] < cases[0][0]["n_fn"]
    for F, seed in cases:
        print(f"[gpu] noalloc tangent case n_fn={F['n_fn']} seed={seed}", flush=True)
        W, mesh, pts, wts = _setup(F)
        T, Td, f = _fields(pts, seed)
        k = (W.K_QUADRATIC, 1.0, 1.0)
        S_ref, R_ref = W.assemble_tangent(pts, wts, T, Td, 10.0, k=k, f=f)
        S = torch.full((pts.nnz,), np.nan, dtype=torch.float64, device="cuda")
        R = torch.full((pts.n_rows,), np.nan, dtype=torch.float64, device="cuda")
        W.assemble_tangent_noalloc(pts, wts, T, Td, 10.0, k=k, f=f, S_out=S, R_out=R)
        torch.cuda.synchronize()
        assert torch.equal(S, S_ref)
        assert torch.equal(R, R_ref)
        del wts, pts, mesh
