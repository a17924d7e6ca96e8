"""Batched meshes (wq_batch_*), the assembly HIP graph and the assembly autotuner.

* Every mesh of a batch gets exactly what it gets alone: the same classification,
  pattern, point sets (shifted by its offsets), weights and matrix values, bit for bit
  (the method is local to each function's support and the kernels sum in fixed orders).
* The captured graph reproduces the eager assembly on every replay, with eager work and
  coefficient updates between the replays.
* The autotuner's choice only reorders the schedule of tiles: values are unchanged.
* Two meshes of the batch (the half strip and the 2 % EP mesh) against the oracle: the
  mass matrix with a variable coefficient end to end (oracle weights) at 1e-12, and the
  stiffness contraction with the batch's own weights at 1e-12.
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


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def batch():
    W = _wq()
    print("[gpu] batch of 5 meshes", flush=True)
    pool = [fx.fixture_grid(8, displace=0.05, seed=11), fx.fixture_half_strip(),
            fx.fixture_eps(32, 0.02, (3, 5, 6), seed=5), fx.fixture_grid(12, displace=0.05, seed=3),
            fx.fixture_grid(10, displace=0.05, seed=7)]
    B = W.Batch(pool).build(1 | 2 | 4)
    return W, pool, B


def _coef(x, shift):
    c = 1 + 0.5 * torch.sin(2 * np.pi * x[:, 0] + shift) * torch.sin(2 * np.pi * x[:, 1])
    k = 1 + 0.5 * torch.cos(np.pi * x[:, 0]) * torch.cos(np.pi * x[:, 1] + shift)
    return c.contiguous(), k.contiguous()


def test_each_mesh_equals_its_own_run(batch):
    W, pool, B = batch
    P, Wt = B.points, B.weights
    x = P.get(W.ARR_X).reshape(-1, 2)
    c, k = _coef(x, 0.3)
    Mb, Kb = W.assemble_mass_stiffness(P, Wt, c, k)
    rp, col = _np(P.get(W.ARR_ROW_PTR)), _np(P.get(W.ARR_COL))
    qp, qi = _np(P.get(W.ARR_QPTR)), _np(P.get(W.ARR_QIDX))
    wb = {f: _np(Wt.weights(f)) for f in (1, 2, 4)}
    for m, F in enumerate(pool):
        o = B.info(m)
        mesh = W.Mesh(F)
        pts = W.Points(mesh)
        wts = W.Weights(mesh, pts, 1 | 2 | 4)
        assert pts.n_rows == o["n_rows"] and pts.nnz == o["nnz"] and pts.n_points == o["n_points"]
        r0, z0, p0 = o["row0"], o["nnz0"], o["pt0"]
        rows = slice(r0, r0 + o["n_rows"] + 1)
        np.testing.assert_array_equal(_np(pts.get(W.ARR_ROW_PTR)), rp[rows] - z0)
        np.testing.assert_array_equal(_np(pts.get(W.ARR_COL)), col[z0:z0 + o["nnz"]] - r0)
        q0 = qp[r0]
        np.testing.assert_array_equal(_np(pts.get(W.ARR_QPTR)), qp[rows] - q0)
        np.testing.assert_array_equal(_np(pts.get(W.ARR_QIDX)), qi[q0:qp[r0 + o["n_rows"]]] - p0)
        for f in (1, 2, 4):
            assert np.array_equal(_np(wts.weights(f)), wb[f][q0:qp[r0 + o["n_rows"]]]), (m, f)
        cs, ks = c[p0:p0 + o["n_points"]].contiguous(), k[p0:p0 + o["n_points"]].contiguous()
        M, K = W.assemble_mass_stiffness(pts, wts, cs, ks)
        assert np.array_equal(_np(M), _np(Mb)[z0:z0 + o["nnz"]]), m
        assert np.array_equal(_np(K), _np(Kb)[z0:z0 + o["nnz"]]), m
    print(f"[gpu] batch: {B.n_meshes} meshes, {P.n_rows} rows, {P.nnz} nnz, report {B.report}")


def test_graph_replays_match_eager(batch):
    W, pool, B = batch
    P, Wt = B.points, B.weights
    x = P.get(W.ARR_X).reshape(-1, 2)
    c, k = _coef(x, 0.0)
    Mg = torch.empty(P.nnz, dtype=torch.float64, device="cuda")
    Kg = torch.empty_like(Mg)
    s = torch.cuda.Stream()  # capture needs a created stream
    torch.cuda.synchronize()
    for rep in range(4):
        c2, k2 = _coef(x, 0.1 * rep)
        c.copy_(c2)
        k.copy_(k2)
        torch.cuda.synchronize()
        B.graph_assemble(c, k, Mg, Kg, stream=s)
        s.synchronize()
        Me, Ke = W.assemble_mass_stiffness(P, Wt, c, k)
        torch.cuda.synchronize()
        assert torch.equal(Mg, Me) and torch.equal(Kg, Ke), rep


def test_autotune_changes_schedule_not_values(batch):
    W, pool, B = batch
    P, Wt = B.points, B.weights
    M0, K0 = W.assemble_mass_stiffness(P, Wt)
    chunk, ms = W.autotune_assembly(P, Wt)
    print(f"[gpu] autotune: chunk {chunk}, {ms:.4f} ms")
    band = -(-P.info()["tiles"] // 8)
    assert (chunk in (4, 8, 16, 32, 64, 128, 256, 512, 1024) and chunk < band or chunk == band) and ms > 0
    M1, K1 = W.assemble_mass_stiffness(P, Wt)
    assert torch.equal(M0, M1) and torch.equal(K0, K1)


def test_autotune_tiles_changes_schedule_not_values(batch):
    """The tile-shape autotuner rebuilds the cell-major tiles: values are unchanged, eager
    and through the batch's captured graph (captured again after the rebuild)."""
    W, pool, B = batch
    P, Wt = B.points, B.weights
    x = P.get(W.ARR_X).reshape(-1, 2)
    c, k = _coef(x, 0.3)
    M0, K0 = W.assemble_mass_stiffness(P, Wt, c, k)
    s = torch.cuda.Stream()
    Mg, Kg = torch.empty_like(M0), torch.empty_like(K0)
    torch.cuda.synchronize()
    B.graph_assemble(c, k, Mg, Kg, stream=s)
    s.synchronize()
    assert torch.equal(Mg, M0) and torch.equal(Kg, K0)
    tiles0 = P.info()["tiles"]
    cap, chunk, ms = W.autotune_tiles(P, Wt)
    tiles1 = P.info()["tiles"]
    print(f"[gpu] autotune tiles: step cap {cap}, chunk {chunk}, {ms:.4f} ms; tiles {tiles0} -> {tiles1}")
    band = -(-tiles1 // 8)
    assert cap in (64, 96, 128, 192, 256, 1 << 30) and ms > 0
    assert chunk in (4, 8, 16, 32, 64, 128, 256, 512, 1024) and chunk < band or chunk == band
    M1, K1 = W.assemble_mass_stiffness(P, Wt, c, k)
    torch.cuda.synchronize()
    assert torch.equal(M0, M1) and torch.equal(K0, K1)
    Mg.zero_()
    Kg.zero_()
    torch.cuda.synchronize()
    for rep in range(3):
        B.graph_assemble(c, k, Mg, Kg, stream=s)
        s.synchronize()
        assert torch.equal(Mg, M0) and torch.equal(Kg, K0), rep


def test_batch_meshes_against_oracle(batch):
    W, pool, B = batch
    P, Wt = B.points, B.weights
    x = P.get(W.ARR_X).reshape(-1, 2)
    c, k = _coef(x, 0.2)
    Mb, Kb = W.assemble_mass_stiffness(P, Wt, c, k)
    Mb, Kb = _np(Mb), _np(Kb)
    wb = {f: _np(Wt.weights(b)) for f, b in (("mass", 1), ("x", 2), ("y", 4))}
    qp = _np(P.get(W.ARR_QPTR))
    for m in (1, 2):
        F = pool[m]
        o = B.info(m)
        r0, z0, p0, n = o["row0"], o["nnz0"], o["pt0"], o["n_rows"]
        print(f"[gpu] batch mesh {m} against the oracle ({n} rows)", flush=True)
        R = O.setup(F, families=("mass", "x", "y"))
        pat, data = R["pat"], R["data"]
        cs = _np(c[p0:p0 + o["n_points"]])
        ks = _np(k[p0:p0 + o["n_points"]])
        Mref = O.wq_assemble(F, pat, data, R["W"], "mass", cs)
        q0, q1 = qp[r0], qp[r0 + n]
        Wm = {f: v[q0:q1] for f, v in wb.items()}
        Kref = O.wq_assemble(F, pat, data, Wm, "stiffness", ks)
        em = float(np.abs(Mb[z0:z0 + o["nnz"]] - Mref).max() / np.abs(Mref).max())
        ek = float(np.abs(Kb[z0:z0 + o["nnz"]] - Kref).max() / np.abs(Kref).max())
        print(f"[gpu] batch mesh {m}: mass (oracle weights) rel err {em:.2e}, "
              f"stiffness (batch weights) rel err {ek:.2e}", flush=True)
        assert em < 1e-12 and ek < 1e-12


def test_side_streams_change_schedule_not_values(batch):
    """The size buckets' launches on 1, 4 or 8 side streams (wq_set_side_streams): the
    weights of the whole batch and its solve report are bit-identical (each system is
    solved by one workgroup; the reports are atomic minima, maxima and counts)."""
    W, pool, _ = batch
    got = {}
    try:
        for ns in (1, 4, 8):
            W.set_side_streams(ns)
            B = W.Batch(pool).build(1 | 2 | 4)
            got[ns] = ({f: _np(B.weights.weights(f)) for f in (1, 2, 4)}, dict(B.report))
            B.close()
        with pytest.raises(W.WQError):
            W.set_side_streams(0)
        with pytest.raises(W.WQError):
            W.set_side_streams(9)
    finally:
        W.set_side_streams(4)
    for ns in (4, 8):
        for f in (1, 2, 4):
            assert np.array_equal(got[ns][0][f], got[1][0][f]), (ns, f)
        assert got[ns][1] == got[1][1], ns
