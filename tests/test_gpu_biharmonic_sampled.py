"""Biharmonic assembly on a mesh shaped like the biharmonic workload: 128 x 128 faces, 0.5%
EPs of valence 3 and 5, seeded smooth displacement (seed 3000). The workload itself is
512 x 512 faces; its fixture and the oracle's whole-mesh setup take minutes on the host,
so this test uses the same recipe at 128 x 128 faces and checks sampled rows one by one:

* CSR columns S_i and point sets Q_i: bit-exact.
* Laplacian weights: the exactness residual in the oracle's system, bounded per row by
  the dropped part of b plus rounding amplified by sigma_1 / sigma_t.
* FP64 biharmonic rows with a variable coefficient: 1e-12 + 8 eps (sigma_1 / sigma_t)
  kappa(Z V_t) relative to the row.
* The low-precision contractions, per matrix against the FP64 rows of the oracle: the
  sliced form within 1e-6; the two-term forms within max(1e-6, 8 * 2^-24 * C), with C
  the cancellation factor of the sampled rows (sum of |terms| over the largest |entry|).
Rows are drawn at random and from the largest systems (next to extraordinary points).
"""
import numpy as np
import pytest

import fixtures as fx
import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _np(t):
    return t.detach().cpu().numpy()


def _coef(p):
    return 1 + 0.5 * np.cos(np.pi * p[:, 0]) * np.cos(np.pi * p[:, 1])


def test_biharmonic_sampled_rows():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_29334_amd.wq as W
    print("[gpu] biharmonic fixture 128x128, 0.5% EPs (3, 5)", flush=True)
    F = fx.fixture_eps(128, 0.005, (3, 5), displace=0.05, seed=3000)
    mesh = W.Mesh(F)
    pts = W.Points(mesh, want_laplacian=True)
    wts = W.Weights(mesh, pts, 8, tau=1e-12)
    x = pts.get(W.ARR_X).reshape(-1, 2)
    d = (1 + 0.5 * torch.cos(np.pi * x[:, 0]) * torch.cos(np.pi * x[:, 1])).contiguous()
    Bg = {0: _np(W.assemble_biharmonic(pts, wts, d))}
    for prec in (1, 2, 3):
        Bg[prec] = _np(W.assemble_biharmonic(pts, wts, d, prec=prec)).astype(np.float64)
    rp, col = _np(pts.get(W.ARR_ROW_PTR)), _np(pts.get(W.ARR_COL))
    qp, qi = _np(pts.get(W.ARR_QPTR)), _np(pts.get(W.ARR_QIDX))
    wl = _np(wts.weights(8))
    n = F["n_fn"]
    rng = np.random.default_rng(3000)
    sizes = np.diff(rp)
    rows = sorted(set(rng.choice(n, 12, replace=False).tolist()) | set(np.argsort(sizes)[-12:].tolist()))
    print(f"[gpu] oracle on {len(rows)} sampled rows (n_i up to {sizes[rows].max()})", flush=True)
    res, _ = O.sample_rows(F, rows, ("lap",), 1e-12)
    eps = np.finfo(np.float64).eps
    worst_w, worst_b = 0.0, 0.0
    err = {1: 0.0, 2: 0.0, 3: 0.0}
    bmax, tmax = 0.0, 0.0
    for i in rows:
        o = res[i]
        np.testing.assert_array_equal(col[rp[i]:rp[i + 1]], o["S"])
        np.testing.assert_array_equal(qi[qp[i]:qp[i + 1]], o["Q"])
        A, b, z = o["A_lap"], o["b_lap"], o["z"]
        w = wl[qp[i]:qp[i + 1]]
        _, sg, Vt = np.linalg.svd(A, full_matrices=False)
        t = int(np.sum(sg > 1e-12 * sg[0]))
        U = np.linalg.svd(A, full_matrices=False)[0][:, :t]
        dropped = np.linalg.norm(b - U @ (U.T @ b))
        bound = 8 * eps * (sg[0] / sg[t - 1] * np.linalg.norm(b) + sg[0] * np.linalg.norm(w)) + 2 * dropped \
            + 1e-13 * np.abs(b).max()  # GPU and oracle Gauss right-hand sides agree to 1e-13
        worst_w = max(worst_w, np.abs(A @ w - b).max() / bound)
        kap = sg[0] / sg[t - 1] * np.linalg.cond(z[:, None] * Vt[:t].T)
        dq = _coef(o["x"])
        ref = A @ (dq * o["W"]["lap"])
        got = Bg[0][rp[i]:rp[i + 1]]
        worst_b = max(worst_b, np.abs(got - ref).max() / np.abs(ref).max() / (1e-12 + 8 * eps * kap))
        bmax = max(bmax, np.abs(ref).max())
        tmax = max(tmax, (np.abs(A) @ np.abs(dq * o["W"]["lap"])).max())
        for prec in (1, 2, 3):
            err[prec] = max(err[prec], np.abs(Bg[prec][rp[i]:rp[i + 1]] - ref).max())
    canc = tmax / bmax
    rel = {p: e / bmax for p, e in err.items()}
    print(f"[gpu] biharmonic: weights residual/bound {worst_w:.2f}, FP64 rows err/bound {worst_b:.2f}; "
          f"low precision rel err fp16x2 {rel[1]:.2e}, bf16x3 {rel[2]:.2e}, sliced {rel[3]:.2e} "
          f"(cancellation factor {canc:.0f})", flush=True)
    assert worst_w <= 1.0
    assert worst_b <= 1.0
    assert rel[3] <= 1e-6
    for p in (1, 2):
        assert rel[p] <= max(1e-6, 8 * 2.0 ** -24 * canc), (p, rel[p])
