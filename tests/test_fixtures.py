"""Properties of the synthetic spline spaces (input generation, not the method).

The evaluator below is written independently of the oracle: it only expands the
Bernstein form of each cell.
"""
import numpy as np
import pytest

import fixtures as fx


def _bern(t):
    return np.array([(1 - t) ** 3, 3 * t * (1 - t) ** 2, 3 * t * t * (1 - t), t ** 3])


def _values(F, f, xi):
    lo, hi = F["ext_ptr"][f], F["ext_ptr"][f + 1]
    fn = F["ext_fn"][lo:hi]
    C = F["coef"][F["coef_ptr"][f]:F["coef_ptr"][f + 1]]
    if F["split"][f]:
        C = C.reshape(4, len(fn), 16)
        sx, sy = min(int(2 * xi[0]), 1), min(int(2 * xi[1]), 1)
        C = C[sx + 2 * sy]
        eta = (2 * xi[0] - sx, 2 * xi[1] - sy)
    else:
        C = C.reshape(len(fn), 16)
        eta = xi
    B = np.outer(_bern(eta[1]), _bern(eta[0])).reshape(16)
    return dict(zip(fn.tolist(), C @ B))


@pytest.fixture(scope="module")
def meshes():
    return {
        "grid": fx.fixture_grid(10),
        "half_strip": fx.fixture_half_strip(),
        "eps": fx.fixture_eps(48, 0.01, (3, 5, 6), seed=11),
    }


@pytest.mark.parametrize("name", ["grid", "half_strip", "eps"])
def test_partition_of_unity_and_nonnegative(meshes, name):
    F = meshes[name]
    assert F["coef"].min() >= 0.0
    nf = len(F["face_vtx"])
    for f in range(nf):
        m = F["ext_ptr"][f + 1] - F["ext_ptr"][f]
        if m == 0:
            continue
        C = F["coef"][F["coef_ptr"][f]:F["coef_ptr"][f + 1]].reshape(-1, m, 16)
        # Bernstein polynomials sum to one, so PU <=> coefficient columns sum to one
        assert np.abs(C.sum(axis=1) - 1.0).max() < 1e-14


@pytest.mark.parametrize("name", ["half_strip", "eps"])
def test_c0_across_edges(meshes, name):
    F = meshes[name]
    fv = F["face_vtx"]
    emap = {}
    for f in range(len(fv)):
        for k in range(4):
            emap[(fv[f][k], fv[f][(k + 1) % 4])] = (f, k)
    par = lambda k, t: [(t, 0.0), (1.0, t), (1.0 - t, 1.0), (0.0, 1.0 - t)][k]  # noqa: E731
    worst = 0.0
    for (a, b), (f, k) in emap.items():
        if (b, a) not in emap:
            continue
        g, kg = emap[(b, a)]
        if F["ext_ptr"][f + 1] == F["ext_ptr"][f] or F["ext_ptr"][g + 1] == F["ext_ptr"][g]:
            continue
        for t in (0.21, 0.5, 0.83):
            v1, v2 = _values(F, f, par(k, t)), _values(F, g, par(kg, 1.0 - t))
            for key in set(v1) | set(v2):
                worst = max(worst, abs(v1.get(key, 0.0) - v2.get(key, 0.0)))
    assert worst < 1e-14


def test_c1_on_regular_grid(meshes):
    """EP-free B-splines are C1: the parametric derivative across a shared edge agrees."""
    F = meshes["grid"]
    N = 10
    h = 1e-6
    worst = 0.0
    for j in range(2, N - 3):
        for i in range(2, N - 3):
            f, g = i + N * j, i + 1 + N * j  # g is the right neighbour of f
            for t in (0.3, 0.7):
                a = _values(F, f, (1.0, t))
                am = _values(F, f, (1.0 - h, t))
                b = _values(F, g, (0.0, t))
                bp = _values(F, g, (h, t))
                for key in a:
                    d1 = (a[key] - am.get(key, 0.0)) / h
                    d2 = (bp.get(key, 0.0) - b.get(key, 0.0)) / h
                    worst = max(worst, abs(d1 - d2))
    assert worst < 1e-4


@pytest.mark.parametrize("name", ["half_strip", "eps"])
def test_linear_independence(meshes, name):
    F = meshes[name]
    rows, cols, vals = [], [], []
    r0 = 0
    for f in range(len(F["face_vtx"])):
        m = F["ext_ptr"][f + 1] - F["ext_ptr"][f]
        if m == 0:
            continue
        fn = F["ext_fn"][F["ext_ptr"][f]:F["ext_ptr"][f + 1]]
        C = F["coef"][F["coef_ptr"][f]:F["coef_ptr"][f + 1]].reshape(-1, m, 16)
        for s in range(C.shape[0]):
            for j in range(m):
                nz = np.nonzero(C[s, j])[0]
                rows.extend((r0 + nz).tolist())
                cols.extend([int(fn[j])] * len(nz))
                vals.extend(C[s, j, nz].tolist())
            r0 += 16
    A = np.zeros((r0, F["n_fn"]))
    A[rows, cols] = vals
    sv = np.linalg.svd(A, compute_uv=False)
    assert sv[-1] / sv[0] > 1e-3


def test_function_counts_per_element(meshes):
    """Irregular faces carry 3 mu + 12 functions (ASUTS Table 1: 3 mu + 13; stated
    deviation), transition faces 16 or 18, all others 16."""
    F = meshes["eps"]
    import oracle  # topology only
    bnd, val, _ = oracle.topology(F["face_vtx"], F["nv"])
    m = np.diff(F["ext_ptr"])
    for f, fv in enumerate(F["face_vtx"]):
        if m[f] == 0:
            assert any(bnd[v] for v in fv)
            continue
        mus = [val[v] for v in fv if (not bnd[v]) and val[v] != 4]
        if mus:
            assert F["split"][f] == 1
            assert m[f] == 3 * mus[0] + 12
        else:
            assert F["split"][f] == 0
            assert m[f] in (16, 18)


def test_ep_valences():
    m, _ = fx.half_strip_mesh()
    vals = sorted(int(m.valence[v]) for v in m.eps())
    assert vals == [3, 5]
    m2, _ = fx.ep_mesh(64, 0.01, (3, 5), seed=3)
    v2 = [int(m2.valence[v]) for v in m2.eps()]
    assert set(v2) <= {3, 5} and v2.count(3) == v2.count(5)
    m3, _ = fx.ep_mesh(64, 0.02, (3, 5, 6), seed=4)
    v3 = [int(m3.valence[v]) for v in m3.eps()]
    # quad-mesh Euler balance on a disk with a regular boundary: #3 = #5 + 2 #6
    assert v3.count(3) == v3.count(5) + 2 * v3.count(6)


def test_domain_is_unit_square(meshes):
    """Boundary control points lie on the sides of [0,1]^2 (open knot vectors)."""
    F = meshes["eps"]
    import oracle
    bnd, _, _ = oracle.topology(F["face_vtx"], F["nv"])
    P = F["vtx_pos"][bnd]
    on_side = np.minimum.reduce([np.abs(P[:, 0]), np.abs(P[:, 1]), np.abs(P[:, 0] - 1), np.abs(P[:, 1] - 1)])
    assert on_side.max() < 1e-14
