"""Pins of the oracle's surface geometry (Section 4.1, Eqs. (13)-(17) on 2-manifolds),
checked against what the mathematics fixes rather than against its own formulas:

* a plane placed in 3-D by a rotation is the planar problem: values, area element and
  Laplace-Beltrami operator unchanged, the surface gradient the rotated planar gradient,
  and the Gauss and WQ matrices (with the third gradient family) equal the planar ones;
* on a curved surface the surface gradient is tangent and reproduces the parametric
  derivatives along the tangent vectors (taken here by central differences of the
  oracle's own x(eta) and N(eta)), and the Laplace-Beltrami operator satisfies Green's
  identity, int N_i Delta_s N_j + int grad_s N_i . grad_s N_j = 0 for a function N_i that
  vanishes on the boundary, integrated with a 10-point Gauss rule per direction.
"""
import numpy as np
import pytest

import fixtures as fx
import oracle as O
from oracle import wq as OW


@pytest.fixture(scope="module")
def plane():
    F = fx.fixture_grid(6, displace=0.05, seed=7)
    return F, fx.rotate_to_3d(F)


def _cells(F):
    cls = OW.classify(F)
    return OW.cells(F, OW.points_per_element(F, cls))


def test_rotated_plane_pointwise(plane):
    F, G = plane
    Rot = G["rotation"]
    cl = _cells(F)
    rng = np.random.default_rng(3)
    for c in rng.choice(len(cl["elem"]), min(12, len(cl["elem"])), replace=False):
        f, k = int(cl["elem"][c]), int(cl["sub"][c])
        eta = tuple(rng.uniform(0.05, 0.95, 2))
        fn, N, Nx, Ny, Lap, x, dJ = OW.eval_cell(F, f, k, eta)
        sfn, sN, sx, sy, sLB, sxx, sg, sz = OW.eval_cell(G, f, k, eta)
        assert np.array_equal(fn, sfn)
        assert np.allclose(sN, N, rtol=0, atol=1e-14)
        grad3 = Rot @ np.vstack([Nx, Ny, np.zeros_like(Nx)])
        scale = np.abs(grad3).max()
        assert np.abs(np.vstack([sx, sy, sz]) - grad3).max() <= 1e-12 * scale
        assert np.abs(sLB - Lap).max() <= 1e-11 * np.abs(Lap).max()
        assert abs(sg - abs(dJ)) <= 1e-13 * abs(dJ)
        assert np.allclose(sxx, Rot @ np.append(x, 0.0), rtol=0, atol=1e-14)


def test_rotated_plane_matrices(plane):
    """Gauss matrices, and WQ stiffness with three gradient families, equal the planar
    ones: stiffness is invariant under rotation, and both WQ stiffnesses reproduce the
    Gauss one to the exactness residual."""
    F, G = plane
    RF = O.setup(F, families=("mass", "x", "y", "lap"))
    RG = O.setup(G, families=("mass", "x", "y", "z", "lap"))
    gf, gg = RF["gq"], RG["gq"]
    Kf = gf["Kx"] + gf["Ky"]
    Kg = gg["Kx"] + gg["Ky"] + gg["Kz"]
    assert abs(gg["M"] - gf["M"]).max() <= 1e-14 * abs(gf["M"]).max()
    assert abs(Kg - Kf).max() <= 1e-13 * abs(Kf).max()
    assert abs(gg["B"] - gf["B"]).max() <= 1e-11 * abs(gf["B"]).max()
    n = F["n_fn"]
    for kind in ("mass", "stiffness", "biharmonic"):
        a = OW.csr(RF["pat"], OW.wq_assemble(F, RF["pat"], RF["data"], RF["W"], kind), n)
        b = OW.csr(RG["pat"], OW.wq_assemble(G, RG["pat"], RG["data"], RG["W"], kind), n)
        assert abs(a - b).max() <= 1e-10 * abs(a).max(), kind


def _fd(fun, eta, h=1e-6):
    e = np.array(eta)
    d1 = (fun((e[0] + h, e[1])) - fun((e[0] - h, e[1]))) / (2 * h)
    d2 = (fun((e[0], e[1] + h)) - fun((e[0], e[1] - h))) / (2 * h)
    return d1, d2


def test_curved_surface_gradient_is_tangent():
    G = fx.fixture_dome(fx.fixture_half_strip(), radius=1.5)
    cl = _cells(G)
    rng = np.random.default_rng(5)
    for c in rng.choice(len(cl["elem"]), 10, replace=False):
        f, k = int(cl["elem"][c]), int(cl["sub"][c])
        eta = tuple(rng.uniform(0.1, 0.9, 2))
        fn, N, gx, gy, LB, x, sg, gz = OW.eval_cell(G, f, k, eta)
        grad = np.vstack([gx, gy, gz])
        a1, a2 = _fd(lambda e: OW.eval_cell(G, f, k, e)[5], eta)
        dN1, dN2 = _fd(lambda e: OW.eval_cell(G, f, k, e)[1], eta)
        nrm = np.cross(a1, a2)
        assert abs(np.linalg.norm(nrm) - sg) <= 1e-7 * sg
        nrm /= np.linalg.norm(nrm)
        s = np.abs(grad).max()
        assert np.abs(nrm @ grad).max() <= 1e-7 * s  # the normal is a central difference
        assert np.abs(a1 @ grad - dN1).max() <= 1e-7 * max(np.abs(dN1).max(), 1.0)
        assert np.abs(a2 @ grad - dN2).max() <= 1e-7 * max(np.abs(dN2).max(), 1.0)


def test_curved_surface_laplace_beltrami_green_identity():
    G = fx.fixture_dome(fx.fixture_half_strip(), radius=1.5)
    cl = _cells(G)
    gp, gw = np.polynomial.legendre.leggauss(10)
    gp, gw = 0.5 * (gp + 1), 0.5 * gw
    supp = OW.supports(G, cl)
    n = G["n_fn"]
    boundary = np.asarray(G["dir1"], dtype=bool)
    # an interior function away from the boundary, and a few trial functions around it
    interior = [i for i in range(n) if not boundary[i] and len(supp[i]) >= 9]
    i = interior[len(interior) // 2]
    lhs = {}
    for c in supp[i]:
        f, k = int(cl["elem"][c]), int(cl["sub"][c])
        for a in range(10):
            for b in range(10):
                fn, N, gx, gy, LB, x, sg, gz = OW.eval_cell(G, f, k, (gp[a], gp[b]))
                w = gw[a] * gw[b] * sg
                li = int(np.nonzero(fn == i)[0][0])
                for lj, j in enumerate(fn):
                    v = w * (N[li] * LB[lj] + gx[li] * gx[lj] + gy[li] * gy[lj] + gz[li] * gz[lj])
                    s = w * (abs(N[li] * LB[lj]) + abs(gx[li] * gx[lj] + gy[li] * gy[lj] + gz[li] * gz[lj]))
                    acc = lhs.setdefault(int(j), [0.0, 0.0])
                    acc[0] += v
                    acc[1] += s
    worst = max(abs(v) / s for v, s in lhs.values())
    assert worst <= 1e-9, worst
