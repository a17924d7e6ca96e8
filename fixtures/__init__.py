"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package generates control meshes and their Bezier extraction operators, i.e. the
*input* of the weighted-quadrature path. It contains none of the method's arithmetic
(no quadrature points, no weights, no classification, no assembly).

A fixture is a dict of NumPy arrays:
  nv                   number of control-mesh vertices
  face_vtx  (nf,4)     int32, counter-clockwise vertex ids per face (row-major order)
  n_fn                 number of basis functions
  ctrl      (n_fn,2)   float64 control points (the geometry map is x = sum_j ctrl_j N_j)
  split     (nf,)      uint8, 1 if the face is split 2x2 into Bezier sub-elements
  ext_ptr   (nf+1,)    int64 offsets into ext_fn
  ext_fn    (...)      int32 global ids of the functions living on each face (ascending)
  coef_ptr  (nf+1,)    int64 offsets (in doubles) into coef
  coef      (...)      float64, per face nsub x m x 16 Bernstein coefficients, index k+4l
                       (k along corner0->corner1, l along corner0->corner3); nsub = 4 for
                       split faces, sub-element s = sx + 2 sy covers [sx/2,(sx+1)/2] x ...
  fn_vertex (n_fn,)    int32 vertex of a vertex function, -1 for face functions
  dir1      (n_fn,)    uint8, function does not vanish on the boundary (Poisson Dirichlet)
  dir2      (n_fn,)    uint8, outer two function layers (clamped biharmonic)
Passive faces (touching the boundary) have no functions (zero parametric area).
"""
from __future__ import annotations

import numpy as np

from . import quadmesh as qm
from .basis import Extraction


def greville_1d(N):
    """Greville abscissae on [0,1] of the open cubic knot vector of an N-face row."""
    u = np.zeros(N + 3)
    for k in range(-1, N + 2):
        if k <= 1:
            val = 0.0
        elif k >= N - 1:
            val = N - 2.0
        else:
            val = k - 1.0
        u[k + 1] = val
    g = np.array([(u[j] + u[j + 1] + u[j + 2]) / 3.0 for j in range(N + 1)])
    return g / (N - 2.0)


def _grid_mesh(N):
    mesh = qm.grid(N)
    g = greville_1d(N)
    P = np.zeros((mesh.nv, 2))
    for j in range(N + 1):
        for i in range(N + 1):
            P[i + (N + 1) * j] = (g[i], g[j])
    return mesh.build(), P


def _finish(mesh, splits, base_pos):
    pos = base_pos
    for _ in range(splits):
        mesh, pos = qm.split_polygons(mesh, pos)
    used = sorted({v for fv in mesh.faces for v in fv})
    remap = {v: i for i, v in enumerate(used)}
    mesh = qm.QuadMesh([[remap[v] for v in fv] for fv in mesh.faces], len(used))
    pos = pos[used]
    mesh.build()
    P = qm.tutte_embed(mesh, guess=pos)
    mesh, P = qm.renumber_spatial(mesh, P)
    mesh.build()
    return mesh, P


def half_strip_mesh(M=4, a=1, b=2, splits=3):
    """One valence-5 and one valence-3 EP (a dislocation reaching the top boundary)."""
    mesh = qm.edit_half_strip(M, a, b)
    base = np.array([[i, j] for j in range(M + 1) for i in range(M + 1)], dtype=float) / M
    return _finish(mesh, splits, base)


def ep_mesh(N, density, valences, seed, splits=2):
    """N x N faces (N divisible by 2**splits) with seeded EPs of the given valences.

    EPs come in clusters from local edits on the coarse grid (rotation: 3,3,5,5;
    collapse: 6,3,3), which the uniform splits separate by 2**splits edges.
    """
    rng = np.random.default_rng(seed)
    f = 2 ** splits
    if N % f:
        raise ValueError("N must be divisible by 2**splits")
    M = N // f
    mesh = qm.grid(M)
    n_int = (N - 1) ** 2
    target = density * n_int
    use6 = 6 in valences
    # slots on a jittered lattice of pitch 4 base cells, margin 2 (EPs at base depth >= 2)
    pitch = 4
    slots = [(i, j) for j in range(2, M - 3, pitch) for i in range(2, M - 3, pitch)]
    rng.shuffle(slots)
    ops = []
    count = 0
    for (i, j) in slots:
        if count >= target:
            break
        kind = 'c' if (use6 and rng.uniform() < 0.35) else 'r'
        ops.append((kind, i, j, int(rng.integers(0, 2))))
        count += 3 if kind == 'c' else 4
    removed = []
    for kind, i, j, o in ops:
        if kind == 'r':
            if o == 0:
                mesh_f, mesh_g = qm._face_at(M, i, j), qm._face_at(M, i + 1, j)
            else:
                mesh_f, mesh_g = qm._face_at(M, i, j), qm._face_at(M, i, j + 1)
            qm.edit_rotate(mesh, mesh_f, mesh_g)
        else:
            removed.append((qm._face_at(M, i, j), o))
    # collapses last, highest face index first so indices stay valid
    for fidx, o in sorted(removed, reverse=True):
        if o == 1:
            fv = mesh.faces[fidx]
            mesh.faces[fidx] = fv[1:] + fv[:1]
        qm.edit_collapse(mesh, fidx)
    base = np.array([[i, j] for j in range(M + 1) for i in range(M + 1)], dtype=float) / M
    return _finish(mesh, splits, base)


def build_fixture(mesh, P, displace=0.0, seed=0):
    """Extraction operators + control points for a built mesh."""
    if displace > 0:
        P = qm.smooth_displacement(P, np.random.default_rng(seed), displace)
    ex = Extraction(mesh).build()
    nf = len(mesh.faces)
    ext_ptr = np.zeros(nf + 1, dtype=np.int64)
    coef_ptr = np.zeros(nf + 1, dtype=np.int64)
    for f in range(nf):
        ext_ptr[f + 1] = ext_ptr[f] + len(ex.face_fns[f])
        coef_ptr[f + 1] = coef_ptr[f] + ex.face_coef[f].size
    ext_fn = np.concatenate([a for a in ex.face_fns]).astype(np.int32) if nf else np.zeros(0, np.int32)
    coef = np.concatenate([c.reshape(-1) for c in ex.face_coef]) if nf else np.zeros(0)
    n_fn = ex.n_fn
    ctrl = np.zeros((n_fn, 2))
    fn_vertex = -np.ones(n_fn, dtype=np.int32)
    for v in range(mesh.nv):
        if ex.vertex_fn[v] >= 0:
            ctrl[ex.vertex_fn[v]] = P[v]
            fn_vertex[ex.vertex_fn[v]] = v
    for (fc, c), gid in ex.face_fn.items():
        e = [v for v in mesh.faces[fc] if ex.is_ep[v]][0]
        ctrl[gid] = P[e]
    depth_fn = np.zeros(n_fn, dtype=np.int64)
    for gid in range(n_fn):
        v = fn_vertex[gid]
        depth_fn[gid] = mesh.depth[v] if v >= 0 else 99
    return {
        "nv": int(mesh.nv),
        "face_vtx": np.array(mesh.faces, dtype=np.int32).reshape(nf, 4),
        "n_fn": int(n_fn),
        "ctrl": ctrl,
        "split": ex.face_split.astype(np.uint8),
        "ext_ptr": ext_ptr,
        "ext_fn": ext_fn,
        "coef_ptr": coef_ptr,
        "coef": coef,
        "fn_vertex": fn_vertex,
        "dir1": (depth_fn == 0).astype(np.uint8),
        "dir2": (depth_fn <= 1).astype(np.uint8),
        "vtx_pos": P,
    }


def fixture_grid(N, displace=0.0, seed=0):
    """EP-free N x N control faces; identity geometry (Greville control points)."""
    mesh, P = _grid_mesh(N)
    return build_fixture(mesh, P, displace, seed)


def fixture_half_strip(displace=0.05, seed=1000, M=4, a=1, b=2, splits=3):
    """Small two-EP mesh (valences 5 and 3), the oracle-sized case."""
    mesh, P = half_strip_mesh(M, a, b, splits)
    return build_fixture(mesh, P, displace, seed)


def fixture_eps(N, density=0.01, valences=(3, 5, 6), displace=0.05, seed=2000):
    """N x N faces with seeded EPs (density = fraction of interior vertices)."""
    mesh, P = ep_mesh(N, density, valences, seed)
    return build_fixture(mesh, P, displace, seed)


# ---------------------------------------------------------------- surfaces (2-manifolds in 3-D)
# The spline space is the planar one; only the control points gain a third coordinate, so
# the surface is x(eta) = sum_j ctrl_j N_j in R^3 (Section 4.1 treats such surfaces).

def rotate_to_3d(F, angles=(0.3, -0.5, 0.7)):
    """The planar domain placed in 3-D by a rotation (about z, y, x in turn): a plane
    whose geometry is the planar one, for invariance checks."""
    az, ay, ax = angles
    Rz = np.array([[np.cos(az), -np.sin(az), 0], [np.sin(az), np.cos(az), 0], [0, 0, 1]])
    Ry = np.array([[np.cos(ay), 0, np.sin(ay)], [0, 1, 0], [-np.sin(ay), 0, np.cos(ay)]])
    Rx = np.array([[1, 0, 0], [0, np.cos(ax), -np.sin(ax)], [0, np.sin(ax), np.cos(ax)]])
    Rot = Rx @ Ry @ Rz
    G = dict(F)
    c = np.asarray(F["ctrl"], dtype=np.float64)
    G["ctrl"] = np.ascontiguousarray(np.hstack([c, np.zeros((len(c), 1))]) @ Rot.T)
    G["rotation"] = Rot
    return G


def fixture_dome(F, radius=1.5):
    """The planar domain lifted onto a sphere of the given radius centred above the
    domain's centre: control point (x, y) -> (x, y, sqrt(radius^2 - |(x, y) - centre|^2)),
    a spherical cap (the spline surface through those control points is close to it).
    With fixture_half_strip as the base: a curved 2-EP surface patch."""
    G = dict(F)
    c = np.asarray(F["ctrl"], dtype=np.float64)
    ctr = 0.5 * (c.min(axis=0) + c.max(axis=0))
    r2 = np.sum((c - ctr) ** 2, axis=1)
    assert np.all(r2 < radius * radius), "radius too small for the domain"
    G["ctrl"] = np.ascontiguousarray(np.hstack([c, np.sqrt(radius * radius - r2)[:, None]]))
    return G
