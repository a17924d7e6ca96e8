"""Seeded quad control meshes on the unit square with interior extraordinary points.

Input generation only: nothing here computes quadrature points, weights or matrices.
The control meshes follow the mild assumptions of the paper's Section 3 (EPs stay away
from the boundary, knot spans are 1 except on edges perpendicular to the boundary).

Construction (all topological, then embedded):
  * a structured M x M base grid;
  * local edits that create extraordinary points while the rest stays structured:
      - edge rotation inside a 2x1 block of quads      -> valences (3, 3, 5, 5)
      - diagonal collapse of one quad                  -> valences (6, 3, 3)
      - removal of a half strip of quads up to the top boundary, zipped shut
        -> one valence-5 vertex and one triangle (whose centre becomes valence 3)
  * r rounds of uniform polygon splitting (centroid + edge midpoints), which keeps the
    valence of every old vertex, turns an n-gon centre into a valence-n vertex and
    doubles all distances, so EPs become separated;
  * spatial renumbering (row-major by position) of vertices and faces;
  * a Tutte (uniform-weight harmonic) embedding with the boundary on [0,1]^2, followed
    by a seeded smooth displacement that vanishes on the boundary.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class QuadMesh:
    """Polygonal mesh (after splitting: all quads), faces listed counter-clockwise."""

    def __init__(self, faces, nv):
        self.faces = [list(map(int, f)) for f in faces]
        self.nv = int(nv)

    # ------------------------------------------------------------------ topology
    def build(self):
        faces = self.faces
        emap = {}
        for fi, fv in enumerate(faces):
            n = len(fv)
            for k in range(n):
                key = (fv[k], fv[(k + 1) % n])
                if key in emap:
                    raise ValueError(f"non-manifold directed edge {key}")
                emap[key] = (fi, k)
        self.emap = emap
        nv = self.nv
        bnd = np.zeros(nv, dtype=bool)
        for (a, b) in emap:
            if (b, a) not in emap:
                bnd[a] = True
                bnd[b] = True
        self.boundary = bnd
        # a face incident to each vertex
        inc = [[] for _ in range(nv)]
        for fi, fv in enumerate(faces):
            for k, v in enumerate(fv):
                inc[v].append((fi, k))
        self.nbrs = [None] * nv
        self.ring_faces = [None] * nv
        for v in range(nv):
            if not inc[v]:
                self.nbrs[v] = []
                self.ring_faces[v] = []
                continue
            # choose a start face: for boundary vertices, the face whose outgoing edge
            # v -> w has no twin (domain on its left when walking counter-clockwise)
            start = inc[v][0]
            if bnd[v]:
                for fi, k in inc[v]:
                    fv = faces[fi]
                    w = fv[(k + 1) % len(fv)]
                    if (w, v) not in emap:
                        start = (fi, k)
                        break
            nb, rf = [], []
            fi, k = start
            fv = faces[fi]
            nb.append(fv[(k + 1) % len(fv)])
            while True:
                fv = faces[fi]
                prev = fv[(k - 1) % len(fv)]
                rf.append(fi)
                nb.append(prev)
                nxt = emap.get((v, prev))
                if nxt is None:
                    break  # reached the boundary
                if nxt[0] == start[0]:
                    nb.pop()  # closed the ring: last neighbour == first
                    break
                fi, k = nxt
            self.nbrs[v] = nb
            self.ring_faces[v] = rf
        self.valence = np.array([len(n) for n in self.nbrs], dtype=np.int32)
        # breadth-first depth from the boundary
        depth = np.full(nv, -1, dtype=np.int64)
        frontier = list(np.nonzero(bnd)[0])
        for v in frontier:
            depth[v] = 0
        d = 0
        while frontier:
            nxt = []
            for v in frontier:
                for w in self.nbrs[v]:
                    if depth[w] < 0:
                        depth[w] = d + 1
                        nxt.append(w)
            frontier = nxt
            d += 1
        self.depth = depth
        return self

    def eps(self):
        """Interior vertices with valence != 4 (the paper's extraordinary points)."""
        return [v for v in range(self.nv)
                if (not self.boundary[v]) and self.valence[v] != 4 and self.nbrs[v]]


# ---------------------------------------------------------------------- base grid

def grid(M):
    """M x M structured quads; vertex (i, j) -> i + (M+1) j; faces CCW."""
    faces = []
    for j in range(M):
        for i in range(M):
            a = i + (M + 1) * j
            faces.append([a, a + 1, a + M + 2, a + M + 1])
    return QuadMesh(faces, (M + 1) ** 2)


def _face_at(M, i, j):
    return i + M * j


def edit_rotate(mesh: QuadMesh, f: int, g: int):
    """Rotate the edge shared by faces f and g inside their hexagon (3,3,5,5 pattern)."""
    F, G = mesh.faces[f], mesh.faces[g]
    shared = None
    for k in range(4):
        a, b = F[k], F[(k + 1) % 4]
        for m in range(4):
            if G[m] == b and G[(m + 1) % 4] == a:
                shared = (k, m)
    if shared is None:
        raise ValueError("faces are not edge-adjacent")
    k, m = shared
    # rotate F so that the shared edge is (F[1], F[2]); then G = (F2, F1, x, y)
    F = F[(k - 1) % 4:] + F[:(k - 1) % 4]
    G = G[m:] + G[:m]
    f0, f1, f2, f3 = F
    assert G[0] == f2 and G[1] == f1
    x, y = G[2], G[3]
    # hexagon (f2, f3, f0, f1, x, y); new diagonal (f3, x)
    mesh.faces[f] = [f3, f0, f1, x]
    mesh.faces[g] = [x, y, f2, f3]


def edit_collapse(mesh: QuadMesh, f: int):
    """Merge the diagonal corners 0 and 2 of face f (6,3,3 pattern); f is removed."""
    a, b, c, d = mesh.faces[f]
    new = []
    for fi, fv in enumerate(mesh.faces):
        if fi == f:
            continue
        new.append([a if v == c else v for v in fv])
    mesh.faces = new  # vertex c is left unused and dropped at renumbering


def edit_half_strip(M, a, b):
    """Base M x M grid with the quads (a, j), j >= b removed and the cut zipped shut.

    Vertex (a+1, j) is identified with (a, j) for j >= b; quad (a, b-1) becomes a
    triangle. Returns a QuadMesh with one triangle (valence-3 EP after splitting) and
    one degree-5 vertex (a, b).
    """
    def vid(i, j):
        return i + (M + 1) * j
    ident = {}
    for j in range(b, M + 1):
        ident[vid(a + 1, j)] = vid(a, j)
    faces = []
    for j in range(M):
        for i in range(M):
            if i == a and j >= b:
                continue
            v0 = vid(i, j)
            fv = [v0, v0 + 1, v0 + M + 2, v0 + M + 1]
            fv = [ident.get(v, v) for v in fv]
            out = []
            for v in fv:
                if not out or out[-1] != v:
                    out.append(v)
            if out[0] == out[-1]:
                out.pop()
            faces.append(out)
    return QuadMesh(faces, (M + 1) ** 2)


def split_polygons(mesh: QuadMesh, positions=None):
    """One round of uniform splitting: every n-gon -> n quads (centre + edge midpoints).

    Old vertices keep their ids; edge midpoints and face centres are appended.
    Returns the new mesh and, if positions were given, new positions (averages).
    """
    nv = mesh.nv
    edge_id = {}
    pos = None if positions is None else [p for p in positions]
    nid = nv
    for fv in mesh.faces:
        n = len(fv)
        for k in range(n):
            a, b = fv[k], fv[(k + 1) % n]
            key = (min(a, b), max(a, b))
            if key not in edge_id:
                edge_id[key] = nid
                nid += 1
                if pos is not None:
                    pos.append(0.5 * (positions[a] + positions[b]))
    faces = []
    for fv in mesh.faces:
        n = len(fv)
        c = nid
        nid += 1
        if pos is not None:
            pos.append(np.mean([positions[v] for v in fv], axis=0))
        for k in range(n):
            v = fv[k]
            m_next = edge_id[(min(v, fv[(k + 1) % n]), max(v, fv[(k + 1) % n]))]
            m_prev = edge_id[(min(v, fv[(k - 1) % n]), max(v, fv[(k - 1) % n]))]
            faces.append([v, m_next, c, m_prev])
    out = QuadMesh(faces, nid)
    return out, (None if pos is None else np.array(pos))


def compact(mesh: QuadMesh):
    """Drop unused vertex ids."""
    used = sorted({v for fv in mesh.faces for v in fv})
    remap = {v: i for i, v in enumerate(used)}
    return QuadMesh([[remap[v] for v in fv] for fv in mesh.faces], len(used))


# -------------------------------------------------------------------- embedding

def boundary_loop(mesh: QuadMesh):
    """Boundary vertices in counter-clockwise order."""
    nxt = {}
    for (a, b) in mesh.emap:
        if (b, a) not in mesh.emap:
            nxt[a] = b
    start = min(nxt)
    loop = [start]
    v = nxt[start]
    while v != start:
        loop.append(v)
        v = nxt[v]
    return loop


def tutte_embed(mesh: QuadMesh, guess=None):
    """Uniform-weight Tutte embedding; boundary on [0,1]^2, corners (valence 2) pinned."""
    loop = boundary_loop(mesh)
    corners = [i for i, v in enumerate(loop) if mesh.valence[v] == 2]
    if len(corners) != 4:
        raise ValueError(f"expected 4 boundary corners, found {len(corners)}")
    # rotate so that the corner nearest the guess's lower-left comes first
    if guess is not None:
        c_ll = min(corners, key=lambda i: guess[loop[i]][0] + guess[loop[i]][1])
    else:
        c_ll = corners[0]
    loop = loop[c_ll:] + loop[:c_ll]
    corners = [i for i, v in enumerate(loop) if mesh.valence[v] == 2]
    targets = [np.array([0.0, 0.0]), np.array([1.0, 0.0]),
               np.array([1.0, 1.0]), np.array([0.0, 1.0])]
    nv = mesh.nv
    P = np.zeros((nv, 2))
    fixed = np.zeros(nv, dtype=bool)
    nb = len(loop)
    for s in range(4):
        i0 = corners[s]
        i1 = corners[(s + 1) % 4] if s < 3 else nb
        seg = list(range(i0, i1))
        L = len(seg)
        for t, i in enumerate(seg):
            P[loop[i]] = targets[s] + (targets[(s + 1) % 4] - targets[s]) * (t / L)
            fixed[loop[i]] = True
    free = np.nonzero(~fixed)[0]
    idx = -np.ones(nv, dtype=np.int64)
    idx[free] = np.arange(len(free))
    rows, cols, vals = [], [], []
    rhs = np.zeros((len(free), 2))
    for v in free:
        r = idx[v]
        nbs = mesh.nbrs[v]
        rows.append(r)
        cols.append(r)
        vals.append(float(len(nbs)))
        for w in nbs:
            if fixed[w]:
                rhs[r] += P[w]
            else:
                rows.append(r)
                cols.append(idx[w])
                vals.append(-1.0)
    A = sp.csc_matrix((vals, (rows, cols)), shape=(len(free), len(free)))
    lu = spla.splu(A)
    P[free, 0] = lu.solve(rhs[:, 0])
    P[free, 1] = lu.solve(rhs[:, 1])
    return P


def renumber_spatial(mesh: QuadMesh, P):
    """Renumber vertices row-major by position and faces row-major by centroid.

    Face vertex lists are rotated so that corner 0 is the one with the smallest x+y
    (frames of structured regions then line up), keeping counter-clockwise order.
    """
    nv = mesh.nv
    h = 0.5 / max(1.0, np.sqrt(nv))
    key_v = np.round(P[:, 1] / h).astype(np.int64) * (10 ** 7) + np.round(P[:, 0] / h).astype(np.int64)
    order_v = np.argsort(key_v, kind="stable")
    new_id = np.empty(nv, dtype=np.int64)
    new_id[order_v] = np.arange(nv)
    faces = []
    cents = []
    for fv in mesh.faces:
        q = [int(new_id[v]) for v in fv]
        pts = P[fv]
        k0 = int(np.argmin(pts[:, 0] + pts[:, 1] + 1e-9 * np.arange(len(fv))))
        q = q[k0:] + q[:k0]
        faces.append(q)
        cents.append(pts.mean(axis=0))
    cents = np.array(cents)
    hf = 0.5 / max(1.0, np.sqrt(len(faces)))
    key_f = np.round(cents[:, 1] / hf).astype(np.int64) * (10 ** 7) + np.round(cents[:, 0] / hf).astype(np.int64)
    order_f = np.argsort(key_f, kind="stable")
    faces = [faces[i] for i in order_f]
    out = QuadMesh(faces, nv)
    return out, P[order_v]


def smooth_displacement(P, rng, amplitude=0.05):
    """d(x,y) = sum_{m,n in {1,2}} (a_mn, b_mn) sin(m pi x) sin(n pi y), max |d| = amplitude."""
    a = rng.uniform(-1.0, 1.0, size=(2, 2))
    b = rng.uniform(-1.0, 1.0, size=(2, 2))

    def d(X, Y):
        dx = np.zeros_like(X)
        dy = np.zeros_like(X)
        for m in (1, 2):
            for n in (1, 2):
                s = np.sin(m * np.pi * X) * np.sin(n * np.pi * Y)
                dx += a[m - 1, n - 1] * s
                dy += b[m - 1, n - 1] * s
        return dx, dy
    g = np.linspace(0.0, 1.0, 101)
    X, Y = np.meshgrid(g, g)
    dx, dy = d(X, Y)
    scale = amplitude / np.max(np.hypot(dx, dy))
    ux, uy = d(P[:, 0], P[:, 1])
    return P + scale * np.stack([ux, uy], axis=1)
