"""Bezier extraction operators of a bicubic spline space on an unstructured quad mesh.

Input generation only. The weighted-quadrature method consumes the per-element
extraction operators produced here (function ids + Bernstein coefficients); it never
depends on how they were made.

The paper (Section 3) sketches the analysis space of bicubic ASUTS: bicubic B-splines
on regular faces; around each extraordinary point (EP) the irregular faces are split
2x2, the EP's own function is removed and 4 face-based functions per irregular face are
added; transition faces blend the two families so that the whole set is a partition of
unity. The D-patch coefficients it relies on come from references that are not
available here, so this module builds its own space with the same structure:

  V0   Every vertex carries a function. The Bezier net of each effective face is built
       from local stencils: on faces whose four corners are regular, the exact
       tensor-product B-spline to Bezier conversion with knot intervals (open knot
       vectors at the boundary: spans perpendicular to the boundary are 0); on faces
       with an EP corner, the uniform edge/interior stencils and, at the EP, the
       valence-mu limit stencil (weights mu/(mu+5), 4/(mu(mu+5)), 1/(mu(mu+5))).
       V0 is a non-negative partition of unity, C1 away from EPs, C0 at spoke edges.
  EP   Each irregular face is split 2x2 (de Casteljau at 1/2). The EP function is
       removed and its Bezier net is partitioned, coefficient by coefficient, among the
       4 face functions (f, c) of its irregular faces (one per corner c of f), with
       bilinear corner weights inside f and fixed splits on shared edges/vertices so
       that every face function is C0. Face function (f, c) is supported on the faces
       around corner c (around the EP: all irregular faces).
Deviations from true ASUTS (stated, not hidden): C0 rather than C1 inside the 2-ring of
an EP; irregular faces carry 3mu+12 functions (ASUTS: 3mu+13); non-enriched transition
faces sharing an edge with an irregular face carry 18 (ASUTS: 17), those sharing a
vertex 16 (same). The hot path is indifferent to these.
"""
from __future__ import annotations

import numpy as np

from .quadmesh import QuadMesh

# 1D de Casteljau split of a cubic at 1/2: 7 x 4
SPLIT = np.array([
    [1.0, 0.0, 0.0, 0.0],
    [0.5, 0.5, 0.0, 0.0],
    [0.25, 0.5, 0.25, 0.0],
    [0.125, 0.375, 0.375, 0.125],
    [0.0, 0.25, 0.5, 0.25],
    [0.0, 0.0, 0.5, 0.5],
    [0.0, 0.0, 0.0, 1.0],
])


def _conv1d(dm2, dm1, d0, d1, d2):
    """4x4 map (c_-1, c0, c1, c2) -> Bezier (b0..b3) on the interval [c0, c1].

    Blossoming with vertex-centred cubic B-splines (vertex j carries the knot vector
    u_{j-2..j+2}); d_k are the knot intervals between consecutive vertices.
    """
    M = np.zeros((4, 4))
    D = dm1 + d0 + d1
    b1 = np.array([0.0, (d0 + d1) / D, dm1 / D, 0.0])
    b2 = np.array([0.0, d1 / D, (dm1 + d0) / D, 0.0])
    Dp = dm2 + dm1 + d0
    b2prev = np.array([d0 / Dp, (dm2 + dm1) / Dp, 0.0, 0.0])
    b0 = (d0 * b2prev + dm1 * b1) / (dm1 + d0)
    Dn = d0 + d1 + d2
    b1next = np.array([0.0, 0.0, (d1 + d2) / Dn, d0 / Dn])
    b3 = (d1 * b2 + d0 * b1next) / (d0 + d1)
    M[0], M[1], M[2], M[3] = b0, b1, b2, b3
    return M


class Extraction:
    """Per-face extraction operators for the EP-enriched bicubic space."""

    def __init__(self, mesh: QuadMesh):
        self.m = mesh
        m = mesh
        self.nv = m.nv
        self.is_ep = np.zeros(m.nv, dtype=bool)
        for v in m.eps():
            self.is_ep[v] = True
        nf = len(m.faces)
        self.effective = np.array([not any(m.boundary[v] for v in fv) for fv in m.faces])
        self.irregular = np.array([self.effective[f] and any(self.is_ep[v] for v in m.faces[f])
                                   for f in range(nf)])
        for f in np.nonzero(self.irregular)[0]:
            if sum(self.is_ep[v] for v in m.faces[f]) != 1:
                raise ValueError(f"face {f} has more than one EP corner; EPs must be separated")
        for v in np.nonzero(self.is_ep)[0]:
            if m.depth[v] < 5:
                raise ValueError(f"EP {v} at depth {m.depth[v]} < 5 from the boundary")
        # the 2-ring of every EP (support of its V0 function) must not reach another
        # EP's irregular faces
        owner = {}
        for v in np.nonzero(self.is_ep)[0]:
            for f in m.ring_faces[v]:
                owner[f] = v
        for v in np.nonzero(self.is_ep)[0]:
            ring1 = {w for f in m.ring_faces[v] for w in m.faces[f]}
            ring2 = {g for w in ring1 for g in m.ring_faces[w]}
            for g in ring2:
                if g in owner and owner[g] != v:
                    raise ValueError(f"EPs {v} and {owner[g]} are too close")

    # ------------------------------------------------------------- small helpers
    def span(self, a, b):
        bd = self.m.boundary
        return 0.0 if bd[a] != bd[b] else 1.0

    def opp(self, v, a):
        m = self.m
        nb = m.nbrs[v]
        if m.boundary[v]:
            if len(nb) == 3:
                if a == nb[0]:
                    return nb[2]
                if a == nb[2]:
                    return nb[0]
            return None
        if len(nb) != 4:
            return None
        i = nb.index(a)
        return nb[(i + 2) % 4]

    def next_span(self, a, b):
        w = self.opp(b, a)
        if w is None:
            return 0.0 if self.m.boundary[b] else 1.0
        return self.span(b, w)

    def diag(self, v, f):
        m = self.m
        rf = m.ring_faces[v]
        i = rf.index(f)
        g = rf[(i + 2) % 4]
        gv = m.faces[g]
        k = gv.index(v)
        return gv[(k + 2) % 4]

    def across(self, a, b):
        """Face across directed edge (a, b) of some face: returns (x, y) with x next to a."""
        g, k = self.m.emap[(b, a)]
        gv = self.m.faces[g]
        # gv[k] = b, gv[k+1] = a, gv[k+2] = x (adjacent to a), gv[k+3] = y (adjacent to b)
        return gv[(k + 2) % 4], gv[(k + 3) % 4]

    # ---------------------------------------------------------------- V0 nets
    def v0_net(self, f):
        """Dict vertex -> 4x4 Bezier coefficients (index [k][l], k along v0->v1)."""
        m = self.m
        v0, v1, v2, v3 = m.faces[f]
        corners = (v0, v1, v2, v3)
        if not any(self.is_ep[v] for v in corners):
            return self._tensor_net(f)
        return self._local_net(f)

    def _tensor_net(self, f):
        m = self.m
        v0, v1, v2, v3 = m.faces[f]
        c = {}
        c[(0, 0)], c[(1, 0)], c[(1, 1)], c[(0, 1)] = v0, v1, v2, v3
        c[(-1, 0)] = self.opp(v0, v1)
        c[(2, 0)] = self.opp(v1, v0)
        c[(-1, 1)] = self.opp(v3, v2)
        c[(2, 1)] = self.opp(v2, v3)
        c[(0, -1)] = self.opp(v0, v3)
        c[(1, -1)] = self.opp(v1, v2)
        c[(0, 2)] = self.opp(v3, v0)
        c[(1, 2)] = self.opp(v2, v1)
        c[(-1, -1)] = self.diag(v0, f)
        c[(2, -1)] = self.diag(v1, f)
        c[(2, 2)] = self.diag(v2, f)
        c[(-1, 2)] = self.diag(v3, f)
        du = (self.next_span(v0, c[(-1, 0)]), self.span(c[(-1, 0)], v0), self.span(v0, v1),
              self.span(v1, c[(2, 0)]), self.next_span(v1, c[(2, 0)]))
        dw = (self.next_span(v0, c[(0, -1)]), self.span(c[(0, -1)], v0), self.span(v0, v3),
              self.span(v3, c[(0, 2)]), self.next_span(v3, c[(0, 2)]))
        U = _conv1d(*du)
        W = _conv1d(*dw)
        net = {}
        for i in range(-1, 3):
            for j in range(-1, 3):
                v = c[(i, j)]
                contrib = np.outer(U[:, i + 1], W[:, j + 1])
                if not np.any(contrib):
                    continue
                if v is None:
                    raise ValueError(f"missing vertex in the 4x4 block of face {f}")
                net[v] = net.get(v, 0.0) + contrib
        return net

    def _limit_stencil(self, v):
        m = self.m
        mu = len(m.nbrs[v])
        out = {v: mu / (mu + 5.0)}
        we = 4.0 / (mu * (mu + 5.0))
        wd = 1.0 / (mu * (mu + 5.0))
        for w in m.nbrs[v]:
            out[w] = out.get(w, 0.0) + we
        for g in m.ring_faces[v]:
            gv = m.faces[g]
            k = gv.index(v)
            d = gv[(k + 2) % 4]
            out[d] = out.get(d, 0.0) + wd
        return out

    def _local_net(self, f):
        """Uniform local stencils (all spans 1 here: EPs are deep)."""
        m = self.m
        fv = m.faces[f]
        net = {}

        def add(v, k, l, w):
            if v not in net:
                net[v] = np.zeros((4, 4))
            net[v][k, l] += w
        cpos = [(0, 0), (3, 0), (3, 3), (0, 3)]
        for ci, v in enumerate(fv):
            for w, wt in self._limit_stencil(v).items():
                add(w, cpos[ci][0], cpos[ci][1], wt)
        # edge points: edge e from fv[e] to fv[e+1]
        # positions at 1/3 and 2/3 from fv[e]
        epos = [[(1, 0), (2, 0)], [(3, 1), (3, 2)], [(2, 3), (1, 3)], [(0, 2), (0, 1)]]
        for e in range(4):
            a, b = fv[e], fv[(e + 1) % 4]
            fa, fb = fv[(e - 1) % 4], fv[(e + 2) % 4]  # far vertices in f next to a, b
            x, y = self.across(a, b)
            for s, (ta, tb) in enumerate(((2.0 / 3.0, 1.0 / 3.0), (1.0 / 3.0, 2.0 / 3.0))):
                k, l = epos[e][s]
                for (va, vb), wr in (((x, y), 1.0 / 6.0), ((a, b), 4.0 / 6.0), ((fa, fb), 1.0 / 6.0)):
                    add(va, k, l, wr * ta)
                    add(vb, k, l, wr * tb)
        al = {1: (2.0 / 3.0, 1.0 / 3.0), 2: (1.0 / 3.0, 2.0 / 3.0)}
        for k in (1, 2):
            for l in (1, 2):
                add(fv[0], k, l, al[k][0] * al[l][0])
                add(fv[1], k, l, al[k][1] * al[l][0])
                add(fv[2], k, l, al[k][1] * al[l][1])
                add(fv[3], k, l, al[k][0] * al[l][1])
        return net

    # --------------------------------------------------------- EP partitioning
    def _faces_with(self, *vs):
        m = self.m
        sets = [set(m.ring_faces[v]) for v in vs]
        return sorted(set.intersection(*sets))

    def _corner(self, f, v):
        return self.m.faces[f].index(v)

    def _rule_vertex(self, e, x):
        m = self.m
        if x == e:
            mu = len(m.ring_faces[e])
            return [((f, self._corner(f, e)), 1.0 / mu) for f in m.ring_faces[e]]
        if x in m.nbrs[e]:
            fs = self._faces_with(e, x)
            return [((f, self._corner(f, x)), 1.0 / len(fs)) for f in fs]
        fs = self._faces_with(e, x)
        if fs:  # diagonal vertex of one irregular face
            return [((fs[0], self._corner(fs[0], x)), 1.0)]
        return None

    def _rule_edge(self, e, a, b, t):
        """Edge (a, b), parameter t from a, 0 < t < 1."""
        m = self.m
        if b == e:
            a, b, t = b, a, 1.0 - t
        if a == e:  # spoke edge (e, b)
            fs = self._faces_with(e, b)
            out = []
            for f in fs:
                out.append(((f, self._corner(f, e)), (1.0 - t) / len(fs)))
                out.append(((f, self._corner(f, b)), t / len(fs)))
            return out
        # outer edge: one endpoint is a neighbour of e, the other a diagonal vertex
        if b in m.nbrs[e]:
            a, b, t = b, a, 1.0 - t
        if a in m.nbrs[e]:
            fs = self._faces_with(e, a, b)
            if len(fs) == 1:
                f = fs[0]
                return [((f, self._corner(f, a)), 1.0 - t), ((f, self._corner(f, b)), t)]
        return None

    def build(self):
        m = self.m
        nf = len(m.faces)
        nets = [None] * nf
        for f in range(nf):
            if self.effective[f]:
                nets[f] = self.v0_net(f)
        # function numbering: non-EP vertices, then (irregular face, corner)
        vid = -np.ones(m.nv, dtype=np.int64)
        nvf = 0
        for v in range(m.nv):
            if not self.is_ep[v]:
                vid[v] = nvf
                nvf += 1
        irr = np.nonzero(self.irregular)[0]
        ffid = {}
        for j, f in enumerate(irr):
            for c in range(4):
                ffid[(int(f), c)] = nvf + 4 * j + c
        self.n_fn = nvf + 4 * len(irr)
        self.vertex_fn = vid
        self.face_fn = ffid
        epset = set(np.nonzero(self.is_ep)[0].tolist())
        face_fns, face_coef, face_split = [], [], []
        tol = 1e-14
        for f in range(nf):
            if not self.effective[f]:
                face_fns.append(np.zeros(0, dtype=np.int64))
                face_coef.append(np.zeros((1, 0, 16)))
                face_split.append(0)
                continue
            net = nets[f]
            fv = m.faces[f]
            split = bool(self.irregular[f])
            acc = {}  # global fn id -> net (4x4 or 7x7)

            def addf(gid, arr):
                if gid in acc:
                    acc[gid] = acc[gid] + arr
                else:
                    acc[gid] = arr.copy()
            for v, N4 in net.items():
                if v in epset:
                    continue
                arr = SPLIT @ N4 @ SPLIT.T if split else N4
                addf(int(vid[v]), arr)
            eps_here = [v for v in net if v in epset and np.max(np.abs(net[v])) > 0]
            for e in eps_here:
                N4 = net[e]
                if split:
                    self._partition_split(f, e, N4, addf)
                else:
                    self._partition_unsplit(f, e, N4, addf)
            ids = sorted(k for k, a in acc.items() if np.max(np.abs(a)) > tol)
            nsub = 4 if split else 1
            C = np.zeros((nsub, len(ids), 16))
            for r, g in enumerate(ids):
                a = acc[g]
                if split:
                    for sy in range(2):
                        for sx in range(2):
                            blk = a[3 * sx:3 * sx + 4, 3 * sy:3 * sy + 4]
                            C[sx + 2 * sy, r] = blk.T.reshape(16)  # index k + 4 l
                else:
                    C[0, r] = a.T.reshape(16)
            face_fns.append(np.array(ids, dtype=np.int64))
            face_coef.append(C)
            face_split.append(1 if split else 0)
        self.face_fns = face_fns
        self.face_coef = face_coef
        self.face_split = np.array(face_split, dtype=np.uint8)
        return self

    def _net_entity(self, f, u, v):
        """Locate parametric (u, v) of face f: ('v', vertex) | ('e', a, b, t) | ('i',)."""
        fv = self.m.faces[f]
        eps = 1e-12
        onu0, onu1, onv0, onv1 = u < eps, u > 1 - eps, v < eps, v > 1 - eps
        if (onu0 or onu1) and (onv0 or onv1):
            ci = {(True, True): 0, (False, True): 1, (False, False): 2, (True, False): 3}[(onu0, onv0)]
            return ('v', fv[ci])
        if onv0:
            return ('e', fv[0], fv[1], u)
        if onu1:
            return ('e', fv[1], fv[2], v)
        if onv1:
            return ('e', fv[2], fv[3], 1.0 - u)
        if onu0:
            return ('e', fv[3], fv[0], 1.0 - v)
        return ('i',)

    def _apply_rule(self, e, ent, f, u, v):
        if ent[0] == 'v':
            r = self._rule_vertex(e, ent[1])
        elif ent[0] == 'e':
            r = self._rule_edge(e, ent[1], ent[2], ent[3])
        else:
            if not self.irregular[f]:
                return None
            r = []
            fv = self.m.faces[f]
            for c, (cx, cy) in enumerate(((0, 0), (1, 0), (1, 1), (0, 1))):
                h = (1.0 - abs(u - cx)) * (1.0 - abs(v - cy))
                if h <= 0:
                    continue
                # the corner's share is split among all face functions attached to that
                # vertex, so each of them is nonzero on every cell of every face it
                # reaches (own face: 1/2 at the EP, 2/3 at a spoke neighbour)
                x = fv[c]
                owners = self._faces_with(e, x)
                if len(owners) == 1:
                    r.append(((f, c), h))
                    continue
                own = 0.5 if x == e else 2.0 / 3.0
                other = (1.0 - own) / (len(owners) - 1)
                for g in owners:
                    r.append(((g, self._corner(g, x)), h * (own if g == f else other)))
        return r

    def _partition_unsplit(self, f, e, N4, addf):
        out = {}
        for k in range(4):
            for l in range(4):
                val = N4[k, l]
                if abs(val) <= 1e-15:
                    continue
                ent = self._net_entity(f, k / 3.0, l / 3.0)
                r = self._apply_rule(e, ent, f, k / 3.0, l / 3.0)
                if r is None:
                    raise ValueError(f"EP {e}: no face function owns net point ({k},{l}) of face {f}")
                for key, w in r:
                    if key not in out:
                        out[key] = np.zeros((4, 4))
                    out[key][k, l] += w * val
        for key, arr in out.items():
            addf(self.face_fn[key], arr)

    def _partition_split(self, f, e, N4, addf):
        N7 = SPLIT @ N4 @ SPLIT.T
        fv = self.m.faces[f]
        ce = fv.index(e)
        out = {}

        def put(key, K, L, val):
            if key not in out:
                out[key] = np.zeros((7, 7))
            out[key][K, L] += val
        # outer edges (not incident to e) are partitioned on their unsplit cubic
        outer = [ei for ei in range(4) if fv[ei] != e and fv[(ei + 1) % 4] != e]
        # edge ei occupies, in the 4x4 net, positions listed from fv[ei] to fv[ei+1]
        edge4 = {0: [(0, 0), (1, 0), (2, 0), (3, 0)], 1: [(3, 0), (3, 1), (3, 2), (3, 3)],
                 2: [(3, 3), (2, 3), (1, 3), (0, 3)], 3: [(0, 3), (0, 2), (0, 1), (0, 0)]}
        edge7 = {0: [(K, 0) for K in range(7)], 1: [(6, L) for L in range(7)],
                 2: [(6 - K, 6) for K in range(7)], 3: [(0, 6 - L) for L in range(7)]}
        done = np.zeros((7, 7), dtype=bool)
        for ei in outer:
            a, b = fv[ei], fv[(ei + 1) % 4]
            vals = np.array([N4[p] for p in edge4[ei]])
            parts = {}
            for s in range(4):
                t = s / 3.0
                if s == 0:
                    r = self._rule_vertex(e, a)
                elif s == 3:
                    r = self._rule_vertex(e, b)
                else:
                    r = self._rule_edge(e, a, b, t)
                if r is None:
                    if abs(vals[s]) > 1e-15:
                        raise ValueError("unowned outer-edge net point")
                    continue
                for key, w in r:
                    parts.setdefault(key, np.zeros(4))[s] += w * vals[s]
            for key, p4 in parts.items():
                p7 = SPLIT @ p4
                for s7, (K, L) in enumerate(edge7[ei]):
                    if not done[K, L]:
                        put(key, K, L, p7[s7])
            for (K, L) in edge7[ei]:
                done[K, L] = True
        for K in range(7):
            for L in range(7):
                if done[K, L]:
                    continue
                val = N7[K, L]
                if abs(val) <= 1e-15:
                    continue
                u, v = K / 6.0, L / 6.0
                ent = self._net_entity(f, u, v)
                r = self._apply_rule(e, ent, f, u, v)
                if r is None:
                    raise ValueError(f"EP {e}: unowned split net point ({K},{L}) of face {f}")
                for key, w in r:
                    put(key, K, L, w * val)
        del ce
        for key, arr in out.items():
            addf(self.face_fn[key], arr)
