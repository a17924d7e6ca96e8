"""Weighted quadrature on unstructured bicubic splines: plain FP64 reference.

TEST INFRASTRUCTURE ONLY (see package docstring). Every function names the passage of
the paper it follows. Readings of silent/ambiguous passages are marked READING.

Inputs are fixtures (see fixtures/__init__.py): control mesh topology, per-face Bezier
extraction operators and control points. Nothing here is shared with the GPU library.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# ----------------------------------------------------------------------------------
# O1  Element classification and points per element
#     Section 3 (definitions of valence, EP, irregular/enriched/transition/boundary/
#     passive/regular elements), Section 4.2 Table 2 and Eq. (18).
# ----------------------------------------------------------------------------------

ET_PASSIVE, ET_REGULAR, ET_BOUNDARY, ET_IRREGULAR, ET_TRANSITION = 0, 1, 2, 3, 4


def topology(face_vtx, nv):
    """Boundary flags, valence (edge count) and vertex->faces of a quad mesh."""
    edges = {}
    for f, fv in enumerate(face_vtx):
        for k in range(4):
            a, b = int(fv[k]), int(fv[(k + 1) % 4])
            key = (min(a, b), max(a, b))
            edges[key] = edges.get(key, 0) + 1
    boundary = np.zeros(nv, dtype=bool)
    valence = np.zeros(nv, dtype=np.int64)
    for (a, b), cnt in edges.items():
        valence[a] += 1
        valence[b] += 1
        if cnt == 1:
            boundary[a] = boundary[b] = True
    vfaces = [[] for _ in range(nv)]
    for f, fv in enumerate(face_vtx):
        for v in fv:
            vfaces[int(v)].append(f)
    return boundary, valence, vfaces


def classify(fx):
    """Element type and points-per-direction s_e for every face (Section 3, Table 2).

    Returns dict with etype (per face), s (per face, 0 for passive), ep (bool per
    vertex). READING (X9): an element in several classes takes the largest s; a
    non-enriched transition element takes 4x4 when an involved EP has valence >= 7 or
    when it touches enriched elements of two different EPs ("clustered"), else 3x3.
    """
    fvs = fx["face_vtx"]
    nv = fx["nv"]
    nf = len(fvs)
    boundary, valence, vfaces = topology(fvs, nv)
    # EP: interior vertex with valence != 4, or boundary vertex with valence > 3
    ep = np.array([(not boundary[v] and valence[v] != 4) or (boundary[v] and valence[v] > 3)
                   for v in range(nv)])
    # 1-ring neighbourhood of the boundary = elements sharing a boundary vertex: passive
    passive = np.array([any(boundary[v] for v in fv) for fv in fvs])
    passive_vtx = np.zeros(nv, dtype=bool)
    for f in np.nonzero(passive)[0]:
        passive_vtx[fvs[f]] = True
    # 2nd ring of the boundary: elements sharing a vertex with the 1-ring, not in it
    bnd2 = np.array([(not passive[f]) and any(passive_vtx[v] for v in fvs[f]) for f in range(nf)])
    irregular = np.array([(not passive[f]) and any(ep[v] for v in fvs[f]) for f in range(nf)])
    enriched = irregular.copy()  # initial mesh: enriched elements = irregular elements
    # transition points: shared by an enriched and a non-enriched element
    tpoint = np.zeros(nv, dtype=bool)
    for v in range(nv):
        fs = vfaces[v]
        if any(enriched[f] for f in fs) and any((not enriched[f]) for f in fs):
            tpoint[v] = True
    transition = np.array([(not passive[f]) and any(tpoint[v] for v in fvs[f]) for f in range(nf)])
    etype = np.full(nf, ET_REGULAR, dtype=np.int64)
    s = np.zeros(nf, dtype=np.int64)
    for f in range(nf):
        if passive[f]:
            etype[f] = ET_PASSIVE
            continue
        cand = []
        if irregular[f]:
            etype[f] = ET_IRREGULAR
            cand.append(4)
        elif transition[f]:
            etype[f] = ET_TRANSITION
        elif bnd2[f]:
            etype[f] = ET_BOUNDARY
        if bnd2[f]:
            cand.append(4)
        if transition[f] and enriched[f]:
            cand.append(4)
        if transition[f] and not enriched[f]:
            involved = set()
            for v in fvs[f]:
                if tpoint[v]:
                    for g in vfaces[v]:
                        if enriched[g]:
                            involved.update(int(w) for w in fvs[g] if ep[w])
            clustered = len(involved) >= 2 or any(valence[w] >= 7 for w in involved)
            cand.append(4 if clustered else 3)
        if not cand:
            cand.append(2)  # regular
        s[f] = max(cand)
    return {"etype": etype, "s": s, "ep": ep, "split": fx["split"].astype(bool)}


def element_functions(fx, f):
    lo, hi = fx["ext_ptr"][f], fx["ext_ptr"][f + 1]
    return fx["ext_fn"][lo:hi]


def element_coef(fx, f):
    fn = element_functions(fx, f)
    C = fx["coef"][fx["coef_ptr"][f]:fx["coef_ptr"][f + 1]]
    nsub = 4 if fx["split"][f] else 1
    return fn, C.reshape(nsub, len(fn), 16)


def cells(fx, s):
    """Bezier cells: each non-passive element is one cell, a split (irregular) element
    four (Section 3: the 2x2 split). Returns dict of per-cell arrays: elem, sub,
    funcs (functions with a nonzero Bernstein coefficient on the cell), and points.

    Points (Section 4.1): s x s per element at ((2a+1)/(2s), (2b+1)/(2s)) in the
    element's parametric square (READING X1: cell-centred). They are numbered cell by
    cell (elements ascending, sub-elements s = sx + 2 sy ascending), and inside a cell
    in (b, a) row-major order; eta is the cell-local coordinate.
    """
    elem, sub, funcs, eta, npts = [], [], [], [], []
    for f in range(len(s)):
        if s[f] == 0:
            continue
        fn, C = element_coef(fx, f)
        sf = int(s[f])
        grid = [((2 * a + 1) / (2 * sf), (2 * b + 1) / (2 * sf)) for b in range(sf) for a in range(sf)]
        nsub = C.shape[0]
        for k in range(nsub):
            if nsub == 1:
                pts = grid
            else:
                sx, sy = k % 2, k // 2
                pts = [(2 * u - sx, 2 * v - sy) for (u, v) in grid
                       if min(int(2 * u), 1) == sx and min(int(2 * v), 1) == sy]
            nz = [j for r, j in enumerate(fn) if np.any(C[k, r] != 0.0)]
            elem.append(f)
            sub.append(k)
            funcs.append(np.array(nz, dtype=np.int64))
            eta.append(pts)
            npts.append(len(pts))
    pt_off = np.zeros(len(elem) + 1, dtype=np.int64)
    pt_off[1:] = np.cumsum(npts)
    return {"elem": np.array(elem), "sub": np.array(sub), "funcs": funcs, "eta": eta,
            "pt_off": pt_off}


def supports(fx, cl):
    """supp(N_i) as ascending cell lists. READING: Section 2 counts the quadrature
    points located in the support of the test function; with piecewise definitions on
    the 2x2 split, the support is taken cell by cell, so Q_i never holds a point where
    N_i vanishes identically."""
    n = fx["n_fn"]
    supp = [[] for _ in range(n)]
    for c, fn in enumerate(cl["funcs"]):
        for j in fn:
            supp[int(j)].append(c)
    return supp


def overlap_sets(fx, cl, supp):
    """S_i of Eq. (10): functions nonzero on some cell of supp(N_i), ascending."""
    out = []
    for i in range(fx["n_fn"]):
        cols = set()
        for c in supp[i]:
            cols.update(int(j) for j in cl["funcs"][c])
        out.append(np.array(sorted(cols), dtype=np.int64))
    return out


def minmax_row_requirement(n_i, elems):
    """Eq. (18) for one test function N_i. elems lists (element type, m_k) for every
    element k of supp(N_i). Regular and boundary elements (the set R) keep the standard
    WQ counts, 4 and 16 points; every other element k gets the share
    r_{i,k} = m_k / (sum over l in supp(N_i) minus R of m_l) * (n_i - 4 e^r_i - 16 e^b_i),
    rounded up (READING X9). Returns r_{i,k} per element, None for elements in R."""
    e_r = sum(1 for t, _ in elems if t == ET_REGULAR)
    e_b = sum(1 for t, _ in elems if t == ET_BOUNDARY)
    msum = sum(mk for t, mk in elems if t not in (ET_REGULAR, ET_BOUNDARY))
    out = []
    for t, mk in elems:
        if t in (ET_REGULAR, ET_BOUNDARY):
            out.append(None)
        else:
            out.append(math.ceil(mk / msum * (n_i - 4 * e_r - 16 * e_b) - 1e-12))
    return out


def minmax_points_per_direction(r_k, split):
    """s_k = smallest s >= 2 with s^2 >= r_k, where r_k = max_i r_{i,k} (Eq. (18) and
    the sentence after it); even on a split element so that no point falls on a
    sub-element edge (READING)."""
    sk = 2
    while sk * sk < r_k or (split and sk % 2):
        sk += 1
    return sk


def points_per_element(fx, cls, s_init=None):
    """Table 2 counts, then the well-posedness check r_i >= n_i and, where it fails,
    the "min-max" allocation of Eq. (18) for the non-regular, non-boundary elements.

    READING: r_k = max_i ceil(r_{i,k}); s_k = smallest s >= 2 with s^2 >= r_k (even for
    split elements so that no point falls on a sub-element edge); repeated until every
    row is well posed. supp(N_i) in Eq. (18) is the set of elements holding a cell of
    the support; m_k counts the functions of element k.
    """
    s = (cls["s"] if s_init is None else np.asarray(s_init, dtype=np.int64)).copy()
    etype = cls["etype"]
    m = np.array([fx["ext_ptr"][f + 1] - fx["ext_ptr"][f] for f in range(len(s))])
    for _ in range(16):
        cl = cells(fx, s)
        supp = supports(fx, cl)
        S = overlap_sets(fx, cl, supp)
        npts = np.diff(cl["pt_off"])
        r = [int(sum(npts[c] for c in supp[i])) for i in range(fx["n_fn"])]
        bad = [i for i in range(fx["n_fn"]) if r[i] < len(S[i])]
        if not bad:
            return s
        need = {}
        for i in range(fx["n_fn"]):
            els = sorted({int(cl["elem"][c]) for c in supp[i]})
            req = minmax_row_requirement(len(S[i]), [(int(etype[f]), int(m[f])) for f in els])
            for f, r_ik in zip(els, req):
                if r_ik is not None:
                    need[f] = max(need.get(f, 0), r_ik)
        changed = False
        for k, rk in need.items():
            sk = minmax_points_per_direction(rk, bool(cls["split"][k]))
            if sk > s[k]:
                s[k] = sk
                changed = True
        if not changed:
            raise RuntimeError(f"min-max allocation cannot make rows {bad[:5]} well posed")
    raise RuntimeError("min-max allocation did not converge")


# ----------------------------------------------------------------------------------
# O2/O3  Points and basis/geometry evaluation (Section 4.1; Section 3 Bezier form;
#        Eqs. (13)-(17) reduced to the plane)
# ----------------------------------------------------------------------------------

def bernstein3(t):
    """Cubic Bernstein values, first and second derivatives at t."""
    b = np.array([(1 - t) ** 3, 3 * t * (1 - t) ** 2, 3 * t * t * (1 - t), t ** 3])
    d1 = np.array([-3 * (1 - t) ** 2, 3 * (1 - t) ** 2 - 6 * t * (1 - t),
                   6 * t * (1 - t) - 3 * t * t, 3 * t * t])
    d2 = np.array([6 * (1 - t), -12 * (1 - t) + 6 * t, 6 * (1 - t) - 12 * t, 6 * t])
    return b, d1, d2


def eval_cell(fx, f, k, eta, fn_subset=None):
    """Basis and geometry at cell-local point eta of sub-element k of element f.

    N_j = sum_kl C[j, k+4l] b_k(eta_1) b_l(eta_2) (Section 3); x = sum_j P_j N_j;
    J = dx/deta; grad_x N = J^{-T} grad_eta N; Hessian by the chain rule
    H_x N = J^{-T} (H_eta N - sum_d (dN/dx_d) H_eta x_d) J^{-1}, Lap N = tr H_x N.
    Returns (fn, N, Nx, Ny, Lap, x, detJ)."""
    fn, C = element_coef(fx, f)
    Ce = C[k]
    b1, d1, s1 = bernstein3(eta[0])
    b2, d2, s2 = bernstein3(eta[1])
    T = lambda u, v: np.outer(v, u).reshape(16)  # noqa: E731  index k + 4 l
    N = Ce @ T(b1, b2)
    N1 = Ce @ T(d1, b2)
    N2 = Ce @ T(b1, d2)
    N11 = Ce @ T(s1, b2)
    N12 = Ce @ T(d1, d2)
    N22 = Ce @ T(b1, s2)
    P = fx["ctrl"][fn]  # (m, 2), or (m, 3) for a surface
    if P.shape[1] == 3:
        out = _eval_surface(fn, P, N, N1, N2, N11, N12, N22)
        if fn_subset is None:
            return out
        sel = np.array([int(np.nonzero(fn == j)[0][0]) for j in fn_subset], dtype=np.int64)
        return (fn[sel], out[1][sel], out[2][sel], out[3][sel], out[4][sel], out[5], out[6], out[7][sel])
    x = P.T @ N
    J = np.stack([P.T @ N1, P.T @ N2], axis=1)  # J[a, b] = d x_a / d eta_b
    detJ = np.linalg.det(J)
    Ji = np.linalg.inv(J)
    grad = Ji.T @ np.stack([N1, N2])  # (2, m)
    Hx = np.array([[[P[:, a] @ N11, P[:, a] @ N12], [P[:, a] @ N12, P[:, a] @ N22]] for a in range(2)])
    lap = np.zeros(len(fn))
    for j in range(len(fn)):
        He = np.array([[N11[j], N12[j]], [N12[j], N22[j]]])
        He = He - grad[0, j] * Hx[0] - grad[1, j] * Hx[1]
        lap[j] = np.trace(Ji.T @ He @ Ji)
    out = (fn, N, grad[0], grad[1], lap, x, detJ)
    if fn_subset is None:
        return out
    sel = np.array([int(np.nonzero(fn == j)[0][0]) for j in fn_subset], dtype=np.int64)
    return (fn[sel], N[sel], grad[0][sel], grad[1][sel], lap[sel], x, detJ)


def is_surface(fx):
    """A 2-manifold in 3-D: control points with three coordinates (Section 4.1)."""
    return np.asarray(fx["ctrl"]).shape[1] == 3


def _eval_surface(fn, P, N, N1, N2, N11, N12, N22):
    """Eqs. (13)-(17) on a parametric surface x(eta) = sum_j P_j N_j in R^3: tangent
    vectors a_a = dx/deta_a, metric g_ab = a_a . a_b, area element sqrt(det g); the
    surface gradient grad_s N = g^{ab} (dN/deta_b) a_a (three components) and the
    Laplace-Beltrami operator Delta_s N = g^{ab} (d2N/deta_a deta_b - Gamma^c_ab dN/deta_c)
    with Gamma^c_ab = g^{cd} a_d . d2x/deta_a deta_b. For a plane they reduce to the
    planar gradient and Laplacian. Returns (fn, N, Nx, Ny, LB, x, sqrt(det g), Nz)."""
    x = P.T @ N
    A = np.stack([P.T @ N1, P.T @ N2], axis=1)  # (3, 2): columns a_1, a_2
    g = A.T @ A
    gi = np.linalg.inv(g)
    sg = math.sqrt(np.linalg.det(g))
    dN = np.stack([N1, N2])  # (2, m)
    grad = A @ (gi @ dN)  # (3, m)
    Xh = {(0, 0): P.T @ N11, (0, 1): P.T @ N12, (1, 1): P.T @ N22}
    Xh[(1, 0)] = Xh[(0, 1)]
    Hn = {(0, 0): N11, (0, 1): N12, (1, 0): N12, (1, 1): N22}
    lb = np.zeros(len(fn))
    for a in range(2):
        for b in range(2):
            gam = gi @ (A.T @ Xh[(a, b)])  # Gamma^c_ab, c = 0, 1
            lb += gi[a, b] * (Hn[(a, b)] - gam[0] * N1 - gam[1] * N2)
    return (fn, N, grad[0], grad[1], lb, x, sg, grad[2])


def wq_points(fx, cl):
    """Basis/geometry at every WQ point, per cell: dict with fn (the cell's nonzero
    functions), N, Nx, Ny (and Nz on a surface: the surface gradient), Lap (the
    Laplacian, or the Laplace-Beltrami operator on a surface) (npts x m), x (npts x 2 or
    3), detJ (npts; sqrt(det g) on a surface)."""
    data = []
    for c in range(len(cl["elem"])):
        f, k = int(cl["elem"][c]), int(cl["sub"][c])
        rows = [eval_cell(fx, f, k, eta, cl["funcs"][c]) for eta in cl["eta"][c]]
        d = {
            "fn": cl["funcs"][c],
            "N": np.array([r[1] for r in rows]),
            "Nx": np.array([r[2] for r in rows]),
            "Ny": np.array([r[3] for r in rows]),
            "Lap": np.array([r[4] for r in rows]),
            "x": np.array([r[5] for r in rows]),
            "detJ": np.array([r[6] for r in rows]),
        }
        if len(rows[0]) > 7:
            d["Nz"] = np.array([r[7] for r in rows])
        data.append(d)
    return data


def pattern(fx, cl):
    """Eq. (10): CSR rows S_i (ascending columns) and point sets Q_i (the point ranges
    of the cells of supp(N_i), cells ascending)."""
    supp = supports(fx, cl)
    S = overlap_sets(fx, cl, supp)
    n = fx["n_fn"]
    pt_off = cl["pt_off"]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    qptr = np.zeros(n + 1, dtype=np.int64)
    cols, qidx = [], []
    for i in range(n):
        row_ptr[i + 1] = row_ptr[i] + len(S[i])
        cols.extend(S[i].tolist())
        q = []
        for c in supp[i]:
            q.extend(range(pt_off[c], pt_off[c + 1]))
        qptr[i + 1] = qptr[i] + len(q)
        qidx.extend(q)
    return {"row_ptr": row_ptr, "col": np.array(cols, dtype=np.int32),
            "qptr": qptr, "qidx": np.array(qidx, dtype=np.int32), "supp": supp, "S": S}


# ----------------------------------------------------------------------------------
# O5  Exact integrals b (Section 2: "precomputed"; Section 4.2: 4x4 Gauss points per
#     Bezier element, 4x4x4 for a split irregular element)
# ----------------------------------------------------------------------------------

def gauss4():
    g, w = np.polynomial.legendre.leggauss(4)
    return 0.5 * (g + 1.0), 0.5 * w


def gq_matrices(fx, cl, coef=None):
    """Element-wise Gauss assembly (4x4 points per Bezier cell, i.e. 4x4x4 for a split
    element) of M = int N_i N_j, Kx = int dxN_i dxN_j, Ky = int dyN_i dyN_j and
    B = int Lap N_i Lap N_j (scipy CSR, n x n); on a surface also Kz, with the surface
    gradient and the Laplace-Beltrami operator. coef(x) optionally multiplies every
    integrand."""
    gp, gw = gauss4()
    n = fx["n_fn"]
    R, Cc = [], []
    surf = is_surface(fx)
    V = {k: [] for k in (("M", "Kx", "Ky", "Kz", "B") if surf else ("M", "Kx", "Ky", "B"))}
    for c in range(len(cl["elem"])):
        f, k = int(cl["elem"][c]), int(cl["sub"][c])
        for bq in range(4):
            for aq in range(4):
                ev = eval_cell(fx, f, k, (gp[aq], gp[bq]), cl["funcs"][c])
                fn, N, Nx, Ny, Lap, x, detJ = ev[:7]
                # derivatives are w.r.t. the cell coordinate eta: |detJ| d eta is the
                # area element on the cell (sqrt(det g) on a surface)
                wq = gw[aq] * gw[bq] * abs(detJ)
                if coef is not None:
                    wq *= coef(x)
                ii, jj = np.meshgrid(fn, fn, indexing="ij")
                R.append(ii.reshape(-1))
                Cc.append(jj.reshape(-1))
                V["M"].append((wq * np.outer(N, N)).reshape(-1))
                V["Kx"].append((wq * np.outer(Nx, Nx)).reshape(-1))
                V["Ky"].append((wq * np.outer(Ny, Ny)).reshape(-1))
                V["B"].append((wq * np.outer(Lap, Lap)).reshape(-1))
                if surf:
                    V["Kz"].append((wq * np.outer(ev[7], ev[7])).reshape(-1))
    R = np.concatenate(R)
    Cc = np.concatenate(Cc)
    return {k: sp.csr_matrix((np.concatenate(v), (R, Cc)), shape=(n, n)) for k, v in V.items()}


def gauss_data(fx, cl):
    """Basis at the 4x4 Gauss points of every Bezier cell, computed ahead (the paper times
    formation and assembly with basis evaluation excluded, Section 6.1): per cell the
    functions, N, dN/dx, dN/dy (16 x m), the points x and the weights g_a g_b |detJ|."""
    gp, gw = gauss4()
    out = []
    for c in range(len(cl["elem"])):
        f, k = int(cl["elem"][c]), int(cl["sub"][c])
        rows = [eval_cell(fx, f, k, (gp[aq], gp[bq]), cl["funcs"][c]) for bq in range(4) for aq in range(4)]
        wts = np.array([gw[aq] * gw[bq] for bq in range(4) for aq in range(4)])
        d = {"fn": cl["funcs"][c], "N": np.array([r[1] for r in rows]), "Nx": np.array([r[2] for r in rows]),
             "Ny": np.array([r[3] for r in rows]), "x": np.array([r[5] for r in rows]),
             "w": wts * np.abs(np.array([r[6] for r in rows]))}
        if len(rows[0]) > 7:
            d["Nz"] = np.array([r[7] for r in rows])
        out.append(d)
    return out


def gq_assemble(fx, gdata, kind, coef=None):
    """Element-wise Gauss formation and assembly with the basis given (gauss_data): per
    cell and Gauss point the outer product of the basis values, weighted, added into the
    global matrix; 'mass' (int c N_i N_j) or 'stiffness' (int k grad N_i . grad N_j).
    coef(x) or None for 1. Returns a scipy CSR matrix."""
    n = fx["n_fn"]
    R, Cc, V = [], [], []
    for d in gdata:
        m = len(d["fn"])
        wq = d["w"] if coef is None else d["w"] * coef(d["x"])
        E = np.zeros((m, m))
        for g in range(len(wq)):
            if kind == "mass":
                E += wq[g] * np.outer(d["N"][g], d["N"][g])
            else:
                E += wq[g] * (np.outer(d["Nx"][g], d["Nx"][g]) + np.outer(d["Ny"][g], d["Ny"][g]))
                if "Nz" in d:
                    E += wq[g] * np.outer(d["Nz"][g], d["Nz"][g])
        ii, jj = np.meshgrid(d["fn"], d["fn"], indexing="ij")
        R.append(ii.reshape(-1))
        Cc.append(jj.reshape(-1))
        V.append(E.reshape(-1))
    return sp.csr_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(Cc))), shape=(n, n))


# ----------------------------------------------------------------------------------
# O6  Weights by truncated SVD (Section 4.3, Eqs. (19)-(22); Section 2 Eqs. (5)-(6))
# ----------------------------------------------------------------------------------

FAMILIES = ("mass", "x", "y", "lap", "z")
_FAM_KEY = {"mass": "N", "x": "Nx", "y": "Ny", "lap": "Lap", "z": "Nz"}
_FAM_GQ = {"mass": "M", "x": "Kx", "y": "Ky", "lap": "B", "z": "Kz"}


def local_matrix(fx, pat, data, i, key):
    """A[l, m] = D N_{S_i[l]}(x_{Q_i[m]}) (Eq. (19); Eq. (5) for the mass family)."""
    S = pat["S"][i]
    pos = {int(j): l for l, j in enumerate(S)}
    blocks = []
    for c in pat["supp"][i]:
        d = data[c]
        A_c = np.zeros((len(S), d[key].shape[0]))
        for k, j in enumerate(d["fn"]):
            A_c[pos[int(j)], :] = d[key][:, k]
        blocks.append(A_c)
    return np.concatenate(blocks, axis=1)


def z_diag(fx, pat, data, i):
    """Z = diag(N_i(x_q)) over Q_i (Eq. (5)); READING X2: the same Z for every family."""
    z = []
    for c in pat["supp"][i]:
        d = data[c]
        k = int(np.nonzero(d["fn"] == i)[0][0])
        z.append(d["N"][:, k])
    return np.concatenate(z)


def tsvd_solve(A, z, b, tau):
    """Eqs. (20)-(22): A = U S V^T, keep sigma_k > tau sigma_1 (READING X4: relative
    cutoff), w = Z^2 V_t (V_t^T Z^2 V_t)^{-1} S_t^{-1} U_t^T b.

    READING: the inverse of V_t^T Z^2 V_t = (Z V_t)^T (Z V_t) is applied through a thin QR
    factorisation Z V_t = Q R, exactly as Section 2 applies (A Z^2 A^T)^{-1} through the
    QR of (A Z)^T (Eq. (7), with its Z^{-1} read as Z): w = Z Q R^{-T} c, c = S_t^{-1} U_t^T b.
    Forming the Gram matrix instead would square its condition number (~1e10 when N_i
    is small at the edge of its support). Returns (w, t, sigma)."""
    U, sig, Vt = np.linalg.svd(A, full_matrices=False)
    t = int(np.sum(sig > tau * sig[0]))
    Ut, st, V = U[:, :t], sig[:t], Vt[:t].T
    c = (Ut.T @ b) / st
    Q, R = np.linalg.qr(z[:, None] * V)
    w = z * (Q @ np.linalg.solve(R.T, c))
    return w, t, sig


def wq_weights(fx, pat, data, gq, families, tau=1e-12, rows=None):
    """Per (row, family) weights aligned with Q_i, plus a report per system."""
    n = fx["n_fn"]
    rows = range(n) if rows is None else rows
    W = {f: np.zeros(len(pat["qidx"])) for f in families}
    rank = {f: np.zeros(n, dtype=np.int64) for f in families}
    resid = {f: np.zeros(n) for f in families}
    for i in rows:
        z = z_diag(fx, pat, data, i)
        S = pat["S"][i]
        for fam in families:
            A = local_matrix(fx, pat, data, i, _FAM_KEY[fam])
            b = np.asarray(gq[_FAM_GQ[fam]][i, S].todense()).reshape(-1)
            w, t, _ = tsvd_solve(A, z, b, tau)
            W[fam][pat["qptr"][i]:pat["qptr"][i + 1]] = w
            rank[fam][i] = t
            nb = np.max(np.abs(b))
            resid[fam][i] = np.max(np.abs(A @ w - b)) / (nb if nb > 0 else 1.0)
    return W, rank, resid


# ----------------------------------------------------------------------------------
# O7  Row-wise assembly (Eqs. (9), (11), (12); Section 6.1 row-by-row formation)
# ----------------------------------------------------------------------------------

def point_values(data, key):
    """Per-point quantity over all points in global point order."""
    return np.concatenate([d[key] for d in data])


def wq_assemble(fx, pat, data, W, kind, coef_pts=None, rows=None):
    """kind: 'mass' (Eq. 9), 'stiffness' (Eq. 11, planar: x and y terms),
    'biharmonic' (Eq. 12). coef_pts: coefficient at every WQ point (None = 1).
    Returns CSR values aligned with pat['col']."""
    n = fx["n_fn"]
    rows = range(n) if rows is None else rows
    vals = np.zeros(len(pat["col"]))
    terms = {"mass": [("mass", "N")], "stiffness": [("x", "Nx"), ("y", "Ny")],
             "biharmonic": [("lap", "Lap")]}[kind]
    if kind == "stiffness" and is_surface(fx):  # the third surface-gradient component
        terms = terms + [("z", "Nz")]
    for i in rows:
        q0, q1 = pat["qptr"][i], pat["qptr"][i + 1]
        c = np.ones(q1 - q0) if coef_pts is None else coef_pts[pat["qidx"][q0:q1]]
        acc = np.zeros(pat["row_ptr"][i + 1] - pat["row_ptr"][i])
        for fam, key in terms:
            A = local_matrix(fx, pat, data, i, key)
            acc += A @ (c * W[fam][q0:q1])
        vals[pat["row_ptr"][i]:pat["row_ptr"][i + 1]] = acc
    return vals


def csr(pat, vals, n):
    return sp.csr_matrix((vals, pat["col"], pat["row_ptr"]), shape=(n, n))


# ----------------------------------------------------------------------------------
# Convenience: the whole WQ setup for a fixture
# ----------------------------------------------------------------------------------

def setup(fx, families=("mass", "x", "y"), tau=1e-12, rows=None):
    cls = classify(fx)
    s = points_per_element(fx, cls)
    cl = cells(fx, s)
    pat = pattern(fx, cl)
    data = wq_points(fx, cl)
    gq = gq_matrices(fx, cl)
    W, rank, resid = wq_weights(fx, pat, data, gq, families, tau, rows)
    return {"cls": cls, "s": s, "cells": cl, "pat": pat, "data": data, "gq": gq,
            "W": W, "rank": rank, "resid": resid}


# ----------------------------------------------------------------------------------
# Row-by-row evaluation for large meshes: the same steps, restricted to sampled rows
# (every row's weights and matrix row depend only on the cells of its support).
# ----------------------------------------------------------------------------------

def row_gauss_rhs(fx, cl, supp_i, S_i, i, fam, cache):
    """b^f_i[l] = integral of D N_i D N_{S_i[l]} by 4x4 Gauss on each cell of supp N_i."""
    gp, gw = gauss4()
    key = _FAM_KEY[fam]
    pos = {int(j): l for l, j in enumerate(S_i)}
    b = np.zeros(len(S_i))
    for c in supp_i:
        if c not in cache:
            f, k = int(cl["elem"][c]), int(cl["sub"][c])
            pts = []
            for bq in range(4):
                for aq in range(4):
                    fn, N, Nx, Ny, Lap, x, dJ = eval_cell(fx, f, k, (gp[aq], gp[bq]), cl["funcs"][c])
                    pts.append((gw[aq] * gw[bq] * abs(dJ), {"N": N, "Nx": Nx, "Ny": Ny, "Lap": Lap}))
            cache[c] = (cl["funcs"][c], pts)
        fn, pts = cache[c]
        ki = int(np.nonzero(fn == i)[0][0])
        for wq_, vals in pts:
            v = vals[key]
            for k, j in enumerate(fn):
                b[pos[int(j)]] += wq_ * v[ki] * v[k]
    return b


def sample_rows(fx, rows, families=("mass", "x", "y"), tau=1e-12, coef=None, glob=None):
    """Everything the method produces for the given rows: S_i, Q_i, the points' coordinates
    x, the system of each family (A_fam, b_fam, z) with its weights, and the mass,
    stiffness and biharmonic rows of the families given (coef: dict kind -> callable of
    x, or None for 1).
    glob: optional precomputed {"cls", "s", "cells"} of the whole mesh."""
    if glob is None:
        cls = classify(fx)
        s = points_per_element(fx, cls)
        glob = {"cls": cls, "s": s, "cells": cells(fx, s)}
    cl = glob["cells"]
    if "supp" not in glob:
        glob["supp"] = supports(fx, cl)
    supp = glob["supp"]
    pat = {"S": {}, "supp": {}}
    for i in rows:
        cols = set()
        for c in supp[i]:
            cols.update(int(j) for j in cl["funcs"][c])
        pat["S"][i] = np.array(sorted(cols), dtype=np.int64)
        pat["supp"][i] = supp[i]
    need = sorted({c for i in rows for c in supp[i]})
    data = {}
    for c in need:
        f, k = int(cl["elem"][c]), int(cl["sub"][c])
        rr = [eval_cell(fx, f, k, eta, cl["funcs"][c]) for eta in cl["eta"][c]]
        data[c] = {"fn": cl["funcs"][c], "N": np.array([r[1] for r in rr]), "Nx": np.array([r[2] for r in rr]),
                   "Ny": np.array([r[3] for r in rr]), "Lap": np.array([r[4] for r in rr]),
                   "x": np.array([r[5] for r in rr]), "detJ": np.array([r[6] for r in rr])}
    gcache = {}
    out = {}
    for i in rows:
        S_i = pat["S"][i]
        z = z_diag(fx, pat, data, i)
        x = np.concatenate([data[c]["x"] for c in supp[i]])
        q = np.concatenate([np.arange(cl["pt_off"][c], cl["pt_off"][c + 1]) for c in supp[i]])
        res = {"S": S_i, "Q": q, "W": {}}
        for fam in families:
            A = local_matrix(fx, pat, data, i, _FAM_KEY[fam])
            b = row_gauss_rhs(fx, cl, supp[i], S_i, i, fam, gcache)
            w, t, _ = tsvd_solve(A, z, b, tau)
            res["W"][fam] = w
            res["b_" + fam] = b
            res["A_" + fam] = A
        res["z"] = z
        res["x"] = x
        cm = np.ones(len(q)) if coef is None or "mass" not in coef else coef["mass"](x)
        ck = np.ones(len(q)) if coef is None or "stiffness" not in coef else coef["stiffness"](x)
        if "mass" in families:
            res["M"] = local_matrix(fx, pat, data, i, "N") @ (cm * res["W"]["mass"])
        if "x" in families and "y" in families:
            res["K"] = (local_matrix(fx, pat, data, i, "Nx") @ (ck * res["W"]["x"])
                        + local_matrix(fx, pat, data, i, "Ny") @ (ck * res["W"]["y"]))
        if "lap" in families:
            cb = np.ones(len(q)) if coef is None or "biharmonic" not in coef else coef["biharmonic"](x)
            res["B"] = local_matrix(fx, pat, data, i, "Lap") @ (cb * res["W"]["lap"])
        out[i] = res
    return out, glob
