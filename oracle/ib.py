"""Immersed boundary coupling: DIBM, FODIBM and FODIBM-R, FP64, on the CPU.

Test infrastructure only (see oracle/__init__.py).

Follows Secs. 2.3-2.5 of the paper:
  Eq. (12)  two-sided interpolation over Omega (DIBM; projection points with d = 1)
  Eq. (14)  one-sided interpolation over Omega' with the scaling factor phi_l
  Eq. (15)  one-sided spreading with phi_l W_l
  Eq. (16)  phi_l = 1 / sum_{Omega'} delta
  Eq. (17)  improved Lagrangian weight W_l
  Eqs. (18-19) tensor-product cosine kernel, radius d = 2 for markers
  Eqs. (20-22) forces with the boundary targets (DIBM / FODIBM)
  Eq. (25)  effective boundary position X*_l
  Eqs. (27), (29) Dirichlet / Neumann target reconstruction at the virtual point
  Eqs. (30-32) FODIBM-R forces
  Sec. 2.5  order of the five sub-steps

Readings of the paper taken here:
  * Omega' is the closed interior: node i is inside iff (x_i - X_l*) . n_l* <= 0
    where l* is the marker nearest to x_i (ties: lowest index); FP64, products
    and sums left to right.
  * Kernel support is strict: |x_ia - X_la| < d on every axis.
  * A marker whose interior support is empty is inactive (phi = 0).
  * d_BV = |X_l - X*_l| (Euclidean), d_PB = d_n = 1.5, P_l = X_l + d_n n_l.
  * In two dimensions the kernel is the product over two axes.
"""
from dataclasses import dataclass

import numpy as np

from .lbm import predicted_macros

DIBM, FODIBM, FODIBM_R = 0, 1, 2
KERNEL_COS, KERNEL_ROMA3 = 0, 1
D_N = 1.5          # d_n / dx, Sec. 2.3
T_NONE, T_DIRICHLET, T_NEUMANN = 0, 1, 2


def cos_kernel(r, d):
    """Eq. (19): (1/(2d)) [1 + cos(pi r / d)] for |r| <= d, 0 otherwise."""
    r = np.asarray(r, dtype=np.float64)
    return np.where(np.abs(r) <= d, (1.0 + np.cos(np.pi * r / d)) / (2.0 * d), 0.0)


def roma3_kernel(r):
    """Three-point kernel of Roma, Peskin & Berger (1999); selectable instead of Eq. (19)."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    inner = (1.0 + np.sqrt(np.maximum(1.0 - 3.0 * a * a, 0.0))) / 3.0
    outer = (5.0 - 3.0 * a - np.sqrt(np.maximum(1.0 - 3.0 * (1.0 - a) ** 2, 0.0))) / 6.0
    return np.where(a <= 0.5, inner, np.where(a <= 1.5, outer, 0.0))


def kernel_radius(kind):
    return 2.0 if kind == KERNEL_COS else 1.5


def kernel_1d(kind, r):
    return cos_kernel(r, 2.0) if kind == KERNEL_COS else roma3_kernel(r)


def linear_index(nodes, dims):
    """x + nx (y + ny z) for integer node coordinates (n, D).

    The map does not wrap: a stencil that leaves the grid is refused (ValueError), as the
    library refuses markers within 3 cells of an edge."""
    nodes = np.asarray(nodes, dtype=np.int64)
    hi = np.asarray(dims, dtype=np.int64)[:nodes.shape[1]]
    if nodes.size and (np.any(nodes < 0) or np.any(nodes >= hi)):
        raise ValueError('marker stencil leaves the grid')
    lin = nodes[:, -1].copy()
    for a in range(nodes.shape[1] - 2, -1, -1):
        lin = lin * dims[a] + nodes[:, a]
    return lin


def box_nodes(center, radius):
    """Integer nodes with |x_a - center_a| < radius on every axis (strict), x fastest."""
    axes = []
    for c in center:
        lo = int(np.ceil(c - radius))
        hi = int(np.floor(c + radius))
        cand = np.arange(lo, hi + 1)
        axes.append(cand[np.abs(cand.astype(np.float64) - c) < radius])
    grids = np.meshgrid(*axes[::-1], indexing='ij')          # slowest axis first
    pts = np.stack([g.ravel() for g in grids[::-1]], axis=1)   # columns x, y[, z]
    return pts


def sq_dist_and_dot(node, X, n):
    """Squared distances and normal projections from a node to every marker, left-to-right sums."""
    d0 = node[0] - X[:, 0]
    dd = d0 * d0
    dot = d0 * n[:, 0]
    for a in range(1, X.shape[1]):
        da = node[a] - X[:, a]
        dd = dd + da * da
        dot = dot + da * n[:, a]
    return dd, dot


def interior_flags(nodes, X, n):
    """Closed-interior test of each node against its nearest marker."""
    nodes = np.asarray(nodes, dtype=np.float64)
    out = np.zeros(len(nodes), dtype=bool)
    for k, p in enumerate(nodes):
        dd, dot = sq_dist_and_dot(p, X, n)
        l = int(np.argmin(dd))
        out[k] = dot[l] <= 0.0
    return out


@dataclass
class Geometry:
    D: int
    dims: tuple
    method: int
    kernel: int
    X: np.ndarray
    n: np.ndarray
    supp_nodes: list      # per marker: (s, D) integer nodes of S'_l (Omega' or Omega), x fastest
    supp_lin: list        # per marker: linear node indices
    supp_w: list          # per marker: delta_il
    phi: np.ndarray
    active: np.ndarray
    Xstar: np.ndarray
    dBV: np.ndarray
    W: np.ndarray
    P: np.ndarray
    proj_lin: list        # per marker: linear indices of the d = 1 support of P
    proj_w: list
    rows: np.ndarray      # CSR row node (linear index), ascending
    row_ptr: np.ndarray
    col_marker: np.ndarray
    col_s: np.ndarray     # s_ik = phi_k delta_ik W_k
    interior_lin: np.ndarray   # candidate nodes flagged interior (FODIBM modes), ascending


def build_geometry(dims, X, n, method=FODIBM_R, kernel=KERNEL_COS):
    """Per-geometry precompute: supports, phi (Eq. 16), X* (Eq. 25), d_BV, W (Eq. 17), CSR.

    dims = (nx, ny[, nz]); X, n: (M, D) marker positions and outward unit normals.
    """
    X = np.asarray(X, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    M, D = X.shape
    radius = kernel_radius(kernel)
    boxes = [box_nodes(X[l], radius) for l in range(M)]

    one_sided = method in (FODIBM, FODIBM_R)
    if one_sided:
        allnodes = np.unique(np.concatenate([linear_index(b, dims) for b in boxes]))
        coords = np.stack(np.unravel_index(allnodes, tuple(dims[::-1]))[::-1], axis=1)
        flags = interior_flags(coords, X, n)
        interior = set(allnodes[flags].tolist())
        interior_lin = allnodes[flags]
    else:
        interior = None
        interior_lin = np.zeros(0, dtype=np.int64)

    supp_nodes, supp_lin, supp_w = [], [], []
    for l in range(M):
        b = boxes[l]
        lin = linear_index(b, dims)
        if one_sided:
            keep = np.array([v in interior for v in lin.tolist()], dtype=bool)
            b, lin = b[keep], lin[keep]
        w = np.ones(len(b))
        for a in range(D):
            w = w * kernel_1d(kernel, b[:, a].astype(np.float64) - X[l, a])
        supp_nodes.append(b)
        supp_lin.append(lin)
        supp_w.append(w)

    phi = np.zeros(M)
    Xstar = X.copy()
    for l in range(M):
        s = supp_w[l].sum()
        if s > 0.0:
            phi[l] = 1.0 / s if one_sided else 1.0
            Xstar[l] = phi[l] * (supp_nodes[l].astype(np.float64) * supp_w[l][:, None]).sum(axis=0)
    active = phi > 0.0
    dBV = np.sqrt(((X - Xstar) ** 2).sum(axis=1))

    # Node density sum_k phi_k delta_ik, then W_l of Eq. (17).
    density = {}
    for l in range(M):
        for v, wv in zip(supp_lin[l].tolist(), supp_w[l].tolist()):
            density[v] = density.get(v, 0.0) + phi[l] * wv
    W = np.zeros(M)
    for l in range(M):
        if active[l]:
            tot = sum(phi[l] * wv * density[v] for v, wv in zip(supp_lin[l].tolist(), supp_w[l].tolist()))
            W[l] = 1.0 / tot

    # Node -> marker CSR of the spreading weights s_ik = phi_k delta_ik W_k (Eq. 15).
    entries = {}
    for l in range(M):
        if not active[l]:
            continue
        for v, wv in zip(supp_lin[l].tolist(), supp_w[l].tolist()):
            entries.setdefault(v, []).append((l, phi[l] * wv * W[l]))
    rows = np.array(sorted(entries), dtype=np.int64)
    row_ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    cols, svals = [], []
    for r, v in enumerate(rows.tolist()):
        ent = sorted(entries[v])
        cols += [e[0] for e in ent]
        svals += [e[1] for e in ent]
        row_ptr[r + 1] = len(cols)

    # Projection points and their two-sided d = 1 cosine support (Sec. 2.3).
    P = X + D_N * n
    proj_lin, proj_w = [], []
    for l in range(M):
        b = box_nodes(P[l], 1.0)
        w = np.ones(len(b))
        for a in range(D):
            w = w * cos_kernel(b[:, a].astype(np.float64) - P[l, a], 1.0)
        proj_lin.append(linear_index(b, dims))
        proj_w.append(w)

    return Geometry(D=D, dims=tuple(dims), method=method, kernel=kernel, X=X, n=n,
                    supp_nodes=supp_nodes, supp_lin=supp_lin, supp_w=supp_w, phi=phi, active=active,
                    Xstar=Xstar, dBV=dBV, W=W, P=P, proj_lin=proj_lin, proj_w=proj_w,
                    rows=rows, row_ptr=row_ptr, col_marker=np.array(cols, dtype=np.int64),
                    col_s=np.array(svals), interior_lin=interior_lin)


def two_sided_interp_lists(dims, points, radius=2.0):
    """Eq. (12) supports and weights at arbitrary points (phi = 1, all nodes)."""
    lins, ws = [], []
    D = points.shape[1]
    for p in points:
        b = box_nodes(p, radius)
        w = np.ones(len(b))
        for a in range(D):
            w = w * cos_kernel(b[:, a].astype(np.float64) - p[a], radius)
        lins.append(linear_index(b, dims))
        ws.append(w)
    return lins, ws


@dataclass
class Markers:
    """Boundary data per marker: wall velocity u^Bt, thermal kind and value."""
    u_wall: np.ndarray    # (M, D)
    t_kind: np.ndarray    # (M,) 0 none, 1 Dirichlet (T_w), 2 Neumann (dT/dn)
    t_value: np.ndarray   # (M,)


def marker_forces(geom, mk, prm, rho, j, ustar, T):
    """Sec. 2.5 steps 1-3 for every marker, from flattened predicted fields.

    Returns a dict with the interpolated values and the Lagrangian forces
    F (M, D), Wib (M,), Qib (M,). Inactive markers get zero forces.
    """
    M, D = geom.X.shape
    out = {k: np.zeros((M, D)) for k in ('F', 'j', 'u', 'uP', 'ut')}
    out.update({k: np.zeros(M) for k in ('Wib', 'Qib', 'rho', 'T', 'TP', 'Tt')})
    for l in range(M):
        if not geom.active[l]:
            continue
        idx, w, ph = geom.supp_lin[l], geom.supp_w[l], geom.phi[l]
        # Eq. (14) (phi = 1 and Omega for DIBM, Eq. (12))
        r_l = ph * (rho[idx] * w).sum()
        j_l = ph * (j[:, idx] * w).sum(axis=1)
        u_l = ph * (ustar[:, idx] * w).sum(axis=1)
        T_l = ph * (T[idx] * w).sum()
        # Eq. (12) with d = 1 at the projection point
        pi, pw = geom.proj_lin[l], geom.proj_w[l]
        uP = (ustar[:, pi] * pw).sum(axis=1)
        TP = (T[pi] * pw).sum()
        ub = mk.u_wall[l]
        kind, tv = int(mk.t_kind[l]), mk.t_value[l]
        if geom.method == FODIBM_R:
            ratio = geom.dBV[l] / D_N
            ut = ub - ratio * (uP - ub)                                    # Eq. (27)
            if kind == T_DIRICHLET:
                Tt = tv - ratio * (TP - tv)                                # Eq. (27)
            elif kind == T_NEUMANN:
                Tt = TP - tv * (D_N + geom.dBV[l])                         # Eq. (29)
            else:
                Tt = T_l
        else:
            ut = ub.copy()
            if kind == T_DIRICHLET:
                Tt = tv
            elif kind == T_NEUMANN:
                Tt = TP - tv * D_N
            else:
                Tt = T_l
        out['F'][l] = 2.0 * (r_l * ut - j_l)                                 # Eqs. (20)/(30)
        out['Wib'][l] = r_l * ((ut * ut).sum() - (u_l * u_l).sum()) / 2.0     # Eqs. (21)/(31)
        out['Qib'][l] = prm.Cv * r_l * (Tt - T_l) if kind != T_NONE else 0.0  # Eqs. (22)/(32)
        out['rho'][l], out['j'][l], out['u'][l], out['T'][l] = r_l, j_l, u_l, T_l
        out['uP'][l], out['TP'][l], out['ut'][l], out['Tt'][l] = uP, TP, ut, Tt
    return out


def spread(geom, F, G):
    """Eq. (15) through the node -> marker CSR: g_i = sum_k s_ik G_k.

    F: (M, D) momentum forces, G: (M,) energy forces W + Q.
    Returns per-row arrays fib (rows, D) and fE (rows,).
    """
    nrow = len(geom.rows)
    D = geom.D
    fib = np.zeros((nrow, D))
    fE = np.zeros(nrow)
    for r in range(nrow):
        a, b = geom.row_ptr[r], geom.row_ptr[r + 1]
        k = geom.col_marker[a:b]
        s = geom.col_s[a:b]
        fib[r] = (s[:, None] * F[k]).sum(axis=0)
        fE[r] = (s * G[k]).sum()
    return fib, fE


def ib_step_forcing(lat, prm, geom, mk, st):
    """Sec. 2.5 steps 1-4: Eulerian forcing fields (fib (D, *grid), fE (*grid)) for the state."""
    D = lat.D
    grid = st.rhoE.shape
    rho, j, u, T = predicted_macros(lat, prm, st.f, st.rhoE)
    flat = lambda a: a.reshape(a.shape[:a.ndim - D] + (-1,))
    mf = marker_forces(geom, mk, prm, flat(rho), flat(j), flat(u), flat(T))
    fib_r, fE_r = spread(geom, mf['F'], mf['Wib'] + mf['Qib'])
    fib = np.zeros((D, int(np.prod(grid))))
    fE = np.zeros(int(np.prod(grid)))
    fib[:, geom.rows] = fib_r.T
    fE[geom.rows] = fE_r
    return fib.reshape((D,) + grid), fE.reshape(grid), mf


__all__ = ['DIBM', 'FODIBM', 'FODIBM_R', 'KERNEL_COS', 'KERNEL_ROMA3', 'D_N', 'T_NONE', 'T_DIRICHLET',
           'T_NEUMANN', 'cos_kernel', 'roma3_kernel', 'box_nodes', 'linear_index', 'interior_flags',
           'Geometry', 'build_geometry', 'two_sided_interp_lists', 'Markers', 'marker_forces', 'spread',
           'ib_step_forcing']
