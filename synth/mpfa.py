"""MPFA-O flow matrices on perturbed 2D quadrilateral grids (input generator).

The multipoint flux approximation O-method (Sec. "MsRSB for non-M matrices",
App. "Incompressible single-phase flow: finite volume formulation", flux
split eq. num_flux_split) computes the flux over every half-edge from the
pressures of the cells sharing the half-edge's vertex.  Around each grid
vertex (its interaction region) the pressure in every adjacent cell is taken
linear, fixed by the cell-centre pressure and by one continuity pressure at
the midpoint of each of the two half-edges of that cell meeting at the
vertex.  Requiring the normal flux -nu . K grad p to agree on both sides of
every interior half-edge (and to vanish on no-flow boundary half-edges)
eliminates the continuity pressures and leaves transmissibilities that
express each half-edge flux through the cell pressures of the region.

The matrix is what the method consumes, so it is generated here and handed
to both the CPU oracle and the GPU library as a CSR matrix.  Row K of A
holds the net outflow of cell K (positive diagonal), matching the bilinear
form of eq. model_flow_bilin_FV.
"""
import numpy as np
import scipy.sparse as sp


def perturbed_nodes(dims, rng, amplitude=0.2, lengths=(1.0, 1.0)):
    """Node coordinates, shape (ny+1, nx+1, 2), of a structured grid of
    dims = (nx, ny) cells on [0, Lx] x [0, Ly]; interior nodes are moved by
    amplitude * U(-1/2, 1/2) * (cell size) in x and in y independently."""
    nx, ny = dims
    hx, hy = lengths[0] / nx, lengths[1] / ny
    xs = np.arange(nx + 1) * hx
    ys = np.arange(ny + 1) * hy
    X = np.empty((ny + 1, nx + 1, 2))
    X[..., 0] = xs[None, :]
    X[..., 1] = ys[:, None]
    if amplitude != 0.0:
        d = rng.uniform(-0.5, 0.5, size=(ny - 1, nx - 1, 2))
        X[1:-1, 1:-1, 0] += amplitude * hx * d[..., 0]
        X[1:-1, 1:-1, 1] += amplitude * hy * d[..., 1]
    return X


def rotated_tensors(logk, ratio=100.0, angle_deg=30.0):
    """K_c = exp(logk_c) * R diag(ratio, 1) R^T with R the rotation by
    angle_deg; shape (n, 2, 2)."""
    a = np.deg2rad(angle_deg)
    R = np.array([[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]])
    base = R @ np.diag([ratio, 1.0]) @ R.T
    return np.exp(logk)[:, None, None] * base[None]


def _cell_centres(X):
    return 0.25 * (X[:-1, :-1] + X[:-1, 1:] + X[1:, 1:] + X[1:, :-1])


def mpfa_o(X, K):
    """Assemble the MPFA-O matrix (no-flow on the whole boundary).

    X: node coordinates (ny+1, nx+1, 2); K: per-cell tensors (nx*ny, 2, 2),
    cells numbered x + nx*y.  Returns CSR (rowptr, col, val) with sorted
    columns; every row has the full 9-point pattern of its neighbourhood."""
    rp, ci, val, _ = mpfa_o_bc(X, K, None)
    return rp, ci, val


def mpfa_o_bc(X, K, dirichlet):
    """MPFA-O with Dirichlet data on some domain sides.

    dirichlet maps a side ("xlo", "xhi", "ylo", "yhi") to a function g(x, y)
    (or a constant); the other sides are no-flow.  On a Dirichlet half-edge
    the continuity pressure of the interaction region is g at the half-edge's
    midpoint, and the half-edge's outflow enters its cell's balance; the part
    of it that does not depend on the cell pressures goes to the right-hand
    side.  Returns (rowptr, col, val, rhs) with A p = rhs."""
    dirichlet = dirichlet or {}
    ny, nx = X.shape[0] - 1, X.shape[1] - 1
    xc = _cell_centres(X)
    rhs = np.zeros(nx * ny)

    def cell(i, j):
        return i + nx * j if (0 <= i < nx and 0 <= j < ny) else -1

    def gval(side, x):
        g = dirichlet[side]
        return float(g(x[0], x[1])) if callable(g) else float(g)

    rows, cols, vals = [], [], []
    for j in range(ny + 1):
        for i in range(nx + 1):
            v = X[j, i]
            # half-edges at the vertex: (far node, first cell, second cell,
            # domain side if on the boundary); the flux orientation runs from
            # the first to the second cell
            edges = []
            if i >= 1:   # west: horizontal edge, cells below / above
                edges.append((X[j, i - 1], cell(i - 1, j - 1), cell(i - 1, j),
                              "ylo" if j == 0 else ("yhi" if j == ny else None)))
            if i < nx:   # east
                edges.append((X[j, i + 1], cell(i, j - 1), cell(i, j),
                              "ylo" if j == 0 else ("yhi" if j == ny else None)))
            if j >= 1:   # south: vertical edge, cells left / right
                edges.append((X[j - 1, i], cell(i - 1, j - 1), cell(i, j - 1),
                              "xlo" if i == 0 else ("xhi" if i == nx else None)))
            if j < ny:   # north
                edges.append((X[j + 1, i], cell(i - 1, j), cell(i, j),
                              "xlo" if i == 0 else ("xhi" if i == nx else None)))
            cells = sorted({c for _, a, b, _ in edges for c in (a, b) if c >= 0})
            has_dir = any(sd in dirichlet for _, _, _, sd in edges)
            if len(cells) < 2 and not has_dir:
                continue  # a no-flow domain corner: no flux at all
            ne, ncl = len(edges), len(cells)
            cpos = {c: q for q, c in enumerate(cells)}
            mid = [0.5 * (v + far) for far, _, _, _ in edges]
            # normal of each half-edge (length = half-edge length), pointing
            # from the first cell to the second one
            xcf = xc.reshape(-1, 2)
            nu = []
            for e, (far, a, b, _) in enumerate(edges):
                t = mid[e] - v
                nrm = np.array([t[1], -t[0]])
                if a >= 0 and b >= 0 and nrm @ (xcf[b] - xcf[a]) < 0:
                    nrm = -nrm
                nu.append(nrm)
            # per cell: its two half-edges and the gradient operator
            cell_edges = {c: [e for e, (_, a, b, _) in enumerate(edges) if c in (a, b)]
                          for c in cells}
            # flux of half-edge e seen from cell c: coefficients on u (ne) and p (ncl)
            def flux_row(c, e):
                ea, eb = cell_edges[c]
                xk = xcf[c]
                M = np.array([mid[ea] - xk, mid[eb] - xk])
                G = np.linalg.inv(M)             # grad = G [u_a - p_c, u_b - p_c]
                w = -(nu[e] @ K[c] @ G)          # flux = w . [u_a - p_c, u_b - p_c]
                cu = np.zeros(ne)
                cp = np.zeros(ncl)
                cu[ea] += w[0]
                cu[eb] += w[1]
                cp[cpos[c]] -= w[0] + w[1]
                return cu, cp
            Cu = np.zeros((ne, ne))
            Cp = np.zeros((ne, ncl))
            bu = np.zeros(ne)
            for e, (_, a, b, sd) in enumerate(edges):
                if a >= 0 and b >= 0:    # continuity of the flux
                    ua, pa = flux_row(a, e)
                    ub, pb = flux_row(b, e)
                    Cu[e], Cp[e] = ua - ub, pa - pb
                elif sd in dirichlet:    # the half-edge pressure is given
                    Cu[e, e] = 1.0
                    bu[e] = gval(sd, mid[e])
                else:                    # no-flow boundary half-edge
                    Cu[e], Cp[e] = flux_row(a if a >= 0 else b, e)
            # Cu u + Cp p = bu  =>  u = U p + u0
            U = -np.linalg.solve(Cu, Cp)
            u0 = np.linalg.solve(Cu, bu)
            for e, (_, a, b, sd) in enumerate(edges):
                if a >= 0 and b >= 0:
                    fu, fp = flux_row(a, e)
                    T = fu @ U + fp              # flux from a to b = T . p + t0
                    t0 = fu @ u0
                    for q, c in enumerate(cells):
                        rows += [a, b]
                        cols += [c, c]
                        vals += [T[q], -T[q]]
                    rhs[a] -= t0
                    rhs[b] += t0
                elif sd in dirichlet:            # outflow of the cell through e
                    c0 = a if a >= 0 else b
                    fu, fp = flux_row(c0, e)
                    sgn = 1.0 if nu[e] @ (mid[e] - xcf[c0]) > 0 else -1.0
                    T = sgn * (fu @ U + fp)
                    for q, c in enumerate(cells):
                        rows.append(c0)
                        cols.append(c)
                        vals.append(T[q])
                    rhs[c0] -= sgn * (fu @ u0)
    n = nx * ny
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return (A.indptr.astype(np.int32), A.indices.astype(np.int32),
            A.data.astype(np.float64), rhs)


def mpfa_case(dims, rng):
    """The 2D MPFA-O workload: perturbed unit-square grid, rotated 100:1
    log-normal tensor (sigma 2), unit source in cell (0,0) and a p = 0 well
    in the opposite corner cell whose index equals that cell's diagonal."""
    nx, ny = dims
    X = perturbed_nodes(dims, rng, 0.2)
    logk = 2.0 * rng.standard_normal(nx * ny)
    K = rotated_tensors(logk)
    rp, ci, val = mpfa_o(X, K)
    val = val.copy()
    sink = nx * ny - 1
    d = rp[sink] + int(np.nonzero(ci[rp[sink]:rp[sink + 1]] == sink)[0][0])
    val[d] *= 2.0            # well index = the cell's own diagonal, p_well = 0
    f = np.zeros(nx * ny)
    f[0] = 1.0
    return dict(nodes=X, logk=logk, matrix=(rp, ci, val), rhs=f)


def e2_case(dims, rng, lengths=(20.0, 150.0)):
    """The 2D MPFA-O test of Sec. 3.2: a 20 m x 150 m rectangle (x by y) of
    dims cells (100 x 100 in the paper), interior vertices moved by
    0.2 Psi times the cell size in x and in y, Psi ~ U(-1/2, 1/2), the
    homogeneous tensor lambda_xx = lambda_yy = 100, lambda_xy = 25, and a
    unit pressure drop from x = 0 (p = 1) to x = 20 m (p = 0); no flow on the
    other two sides."""
    nx, ny = dims
    X = perturbed_nodes(dims, rng, 0.2, lengths=lengths)
    K = np.array([[100.0, 25.0], [25.0, 100.0]])[None].repeat(nx * ny, 0)
    rp, ci, val, f = mpfa_o_bc(X, K, {"xlo": 1.0, "xhi": 0.0})
    return dict(nodes=X, matrix=(rp, ci, val), rhs=f)
