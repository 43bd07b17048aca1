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
    ny, nx = X.shape[0] - 1, X.shape[1] - 1
    xc = _cell_centres(X)

    def cell(i, j):
        return i + nx * j if (0 <= i < nx and 0 <= j < ny) else -1

    rows, cols, vals = [], [], []
    for j in range(ny + 1):
        for i in range(nx + 1):
            v = X[j, i]
            # half-edges at the vertex: (far node, first cell, second cell);
            # the flux orientation runs from the first to the second cell
            edges = []
            if i >= 1:   # west: horizontal edge, cells below / above
                edges.append((X[j, i - 1], cell(i - 1, j - 1), cell(i - 1, j)))
            if i < nx:   # east
                edges.append((X[j, i + 1], cell(i, j - 1), cell(i, j)))
            if j >= 1:   # south: vertical edge, cells left / right
                edges.append((X[j - 1, i], cell(i - 1, j - 1), cell(i, j - 1)))
            if j < ny:   # north
                edges.append((X[j + 1, i], cell(i - 1, j), cell(i, j)))
            cells = sorted({c for _, a, b in edges for c in (a, b) if c >= 0})
            if len(cells) < 2:
                continue  # a domain corner: no interior half-edge
            ne, ncl = len(edges), len(cells)
            cpos = {c: q for q, c in enumerate(cells)}
            mid = [0.5 * (v + far) for far, _, _ in edges]
            # normal of each half-edge (length = half-edge length), pointing
            # from the first cell to the second one
            xcf = xc.reshape(-1, 2)
            nu = []
            for e, (far, a, b) in enumerate(edges):
                t = mid[e] - v
                nrm = np.array([t[1], -t[0]])
                if a >= 0 and b >= 0 and nrm @ (xcf[b] - xcf[a]) < 0:
                    nrm = -nrm
                nu.append(nrm)
            # per cell: its two half-edges and the gradient operator
            cell_edges = {c: [e for e, (_, a, b) in enumerate(edges) if c in (a, b)] for c in cells}
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
            for e, (_, a, b) in enumerate(edges):
                if a >= 0 and b >= 0:    # continuity of the flux
                    ua, pa = flux_row(a, e)
                    ub, pb = flux_row(b, e)
                    Cu[e], Cp[e] = ua - ub, pa - pb
                else:                    # no-flow boundary half-edge
                    Cu[e], Cp[e] = flux_row(a if a >= 0 else b, e)
            # Cu u + Cp p = 0  =>  u = -Cu^{-1} Cp p
            U = -np.linalg.solve(Cu, Cp)
            for e, (_, a, b) in enumerate(edges):
                if a < 0 or b < 0:
                    continue
                fu, fp = flux_row(a, e)
                T = fu @ U + fp                  # flux from a to b = T . p
                for q, c in enumerate(cells):
                    rows += [a, b]
                    cols += [c, c]
                    vals += [T[q], -T[q]]
    n = nx * ny
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return (A.indptr.astype(np.int32), A.indices.astype(np.int32),
            A.data.astype(np.float64))


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
