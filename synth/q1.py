"""Q1 (bi/trilinear) finite element linear elasticity (input generator).

Galerkin displacement formulation of App. "Linear elastostatics: Galerkin
finite element formulation" (eq. model_elastostatics_bilin_FE) on a
Cartesian grid of equal elements, with 2 x 2 (x 2) Gauss quadrature (exact
for these elements).  Degrees of freedom are interleaved: dof = d * node + l
for displacement component l, nodes numbered x + (nx+1) (y + (ny+1) z).
Dirichlet conditions use the symmetric diagonalisation of Remark
"FEM_Dir_BC": the row and column of a fixed dof are zeroed, its diagonal
is kept, the right-hand side there is A_ii g_i.  The matrix keeps the full
pattern (3^d neighbouring nodes times d components per row, zeros
included), so every row of a grid interior looks alike.

Like the MPFA-O matrix this is an input of the method: both the CPU oracle
and the GPU library receive the CSR matrix built here.
"""
import itertools

import numpy as np
import scipy.sparse as sp

from .fields import gaussian_smoothed


def lame(E, nu):
    """Lame parameters (lambda, mu = G) of Young's modulus E and Poisson's
    ratio nu."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def _shape_gradients(h, point):
    """Physical gradients (2^d, d) of the Q1 shape functions on an element of
    sizes h at reference point in [-1, 1]^d; local node q has corner bits
    (q >> k) & 1 per axis k."""
    d = len(h)
    nloc = 1 << d
    g = np.zeros((nloc, d))
    for q in range(nloc):
        s = [1.0 if (q >> k) & 1 else -1.0 for k in range(d)]
        for k in range(d):
            v = s[k] / 2.0
            for m in range(d):
                if m != k:
                    v *= (1.0 + s[m] * point[m]) / 2.0
            g[q, k] = v * 2.0 / h[k]      # d xi / d x = 2 / h
    return g


def element_stiffness(h, nu, E=1.0):
    """(d 2^d) x (d 2^d) stiffness of one element, dofs ordered d*q + l."""
    d = len(h)
    lam, mu = lame(E, nu)
    nv = 3 if d == 2 else 6
    D = np.zeros((nv, nv))
    D[:d, :d] = lam
    D[np.arange(d), np.arange(d)] += 2.0 * mu
    D[np.arange(d, nv), np.arange(d, nv)] = mu
    # engineering shear strains: pairs (a, b) in Voigt order
    shear = [(0, 1)] if d == 2 else [(1, 2), (0, 2), (0, 1)]
    nloc = 1 << d
    K = np.zeros((d * nloc, d * nloc))
    gp = 1.0 / np.sqrt(3.0)
    detJ = np.prod(h) / (1 << d)
    for point in itertools.product((-gp, gp), repeat=d):
        G = _shape_gradients(h, point)
        B = np.zeros((nv, d * nloc))
        for q in range(nloc):
            for k in range(d):
                B[k, d * q + k] = G[q, k]
            for r, (a, b) in enumerate(shear):
                B[d + r, d * q + a] = G[q, b]
                B[d + r, d * q + b] = G[q, a]
        K += B.T @ D @ B * detJ
    return K


def q1_elasticity(elems, h, E, nu, fixed=None):
    """Assemble the stiffness matrix on `elems` elements per axis of sizes
    `h`, element moduli E (x fastest, one per element), Poisson ratio nu.
    `fixed`: boolean per dof (or None) for homogeneous Dirichlet conditions.
    Returns CSR (rowptr, col, val) with sorted columns."""
    d = len(elems)
    nodes = tuple(e + 1 for e in elems)
    nn = int(np.prod(nodes))
    nloc = 1 << d
    K0 = element_stiffness(h, nu)
    Eg = np.asarray(E, dtype=np.float64).reshape(tuple(reversed(elems)))
    offs = list(itertools.product((-1, 0, 1), repeat=d))        # (dz, dy, dx) / (dy, dx)
    oidx = {o: t for t, o in enumerate(offs)}
    # blocks[t][node] = coupling block (d x d) of node with node + offs[t]
    blocks = np.zeros((len(offs),) + tuple(reversed(nodes)) + (d, d))
    for qi in range(nloc):
        bi = [(qi >> k) & 1 for k in range(d)]                   # x, y, (z)
        for qj in range(nloc):
            bj = [(qj >> k) & 1 for k in range(d)]
            delta = tuple(bj[k] - bi[k] for k in reversed(range(d)))
            sl = tuple(slice(bi[k], bi[k] + elems[k]) for k in reversed(range(d)))
            blk = K0[d * qi:d * qi + d, d * qj:d * qj + d]
            blocks[(oidx[delta],) + sl] += Eg[..., None, None] * blk
    # CSR: row (node, l) lists neighbours in ascending node index (offsets in
    # lexicographic (dz, dy, dx) order), d components each
    coords = np.stack(np.meshgrid(*[np.arange(m) for m in reversed(nodes)], indexing="ij"),
                      axis=-1).reshape(-1, d)                     # (nn, d) as (z, y, x)
    strides = np.cumprod((1,) + tuple(nodes[:-1]))[::-1]          # for (z, y, x)
    valid = np.zeros((nn, len(offs)), dtype=bool)
    for t, o in enumerate(offs):
        c = coords + np.array(o)
        valid[:, t] = np.all((c >= 0) & (c < np.array(tuple(reversed(nodes)))), axis=1)
    cnt = valid.sum(axis=1) * d                                   # per row of node
    rowcnt = np.repeat(cnt, d)
    rp = np.zeros(nn * d + 1, dtype=np.int64)
    rp[1:] = np.cumsum(rowcnt)
    blk = blocks.reshape(len(offs), nn, d, d)                      # (t, node, l, m)
    node_off = np.array([int(np.dot(o, strides)) for o in offs])
    # (node, l, t, m) layout, masked by valid[node, t]
    vals = np.transpose(blk, (1, 2, 0, 3))
    colnode = np.arange(nn)[:, None] + node_off[None, :]          # (node, t)
    cols = (d * colnode[:, None, :, None] + np.arange(d)[None, None, None, :])
    cols = np.broadcast_to(cols, (nn, d, len(offs), d))
    mask = np.broadcast_to(valid[:, None, :, None], (nn, d, len(offs), d))
    ci = cols[mask].astype(np.int32)
    a = vals[mask].astype(np.float64)
    # element sums reach A_ij and A_ji in different orders: average the two
    # so the matrix is symmetric to the bit (the pattern is symmetric)
    At = sp.csr_matrix((a, ci, rp), shape=(nn * d, nn * d)).T.tocsr()
    At.sort_indices()
    assert np.array_equal(At.indices, ci) and np.array_equal(At.indptr, rp)
    a = 0.5 * (a + At.data)
    if fixed is not None:
        fixed = np.asarray(fixed, dtype=bool)
        row = np.repeat(np.arange(nn * d), rowcnt)
        kill = (fixed[row] | fixed[ci]) & (row != ci)
        a = np.where(kill, 0.0, a)
    return rp.astype(np.int32), ci, a


def q1_case(elems, rng, sigma=1.5, corr=8.0, nu=0.25):
    """The 3D elasticity workload on the unit cube: log E = sigma g with g
    Gaussian-smoothed white noise (std `corr` elements, standardised), the
    z = 0 face fixed, a unit downward traction on z = 1 with consistent
    nodal loads."""
    assert len(elems) == 3
    nx, ny, nz = elems
    h = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    logE = sigma * gaussian_smoothed(elems, corr, rng)
    nodes = (nx + 1, ny + 1, nz + 1)
    nn = int(np.prod(nodes))
    z = np.arange(nn) // (nodes[0] * nodes[1])
    fixed = np.repeat(z == 0, 3)
    rp, ci, a = q1_elasticity(elems, h, np.exp(logE), nu, fixed)
    # traction (0, 0, -1) on the top face: each face quad puts a quarter of
    # its area on each of its corners
    f = np.zeros(3 * nn)
    top = np.zeros((ny + 1, nx + 1))
    top[:-1, :-1] += 1
    top[1:, :-1] += 1
    top[:-1, 1:] += 1
    top[1:, 1:] += 1
    top_nodes = np.arange(nn)[z == nz]
    f[3 * top_nodes + 2] = -0.25 * h[0] * h[1] * top.ravel()
    return dict(logE=logE, matrix=(rp, ci, a), rhs=f, fixed=fixed, h=h, nu=nu)
