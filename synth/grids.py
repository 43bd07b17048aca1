"""Coarse partitions and support regions on Cartesian grids.

The paper defines the coarse grid structure in words (Sec. 2.1, Fig. 1):
a primal partition with one coarse node per coarse block; support boundary
cells connect neighbouring coarse nodes; support edge cells connect a coarse
node to its neighbours.  On a Cartesian grid we read this as follows.

Cell-centred (finite volume).  Along each axis with N cells and block size
b, coarse node a sits in cell c_a = a*b + floor(b/2).  The support of node a
along that axis is the open interval (c_{a-1}, c_{a+1}) with c_{-1} = -1 and
c_m = N at the domain ends; in d dimensions the support is the tensor
product.  A fine row's pattern is the sorted list of coarse nodes whose
support contains it (at most 2^d).  Cells lying on a node plane of any axis
form the global boundary; every other cell is interior and counts in e_it.

Vertex-centred (finite element).  Along an axis with N elements (N+1
nodes), coarse vertex a sits at node v_a = a*b.  Its support is the open
interval (v_{a-1}, v_{a+1}) with the ends extended past the domain.  The
initial basis assigns node x to the nearest coarse vertex (ties to the
higher vertex; floor((2x + b) / (2b)) where the spacing is b).  Nodes on a coarse
element face (x = v_a on some axis) are not interior.
"""
import numpy as np


def tensor_index(coords, dims):
    """Linear index x + nx*(y + ny*z) of integer coordinate arrays."""
    idx = np.zeros_like(np.asarray(coords[0]), dtype=np.int64)
    for d in reversed(range(len(dims))):
        idx = idx * dims[d] + np.asarray(coords[d], dtype=np.int64)
    return idx


def _axis_cells(N, b):
    m = -(-N // b)
    nodes = np.minimum(np.arange(m) * b + b // 2, N - 1)
    lo = np.concatenate([[-1], nodes[:-1]])
    hi = np.concatenate([nodes[1:], [N]])
    x = np.arange(N)
    member = (x[:, None] > lo[None, :]) & (x[:, None] < hi[None, :])
    part = np.minimum(x // b, m - 1)
    on_node = np.isin(x, nodes)
    return m, member, part, on_node


def _axis_vertices(N, b):
    M = -(-N // b)
    verts = np.minimum(np.arange(M + 1) * b, N)
    lo = np.concatenate([[-1], verts[:-1]])
    hi = np.concatenate([verts[1:], [N + 1]])
    x = np.arange(N + 1)
    member = (x[:, None] > lo[None, :]) & (x[:, None] < hi[None, :])
    # nearest coarse vertex, ties to the higher one (equal to
    # floor((2x + b) / 2b) where the spacing is b; also right for a shorter
    # last coarse element)
    dist = np.abs(x[:, None] - verts[None, :])
    part = verts.size - 1 - np.argmin(dist[:, ::-1], axis=1)
    on_vert = np.isin(x, verts)
    return M + 1, member, part, on_vert


def _tensor_supports(axes):
    """Combine per-axis (m, member, part, on_plane) into a row pattern CSR."""
    dim = len(axes)
    ms = [a[0] for a in axes]
    Ns = [a[1].shape[0] for a in axes]
    mem_idx, mem_cnt = [], []
    for (m, member, part, on) in axes:
        cnt = member.sum(axis=1)
        assert cnt.max() <= 2 and cnt.min() >= 1
        idx = np.full((member.shape[0], 2), -1, dtype=np.int64)
        for x in range(member.shape[0]):
            w = np.nonzero(member[x])[0]
            idx[x, :len(w)] = w
        mem_idx.append(idx)
        mem_cnt.append(cnt)
    grids = np.meshgrid(*[np.arange(N) for N in reversed(Ns)], indexing="ij")
    coords = [g.ravel() for g in reversed(grids)]  # x fastest
    n = coords[0].size
    cand = []
    valid = []
    for combo in range(1 << dim):
        sel = [(combo >> d) & 1 for d in range(dim)]
        ok = np.ones(n, dtype=bool)
        cc = np.zeros(n, dtype=np.int64)
        for d in reversed(range(dim)):
            s = sel[d]
            ok &= s < mem_cnt[d][coords[d]]
            cc = cc * ms[d] + np.where(ok, mem_idx[d][coords[d], s], 0)
        cand.append(np.where(ok, cc, np.iinfo(np.int64).max))
        valid.append(ok)
    cand = np.sort(np.stack(cand, axis=1), axis=1)
    cnt = np.stack(valid, axis=1).sum(axis=1)
    prp = np.zeros(n + 1, dtype=np.int32)
    prp[1:] = np.cumsum(cnt)
    pci = cand[np.arange(cand.shape[1])[None, :] < cnt[:, None]].astype(np.int32)
    part = tensor_index([axes[d][2][coords[d]] for d in range(dim)], ms).astype(np.int32)
    on = np.zeros(n, dtype=bool)
    for d in range(dim):
        on |= axes[d][3][coords[d]]
    interior = (~on).astype(np.uint8)
    nc = int(np.prod(ms))
    return dict(nc=nc, part=part, prp=prp, pci=pci, interior=interior,
                coarse_dims=tuple(ms))


def cell_supports(dims, block):
    """Cell-centred coarse partition and supports for a grid of `dims` cells
    with coarse blocks of `block` cells per axis (int or per-axis tuple)."""
    if np.isscalar(block):
        block = (block,) * len(dims)
    return _tensor_supports([_axis_cells(N, b) for N, b in zip(dims, block)])


def vertex_supports(elems, block):
    """Vertex-centred partition and supports for a grid with `elems`
    elements per axis (elems+1 nodes) and coarse elements of `block`."""
    if np.isscalar(block):
        block = (block,) * len(elems)
    return _tensor_supports([_axis_vertices(N, b) for N, b in zip(elems, block)])


def vector_supports(sup, bs):
    """Block-diagonal (per displacement component) supports: dof bs*i + l
    couples to coarse dofs bs*j + l for j in node i's pattern."""
    prp, pci = sup["prp"], sup["pci"].astype(np.int64)
    n = prp.size - 1
    cnt = np.diff(prp)
    dof_cnt = np.repeat(cnt, bs)
    dprp = np.zeros(n * bs + 1, dtype=np.int32)
    dprp[1:] = np.cumsum(dof_cnt)
    # entries of dof (i, l) are bs*pci[prp[i]:prp[i+1]] + l
    rows = np.repeat(np.arange(n), cnt)
    ent = np.empty(dprp[-1], dtype=np.int32)
    for l in range(bs):
        # position of dof (i, l)'s block inside the dof CSR
        start = dprp[bs * np.arange(n) + l]
        off = np.arange(prp[-1]) - prp[rows]
        ent[start[rows] + off] = bs * pci + l
    part = (bs * sup["part"].astype(np.int64)[:, None] + np.arange(bs)[None, :]).ravel()
    interior = np.repeat(sup["interior"], bs)
    return dict(nc=sup["nc"] * bs, part=part.astype(np.int32), prp=dprp, pci=ent,
                interior=interior.astype(np.uint8), coarse_dims=sup["coarse_dims"],
                block_size=bs)
