"""Adjacency builders for the graph-TV tests (CSR over masked voxels or
vertices; no arithmetic of the method)."""
import numpy as np


def grid_graph(mask, dim=3):
    """CSR adjacency of the masked voxels (grid order) under the 2*dim-neighbourhood."""
    nz, ny, nx = mask.shape
    idx = -np.ones(mask.size, np.int64)
    flat = np.flatnonzero(mask.reshape(-1))
    idx[flat] = np.arange(flat.size)
    rows = []
    for g in flat:
        z, r = divmod(g, ny * nx)
        y, x = divmod(r, nx)
        nb = []
        for dz, dy, dx in [(0, 0, -1), (0, 0, 1), (0, -1, 0), (0, 1, 0), (-1, 0, 0), (1, 0, 0)]:
            if dim == 2 and dz != 0:
                continue
            zz, yy, xx = z + dz, y + dy, x + dx
            if 0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx:
                k = idx[(zz * ny + yy) * nx + xx]
                if k >= 0:
                    nb.append(k)
        rows.append(nb)
    rowptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    col = np.array([k for r in rows for k in r], np.int32)
    return rowptr, col


def random_graph(n, deg, seed):
    """Symmetric random adjacency (no self loops) as CSR."""
    rng = np.random.default_rng(seed)
    adj = [set() for _ in range(n)]
    for i in range(n):
        for j in rng.choice(n, size=deg, replace=False):
            if j != i:
                adj[i].add(int(j))
                adj[int(j)].add(i)
    rowptr = np.concatenate([[0], np.cumsum([len(a) for a in adj])]).astype(np.int64)
    col = np.array([j for a in adj for j in sorted(a)], np.int32)
    return rowptr, col
