"""Synthetic simplicial meshes for the volume-constrained problem.

Every generator returns a :class:`Mesh` whose first ``n_dofs`` nodes are the
nodes strictly inside the interior region (the unknowns of the problem, Sec. 2.3
of the paper), followed by the nodes on the interface and in the exterior
region.  Cells are stored structure-of-arrays: ``cells[a, c]`` is vertex ``a`` of
cell ``c``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    dim: int
    coords: np.ndarray          # (dim, M) float64
    cells: np.ndarray           # (dim+1, n_cells) int32
    cell_interior: np.ndarray   # (n_cells,) uint8, 1 if the cell lies in the interior region
    n_dofs: int                 # N: nodes [0, N) are interior
    exterior_radius: float = 0.0  # R > 0: the exterior continues beyond the ball of radius R
    info: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[1])

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[1])

    def h_max(self) -> float:
        """Largest cell diameter."""
        x = self.coords[:, self.cells]          # (dim, dim+1, nc)
        best = 0.0
        k = self.dim + 1
        for a in range(k):
            for b in range(a + 1, k):
                d = np.sqrt(((x[:, a] - x[:, b]) ** 2).sum(axis=0)).max()
                best = max(best, float(d))
        return best


def _renumber(is_dof: np.ndarray):
    """Return old->new map that puts the dof nodes first (stable)."""
    order = np.concatenate([np.flatnonzero(is_dof), np.flatnonzero(~is_dof)])
    new_of_old = np.empty_like(order)
    new_of_old[order] = np.arange(order.size)
    return order, new_of_old


def interval_mesh(n_int: int, n_ext: int, lo: float = -1.0, hi: float = 1.0,
                  exterior_radius: float = 0.0) -> Mesh:
    """Uniform P1 mesh of (lo - n_ext h, hi + n_ext h), interior (lo, hi), h=(hi-lo)/n_int."""
    h = (hi - lo) / n_int
    n_tot = n_int + 2 * n_ext
    x = lo - n_ext * h + h * np.arange(n_tot + 1, dtype=np.float64)
    idx = np.arange(n_tot + 1)
    is_dof = (idx > n_ext) & (idx < n_ext + n_int)
    order, new = _renumber(is_dof)
    coords = x[order][None, :].copy()
    c = np.arange(n_tot)
    cells = np.stack([new[c], new[c + 1]]).astype(np.int32)
    interior = ((c >= n_ext) & (c < n_ext + n_int)).astype(np.uint8)
    return Mesh(1, coords, cells, interior, int(is_dof.sum()), float(exterior_radius),
                {"h": h, "kind": "interval", "n_int": n_int, "n_ext": n_ext})


def square_mesh(n: int, pad: int, jitter: float = 0.0, seed: int = 0,
                lo: float = 0.0, hi: float = 1.0) -> Mesh:
    """Interior (lo,hi)^2 with n x n squares, padded by ``pad`` squares of the same size.

    Each square (i,j)-(i+1,j)-(i+1,j+1)-(i,j+1) is split along the same diagonal
    into (A,B,C) and (A,C,D).  Interior nodes are displaced by U(-jitter*h,
    jitter*h) per coordinate, drawn from ``numpy.random.default_rng(seed)`` in
    dof order.
    """
    h = (hi - lo) / n
    m = n + 2 * pad
    i, j = np.meshgrid(np.arange(m + 1), np.arange(m + 1), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    xy = np.stack([lo + (i - pad) * h, lo + (j - pad) * h]).astype(np.float64)
    is_dof = (i > pad) & (i < pad + n) & (j > pad) & (j < pad + n)
    order, new = _renumber(is_dof)
    coords = xy[:, order].copy()
    n_dofs = int(is_dof.sum())
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        coords[:, :n_dofs] += rng.uniform(-jitter * h, jitter * h, size=(n_dofs, 2)).T

    def nid(a, b):
        return new[a * (m + 1) + b]

    si, sj = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    si = si.ravel()
    sj = sj.ravel()
    A = nid(si, sj)
    B = nid(si + 1, sj)
    C = nid(si + 1, sj + 1)
    D = nid(si, sj + 1)
    t1 = np.stack([A, B, C])
    t2 = np.stack([A, C, D])
    cells = np.empty((3, 2 * si.size), dtype=np.int32)
    cells[:, 0::2] = t1
    cells[:, 1::2] = t2
    sq_int = (si >= pad) & (si < pad + n) & (sj >= pad) & (sj < pad + n)
    interior = np.repeat(sq_int, 2).astype(np.uint8)
    return Mesh(2, coords, cells, interior, n_dofs, 0.0,
                {"h": h, "kind": "square", "n": n, "pad": pad, "jitter": jitter, "seed": seed})


def graded_band(h: float, width: float, q: float) -> np.ndarray:
    """Offsets 0 < t_1 < ... < t_m = width of the exterior grid lines beyond an interface:
    the first layer has the interior spacing h, each next one q times the previous, and the
    graded part is scaled so that the last line lands on ``width``."""
    w = [h]
    while sum(w) < width:
        w.append(w[-1] * q)
    t = np.cumsum(w)
    if len(w) > 1:   # keep the first layer at h, stretch the others to end at width
        t[1:] = h + (t[1:] - h) * (width - h) / (t[-1] - h)
    else:
        t[:] = width
    return t


def square_mesh_graded(n: int, width: float, q: float, jitter: float = 0.0, seed: int = 0,
                       lo: float = 0.0, hi: float = 1.0) -> Mesh:
    """Interior (lo,hi)^2 with n x n squares inside a band of the given width whose grid lines
    are graded geometrically away from the interface (``graded_band``), so that the exterior
    has O(log) instead of O(n) layers.  Squares are split along the same diagonal as in
    ``square_mesh``; interior nodes are jittered the same way."""
    h = (hi - lo) / n
    t = graded_band(h, width, q)
    g = np.concatenate([lo - t[::-1], lo + h * np.arange(n + 1), hi + t])
    m = g.size - 1
    pad = t.size
    i, j = np.meshgrid(np.arange(m + 1), np.arange(m + 1), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    xy = np.stack([g[i], g[j]]).astype(np.float64)
    is_dof = (i > pad) & (i < pad + n) & (j > pad) & (j < pad + n)
    order, new = _renumber(is_dof)
    coords = xy[:, order].copy()
    n_dofs = int(is_dof.sum())
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        coords[:, :n_dofs] += rng.uniform(-jitter * h, jitter * h, size=(n_dofs, 2)).T

    def nid(a, b):
        return new[a * (m + 1) + b]

    si, sj = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    si = si.ravel()
    sj = sj.ravel()
    t1 = np.stack([nid(si, sj), nid(si + 1, sj), nid(si + 1, sj + 1)])
    t2 = np.stack([nid(si, sj), nid(si + 1, sj + 1), nid(si, sj + 1)])
    cells = np.empty((3, 2 * si.size), dtype=np.int32)
    cells[:, 0::2] = t1
    cells[:, 1::2] = t2
    sq_int = (si >= pad) & (si < pad + n) & (sj >= pad) & (sj < pad + n)
    interior = np.repeat(sq_int, 2).astype(np.uint8)
    return Mesh(2, coords, cells, interior, n_dofs, 0.0,
                {"h": h, "kind": "square_graded", "n": n, "layers": pad, "q": q, "width": width,
                 "jitter": jitter, "seed": seed})


def disk_mesh(n: int, layers: int, radius_out: float, exterior_radius: float = 0.0) -> Mesh:
    """Unit disk from the elliptical square-to-disk map of an n x n grid, plus an annulus.

    The grid on [-1,1]^2 is mapped by (u,v) -> (u sqrt(1-v^2/2), v sqrt(1-u^2/2)),
    which sends the square's boundary onto the unit circle.  The annulus
    1 < |x| < radius_out is meshed by ``layers`` rings of nodes placed on the
    rays through the 4n boundary nodes; each ring quad is split into two
    triangles.  ``exterior_radius`` > 0 declares that the exterior continues
    beyond |x| = exterior_radius (normally radius_out).
    """
    g = np.linspace(-1.0, 1.0, n + 1)
    u, v = np.meshgrid(g, g, indexing="ij")
    X = u * np.sqrt(1.0 - v * v / 2.0)
    Y = v * np.sqrt(1.0 - u * u / 2.0)
    gid = np.arange((n + 1) ** 2).reshape(n + 1, n + 1)
    # boundary loop of the grid, counter-clockwise starting at (n, 0)... as index list
    loop = []
    for jj in range(0, n):            # right edge, bottom to top (i = n)
        loop.append(gid[n, jj])
    for ii in range(n, 0, -1):        # top edge, right to left (j = n)
        loop.append(gid[ii, n])
    for jj in range(n, 0, -1):        # left edge, top to bottom (i = 0)
        loop.append(gid[0, jj])
    for ii in range(0, n):            # bottom edge, left to right (j = 0)
        loop.append(gid[ii, 0])
    loop = np.array(loop)
    nb = loop.size                    # 4n
    xs = [X.ravel(), Y.ravel()]
    bx = X.ravel()[loop]
    by = Y.ravel()[loop]
    ring_ids = [loop]
    next_id = (n + 1) ** 2
    px = [xs[0]]
    py = [xs[1]]
    for k in range(1, layers + 1):
        r = 1.0 + (radius_out - 1.0) * k / layers
        px.append(bx * r)
        py.append(by * r)
        ring_ids.append(next_id + np.arange(nb))
        next_id += nb
    xy = np.stack([np.concatenate(px), np.concatenate(py)])
    # grid triangles
    si, sj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    si = si.ravel()
    sj = sj.ravel()
    A = gid[si, sj]
    B = gid[si + 1, sj]
    C = gid[si + 1, sj + 1]
    D = gid[si, sj + 1]
    tri = [np.stack([A, B, C]), np.stack([A, C, D])]
    n_int_cells = 2 * si.size
    for k in range(layers):
        r0 = ring_ids[k]
        r1 = ring_ids[k + 1]
        a = r0
        b = np.roll(r0, -1)
        c = np.roll(r1, -1)
        d = r1
        tri.append(np.stack([a, b, c]))
        tri.append(np.stack([a, c, d]))
    cells_old = np.concatenate(tri, axis=1)
    interior = np.zeros(cells_old.shape[1], dtype=np.uint8)
    interior[:n_int_cells] = 1
    is_dof = np.zeros(xy.shape[1], dtype=bool)
    is_dof[: (n + 1) ** 2] = True
    is_dof[loop] = False
    order, new = _renumber(is_dof)
    coords = xy[:, order].copy()
    cells = new[cells_old].astype(np.int32)
    # make every triangle counter-clockwise (orientation is irrelevant to the method,
    # but keeps the generated meshes uniform)
    p = coords[:, cells]
    det = (p[0, 1] - p[0, 0]) * (p[1, 2] - p[1, 0]) - (p[1, 1] - p[1, 0]) * (p[0, 2] - p[0, 0])
    flip = det < 0
    cells[1, flip], cells[2, flip] = cells[2, flip].copy(), cells[1, flip].copy()
    return Mesh(2, coords, cells, interior, int(is_dof.sum()), float(exterior_radius),
                {"h": 2.0 / n, "kind": "disk", "n": n, "layers": layers, "radius_out": radius_out})


def grid_values(mesh: Mesh, u_dofs: np.ndarray):
    """Nodal values of a P1 function on the full node grid of a ``square_mesh`` without
    jitter: returns (G, idx) with G[i, k] the value at grid node (i, k) (zero off the dofs)
    and idx (2, M) the grid index of every mesh node."""
    h = mesh.info["h"]
    lo = mesh.coords.min(axis=1)
    full = np.zeros(mesh.n_nodes)
    full[:mesh.n_dofs] = u_dofs
    idx = np.rint((mesh.coords - lo[:, None]) / h).astype(np.int64)
    G = np.zeros((idx[0].max() + 1, idx[1].max() + 1))
    G[idx[0], idx[1]] = full
    return G, idx


def prolong_p1(Gc: np.ndarray) -> np.ndarray:
    """P1 interpolation of grid values onto the grid of half the spacing.  The squares are
    split along the diagonal (i, k)-(i+1, k+1), so a square's centre lies on that edge and
    takes the mean of its two end nodes."""
    n1, n2 = Gc.shape
    Gf = np.zeros((2 * n1 - 1, 2 * n2 - 1))
    Gf[0::2, 0::2] = Gc
    Gf[1::2, 0::2] = 0.5 * (Gc[:-1, :] + Gc[1:, :])
    Gf[0::2, 1::2] = 0.5 * (Gc[:, :-1] + Gc[:, 1:])
    Gf[1::2, 1::2] = 0.5 * (Gc[:-1, :-1] + Gc[1:, 1:])
    return Gf
