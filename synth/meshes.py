"""Seeded P1 mesh generators: triangles in 2D, tetrahedra in 3D.

Geometry only: node coordinates (float64, node-major) and element
connectivity (int32, one row per element).  Element orientation is left as
the generator produces it; consumers accept either sign of the Jacobian.
"""
import numpy as np
from scipy.spatial import Delaunay
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _compact(coords, conn):
    """Drop nodes that no element references; renumber densely."""
    used = np.zeros(coords.shape[0], dtype=bool)
    used[conn.reshape(-1)] = True
    new_id = np.cumsum(used) - 1
    return coords[used].copy(), new_id[conn].astype(np.int32)


def _relabel(coords, conn, rng):
    """Random node relabelling and element shuffle (so ordering has work)."""
    n = coords.shape[0]
    perm = rng.permutation(n)           # old -> new
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    coords2 = coords[inv]
    conn2 = perm[conn].astype(np.int32)
    conn2 = conn2[rng.permutation(conn2.shape[0])]
    return np.ascontiguousarray(coords2), np.ascontiguousarray(conn2)


# ---------------------------------------------------------------- 2D meshes
def grid_triangles(n=33):
    """Structured n x n node grid on the unit square, two triangles per cell.

    Node id = j*n + i at (i/(n-1), j/(n-1)).  Cells are visited row by row
    (j outer, i inner); cell (i, j) gives the lower triangle
    (n_ij, n_i+1,j, n_i+1,j+1) followed by the upper one
    (n_ij, n_i+1,j+1, n_i,j+1).
    """
    t = np.linspace(0.0, 1.0, n)
    X, Y = np.meshgrid(t, t)                      # [j, i]
    coords = np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)
    i, j = np.meshgrid(np.arange(n - 1), np.arange(n - 1))
    i = i.reshape(-1)
    j = j.reshape(-1)
    a = j * n + i
    b = j * n + i + 1
    c = (j + 1) * n + i + 1
    d = (j + 1) * n + i
    lower = np.stack([a, b, c], axis=1)
    upper = np.stack([a, c, d], axis=1)
    conn = np.stack([lower, upper], axis=1).reshape(-1, 3).astype(np.int32)
    return coords, conn


def sample_holes(rng, n_holes, rmin=0.03, rmax=0.08, gap=0.02, margin=0.02,
                 max_tries=100000):
    """Non-overlapping circular holes inside the unit square."""
    holes = []
    tries = 0
    while len(holes) < n_holes:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place holes")
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(r + margin, 1.0 - r - margin, size=2)
        if all(np.hypot(*(c - hc)) >= r + hr + gap for hc, hr in holes):
            holes.append((c, r))
    return holes


def plate_with_holes(rng, n_holes, target_tris):
    """Unit plate with circular holes: jittered triangular lattice + Delaunay.

    Returns coords (N, 2), conn (E, 3), holes list [(centre, radius)].
    Boundary points are placed exactly on the square's edges (so y == 0 and
    y == 1 identify the bottom and top edges) and on each hole circle.
    """
    holes = sample_holes(rng, n_holes)
    area = 1.0 - sum(np.pi * r * r for _, r in holes)
    n_pts = max(target_tris / 2.0, 50.0)
    h = np.sqrt(area / (n_pts * np.sqrt(3.0) / 2.0))
    dy = h * np.sqrt(3.0) / 2.0
    ny = int(np.floor(1.0 / dy)) + 1
    nx = int(np.floor(1.0 / h)) + 2
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    px = ii * h + (jj % 2) * 0.5 * h
    py = jj * dy
    pts = np.stack([px.reshape(-1), py.reshape(-1)], axis=1)
    pts += rng.uniform(-0.08 * h, 0.08 * h, size=pts.shape)
    keep = ((pts[:, 0] > 0.55 * h) & (pts[:, 0] < 1.0 - 0.55 * h) &
            (pts[:, 1] > 0.55 * h) & (pts[:, 1] < 1.0 - 0.55 * h))
    for c, r in holes:
        keep &= np.hypot(pts[:, 0] - c[0], pts[:, 1] - c[1]) > r + 0.6 * h
    pts = pts[keep]
    ne = max(int(round(1.0 / h)), 2)
    s = np.arange(ne) / ne
    edge = np.concatenate([
        np.stack([s, np.zeros(ne)], 1),          # bottom, from (0,0)
        np.stack([np.ones(ne), s], 1),           # right, from (1,0)
        np.stack([1.0 - s, np.ones(ne)], 1),     # top, from (1,1)
        np.stack([np.zeros(ne), 1.0 - s], 1),    # left, from (0,1)
    ])
    circ = []
    for c, r in holes:
        nc = max(12, int(round(2.0 * np.pi * r / h)))
        th = rng.uniform(0, 2 * np.pi) + 2.0 * np.pi * np.arange(nc) / nc
        circ.append(np.stack([c[0] + r * np.cos(th), c[1] + r * np.sin(th)], 1))
    allp = np.concatenate([edge] + circ + [pts])
    tri = Delaunay(allp).simplices.astype(np.int64)
    cen = allp[tri].mean(axis=1)
    keep = np.ones(tri.shape[0], dtype=bool)
    for c, r in holes:
        keep &= np.hypot(cen[:, 0] - c[0], cen[:, 1] - c[1]) > r
    tri = tri[keep]
    coords, conn = _compact(allp, tri)
    return coords, conn, holes


def structured_plate(nx, ny, rng, jitter=0.1):
    """Unit square, nx x ny cells, two triangles per cell, jittered interior
    nodes, random relabelling.  Cheap at tens of millions of triangles."""
    tx = np.linspace(0.0, 1.0, nx + 1)
    ty = np.linspace(0.0, 1.0, ny + 1)
    X, Y = np.meshgrid(tx, ty)
    coords = np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)
    interior = ((coords[:, 0] > 0) & (coords[:, 0] < 1) &
                (coords[:, 1] > 0) & (coords[:, 1] < 1))
    hmin = min(1.0 / nx, 1.0 / ny)
    coords[interior] += rng.uniform(-jitter * hmin, jitter * hmin,
                                    size=(int(interior.sum()), 2))
    i, j = np.meshgrid(np.arange(nx, dtype=np.int64),
                       np.arange(ny, dtype=np.int64))
    i = i.reshape(-1)
    j = j.reshape(-1)
    w = nx + 1
    a = j * w + i
    b = a + 1
    c = a + w + 1
    d = a + w
    # alternate the diagonal so the mesh is not a single repeated stencil
    flip = ((i + j) % 2) == 1
    t1 = np.where(flip[:, None], np.stack([a, b, d], 1), np.stack([a, b, c], 1))
    t2 = np.where(flip[:, None], np.stack([b, c, d], 1), np.stack([a, c, d], 1))
    conn = np.stack([t1, t2], axis=1).reshape(-1, 3)
    return _relabel(coords, conn, rng)


# ---------------------------------------------------------------- 3D meshes
_KUHN = None


def _kuhn_pattern():
    """The 6 Kuhn tetrahedra of the unit cube, as corner bit-indices.

    Corner c has offset (c & 1, (c >> 1) & 1, (c >> 2) & 1).  Each tetrahedron
    walks from corner 0 to corner 7 along one permutation of the three axes;
    using the same pattern in every cell gives a conforming mesh.
    """
    global _KUHN
    if _KUHN is None:
        perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
        tets = []
        for p in perms:
            c0 = 0
            c1 = c0 | (1 << p[0])
            c2 = c1 | (1 << p[1])
            tets.append((c0, c1, c2, 7))
        _KUHN = np.array(tets, dtype=np.int64)
    return _KUHN


def kuhn_box(nx, ny, nz, lx, ly, lz):
    """Hex grid of nx*ny*nz cells on [0,lx]x[0,ly]x[0,lz], 6 tets per cell."""
    gx = np.linspace(0, lx, nx + 1)
    gy = np.linspace(0, ly, ny + 1)
    gz = np.linspace(0, lz, nz + 1)
    Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
    coords = np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)
    k, j, i = np.meshgrid(np.arange(nz, dtype=np.int64),
                          np.arange(ny, dtype=np.int64),
                          np.arange(nx, dtype=np.int64), indexing="ij")
    base = (i + (nx + 1) * (j + (ny + 1) * k)).reshape(-1)
    corner_off = np.array([(c & 1) + (nx + 1) * (((c >> 1) & 1) +
                           (ny + 1) * ((c >> 2) & 1)) for c in range(8)],
                          dtype=np.int64)
    pat = _kuhn_pattern()
    conn = base[:, None, None] + corner_off[pat][None, :, :]
    return coords, conn.reshape(-1, 4)


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([
        [a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
        [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
        [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


def sample_voids(rng, n_voids, dims, smin=0.05, smax=0.15, face_gap=0.03,
                 gap=0.02, max_tries=200000):
    """Non-overlapping ellipsoids (bounding-sphere test) inside a box."""
    voids = []
    tries = 0
    dims = np.asarray(dims, dtype=np.float64)
    while len(voids) < n_voids:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place voids")
        s = rng.uniform(smin, smax, size=3)
        R = _random_rotation(rng)
        rb = s.max()
        lo = rb + face_gap
        c = rng.uniform(lo, dims - lo)
        if all(np.linalg.norm(c - vc) >= rb + vr + gap for vc, _, _, vr in voids):
            voids.append((c, s, R, rb))
    return voids


def _face_component(conn):
    """Label face-connected components of a tetrahedral mesh."""
    ne = conn.shape[0]
    faces = np.concatenate([conn[:, [1, 2, 3]], conn[:, [0, 2, 3]],
                            conn[:, [0, 1, 3]], conn[:, [0, 1, 2]]])
    faces = np.sort(faces, axis=1)
    owner = np.tile(np.arange(ne), 4)
    order = np.lexsort((faces[:, 2], faces[:, 1], faces[:, 0]))
    fs = faces[order]
    same = np.all(fs[1:] == fs[:-1], axis=1)
    a = owner[order][:-1][same]
    b = owner[order][1:][same]
    g = coo_matrix((np.ones(a.size), (a, b)), shape=(ne, ne))
    return connected_components(g, directed=False)[1]


def box_with_voids(rng, n_per_unit, n_voids, dims=(1.0, 1.0, 4.0), jitter=0.08):
    """Box with ellipsoidal voids on a Kuhn tetrahedral grid.

    Tetrahedra whose centroid lies inside a void are removed; only the
    largest face-connected component is kept (so no piece hangs by an edge
    or a vertex); interior nodes are jittered by up to ``jitter`` * h.
    Outer-face nodes keep exact coordinates (x, y in {0, 1}, z in {0, lz}).
    """
    nx = max(int(round(n_per_unit * dims[0])), 1)
    ny = max(int(round(n_per_unit * dims[1])), 1)
    nz = max(int(round(n_per_unit * dims[2])), 1)
    coords, conn = kuhn_box(nx, ny, nz, *dims)
    voids = sample_voids(rng, n_voids, dims)
    cen = coords[conn].mean(axis=1)
    keep = np.ones(conn.shape[0], dtype=bool)
    for c, s, R, _ in voids:
        loc = (cen - c) @ R            # coordinates in the void's frame
        keep &= ((loc / s) ** 2).sum(axis=1) >= 1.0
    conn = conn[keep]
    lab = _face_component(conn)
    big = np.bincount(lab).argmax()
    conn = conn[lab == big]
    coords, conn = _compact(coords, conn)
    h = min(dims[0] / nx, dims[1] / ny, dims[2] / nz)
    on_face = ((coords[:, 0] <= 0) | (coords[:, 0] >= dims[0]) |
               (coords[:, 1] <= 0) | (coords[:, 1] >= dims[1]) |
               (coords[:, 2] <= 0) | (coords[:, 2] >= dims[2]))
    inner = ~on_face
    coords[inner] += rng.uniform(-jitter * h, jitter * h,
                                 size=(int(inner.sum()), 3))
    coords, conn = _relabel(coords, conn, rng)
    return coords, conn, voids


def structured_box(nx, ny, nz, rng, dims=(1.0, 1.0, 4.0), jitter=0.08):
    """Void-free Kuhn box with jitter and random relabelling (size sweeps)."""
    coords, conn = kuhn_box(nx, ny, nz, *dims)
    h = min(dims[0] / nx, dims[1] / ny, dims[2] / nz)
    on_face = ((coords[:, 0] <= 0) | (coords[:, 0] >= dims[0]) |
               (coords[:, 1] <= 0) | (coords[:, 1] >= dims[1]) |
               (coords[:, 2] <= 0) | (coords[:, 2] >= dims[2]))
    inner = ~on_face
    coords[inner] += rng.uniform(-jitter * h, jitter * h,
                                 size=(int(inner.sum()), 3))
    return _relabel(coords, conn.astype(np.int64), rng)


# ---------------------------------------------------- quadrilateral meshes
def quad_grid(nx, ny, mapping, elem="q4", rng=None):
    """Structured nx x ny quadrilateral mesh of the image of [0,1]^2 under
    ``mapping`` ((N, 2) parameters -> (N, 2) points, orientation-preserving).

    Q4: corner nodes; Q8: corners, then the midside nodes of edges (0,1),
    (1,2), (2,3), (3,0) of each element, placed at the image of the
    parameter-space midpoint.  Returns coords, conn and the node ids of the
    left (u = 0) and right (u = 1) edges sorted by v: for Q8 the right-edge
    list alternates corner, midside, corner, ...  With ``rng`` the nodes are
    relabelled and the elements shuffled."""
    ci = lambda i, j: j * (nx + 1) + i                               # corners
    nc = (nx + 1) * (ny + 1)
    u, v = np.meshgrid(np.arange(nx + 1) / nx, np.arange(ny + 1) / ny, indexing="xy")
    par = [np.stack([u.ravel(), v.ravel()], axis=1)]
    I, J = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    I, J = I.ravel(), J.ravel()
    corners = np.stack([ci(I, J), ci(I + 1, J), ci(I + 1, J + 1), ci(I, J + 1)], axis=1)
    left = [ci(0, j) for j in range(ny + 1)]
    right = [ci(nx, j) for j in range(ny + 1)]
    if elem == "q8":
        hi = lambda i, j: nc + j * nx + i                            # edge (i,j)-(i+1,j)
        nh = nx * (ny + 1)
        vi = lambda i, j: nc + nh + j * (nx + 1) + i                 # edge (i,j)-(i,j+1)
        hu, hv = np.meshgrid((np.arange(nx) + 0.5) / nx, np.arange(ny + 1) / ny, indexing="xy")
        vu, vv = np.meshgrid(np.arange(nx + 1) / nx, (np.arange(ny) + 0.5) / ny, indexing="xy")
        par += [np.stack([hu.ravel(), hv.ravel()], axis=1),
                np.stack([vu.ravel(), vv.ravel()], axis=1)]
        mids = np.stack([hi(I, J), vi(I + 1, J), hi(I, J + 1), vi(I, J)], axis=1)
        conn = np.concatenate([corners, mids], axis=1)
        left = [x for j in range(ny) for x in (ci(0, j), vi(0, j))] + [ci(0, ny)]
        right = [x for j in range(ny) for x in (ci(nx, j), vi(nx, j))] + [ci(nx, ny)]
    else:
        conn = corners
    coords = np.ascontiguousarray(mapping(np.concatenate(par, axis=0)), dtype=np.float64)
    conn = conn.astype(np.int32)
    left, right = np.asarray(left, np.int64), np.asarray(right, np.int64)
    if rng is not None:
        n = coords.shape[0]
        perm = rng.permutation(n)
        inv = np.empty(n, dtype=np.int64)
        inv[perm] = np.arange(n)
        coords = np.ascontiguousarray(coords[inv])
        conn = np.ascontiguousarray(perm[conn][rng.permutation(conn.shape[0])].astype(np.int32))
        left, right = perm[left], perm[right]
    return coords, conn, left.astype(np.int32), right.astype(np.int32)


def rectangle_map(W, H):
    """[0,1]^2 -> [0, W] x [0, H]."""
    return lambda p: np.stack([W * p[:, 0], H * p[:, 1]], axis=1)


def cook_map(left_height=44.0, right_low=44.0, right_high=60.0, width=48.0):
    """Bilinear map of [0,1]^2 onto Cook's tapered membrane: left edge from
    (0, 0) to (0, left_height), right edge from (width, right_low) to
    (width, right_high)."""
    def f(p):
        s, t = p[:, 0], p[:, 1]
        y_lo = s * right_low
        y_hi = left_height + s * (right_high - left_height)
        return np.stack([width * s, y_lo + t * (y_hi - y_lo)], axis=1)
    return f
