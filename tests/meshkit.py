"""Small hand-built problems used by the pin and parity tests."""
import numpy as np

from synth import Problem, meshes
from synth.problems import _rng


def boundary_faces(conn):
    """Facets (edges in 2D, triangles in 3D) that belong to one element only."""
    conn = np.asarray(conn, dtype=np.int64)
    k = conn.shape[1]
    subs = [np.delete(conn, i, axis=1) for i in range(k)]
    f = np.sort(np.concatenate(subs), axis=1)
    u, cnt = np.unique(f, axis=0, return_counts=True)
    return u[cnt == 1]


def patch_2d(n=4, seed=0, jitter=0.2):
    coords, conn = meshes.structured_plate(n, n, _rng(seed), jitter=jitter)
    return coords, conn.astype(np.int32)


def patch_3d(n=3, seed=0, dims=(1.0, 1.0, 1.0), jitter=0.1):
    coords, conn = meshes.kuhn_box(n, n, n, *dims)
    rng = _rng(seed)
    h = min(dims) / n
    inner = np.all((coords > 0) & (coords < np.asarray(dims)), axis=1)
    coords = coords.copy()
    coords[inner] += rng.uniform(-jitter * h, jitter * h, size=(int(inner.sum()), 3))
    coords, conn = meshes._relabel(coords, conn, rng)
    return coords, conn.astype(np.int32)


def make_problem(model, coords, conn, E=1.0, nu=0.3, dir_nodes=(), dir_comps=(),
                 dir_values=(), facets=None, traction=None, n_load_steps=1,
                 param_kind="E_nu", p0=None, p1=None, name="test"):
    d = coords.shape[1]
    ne = conn.shape[0]
    if p0 is None:
        p0 = np.full(ne, E) if np.isscalar(E) else np.asarray(E, dtype=np.float64)
    if p1 is None:
        p1 = np.full(ne, nu) if np.isscalar(nu) else np.asarray(nu, dtype=np.float64)
    if facets is None:
        facets = np.zeros((0, d), np.int32)
        traction = np.zeros((0, d))
    return Problem(name, model, np.asarray(coords, np.float64),
                   np.asarray(conn, np.int32), param_kind, p0, p1,
                   np.asarray(dir_nodes, np.int32), np.asarray(dir_comps, np.int8),
                   np.asarray(dir_values, np.float64),
                   np.asarray(facets, np.int32), np.asarray(traction, np.float64),
                   n_load_steps)


def dirichlet_from_field(nodes, field_fn, coords, d):
    """Dirichlet triples prescribing u = field_fn(x) on ``nodes``."""
    nodes = np.asarray(nodes, dtype=np.int64)
    vals = field_fn(coords[nodes])            # (n, d)
    dn = np.repeat(nodes, d)
    dc = np.tile(np.arange(d), nodes.size)
    return dn, dc, vals.reshape(-1)


def fan_problem(m=70000, model="lin_plane_strain"):
    """m triangles around one centre node (node 0) with the rim on the unit
    circle: under plain RCM the centre is numbered next to one end, so the
    element node offsets exceed 16 bits (unpacked connectivity).  Rim nodes
    1..200 clamped, u_x = 0.01 prescribed on rim nodes m/2 .. m/2 + 200."""
    th = 2.0 * np.pi * np.arange(m) / m
    coords = np.vstack([[0.0, 0.0], np.stack([np.cos(th), np.sin(th)], axis=1)])
    i = np.arange(m)
    conn = np.stack([np.zeros(m, np.int64), 1 + i, 1 + (i + 1) % m], axis=1)
    clamp = np.arange(1, 201)
    pull = np.arange(m // 2, m // 2 + 201)
    dn = np.concatenate([np.repeat(clamp, 2), pull])
    dc = np.concatenate([np.tile([0, 1], clamp.size), np.zeros(pull.size, np.int64)])
    dv = np.concatenate([np.zeros(2 * clamp.size), np.full(pull.size, 0.01)])
    return make_problem(model, coords, conn, dir_nodes=dn, dir_comps=dc, dir_values=dv,
                        name="fan")
