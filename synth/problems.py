"""Problem descriptions: mesh + material + boundary sets, for every workload.

A ``Problem`` carries exactly what a user hands to a finite-element solver:
node coordinates, element connectivity, per-element material parameters,
the Dirichlet set (node, component, final value), the Neumann set (boundary
facets with a constant traction each) and the number of load steps.  How
those become stiffness, forces or solutions is not decided here.

Material parameters are given as the workload states them:
``param_kind == "E_nu"`` -> (p0, p1) = (Young's modulus, Poisson ratio);
``param_kind == "lame"`` -> (p0, p1) = (mu, lambda).
"""
from dataclasses import dataclass, field
import numpy as np

from . import meshes
from .fields import rff_field, lifting_weight

MODELS = ("lin_plane_stress", "lin_plane_strain", "lin_3d",
          "nh_plane_strain", "nh_3d")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Problem:
    name: str
    model: str
    coords: np.ndarray            # (N_n, d) float64
    conn: np.ndarray              # (N_e, d+1) int32 (P1); (N_e, 4 | 8) quadrilaterals
    param_kind: str               # "E_nu" | "lame"
    p0: np.ndarray                # (N_e,) float64
    p1: np.ndarray                # (N_e,) float64
    dir_nodes: np.ndarray         # (n_D,) int32
    dir_comps: np.ndarray         # (n_D,) int8
    dir_values: np.ndarray        # (n_D,) float64, final-load values
    neu_facets: np.ndarray        # (n_F, d) int32; Q8 edges: (n_F, 3) ends, then middle
    neu_traction: np.ndarray      # (n_F, d) float64
    n_load_steps: int = 1
    meta: dict = field(default_factory=dict)
    elem: str = "p1"              # "p1" (triangles / tetrahedra), "q4", "q8"

    @property
    def dim(self):
        return self.coords.shape[1]

    @property
    def n_nodes(self):
        return self.coords.shape[0]

    @property
    def n_elems(self):
        return self.conn.shape[0]

    @property
    def n_dof(self):
        return self.coords.shape[0] * self.coords.shape[1]

    @property
    def nonlinear(self):
        return self.model.startswith("nh")


def _clamp(nodes, dim, value=0.0):
    nodes = np.asarray(nodes, dtype=np.int32)
    n = nodes.size
    dn = np.repeat(nodes, dim)
    dc = np.tile(np.arange(dim, dtype=np.int8), n)
    return dn, dc, np.full(dn.size, value)


def _edge_facets(coords, on_edge, axis):
    """Consecutive boundary-node pairs along one straight edge."""
    idx = np.nonzero(on_edge)[0]
    idx = idx[np.argsort(coords[idx, axis])]
    return np.stack([idx[:-1], idx[1:]], axis=1).astype(np.int32)


def unit_square_c1(n=33, E=1.0, nu=0.3, tx=0.01):
    """33x33 nodes, 2048 triangles, plane stress, left edge clamped,
    traction (tx, 0) on the right edge."""
    coords, conn = meshes.grid_triangles(n)
    left = np.nonzero(coords[:, 0] == 0.0)[0]
    dn, dc, dv = _clamp(left, 2)
    facets = _edge_facets(coords, coords[:, 0] == 1.0, axis=1)
    trac = np.tile([tx, 0.0], (facets.shape[0], 1))
    ne = conn.shape[0]
    return Problem("c1_unit_square", "lin_plane_stress", coords, conn, "E_nu",
                   np.full(ne, E), np.full(ne, nu), dn, dc, dv, facets, trac, 1,
                   {"n": n})


def _plate_bcs(coords, rng_bc):
    """Clamped bottom edge; random traction segment on the top edge."""
    bottom = np.nonzero(coords[:, 1] == 0.0)[0]
    dn, dc, dv = _clamp(bottom, 2)
    top = np.nonzero(coords[:, 1] == 1.0)[0]
    top = top[np.argsort(coords[top, 0])]
    centre = rng_bc.uniform(0.2, 0.8)
    length = rng_bc.uniform(0.1, 0.4)
    mag = rng_bc.uniform(0.005, 0.02)
    ang = rng_bc.uniform(0.0, np.pi)
    xs = coords[top, 0]
    a = int(np.argmin(np.abs(xs - (centre - 0.5 * length))))
    b = int(np.argmin(np.abs(xs - (centre + 0.5 * length))))
    if b == a:
        b = min(a + 1, top.size - 1)
        if b == a:
            a = a - 1
    seg = top[a:b + 1]
    facets = np.stack([seg[:-1], seg[1:]], axis=1).astype(np.int32)
    trac = np.tile([mag * np.cos(ang), mag * np.sin(ang)], (facets.shape[0], 1))
    return dn, dc, dv, facets, trac, {"traction": (mag, ang, centre, length)}


def log_e_field(centroids, seed, sigma=0.5, length=0.1, n_features=1024):
    """Gaussian-random-field log-modulus at element centroids."""
    return sigma * rff_field(centroids, seed, length, n_features)


def plate_problem(seed_geom, seed_mat, seed_bc, n_holes=8, target_tris=200000,
                  model="lin_plane_strain", nu=0.3, name=None, e_features=1024):
    """Unit plate with random circular holes and a lognormal E field
    (``e_features`` random Fourier features)."""
    coords, conn, holes = meshes.plate_with_holes(_rng(seed_geom), n_holes,
                                                  target_tris)
    coords, conn = meshes._relabel(coords, conn, _rng(seed_geom + 7919))
    cen = coords[conn].mean(axis=1)
    E = np.exp(log_e_field(cen, seed_mat, n_features=e_features))
    dn, dc, dv, facets, trac, bmeta = _plate_bcs(coords, _rng(seed_bc))
    ne = conn.shape[0]
    meta = {"holes": holes, **bmeta}
    return Problem(name or f"plate_{seed_geom}", model, coords, conn, "E_nu",
                   E, np.full(ne, nu), dn, dc, dv, facets, trac, 1, meta)


def box_problem(seed_geom, seed_mat, n_per_unit=35, n_voids=20, uz=0.4,
                n_load_steps=10, model="nh_3d", name=None):
    """1x1x4 box with ellipsoidal voids; bimaterial mu in {1, 10} split by a
    random plane, lambda = 4 mu; z=0 clamped, u_z = uz prescribed on z=4."""
    coords, conn, voids = meshes.box_with_voids(_rng(seed_geom), n_per_unit,
                                                n_voids)
    rm = _rng(seed_mat)
    p = rm.uniform([0, 0, 0], [1, 1, 4])
    nrm = rm.normal(size=3)
    nrm /= np.linalg.norm(nrm)
    cen = coords[conn].mean(axis=1)
    mu = np.where((cen - p) @ nrm < 0.0, 1.0, 10.0)
    lam = 4.0 * mu
    z0 = np.nonzero(coords[:, 2] == 0.0)[0]
    z4 = np.nonzero(coords[:, 2] == 4.0)[0]
    dn0, dc0, dv0 = _clamp(z0, 3)
    dn = np.concatenate([dn0, z4.astype(np.int32)])
    dc = np.concatenate([dc0, np.full(z4.size, 2, dtype=np.int8)])
    dv = np.concatenate([dv0, np.full(z4.size, uz)])
    return Problem(name or f"box_{seed_geom}", model, coords, conn, "lame",
                   mu, lam, dn, dc, dv, np.zeros((0, 3), np.int32),
                   np.zeros((0, 3)), n_load_steps,
                   {"voids": len(voids), "plane": (p, nrm)})


def structured_plate(nx, ny, seed, model="lin_plane_strain", nu=0.3):
    """Void-free jittered plate for size sweeps (no Delaunay needed)."""
    coords, conn = meshes.structured_plate(nx, ny, _rng(seed))
    cen = coords[conn].mean(axis=1)
    E = np.exp(log_e_field(cen, seed + 1000, n_features=64))
    dn, dc, dv, facets, trac, _ = _plate_bcs(coords, _rng(seed + 2000))
    ne = conn.shape[0]
    return Problem(f"splate_{nx}x{ny}", model, coords, conn, "E_nu", E,
                   np.full(ne, nu), dn, dc, dv, facets, trac, 1, {})


def structured_box(nx, ny, nz, seed, model="lin_3d", nu=0.3):
    """Void-free jittered Kuhn box for size sweeps."""
    coords, conn = meshes.structured_box(nx, ny, nz, _rng(seed))
    cen = coords[conn].mean(axis=1)
    E = np.exp(log_e_field(cen, seed + 1000, n_features=64))
    z0 = np.nonzero(coords[:, 2] == 0.0)[0]
    dn, dc, dv = _clamp(z0, 3)
    top = coords[:, 2] == 4.0
    # z = 4 face triangles carry a uniform traction
    ne = conn.shape[0]
    return Problem(f"sbox_{nx}x{ny}x{nz}", model, coords, conn, "E_nu", E,
                   np.full(ne, nu), dn, dc, dv, np.zeros((0, 3), np.int32),
                   np.zeros((0, 3)), 1, {"top_nodes": int(top.sum())})


def c4_member(i, target=None):
    """One mesh of the differentiable-energy batch and its predicted field."""
    seed = 4000 + i
    rng = _rng(seed)
    if target is None:
        target = float(np.exp(rng.uniform(np.log(5e3), np.log(2e4))))
    n_holes = int(rng.integers(1, 9))
    model = "lin_plane_strain" if i % 2 == 0 else "nh_plane_strain"
    prob = plate_problem(seed, seed + 100000, seed + 200000, n_holes=n_holes,
                         target_tris=target, model=model, name=f"c4_{i}")
    g = rff_field(prob.coords, seed + 300000, 0.1, 256, n_comp=2)
    w = lifting_weight(prob.coords, prob.dir_nodes)
    u = (0.01 * g * w[:, None]).reshape(-1).astype(np.float32)
    return prob, u


def batch_c4(n=64):
    """64 plates, 5k-20k triangles, alternating linear / Neo-Hookean."""
    return [c4_member(i) for i in range(n)]


def serving_stream(n_requests=512, rate=200.0, frac_2d=0.7, smin=1e4,
                   smax=5e5, seed=5999):
    """Request descriptors for the serving stream (meshes built lazily).

    Returns a list of dicts with arrival time (s), kind ("2d" or "3d"),
    target element count and per-request seed.
    """
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for k in range(n_requests):
        rk = _rng(5000 + k)
        kind = "2d" if rk.uniform() < frac_2d else "3d"
        size = float(np.exp(rk.uniform(np.log(smin), np.log(smax))))
        out.append({"id": k, "t_arrive": float(t[k]), "kind": kind,
                    "target_elems": size, "seed": 5000 + k})
    return out


# random Fourier features of the serving stream's fields: 128 for log E and
# 64 for the warm-start noise (against 1024 / 256 elsewhere), so that the
# 512 meshes of a stream are generated in seconds; still unit-variance
# smooth fields of the stated correlation length
SERVING_E_FEATURES = 128
SERVING_NOISE_FEATURES = 64


def serving_problem(desc):
    """Build the mesh/problem for one serving-stream request descriptor."""
    s = desc["seed"]
    if desc["kind"] == "2d":
        return plate_problem(s, s + 100000, s + 200000, n_holes=8,
                             target_tris=desc["target_elems"],
                             model="lin_plane_strain", name=f"req{desc['id']}",
                             e_features=SERVING_E_FEATURES)
    n = max(int(round((desc["target_elems"] / (24.0 * 0.98)) ** (1.0 / 3.0))), 4)
    return box_problem(s, s + 100000, n_per_unit=n, n_voids=20,
                       name=f"req{desc['id']}")


# ------------------------------------------------- quadrilateral benchmarks
def _edge_segments(nodes, elem):
    """Boundary edges along a sorted edge-node list (Q8: corner, mid, corner
    triples, written ends first, then the middle node)."""
    nodes = np.asarray(nodes, dtype=np.int32)
    if elem == "q8":
        return np.stack([nodes[0:-1:2], nodes[2::2], nodes[1::2]], axis=1)
    return np.stack([nodes[:-1], nodes[1:]], axis=1)


def _quad_problem(name, coords, conn, left, right, elem, seed, model, e_mean, trac_mean,
                  n_load_steps, trac_range=(0.0, 1.0), clamp_range=(0.0, 1.0)):
    rng = _rng(seed)
    cen = coords[conn[:, :4]].mean(axis=1)
    scale = np.ptp(coords, axis=0).max()
    E = e_mean * np.exp(0.3 * rff_field(cen / scale, seed + 1, 0.25, 256))
    nu = 0.35 + 0.08 * np.tanh(rff_field(cen / scale, seed + 2, 0.25, 256))
    lo, hi = clamp_range
    nl = len(left)
    clamp = left[int(round(lo * (nl - 1))):int(round(hi * (nl - 1))) + 1]
    dn, dc, dv = _clamp(clamp, 2)
    facets = _edge_segments(right, elem)
    mid = coords[facets[:, :2]].mean(axis=1)
    ys = coords[right, 1]
    a, b = trac_range
    yl = ys.min() + a * (ys.max() - ys.min())
    yh = ys.min() + b * (ys.max() - ys.min())
    on = (mid[:, 1] >= yl - 1e-12) & (mid[:, 1] <= yh + 1e-12)
    facets = facets[on]
    ty = trac_mean * (1.0 + 0.4 * rff_field(mid[on] / scale, seed + 3, 0.3, 128))
    trac = np.stack([np.zeros_like(ty), ty], axis=1)
    return Problem(name, model, coords, conn, "E_nu", E, nu, dn, dc, dv,
                   facets.astype(np.int32), trac, n_load_steps,
                   {"seed": seed}, elem)


def beam_problem(seed, nx=50, ny=50, elem="q4", model="nh_plane_strain", W=4.0, H=1.0,
                 e_mean=10.0, traction=-0.08, n_load_steps=5):
    """Hyperelastic beam (Sec. 'Nonlinear hyperelasticity'): W x H = 4 x 1,
    left end clamped, a downward traction t_y on the right end varying along
    it, lognormal E and nu fields; a uniform nx x ny mesh (50 x 50 Q4 in the
    paper), plane strain."""
    coords, conn, left, right = meshes.quad_grid(nx, ny, meshes.rectangle_map(W, H), elem,
                                                 _rng(seed))
    return _quad_problem(f"beam_{elem}_{nx}x{ny}", coords, conn, left, right, elem, seed,
                         model, e_mean, traction, n_load_steps)


def cook_problem(seed, n=30, elem="q8", model="nh_plane_strain", e_mean=10.0,
                 traction=0.3, n_load_steps=5):
    """Cook's membrane (Sec. 'Nonlinear hyperelasticity'): the tapered panel
    with corners (0,0), (48,44), (48,60), (0,44), on a uniform n x n mesh
    (30 x 30 Q8 in the paper); the clamped part of the left edge and the
    loaded part of the right edge are drawn from the seed, the traction t_y
    varies along it, lognormal E and nu fields, plane strain."""
    rng = _rng(seed + 7)
    c0 = rng.uniform(0.0, 0.2)
    c1 = rng.uniform(0.8, 1.0)
    t0 = rng.uniform(0.0, 0.3)
    t1 = rng.uniform(0.7, 1.0)
    coords, conn, left, right = meshes.quad_grid(n, n, meshes.cook_map(), elem, _rng(seed))
    return _quad_problem(f"cook_{elem}_{n}x{n}", coords, conn, left, right, elem, seed,
                         model, e_mean, traction, n_load_steps, (t0, t1), (c0, c1))
