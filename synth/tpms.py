"""Periodic unit cells of triply periodic minimal surfaces (TPMS) for the
homogenisation workload.

The solid phase of a cell is a level set of one of three TPMS fields (App.
E, TPMS-type equation): Schoen gyroid, Schwarz diamond or Fischer-Koch S,
either as a "solid network" (phi > c) or a "sheet network" (|phi| <= c).
The cell [0, 1]^3 is cut into n^3 voxels; a voxel is solid when its centre
is, the level c is set by bisection so that the solid voxel fraction
matches the requested volume fraction, only the largest solid component
(connected through faces, across the periodic boundary too) is kept, and
every solid voxel becomes 6 Kuhn tetrahedra (the same pattern in every
voxel, so the triangulations of opposite faces are translates of each
other).  Opposite-face node pairs carry the periodic coupling; one node is
pinned to remove the rigid translations.  Nothing here computes stiffness,
strains or moduli.
"""
from dataclasses import dataclass, field

import numpy as np

from .meshes import _kuhn_pattern

TPMS_KINDS = ("gyroid", "diamond", "fks")
NETWORKS = ("solid", "sheet")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def tpms_field(kind, x, y, z):
    """The level-set field phi of App. E (TPMS-type equation) on [0, 1]^3."""
    t = 2.0 * np.pi
    if kind == "gyroid":
        return (np.sin(t * x) * np.cos(t * y) + np.sin(t * y) * np.cos(t * z)
                + np.sin(t * z) * np.cos(t * x))
    if kind == "diamond":
        return (np.cos(t * x) * np.cos(t * y) * np.cos(t * z)
                - np.sin(t * x) * np.sin(t * y) * np.sin(t * z))
    if kind == "fks":
        return (np.cos(2 * t * x) * np.sin(t * y) * np.cos(t * z)
                + np.cos(t * x) * np.cos(2 * t * y) * np.sin(t * z)
                + np.sin(t * x) * np.cos(t * y) * np.cos(2 * t * z))
    raise ValueError(kind)


def _solid(phi, network, c):
    return phi > c if network == "solid" else np.abs(phi) <= c


def voxel_mask(kind, network, vf, n):
    """(n, n, n) bool mask indexed [i, j, k] = voxel (x, y, z), solid where
    the voxel centre is; c chosen by bisection so the solid fraction is as
    close to vf as the voxel count allows."""
    g = (np.arange(n) + 0.5) / n
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    phi = tpms_field(kind, X, Y, Z)
    lo, hi = float(phi.min()) - 1.0, float(phi.max()) + 1.0
    if network == "sheet":
        lo = 0.0
    for _ in range(60):
        c = 0.5 * (lo + hi)
        frac = _solid(phi, network, c).mean()
        # solid: fraction falls as c rises; sheet: fraction rises with c
        if (frac > vf) == (network == "solid"):
            lo = c
        else:
            hi = c
    return _solid(phi, network, 0.5 * (lo + hi))


def largest_periodic_component(mask):
    """Keep the largest face-connected component of the solid voxels, with
    connections across opposite faces of the periodic cell."""
    from scipy import ndimage
    lab, nlab = ndimage.label(mask)
    if nlab <= 1:
        return mask.copy()
    parent = list(range(nlab + 1))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for ax in range(3):
        a = np.take(lab, 0, axis=ax)
        b = np.take(lab, -1, axis=ax)
        both = (a > 0) & (b > 0)
        for la, lb in set(zip(a[both].tolist(), b[both].tolist())):
            ra, rb = find(la), find(lb)
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
    root = np.array([find(k) for k in range(nlab + 1)])
    size = np.bincount(root[lab[mask]], minlength=nlab + 1)
    return root[lab] == int(size.argmax()) if size.any() else mask.copy()


def voxel_tets(mask):
    """Kuhn tetrahedra of the solid voxels on the (n+1)^3 node lattice of
    [0, 1]^3; only nodes used by a tetrahedron are kept.  Returns coords,
    conn and the lattice index (i, j, k) of every kept node."""
    n = mask.shape[0]
    m1 = n + 1
    vox = np.argwhere(mask)                                 # (V, 3): i, j, k
    base = vox[:, 0] + m1 * (vox[:, 1] + m1 * vox[:, 2])
    off = np.array([(c & 1) + m1 * (((c >> 1) & 1) + m1 * ((c >> 2) & 1))
                    for c in range(8)], dtype=np.int64)
    lat = (base[:, None, None] + off[_kuhn_pattern()][None, :, :]).reshape(-1, 4)
    used, inv = np.unique(lat, return_inverse=True)
    conn = inv.reshape(-1, 4).astype(np.int32)
    ijk = np.stack([used % m1, (used // m1) % m1, used // (m1 * m1)], axis=1)
    coords = ijk.astype(np.float64) / n
    return coords, conn, ijk


def periodic_pairs(ijk, n):
    """Node pairs (a, b) with b the image of a across one face pair: a on the
    face x_ax = 0, b on x_ax = 1, same other two lattice indices.  Nodes on
    edges and corners pair along every axis, which couples their images in
    a ring."""
    m1 = n + 1
    key = ijk[:, 0] + m1 * (ijk[:, 1] + m1 * ijk[:, 2])
    lookup = dict(zip(key.tolist(), range(len(key))))
    pairs = []
    for ax in range(3):
        on0 = np.nonzero(ijk[:, ax] == 0)[0]
        img = ijk[on0].copy()
        img[:, ax] = n
        kk = img[:, 0] + m1 * (img[:, 1] + m1 * img[:, 2])
        for a, k in zip(on0.tolist(), kk.tolist()):
            b = lookup.get(k)
            if b is not None:
                pairs.append((a, b))
    return np.array(pairs, dtype=np.int32).reshape(-1, 2)


@dataclass
class CellProblem:
    """A periodic unit cell: mesh, per-element (E, nu), periodic node pairs
    with their penalty stiffness, and the pinned node."""
    name: str
    coords: np.ndarray            # (N_n, 3) float64
    conn: np.ndarray              # (N_e, 4) int32
    p0: np.ndarray                # (N_e,) Young's modulus
    p1: np.ndarray                # (N_e,) Poisson ratio
    pairs: np.ndarray             # (P, 2) int32 periodic node pairs
    penalty: float                # spring stiffness of each pair
    pin: int                      # node whose fluctuation is held at zero
    meta: dict = field(default_factory=dict)
    model: str = "lin_3d"
    param_kind: str = "E_nu"

    dim = 3

    @property
    def n_nodes(self):
        return self.coords.shape[0]

    @property
    def n_elems(self):
        return self.conn.shape[0]

    @property
    def n_dof(self):
        return 3 * self.coords.shape[0]


# Penalty of the periodic coupling, in units of E h (h the voxel edge): the
# springs are this many times stiffer than an element edge.
PENALTY_EH = 1.0e3


def cell_from_mask(mask, E, nu, name="cell", penalty_eh=PENALTY_EH, meta=None):
    n = mask.shape[0]
    coords, conn, ijk = voxel_tets(mask)
    pairs = periodic_pairs(ijk, n)
    ne = conn.shape[0]
    p0 = np.broadcast_to(np.asarray(E, dtype=np.float64), (ne,)).copy()
    p1 = np.broadcast_to(np.asarray(nu, dtype=np.float64), (ne,)).copy()
    pin = int(np.lexsort((ijk[:, 0], ijk[:, 1], ijk[:, 2]))[0])
    k = penalty_eh * float(np.max(p0)) / n
    return CellProblem(name, coords, conn, p0, p1, pairs, k, pin, dict(meta or {}))


def tpms_cell(seed, n=64, kind=None, network=None, vf=None, nu=None,
              penalty_eh=PENALTY_EH):
    """One seeded TPMS cell: kind (3), network (2), volume fraction
    U[0.26, 0.66] and Poisson ratio U[0.1, 0.4] drawn unless given; E = 1."""
    rng = _rng(seed)
    kind = kind or TPMS_KINDS[int(rng.integers(3))]
    network = network or NETWORKS[int(rng.integers(2))]
    vf = float(rng.uniform(0.26, 0.66)) if vf is None else vf
    nu = float(rng.uniform(0.1, 0.4)) if nu is None else nu
    mask = largest_periodic_component(voxel_mask(kind, network, vf, n))
    meta = {"kind": kind, "network": network, "vf_target": vf,
            "vf": float(mask.mean()), "nu": nu, "n": n}
    return cell_from_mask(mask, 1.0, nu, name=f"tpms_{kind}_{network}_{seed}",
                          penalty_eh=penalty_eh, meta=meta)


def laminate_cell(n, layers, E, nu, penalty_eh=PENALTY_EH):
    """A fully solid cell of layers normal to z: voxel layer k has material
    (E[layers[k]], nu[layers[k]]).  Its homogenised tensor has a closed form
    (continuity of traction across the layers), which pins the oracle."""
    mask = np.ones((n, n, n), dtype=bool)
    cell = cell_from_mask(mask, 1.0, 0.3, name="laminate", penalty_eh=penalty_eh)
    zc = cell.coords[cell.conn].mean(axis=1)[:, 2]
    k = np.minimum((zc * n).astype(int), n - 1)
    lay = np.asarray(layers)[k]
    cell.p0 = np.asarray(E, dtype=np.float64)[lay]
    cell.p1 = np.asarray(nu, dtype=np.float64)[lay]
    cell.penalty = penalty_eh * float(np.max(cell.p0)) / n
    cell.meta = {"layers": list(layers), "E": list(E), "nu": list(nu), "n": n}
    return cell
