"""Pins of the quadrilateral-element oracle (CPU).

Each pin fixes part of `oracle/quad.py` (and the quadrature-point path of
`oracle/fe.Model`) with something independent of its code:

* shape functions: partition of unity, zero-sum derivatives, Kronecker
  property at the nodes, derivatives against central differences;
* Gauss rules: the element areas sum to the shoelace area of the mesh;
* the Q4 and Q8 stiffness of a rectangle equals the exact integral of
  B^T D B, computed symbolically (sympy) from shape functions written here
  in physical coordinates;
* patch test: a linear field on the boundary of a distorted, curved-edge
  mesh is reproduced inside (Q4 and Q8);
* Q8 reproduces quadratic fields: on a parallelogram mesh the strain energy
  of a quadratic displacement equals its exact integral (Q4 cannot, so the
  pin checks the midside functions);
* a bar under an end traction has the textbook linear solution (consistent
  edge loads, including the 1/6, 2/3, 1/6 split of a Q8 edge);
* Neo-Hookean: zero energy and force under a finite rotation, the tangent
  at u = 0 equals the linear plane-strain stiffness, forces and tangents
  against central differences of the energy / force;
* the assembled stiffness with a clamped edge is symmetric positive definite.

Planted mistakes (a swapped 3-point Gauss weight, a sign in a Q8 midside
function, P1-style loads on Q8 edges, J^-1 in place of J^-T) each fail a pin.
"""
import functools

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import sympy as sy

import synth
from oracle import fe, quad, solve

ELEMS = ("q4", "q8")


def _problem(coords, conn, elem, model="lin_plane_strain", E=1.3, nu=0.3, dir_nodes=(),
             dir_comps=(), dir_values=(), facets=None, traction=None, n_load_steps=1):
    ne = conn.shape[0]
    nf = 3 if elem == "q8" else 2
    return synth.Problem(
        f"quad_{elem}", model, np.asarray(coords, np.float64), np.asarray(conn, np.int32),
        "E_nu", np.full(ne, E), np.full(ne, nu), np.asarray(dir_nodes, np.int32),
        np.asarray(dir_comps, np.int8), np.asarray(dir_values, np.float64),
        np.zeros((0, nf), np.int32) if facets is None else np.asarray(facets, np.int32),
        np.zeros((0, 2)) if traction is None else np.asarray(traction, np.float64),
        n_load_steps, {}, elem)


def _wavy(p):
    """A smooth orientation-preserving map of [0,1]^2 (curved mesh lines)."""
    x, y = p[:, 0], p[:, 1]
    return np.stack([2.0 * x + 0.15 * np.sin(3.0 * y) * x * (1 - x),
                     1.5 * y + 0.1 * np.sin(4.0 * x) * y * (1 - y) + 0.2 * x], axis=1)


def _parallelogram(p):
    return np.stack([2.0 * p[:, 0] + 0.5 * p[:, 1], 0.3 * p[:, 0] + 1.2 * p[:, 1]], axis=1)


def _boundary_nodes(coords, conn, elem):
    """Nodes on edges used by exactly one element."""
    corners = conn[:, :4]
    edges = {}
    for e in range(conn.shape[0]):
        for k in range(4):
            a, b = corners[e, k], corners[e, (k + 1) % 4]
            key = (min(a, b), max(a, b))
            mid = conn[e, 4 + k] if elem == "q8" else -1
            edges.setdefault(key, []).append(mid)
    nodes = set()
    for (a, b), mids in edges.items():
        if len(mids) == 1:
            nodes.update([a, b])
            if mids[0] >= 0:
                nodes.add(mids[0])
    return np.array(sorted(nodes))


# ------------------------------------------------------------------- pins
def pin_shape_functions():
    rng = np.random.default_rng(0)
    pts = rng.uniform(-1, 1, size=(20, 2))
    for elem in ELEMS:
        N, dN = quad.shape(elem, pts)
        assert np.abs(N.sum(axis=1) - 1).max() <= 1e-14
        assert np.abs(dN.sum(axis=1)).max() <= 1e-13
        nodes = np.concatenate([quad.CORNERS, quad.MIDSIDES])[:N.shape[1]]
        Nn, _ = quad.shape(elem, nodes)
        assert np.abs(Nn - np.eye(N.shape[1])).max() <= 1e-14
        h = 1e-6
        for k in range(2):
            e = np.zeros(2)
            e[k] = h
            fd = (quad.shape(elem, pts + e)[0] - quad.shape(elem, pts - e)[0]) / (2 * h)
            assert np.abs(fd - dN[:, :, k]).max() <= 1e-8


def pin_area():
    for elem in ELEMS:
        coords, conn, _, _ = synth.meshes.quad_grid(6, 5, _parallelogram, elem)
        m = fe.Model(_problem(coords, conn, elem))
        # shoelace area of the parallelogram image of the unit square
        c = _parallelogram(np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float))
        area = 0.5 * abs(sum(c[i, 0] * c[(i + 1) % 4, 1] - c[(i + 1) % 4, 0] * c[i, 1]
                             for i in range(4)))
        assert abs(m.vol.sum() - area) <= 1e-13 * area


@functools.lru_cache(maxsize=None)
def _exact_rect_stiffness(elem, a, b, E, nu):
    """Plane-strain stiffness of the rectangle [0, a] x [0, b] by exact
    integration of B^T D B with physical-coordinate shape functions
    (polynomials integrated term by term in rational arithmetic)."""
    x, y = sy.symbols("x y")
    s, t = 2 * x / a - 1, 2 * y / b - 1            # reference coordinates
    cs = [(-1, -1), (1, -1), (1, 1), (-1, 1)]
    if elem == "q4":
        Ns = [(1 + s * p) * (1 + t * q) / 4 for p, q in cs]
    else:
        Ns = [(1 + s * p) * (1 + t * q) * (s * p + t * q - 1) / 4 for p, q in cs]
        Ns += [(1 - s ** 2) * (1 - t) / 2, (1 + s) * (1 - t ** 2) / 2,
               (1 - s ** 2) * (1 + t) / 2, (1 - s) * (1 - t ** 2) / 2]
    nv = len(Ns)
    dx = [sy.Poly(sy.diff(N, x), x, y) for N in Ns]
    dy = [sy.Poly(sy.diff(N, y), x, y) for N in Ns]

    def integ(P):
        Q = P.integrate(x).integrate(y)
        return (Q.eval({x: a, y: b}) - Q.eval({x: 0, y: b}) - Q.eval({x: a, y: 0})
                + Q.eval({x: 0, y: 0}))

    lam = sy.Rational(E) * nu / ((1 + nu) * (1 - 2 * nu))
    mu = sy.Rational(E) / (2 * (1 + nu))
    K = np.zeros((2 * nv, 2 * nv))
    for i in range(nv):
        for j in range(nv):
            xx, yy = integ(dx[i] * dx[j]), integ(dy[i] * dy[j])
            xy, yx = integ(dx[i] * dy[j]), integ(dy[i] * dx[j])
            K[2 * i, 2 * j] = float((lam + 2 * mu) * xx + mu * yy)
            K[2 * i, 2 * j + 1] = float(lam * xy + mu * yx)
            K[2 * i + 1, 2 * j] = float(lam * yx + mu * xy)
            K[2 * i + 1, 2 * j + 1] = float((lam + 2 * mu) * yy + mu * xx)
    return K


def pin_rectangle_stiffness():
    a, b, E, nu = sy.Rational(3, 2), sy.Rational(1, 2), 2, sy.Rational(3, 10)
    for elem in ELEMS:
        c = np.array([[0, 0], [1.5, 0], [1.5, 0.5], [0, 0.5]])
        if elem == "q8":
            c = np.concatenate([c, 0.5 * (c + np.roll(c, -1, axis=0))])
        conn = np.arange(len(c))[None, :]
        m = fe.Model(_problem(c, conn, elem, E=2.0, nu=0.3))
        K = m.assemble().toarray()
        Kx = _exact_rect_stiffness(elem, a, b, E, nu)
        assert np.abs(K - Kx).max() <= 1e-12 * np.abs(Kx).max()


def pin_patch():
    A = np.array([[0.3, -0.1], [0.25, 0.05]])
    c0 = np.array([0.1, -0.2])
    field = lambda X: c0 + X @ A.T
    for elem in ELEMS:
        coords, conn, _, _ = synth.meshes.quad_grid(5, 4, _wavy, elem,
                                                    np.random.default_rng(3))
        bnd = _boundary_nodes(coords, conn, elem)
        vals = field(coords[bnd])
        prob = _problem(coords, conn, elem, dir_nodes=np.repeat(bnd, 2),
                        dir_comps=np.tile([0, 1], len(bnd)), dir_values=vals.reshape(-1))
        u, _ = solve.solve_linear(prob, method="direct")
        assert np.abs(u.reshape(-1, 2) - field(coords)).max() <= 1e-11


def _quadratic_field(X):
    x, y = X[..., 0], X[..., 1]
    return np.stack([0.1 * x * x - 0.05 * x * y + 0.02 * y * y + 0.1 * x,
                     -0.03 * x * x + 0.07 * x * y + 0.04 * y * y - 0.2 * y], axis=-1)


def _quadratic_field_exact_energy(E, nu):
    """Strain energy of the quadratic field over the parallelogram, from a
    20 x 20 Gauss rule on the affine map of the unit square (exact: the
    integrand is a polynomial of degree 2 in the parameters)."""
    lam = nu * E / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    g, w = np.polynomial.legendre.leggauss(20)
    g, w = 0.5 * (g + 1), 0.5 * w
    P = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    W = np.outer(w, w).reshape(-1)
    X = _parallelogram(P)
    detJ = abs(2.0 * 1.2 - 0.5 * 0.3)
    x, y = X[:, 0], X[:, 1]
    # displacement gradient of the quadratic field (by hand)
    H = np.empty((len(x), 2, 2))
    H[:, 0, 0] = 0.2 * x - 0.05 * y + 0.1
    H[:, 0, 1] = -0.05 * x + 0.04 * y
    H[:, 1, 0] = -0.06 * x + 0.07 * y
    H[:, 1, 1] = 0.07 * x + 0.08 * y - 0.2
    eps = 0.5 * (H + np.transpose(H, (0, 2, 1)))
    tr = eps[:, 0, 0] + eps[:, 1, 1]
    psi = mu * np.einsum("eij,eij->e", eps, eps) + 0.5 * lam * tr * tr
    return float(np.sum(W * detJ * psi))


def pin_q8_quadratic():
    coords, conn, _, _ = synth.meshes.quad_grid(4, 3, _parallelogram, "q8",
                                                np.random.default_rng(4))
    m = fe.Model(_problem(coords, conn, "q8", E=1.7, nu=0.3))
    u = _quadratic_field(coords).reshape(-1)
    exact = _quadratic_field_exact_energy(1.7, 0.3)
    assert abs(m.energy(u) - exact) <= 1e-12 * exact


def pin_bar():
    """Plane-stress bar [0, L] x [0, H]: u_x = 0 on the left edge, u_y = 0 at
    its lower corner, traction t on the right edge: u = (t x / E, -nu t y / E)."""
    L, H, E, nu, t = 3.0, 1.0, 2.5, 0.3, 0.04
    for elem in ELEMS:
        coords, conn, left, right = synth.meshes.quad_grid(
            6, 3, synth.meshes.rectangle_map(L, H), elem, np.random.default_rng(5))
        corner = left[np.argmin(coords[left, 1])]
        facets = synth.problems._edge_segments(right, elem)
        prob = _problem(coords, conn, elem, "lin_plane_stress", E, nu,
                        dir_nodes=np.concatenate([left, [corner]]),
                        dir_comps=np.concatenate([np.zeros(len(left)), [1]]),
                        dir_values=np.zeros(len(left) + 1), facets=facets,
                        traction=np.tile([t, 0.0], (len(facets), 1)))
        u, _ = solve.solve_linear(prob, method="direct")
        ex = np.stack([t * coords[:, 0] / E, -nu * t * coords[:, 1] / E], axis=1)
        assert np.abs(u.reshape(-1, 2) - ex).max() <= 1e-12 * np.abs(ex).max()


def pin_edge_loads():
    """A Q8 edge carries t L/6 at each end and 2 t L/3 at its middle node."""
    c = np.array([[0.0, 0.0], [0.0, 2.0], [0.0, 1.0]])
    f = quad.edge_loads(c, np.array([[0, 1, 2]]), np.array([[0.0, 3.0]]))
    assert np.allclose(f[0, :, 1], [1.0, 1.0, 4.0], rtol=0, atol=1e-14)


def _nh_problem(elem, seed=6):
    coords, conn, left, right = synth.meshes.quad_grid(3, 2, _wavy, elem,
                                                       np.random.default_rng(seed))
    return _problem(coords, conn, elem, "nh_plane_strain", E=1.5, nu=0.35)


def pin_nh_rigid():
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    for elem in ELEMS:
        p = _nh_problem(elem)
        m = fe.Model(p)
        u = (p.coords @ R.T - p.coords + np.array([0.3, -0.2])).reshape(-1)
        assert abs(m.energy(u)) <= 1e-13
        assert np.abs(m.internal_force(u)).max() <= 1e-12


def pin_nh_small_strain():
    for elem in ELEMS:
        p = _nh_problem(elem)
        q = _problem(p.coords, p.conn, elem, "lin_plane_strain", E=1.5, nu=0.35)
        KT = fe.Model(p).assemble(np.zeros(p.n_dof)).toarray()
        K = fe.Model(q).assemble().toarray()
        assert np.abs(KT - K).max() <= 1e-12 * np.abs(K).max()


def pin_nh_derivatives():
    rng = np.random.default_rng(7)
    for elem in ELEMS:
        p = _nh_problem(elem)
        m = fe.Model(p)
        u = 0.05 * rng.normal(size=p.n_dof)
        v = rng.normal(size=p.n_dof)
        h = 1e-6
        g = m.internal_force(u)
        fd = (m.energy(u + h * v) - m.energy(u - h * v)) / (2 * h)
        assert abs(fd - g @ v) <= 1e-7 * abs(g @ v)
        Kv = m.assemble(u) @ v
        fdk = (m.internal_force(u + h * v) - m.internal_force(u - h * v)) / (2 * h)
        assert np.abs(fdk - Kv).max() <= 1e-6 * np.abs(Kv).max()


def pin_spd():
    for elem in ELEMS:
        coords, conn, left, right = synth.meshes.quad_grid(4, 3, _wavy, elem,
                                                           np.random.default_rng(8))
        prob = _problem(coords, conn, elem, dir_nodes=np.repeat(left, 2),
                        dir_comps=np.tile([0, 1], len(left)), dir_values=np.zeros(2 * len(left)))
        m = fe.Model(prob)
        K = m.assemble()[m.free_dofs][:, m.free_dofs].toarray()
        assert np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()
        assert np.linalg.eigvalsh(K).min() > 0


def pin_newton_beam():
    """The oracle's Newton on a small beam: converged states satisfy the
    residual test and the load steps agree with a one-step solve from the
    converged state (Sec. 'Nonlinear hyperelasticity', App. B)."""
    p = synth.beam_problem(21, 10, 4, elem="q8", n_load_steps=3)
    u, rep = solve.newton(p, tol=1e-10)
    assert rep["status"] == 0
    m = fe.Model(p)
    r = m.gradient(u)[m.free_dofs]
    den = np.linalg.norm(m.gradient(m.lifted())[m.free_dofs])
    assert np.linalg.norm(r) <= 1e-10 * den
    KT = m.assemble(u)[m.free_dofs][:, m.free_dofs]
    assert spla.eigsh(KT.tocsc(), k=1, sigma=0, which="LM", return_eigenvectors=False)[0] > 0


PINS = [pin_shape_functions, pin_area, pin_rectangle_stiffness, pin_patch, pin_q8_quadratic,
        pin_bar, pin_edge_loads, pin_nh_rigid, pin_nh_small_strain, pin_nh_derivatives,
        pin_spd, pin_newton_beam]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin()


# -------------------------------------------------------- planted mistakes
_orig_gauss = quad.gauss_1d
_orig_shape = quad.shape
_orig_edge = quad.edge_loads
_orig_geom = quad.point_geometry


def _gauss_swapped(n):
    x, w = _orig_gauss(n)
    if n == 3:
        w = np.array([8.0, 5.0, 8.0]) / 9.0 * (2.0 / (21.0 / 9.0))   # still sums to 2
    return x, w


def _shape_bad_mid(elem, pts):
    N, dN = _orig_shape(elem, pts)
    if elem == "q8":
        N = N.copy()
        dN = dN.copy()
        N[:, 5] = -N[:, 5]                # sign flipped
        dN[:, 5] = -dN[:, 5]
    return N, dN


def _edge_p1_style(coords, facets, traction):
    P = np.asarray(coords)[np.asarray(facets)]
    L = np.linalg.norm(P[:, 1] - P[:, 0], axis=1)
    nf = P.shape[1]
    return np.repeat((L / nf)[:, None, None], nf, axis=1) * np.asarray(traction)[:, None, :]


def _geom_transposed(coords, conn, elem):
    X = np.asarray(coords, dtype=np.float64)[np.asarray(conn, dtype=np.int64)]
    pts, w = quad.gauss_rule(elem)
    _, dN = quad.shape(elem, pts)
    J = np.einsum("eai,qaj->eqij", X, dN)
    det = J[..., 0, 0] * J[..., 1, 1] - J[..., 0, 1] * J[..., 1, 0]
    Jinv = np.linalg.inv(J)
    G = np.einsum("qaj,eqij->eqai", dN, Jinv)      # J^-1 instead of J^-T
    E, nq = det.shape
    return (G.reshape(E * nq, -1, 2), (np.abs(det) * w[None, :]).reshape(-1),
            det.reshape(-1), np.repeat(np.arange(E), nq))


@pytest.mark.parametrize("name,attr,fn", [("gauss_weights", "gauss_1d", _gauss_swapped),
                                          ("q8_mid_sign", "shape", _shape_bad_mid),
                                          ("q8_edge_loads", "edge_loads", _edge_p1_style),
                                          ("jacobian_transposed", "point_geometry",
                                           _geom_transposed)])
def test_planted_mistake_fails_a_pin(monkeypatch, name, attr, fn):
    monkeypatch.setattr(quad, attr, fn)
    failed = 0
    for pin in PINS:
        try:
            pin()
        except (AssertionError, np.linalg.LinAlgError, ValueError, RuntimeError):
            failed += 1
    assert failed > 0, name
