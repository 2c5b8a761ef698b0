"""Quadrilateral elements in float64 (oracle; test infrastructure only: only
tests/, the smoke check and the benchmark's CPU leg use it).

The paper's nonlinear benchmarks (Sec. 'Nonlinear hyperelasticity': the
hyperelastic beam on a 50 x 50 mesh of bilinear quadrilaterals, Cook's
membrane on a 30 x 30 mesh of 8-node serendipity quadrilaterals) discretise
the same total-Lagrangian weak form as the P1 path (App. B: X = N_I X_I,
u = N_I u_I, f_int = int dN_I/dX P dV_0) with isoparametric quadrilaterals.
The paper does not state the quadrature; the reading here is the full Gauss
rule of each element (2 x 2 points for Q4, 3 x 3 for Q8), which integrates
the linear stiffness of an affinely mapped element exactly.

Node order (either orientation is accepted): corners 0..3 around the
element, then for Q8 the midside nodes of edges (0,1), (1,2), (2,3), (3,0).
Reference square [-1, 1]^2 with corners (-1,-1), (1,-1), (1,1), (-1,1).

Shape functions (textbook isoparametric families):
  Q4:  N_a = (1 + xi xi_a)(1 + eta eta_a) / 4
  Q8:  corners  N_a = (1 + xi xi_a)(1 + eta eta_a)(xi xi_a + eta eta_a - 1) / 4
       midsides N_a = (1 - xi^2)(1 + eta eta_a) / 2   (xi_a = 0)
                N_a = (1 + xi xi_a)(1 - eta^2) / 2   (eta_a = 0)

Each quadrature point (element e, point q) is handed to the P1 machinery of
`fe.Model` as a point with its own shape-function gradients dN/dX (nv x 2)
and weight w_q |det J_eq|: energies, forces and element matrices are sums
over points exactly as over P1 elements, with the element's DOFs repeated
per point.
"""
import numpy as np

CORNERS = np.array([[-1.0, -1.0], [1.0, -1.0], [1.0, 1.0], [-1.0, 1.0]])
MIDSIDES = np.array([[0.0, -1.0], [1.0, 0.0], [0.0, 1.0], [-1.0, 0.0]])

NODES_PER_ELEM = {"q4": 4, "q8": 8}


def gauss_1d(n):
    """Gauss-Legendre points and weights on [-1, 1] (n = 2 or 3)."""
    if n == 2:
        a = 1.0 / np.sqrt(3.0)
        return np.array([-a, a]), np.array([1.0, 1.0])
    if n == 3:
        a = np.sqrt(3.0 / 5.0)
        return np.array([-a, 0.0, a]), np.array([5.0, 8.0, 5.0]) / 9.0
    raise ValueError(n)


def gauss_rule(elem):
    """Tensor-product Gauss rule of the element: points (nq, 2), weights (nq,)."""
    x, w = gauss_1d(2 if elem == "q4" else 3)
    xi, eta = np.meshgrid(x, x, indexing="ij")
    wx, wy = np.meshgrid(w, w, indexing="ij")
    return np.stack([xi.ravel(), eta.ravel()], axis=1), (wx * wy).ravel()


def shape(elem, pts):
    """N (np, nv) and dN/dxi (np, nv, 2) at reference points pts (np, 2)."""
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    xi, eta = pts[:, 0:1], pts[:, 1:2]
    ca, cb = CORNERS[:, 0][None, :], CORNERS[:, 1][None, :]
    if elem == "q4":
        N = 0.25 * (1 + xi * ca) * (1 + eta * cb)
        dxi = 0.25 * ca * (1 + eta * cb)
        deta = 0.25 * cb * (1 + xi * ca)
        return N, np.stack([dxi, deta], axis=2)
    if elem != "q8":
        raise ValueError(elem)
    s = xi * ca + eta * cb - 1.0
    Nc = 0.25 * (1 + xi * ca) * (1 + eta * cb) * s
    dNc_xi = 0.25 * ca * (1 + eta * cb) * s + 0.25 * (1 + xi * ca) * (1 + eta * cb) * ca
    dNc_eta = 0.25 * cb * (1 + xi * ca) * s + 0.25 * (1 + xi * ca) * (1 + eta * cb) * cb
    Nm = np.empty((pts.shape[0], 4))
    dNm_xi = np.empty_like(Nm)
    dNm_eta = np.empty_like(Nm)
    for k, (mx, my) in enumerate(MIDSIDES):
        if mx == 0.0:      # edge along xi: (1 - xi^2)(1 + eta eta_a) / 2
            Nm[:, k] = 0.5 * (1 - xi[:, 0] ** 2) * (1 + eta[:, 0] * my)
            dNm_xi[:, k] = -xi[:, 0] * (1 + eta[:, 0] * my)
            dNm_eta[:, k] = 0.5 * (1 - xi[:, 0] ** 2) * my
        else:              # edge along eta: (1 + xi xi_a)(1 - eta^2) / 2
            Nm[:, k] = 0.5 * (1 + xi[:, 0] * mx) * (1 - eta[:, 0] ** 2)
            dNm_xi[:, k] = 0.5 * mx * (1 - eta[:, 0] ** 2)
            dNm_eta[:, k] = -(1 + xi[:, 0] * mx) * eta[:, 0]
    N = np.concatenate([Nc, Nm], axis=1)
    dN = np.stack([np.concatenate([dNc_xi, dNm_xi], axis=1),
                   np.concatenate([dNc_eta, dNm_eta], axis=1)], axis=2)
    return N, dN


def point_geometry(coords, conn, elem):
    """Per quadrature point: gradients dN/dX (E*nq, nv, 2), weights
    w_q |det J| (E*nq,), det J (E*nq,) and the owning element (E*nq,).

    J = sum_a X_a (x) dN_a/dxi (App. B, X = N_I X_I); dN/dX = J^{-T} dN/dxi.
    """
    X = np.asarray(coords, dtype=np.float64)[np.asarray(conn, dtype=np.int64)]  # (E, nv, 2)
    pts, w = gauss_rule(elem)
    _, dN = shape(elem, pts)                                  # (nq, nv, 2)
    J = np.einsum("eai,qaj->eqij", X, dN)                      # (E, nq, 2, 2)
    det = J[..., 0, 0] * J[..., 1, 1] - J[..., 0, 1] * J[..., 1, 0]
    Jinv = np.linalg.inv(J)                                    # (E, nq, 2, 2)
    G = np.einsum("qaj,eqji->eqai", dN, Jinv)                  # dN/dX_i = dN/dxi_j Jinv_ji
    E, nq = det.shape
    elem_of = np.repeat(np.arange(E), nq)
    return (G.reshape(E * nq, -1, 2), (np.abs(det) * w[None, :]).reshape(-1),
            det.reshape(-1), elem_of)


def edge_shape(n_nodes, s):
    """Shape functions of a 2-node (linear) or 3-node (quadratic: ends, then
    the middle node) edge at s in [-1, 1], and their derivatives."""
    s = np.asarray(s, dtype=np.float64)
    if n_nodes == 2:
        return (np.stack([0.5 * (1 - s), 0.5 * (1 + s)], axis=-1),
                np.stack([-0.5 + 0 * s, 0.5 + 0 * s], axis=-1))
    return (np.stack([0.5 * s * (s - 1), 0.5 * s * (s + 1), 1 - s * s], axis=-1),
            np.stack([s - 0.5, s + 0.5, -2 * s], axis=-1))


def edge_loads(coords, facets, traction):
    """Consistent nodal loads of a constant traction on each edge:
    f_a = t int N_a dGamma (App. B, f_ext), 3-point Gauss along the edge
    (exact for straight and for parabolic edges' polynomial part)."""
    P = np.asarray(coords, dtype=np.float64)[np.asarray(facets, dtype=np.int64)]  # (F, nf, 2)
    nf = P.shape[1]
    s, w = gauss_1d(3)
    N, dN = edge_shape(nf, s)                    # (3, nf)
    tang = np.einsum("qa,fai->fqi", dN, P)       # dx/ds at each point
    ds = np.linalg.norm(tang, axis=2)            # (F, 3)
    wN = np.einsum("q,fq,qa->fa", w, ds, N)      # int N_a dGamma per facet node
    return wN[:, :, None] * np.asarray(traction, dtype=np.float64)[:, None, :]
