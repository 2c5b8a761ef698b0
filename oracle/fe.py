"""P1 finite-element physics in float64 (oracle; test infrastructure only).

Notation follows the paper: u displacement, F = I + grad u deformation
gradient, J = det F, C = F^T F, I1 = tr C, (lambda, mu) Lame parameters,
Psi strain-energy density, P first Piola-Kirchhoff stress, f_int / f_ext
internal / external nodal forces, K stiffness, K_T tangent stiffness.

Conventions
-----------
* DOF g = node * d + component (node-major).
* Element arrays are vectorised over elements with numpy; each formula is
  the textbook definition with no reordering beyond that.
"""
import numpy as np
import scipy.sparse as sp

LINEAR = ("lin_plane_stress", "lin_plane_strain", "lin_3d")
NEOHOOKE = ("nh_plane_strain", "nh_3d")


# --------------------------------------------------------------- materials
def lame_parameters(model, param_kind, p0, p1):
    """Per-element (mu, lambda).

    Sec. 'Nonlinear hyperelasticity', Lame-parameter equation:
        lambda = nu E / ((1 + nu)(1 - 2 nu)),  mu = E / (2 (1 + nu)).
    For the linear plate the paper states plane stress (Sec. 'Linear elastic
    plate with arbitrary holes') but prints the plane-strain/3D law; the
    reading used here is the textbook plane-stress law, obtained by
    replacing lambda with lambda* = E nu / (1 - nu^2)
    (= 2 mu lambda / (lambda + 2 mu) when Lame parameters are given).
    """
    p0 = np.asarray(p0, dtype=np.float64)
    p1 = np.asarray(p1, dtype=np.float64)
    if param_kind == "E_nu":
        E, nu = p0, p1
        mu = E / (2.0 * (1.0 + nu))
        if model == "lin_plane_stress":
            lam = E * nu / (1.0 - nu * nu)
        else:
            lam = nu * E / ((1.0 + nu) * (1.0 - 2.0 * nu))
    elif param_kind == "lame":
        mu, lam = p0.copy(), p1.copy()
        if model == "lin_plane_stress":
            lam = 2.0 * mu * lam / (lam + 2.0 * mu)
    else:
        raise ValueError(param_kind)
    return mu, lam


# -------------------------------------------------------------- kinematics
def shape_gradients(coords, conn):
    """Gradients of the P1 shape functions and element measures.

    App. B (total-Lagrangian discretisation, X_i = N_I X_iI): with
    J_e = [X_1 - X_0, ..., X_d - X_0] the rows of J_e^{-1} are grad N_1 ..
    grad N_d, grad N_0 = -sum_{a>=1} grad N_a, and the element measure is
    |det J_e| / d!.  Returns G (N_e, d+1, d) and vol (N_e,).
    """
    X = np.asarray(coords, dtype=np.float64)[conn]          # (E, d+1, d)
    d = X.shape[2]
    Je = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))  # columns X_a-X_0
    det = np.linalg.det(Je)
    inv = np.linalg.inv(Je)                                  # rows = grad N_a
    G = np.empty((X.shape[0], d + 1, d))
    G[:, 1:, :] = inv
    G[:, 0, :] = -inv.sum(axis=1)
    vol = np.abs(det) / (2.0 if d == 2 else 6.0)
    return G, vol


def displacement_gradient(u, conn, G):
    """H = grad u = sum_a u_a (x) grad N_a per element (E, d, d)."""
    d = G.shape[2]
    ue = np.asarray(u, dtype=np.float64).reshape(-1, d)[conn]   # (E, d+1, d)
    return np.einsum("eai,eaj->eij", ue, G)


# ---------------------------------------------------------- linear elastic
def linear_stress(H, mu, lam):
    """sigma = 2 mu eps + lambda tr(eps) I,  eps = sym(H).

    Sec. 'Linear elastic plate with arbitrary holes', loss equation
    (E/(1+nu) = 2 mu; E nu/((1+nu)(1-2nu)) = lambda).
    """
    eps = 0.5 * (H + np.transpose(H, (0, 2, 1)))
    tr = np.trace(eps, axis1=1, axis2=2)
    d = H.shape[1]
    return 2.0 * mu[:, None, None] * eps + (lam * tr)[:, None, None] * np.eye(d)


def linear_energy_density(H, mu, lam):
    """Psi = 1/2 sigma : eps (same equation)."""
    eps = 0.5 * (H + np.transpose(H, (0, 2, 1)))
    sig = linear_stress(H, mu, lam)
    return 0.5 * np.einsum("eij,eij->e", sig, eps)


# ------------------------------------------------------------ Neo-Hookean
def nh_invariants(H):
    """j = J - 1, log J and |H|^2 from H without forming F.

    J = det(I + H).  In 2D det(I + H) - 1 = tr H + det H; in 3D it is
    tr H + 1/2((tr H)^2 - tr(H^2)) + det H.  These are exact identities,
    used so that J - 1 keeps its relative accuracy at small strain.
    """
    d = H.shape[1]
    tr = np.trace(H, axis1=1, axis2=2)
    detH = np.linalg.det(H)
    if d == 2:
        j = tr + detH
    else:
        trH2 = np.einsum("eij,eji->e", H, H)
        j = tr + 0.5 * (tr * tr - trH2) + detH
    return j, tr, detH


def nh_energy_density(H, mu, lam):
    """Psi = 1/2 lambda (ln J)^2 - mu ln J + 1/2 mu (I1 - d).

    Sec. 'Nonlinear hyperelasticity', Neo-Hookean loss equation, with
    J = det F, I1 = tr(F^T F), F = I + H.  The paper writes I1 - 2 for its
    plane-strain examples; the reading here is I1 - d (d = 2 plane strain,
    d = 3 in 3D) so that Psi(I) = 0.  Returns +inf where J <= 0.

    Evaluated as mu[(tr H - j) + 1/2 |H|^2 + (j - log1p j)] + 1/2 lambda
    (log1p j)^2, which is the same expression: I1 - d = 2 tr H + |H|^2 and
    ln J = log1p(j).
    """
    d = H.shape[1]
    j, tr, detH = nh_invariants(H)
    bad = j <= -1.0
    jj = np.where(bad, 0.0, j)
    lnJ = np.log1p(jj)
    h2 = np.einsum("eij,eij->e", H, H)
    psi = mu * ((tr - jj) + 0.5 * h2 + (jj - lnJ)) + 0.5 * lam * lnJ * lnJ
    return np.where(bad, np.inf, psi)


def nh_energy_density_direct(H, mu, lam):
    """The same density evaluated literally from F (for cross-checks)."""
    d = H.shape[1]
    F = np.eye(d) + H
    J = np.linalg.det(F)
    C = np.einsum("eki,ekj->eij", F, F)
    I1 = np.trace(C, axis1=1, axis2=2)
    with np.errstate(invalid="ignore", divide="ignore"):
        lnJ = np.log(J)
    psi = 0.5 * lam * lnJ ** 2 - mu * lnJ + 0.5 * mu * (I1 - d)
    return np.where(J > 0, psi, np.inf)


def nh_piola(H, mu, lam):
    """P = dPsi/dF = mu (F - F^{-T}) + lambda ln J F^{-T}.

    App. B writes the internal force with F S (S the second Piola-Kirchhoff
    stress); F S = P.  F - F^{-T} is evaluated as H + F^{-T} H^T (exact
    identity, I - F^{-T} = F^{-T} (F^T - I)).
    """
    d = H.shape[1]
    F = np.eye(d) + H
    FinvT = np.transpose(np.linalg.inv(F), (0, 2, 1))
    j, _, _ = nh_invariants(H)
    lnJ = np.log1p(j)
    FmFinvT = H + np.einsum("eik,ejk->eij", FinvT, H)
    return mu[:, None, None] * FmFinvT + (lam * lnJ)[:, None, None] * FinvT


def nh_tangent_moduli(H, mu, lam):
    """A_iJkL = dP_iJ / dF_kL (E, d, d, d, d).

    A = mu d_ik d_JL + lambda Finv_Ji Finv_Lk + (mu - lambda ln J) Finv_Li Finv_Jk,
    the material + geometric tangent of App. B (K_mat + K_geo) written in
    first-Piola form.
    """
    d = H.shape[1]
    F = np.eye(d) + H
    Fi = np.linalg.inv(F)
    j, _, _ = nh_invariants(H)
    lnJ = np.log1p(j)
    I = np.eye(d)
    A = (mu[:, None, None, None, None] * np.einsum("ik,JL->iJkL", I, I)[None]
         + lam[:, None, None, None, None] * np.einsum("eJi,eLk->eiJkL", Fi, Fi)
         + (mu - lam * lnJ)[:, None, None, None, None]
         * np.einsum("eLi,eJk->eiJkL", Fi, Fi))
    return A


def linear_moduli(mu, lam, d):
    """C_ijkl = lambda d_ij d_kl + mu (d_ik d_jl + d_il d_jk)."""
    I = np.eye(d)
    base_l = np.einsum("ij,kl->ijkl", I, I)
    base_m = np.einsum("ik,jl->ijkl", I, I) + np.einsum("il,jk->ijkl", I, I)
    return lam[:, None, None, None, None] * base_l + mu[:, None, None, None, None] * base_m


# -------------------------------------------------------------- assembly
class Model:
    """Oracle view of one problem: geometry, materials, f_ext, Dirichlet.

    P1 meshes evaluate one point per element (G = grad N, vol = element
    measure).  Quadrilateral meshes (prob.elem 'q4' / 'q8', see quad.py)
    evaluate one point per Gauss point: `conn`, `G`, `vol`, `mu`, `lam` and
    `dofs` are then per quadrature point (the element's row repeated), and
    every sum below is a sum over those points.
    """

    def __init__(self, prob):
        self.prob = prob
        self.model = prob.model
        self.d = prob.dim
        self.elem = getattr(prob, "elem", "p1")
        conn = np.asarray(prob.conn, dtype=np.int64)
        self.coords = np.asarray(prob.coords, dtype=np.float64)
        self.n_dof = self.coords.shape[0] * self.d
        mu, lam = lame_parameters(prob.model, prob.param_kind, prob.p0, prob.p1)
        if self.elem == "p1":
            self.conn = conn
            self.G, self.vol = shape_gradients(self.coords, conn)
            self.elem_of = np.arange(len(conn))
        else:
            from . import quad
            self.G, self.vol, _, self.elem_of = quad.point_geometry(self.coords, conn,
                                                                    self.elem)
            self.conn = conn[self.elem_of]
        self.mu, self.lam = mu[self.elem_of], lam[self.elem_of]
        self.dofs = (self.conn[:, :, None] * self.d
                     + np.arange(self.d)[None, None, :]).reshape(len(self.conn), -1)
        self.f_ext = external_force(prob)
        dg = (np.asarray(prob.dir_nodes, np.int64) * self.d
              + np.asarray(prob.dir_comps, np.int64))
        self.dir_dofs = dg
        self.dir_vals = np.asarray(prob.dir_values, dtype=np.float64)
        free = np.ones(self.n_dof, dtype=bool)
        free[dg] = False
        self.free = free
        self.free_dofs = np.nonzero(free)[0]

    @property
    def linear(self):
        return self.model in LINEAR

    def H(self, u):
        return displacement_gradient(u, self.conn, self.G)

    def energy_density(self, u):
        H = self.H(u)
        if self.linear:
            return linear_energy_density(H, self.mu, self.lam)
        return nh_energy_density(H, self.mu, self.lam)

    def energy(self, u):
        """Pi(u) = sum_e vol_e Psi_e - f_ext . u.

        Loss equations of Sec. 'Linear elastic plate...' and Sec. 'Nonlinear
        hyperelasticity' with body force f = 0 (every workload here).
        """
        psi = self.energy_density(u)
        return float(np.sum(self.vol * psi) - self.f_ext @ u)

    def stress(self, u):
        H = self.H(u)
        if self.linear:
            return linear_stress(H, self.mu, self.lam)
        return nh_piola(H, self.mu, self.lam)

    def internal_force(self, u):
        """f_int,iI = sum_e vol_e P_iJ dN_I/dX_J (App. B, total Lagrangian).

        For the linear models P is replaced by sigma (small strain).
        """
        P = self.stress(u)
        fe = self.vol[:, None, None] * np.einsum("eij,eaj->eai", P, self.G)
        f = np.zeros(self.n_dof)
        np.add.at(f, self.dofs.reshape(-1), fe.reshape(-1))
        return f

    def gradient(self, u):
        """dPi/du = f_int(u) - f_ext (App. B residual r = f_int - f_ext)."""
        return self.internal_force(u) - self.f_ext

    def element_matrices(self, u=None):
        """Element stiffness / tangent blocks (E, (d+1)d, (d+1)d); per
        quadrature point (E*nq, nv d, nv d) on quadrilateral meshes.

        K_e[(a,i),(b,k)] = vol_e sum_{J,L} dN_a/dX_J  A_iJkL  dN_b/dX_L
        with A the linear moduli C (linear models) or the Neo-Hookean
        tangent of App. B (K_mat + K_geo).
        """
        d = self.d
        if self.linear:
            A = linear_moduli(self.mu, self.lam, d)
        else:
            A = nh_tangent_moduli(self.H(u), self.mu, self.lam)
        Ke = np.einsum("e,eaJ,eiJkL,ebL->eaibk", self.vol, self.G, A, self.G,
                       optimize=True)
        n = self.conn.shape[1] * d
        return Ke.reshape(len(self.conn), n, n)

    def assemble(self, u=None):
        """Global K (linear) or K_T(u) (Neo-Hookean) as scipy CSR."""
        Ke = self.element_matrices(u)
        n = Ke.shape[1]
        rows = np.repeat(self.dofs, n, axis=1).reshape(-1)
        cols = np.tile(self.dofs, (1, n)).reshape(-1)
        K = sp.coo_matrix((Ke.reshape(-1), (rows, cols)),
                          shape=(self.n_dof, self.n_dof)).tocsr()
        K.sum_duplicates()
        return K

    def lifted(self, scale=1.0):
        """Zero on free DOFs, scale * Dirichlet value on constrained DOFs."""
        u = np.zeros(self.n_dof)
        u[self.dir_dofs] = scale * self.dir_vals
        return u


def external_force(prob):
    """Consistent nodal loads of piecewise-constant tractions.

    App. B: f_ext,iI = int_{Gamma_t} N_I t_i dGamma.  For a P1 facet with a
    constant traction this puts t * |facet| / n_f on each of its n_f nodes
    (n_f = 2 for an edge, 3 for a triangle).  A 3-node edge of a Q8 mesh
    (ends, then the middle node) integrates its quadratic shape functions
    (quad.edge_loads).  Body force is zero.
    """
    d = prob.dim
    f = np.zeros(prob.n_dof)
    fac = np.asarray(prob.neu_facets, dtype=np.int64)
    if fac.size == 0:
        return f
    if d == 2 and fac.shape[1] == 3:
        from . import quad
        fl = quad.edge_loads(prob.coords, fac, prob.neu_traction)
        for a in range(3):
            for i in range(2):
                np.add.at(f, fac[:, a] * 2 + i, fl[:, a, i])
        return f
    P = np.asarray(prob.coords, dtype=np.float64)[fac]
    if d == 2:
        meas = np.linalg.norm(P[:, 1] - P[:, 0], axis=1)
    else:
        meas = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0],
                                             P[:, 2] - P[:, 0]), axis=1)
    nf = fac.shape[1]
    t = np.asarray(prob.neu_traction, dtype=np.float64)
    for a in range(nf):
        for i in range(d):
            np.add.at(f, fac[:, a] * d + i, t[:, i] * meas / nf)
    return f
