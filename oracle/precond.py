"""Two-level additive preconditioner in float64 (oracle; test infrastructure
only: only tests/, the smoke check and the benchmark's CPU leg use it).

The paper leaves the preconditioner of its conjugate-gradient solves open
and notes (§5.6) that a stronger preconditioner and the warm start are
complementary.  The stronger one built here is the additive two-level
preconditioner
    M^-1 = D^-1 + P (P^T K P)^-1 P^T
on the free DOFs: D the diagonal of K_ff (the Jacobi part), and P the coarse
space spanned on each aggregate of nodes by the rigid-body modes of linear
elasticity (in 2D two translations and the rotation (-(y - c_y), x - c_x);
in 3D three translations and three rotations omega x (X - c)), zero outside
the aggregate and at prescribed DOFs, c the aggregate's centroid.  The
coarse term is basis-free -- P (P^T K P)^-1 P^T depends only on the span of
P -- so this oracle spans it with the raw modes after dropping those an
aggregate does not resolve (a QR with a rank test); any basis of the same
span gives the same M^-1.  Aggregates are given by the caller (a partition
of the nodes), not decided here.
"""
import numpy as np
import scipy.linalg as sla


def rigid_modes(coords, nodes, dim):
    """Raw rigid-body modes of the node set, (len(nodes) * dim, n_rb)."""
    X = np.asarray(coords, dtype=np.float64)[nodes]
    c = X.mean(axis=0)
    Y = X - c
    n = len(nodes)
    if dim == 2:
        R = np.zeros((n, 2, 3))
        R[:, 0, 0] = 1.0
        R[:, 1, 1] = 1.0
        R[:, 0, 2] = -Y[:, 1]
        R[:, 1, 2] = Y[:, 0]
        return R.reshape(2 * n, 3)
    R = np.zeros((n, 3, 6))
    for i in range(3):
        R[:, i, i] = 1.0
    # omega x Y for unit omega along x, y, z
    R[:, 1, 3], R[:, 2, 3] = -Y[:, 2], Y[:, 1]
    R[:, 0, 4], R[:, 2, 4] = Y[:, 2], -Y[:, 0]
    R[:, 0, 5], R[:, 1, 5] = -Y[:, 1], Y[:, 0]
    return R.reshape(3 * n, 6)


def coarse_basis(coords, aggregates, dim, free_mask, rank_tol=1e-10):
    """P (n_dof, n_c): per aggregate an orthonormal basis of its rigid modes
    restricted to its free DOFs (columns the aggregate does not resolve are
    dropped)."""
    n_dof = len(coords) * dim
    cols = []
    agg = np.asarray(aggregates)
    for a in np.unique(agg):
        nodes = np.nonzero(agg == a)[0]
        dofs = (nodes[:, None] * dim + np.arange(dim)[None, :]).reshape(-1)
        R = rigid_modes(coords, nodes, dim)
        R[~free_mask[dofs]] = 0.0
        if not np.any(R):
            continue
        Q, T, piv = sla.qr(R, mode="economic", pivoting=True)
        diag = np.abs(np.diag(T))
        keep = diag > rank_tol * diag.max()
        for k in np.nonzero(keep)[0]:
            col = np.zeros(n_dof)
            col[dofs] = Q[:, k]
            cols.append(col)
    return np.array(cols).T if cols else np.zeros((n_dof, 0))


def two_level(Kff, free_dofs, coords, aggregates, dim):
    """M^-1 on the free DOFs as a function r_f -> z_f."""
    n_dof = len(coords) * dim
    free_mask = np.zeros(n_dof, dtype=bool)
    free_mask[free_dofs] = True
    P = coarse_basis(coords, aggregates, dim, free_mask)[free_dofs]
    Ac = P.T @ (Kff @ P)
    cho = sla.cho_factor(Ac)
    dinv = 1.0 / Kff.diagonal()

    def apply(r):
        return dinv * r + P @ sla.cho_solve(cho, P.T @ r)

    apply.P = P
    apply.Ac = Ac
    return apply
