"""Random-Fourier-feature fields, boundary lifting and warm-start noise.

A random-Fourier-feature (RFF) field g(x) = sqrt(2/M) * sum_m cos(w_m . x + b_m)
with w_m ~ N(0, l^-2 I) and b_m ~ U[0, 2 pi) has unit marginal variance and
approaches a Gaussian random field with the squared-exponential covariance
exp(-|r|^2 / (2 l^2)) as M grows (Rahimi & Recht, 2007).
"""
import numpy as np
from scipy.spatial import cKDTree


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def rff_field(points, seed, length, n_features=256, n_comp=1):
    """Evaluate ``n_comp`` independent unit-variance RFF fields at ``points``.

    points: (N, d) float64.  Returns (N, n_comp) float64 (or (N,) if n_comp=1).
    """
    pts = np.asarray(points, dtype=np.float64)
    d = pts.shape[1]
    rng = _rng(seed)
    out = np.empty((pts.shape[0], n_comp))
    scale = np.sqrt(2.0 / n_features)
    for c in range(n_comp):
        w = rng.normal(0.0, 1.0 / length, size=(n_features, d))
        b = rng.uniform(0.0, 2.0 * np.pi, size=n_features)
        acc = np.zeros(pts.shape[0])
        # chunk over features to bound memory on million-point meshes
        for m0 in range(0, n_features, 64):
            acc += np.cos(pts @ w[m0:m0 + 64].T + b[m0:m0 + 64]).sum(axis=1)
        out[:, c] = scale * acc
    return out[:, 0] if n_comp == 1 else out


def lifting_weight(coords, dirichlet_nodes, width=0.1):
    """min(1, dist(x, Dirichlet nodes)/width): vanishes on the Dirichlet set."""
    coords = np.asarray(coords, dtype=np.float64)
    if len(dirichlet_nodes) == 0:
        return np.ones(coords.shape[0])
    tree = cKDTree(coords[np.unique(dirichlet_nodes)])
    dist, _ = tree.query(coords, k=1)
    return np.minimum(1.0, dist / width)


def warm_start_noise(coords, dirichlet_nodes, seed, length=0.2, n_features=256):
    """The unscaled noise l(x) g(x) of ``warm_start_guess`` (node-major,
    zero on the Dirichlet nodes)."""
    coords = np.asarray(coords, dtype=np.float64)
    n, d = coords.shape
    g = rff_field(coords, seed, length, n_features, n_comp=d)
    w = lifting_weight(coords, dirichlet_nodes)
    return (g * w[:, None]).reshape(-1)


def warm_start_guess(u_star, coords, dirichlet_nodes, seed, rel=0.01,
                     length=0.2, n_features=256, noise=None):
    """Synthetic network prediction: u_star + s * l(x) * g(x).

    u_star: (N_n*d,) node-major reference displacement (it already carries the
    Dirichlet values).  The smooth noise g is one RFF field per component,
    multiplied by the boundary lifting l(x) so the guess keeps the Dirichlet
    values exactly, and scaled so its 2-norm is ``rel`` * |u_star|.  A noise
    precomputed by ``warm_start_noise`` may be passed in.
    """
    if noise is None:
        noise = warm_start_noise(coords, dirichlet_nodes, seed, length, n_features)
    nn = np.linalg.norm(noise)
    s = 0.0 if nn == 0.0 else rel * np.linalg.norm(u_star) / nn
    return np.asarray(u_star, dtype=np.float64) + s * noise
