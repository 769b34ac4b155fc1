"""Seeded element-wise diffusion coefficients and analytic sources."""
import numpy as np


def _centroids(mesh):
    return mesh.coords[mesh.e2v].mean(axis=1)


def kappa_grf(mesh, seed, corr_len=0.1, n_features=2048):
    """kappa_e = exp(g(c_e)), g a unit-variance Gaussian field with squared-
    exponential covariance exp(-r^2 / (2 l^2)), sampled with random Fourier
    features (Rahimi & Recht 2007) at the element centroids c_e."""
    rng = np.random.default_rng(seed)
    d = mesh.dim
    omega = rng.normal(0.0, 1.0 / corr_len, size=(n_features, d))
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n_features)
    c = _centroids(mesh)
    g = np.sqrt(2.0 / n_features) * np.cos(c @ omega.T + phase).sum(axis=1)
    return np.exp(g)


def kappa_spheres(mesh, seed, n_spheres=32, rmin=0.05, rmax=0.15, high=1e3, low=1.0):
    """kappa_e = high if the centroid of element e lies in any of n_spheres
    spheres with centres ~ U[0,1]^d and radii ~ U[rmin, rmax], else low."""
    rng = np.random.default_rng(seed)
    d = mesh.dim
    centres = rng.uniform(0.0, 1.0, size=(n_spheres, d))
    radii = rng.uniform(rmin, rmax, size=n_spheres)
    c = _centroids(mesh)
    inside = np.zeros(c.shape[0], dtype=bool)
    for k in range(n_spheres):
        inside |= np.sum((c - centres[k]) ** 2, axis=1) <= radii[k] ** 2
    return np.where(inside, high, low).astype(np.float64)


def exact_sine(x):
    """u(x) = prod_i sin(pi x_i)."""
    return np.prod(np.sin(np.pi * x), axis=-1)


def source_sine(x):
    """f = -Laplace(u) = d pi^2 u for u = prod_i sin(pi x_i)."""
    d = x.shape[-1]
    return d * np.pi ** 2 * exact_sine(x)
