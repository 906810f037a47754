"""Independent references that pin the oracle (tests only).

Each one follows from the mathematics of the discrete problem, not from the
oracle's code:

* ``gradient_matrix`` / ``dense_operator``: the finite-volume operator in its
  factorised form L = -G^T B G / h^2 (G: signed face differences, B: diagonal
  of face coefficients), which is how a flux-form discretisation is defined;
* ``dense_solve``: the zero-mean solution of the bordered system by numpy's
  dense solver (tiny grids);
* ``dct_solve``: constant coefficient -- the DCT-II diagonalises the
  cell-centred Neumann Laplacian, eigenvalue -(4/h^2) sum_d sin^2(pi m_d / 2N_d);
* ``layered_solve``: coefficient varying in z only and a right-hand side
  cos(pi mx x) cos(pi my y) g(z) reduce exactly to one tridiagonal system in z;
* ``closed_form``: the discrete solution for b = -3 pi^2 cos(pi x)cos(pi y)cos(pi z)
  at constant coefficient 1.
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.linalg
import scipy.sparse as sp


def gradient_matrix(dims):
    """Sparse G mapping cell values to interior-face differences, and face index maps.

    Rows are the interior faces in the order x-faces, y-faces, z-faces, each in the
    public face layout order restricted to interior faces.  Returns (G, masks) with
    masks the boolean interior masks of the three face arrays.
    """
    nx, ny, nz = dims
    idx = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []
    r0 = 0
    masks = []
    # x faces: between (k,j,i-1) and (k,j,i), i = 1..nx-1
    for axis, shape in ((2, (nz, ny, nx + 1)), (1, (nz, ny + 1, nx)), (0, (nz + 1, ny, nx))):
        m = np.zeros(shape, dtype=bool)
        if axis == 2:
            m[:, :, 1:nx] = True
            left, right = idx[:, :, :-1], idx[:, :, 1:]
        elif axis == 1:
            m[:, 1:ny, :] = True
            left, right = idx[:, :-1, :], idx[:, 1:, :]
        else:
            m[1:nz, :, :] = True
            left, right = idx[:-1, :, :], idx[1:, :, :]
        nf = left.size
        r = np.arange(r0, r0 + nf)
        rows += [r, r]
        cols += [right.ravel(), left.ravel()]
        vals += [np.ones(nf), -np.ones(nf)]
        r0 += nf
        masks.append(m)
    G = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(r0, nx * ny * nz))
    return G, masks


def interior_faces(beta, masks):
    return np.concatenate([b[m] for b, m in zip(beta, masks)])


def dense_operator(beta, h):
    """L = -G^T diag(beta_interior) G / h^2 as a dense matrix (tiny grids)."""
    bx = beta[0]
    nz, ny, nx1 = bx.shape
    dims = (nx1 - 1, ny, nz)
    G, masks = gradient_matrix(dims)
    B = sp.diags(interior_faces(beta, masks))
    return -(G.T @ B @ G).toarray() / (h * h)


def sparse_operator(beta, h):
    bx = beta[0]
    nz, ny, nx1 = bx.shape
    G, masks = gradient_matrix((nx1 - 1, ny, nz))
    B = sp.diags(interior_faces(beta, masks))
    return (-(G.T @ B @ G) / (h * h)).tocsr()


def bilinear(beta, x, y, h):
    """-sum_f beta_f (dx)_f (dy)_f / h^2 over interior faces, via numpy differences."""
    bx, by, bz = beta
    s = 0.0
    s += np.sum(bx[:, :, 1:-1] * np.diff(x, axis=2) * np.diff(y, axis=2))
    s += np.sum(by[:, 1:-1, :] * np.diff(x, axis=1) * np.diff(y, axis=1))
    s += np.sum(bz[1:-1, :, :] * np.diff(x, axis=0) * np.diff(y, axis=0))
    return -s / (h * h)


def dense_solve(beta, rhs, h):
    """Zero-mean p with L p = rhs - mean(rhs) from the bordered dense system."""
    L = dense_operator(beta, h)
    n = L.shape[0]
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = L
    M[:n, n] = 1.0
    M[n, :n] = 1.0
    f = np.concatenate([rhs.ravel(), [0.0]])
    sol = np.linalg.solve(M, f)
    return sol[:n].reshape(rhs.shape)


def sparse_direct_solve(beta, rhs, h):
    """Bordered sparse direct solve (scipy); moderate grids only."""
    from scipy.sparse.linalg import spsolve
    A = sparse_operator(beta, h)
    n = A.shape[0]
    one = sp.csr_matrix(np.ones((n, 1)))
    M = sp.bmat([[A, one], [one.T, None]], format="csc")
    f = np.concatenate([rhs.ravel() - rhs.mean(), [0.0]])
    sol = spsolve(M, f)
    return sol[:n].reshape(rhs.shape)


def neumann_eigenvalues(n, h):
    m = np.arange(n)
    return -(4.0 / (h * h)) * np.sin(np.pi * m / (2.0 * n)) ** 2


def dct_solve(rhs, h, beta0=1.0):
    """Constant face coefficient beta0: zero-mean solution via the DCT-II."""
    nz, ny, nx = rhs.shape
    bh = scipy.fft.dctn(rhs, type=2, norm="ortho")
    lam = (neumann_eigenvalues(nz, h)[:, None, None] + neumann_eigenvalues(ny, h)[None, :, None]
           + neumann_eigenvalues(nx, h)[None, None, :]) * beta0
    lam[0, 0, 0] = 1.0
    ph = bh / lam
    ph[0, 0, 0] = 0.0
    return scipy.fft.idctn(ph, type=2, norm="ortho")


def constant_beta(dims, value=1.0):
    nx, ny, nz = dims
    bx = np.full((nz, ny, nx + 1), value)
    by = np.full((nz, ny + 1, nx), value)
    bz = np.full((nz + 1, ny, nx), value)
    bx[:, :, 0] = bx[:, :, nx] = 0.0
    by[:, 0, :] = by[:, ny, :] = 0.0
    bz[0] = bz[nz] = 0.0
    return bx, by, bz


def layered_beta(dims, rho_layers):
    """Face coefficients of a density that depends on z only (rho_layers[k])."""
    nx, ny, nz = dims
    rho = np.asarray(rho_layers, dtype=np.float64)
    bx = np.zeros((nz, ny, nx + 1))
    by = np.zeros((nz, ny + 1, nx))
    bz = np.zeros((nz + 1, ny, nx))
    cell = 2.0 / (rho + rho)
    bx[:, :, 1:nx] = cell[:, None, None]
    by[:, 1:ny, :] = cell[:, None, None]
    bz[1:nz, :, :] = (2.0 / (rho[:-1] + rho[1:]))[:, None, None]
    return bx, by, bz


def layered_solve(dims, h, rho_layers, mx, my, g):
    """Exact solution of L p = cos(pi mx x) cos(pi my y) g(z) for z-layered density.

    With p = cos(pi mx x) cos(pi my y) q(z), q solves the tridiagonal system
      [bz_{k+1}(q_{k+1} - q_k) - bz_k (q_k - q_{k-1})]/h^2 + (1/rho_k) mu q_k = g_k,
    mu = -(4/h^2)(sin^2(pi mx h/2) + sin^2(pi my h/2)); (mx, my) != (0, 0).
    Returns (rhs, p) as [nz, ny, nx] arrays.
    """
    nx, ny, nz = dims
    assert (mx, my) != (0, 0)
    rho = np.asarray(rho_layers, dtype=np.float64)
    bzf = np.zeros(nz + 1)
    bzf[1:nz] = 2.0 / (rho[:-1] + rho[1:])
    bcell = 1.0 / rho
    mu = -(4.0 / (h * h)) * (np.sin(np.pi * mx * h / 2.0) ** 2 + np.sin(np.pi * my * h / 2.0) ** 2)
    lower = bzf[1:nz] / (h * h)            # coefficient of q_{k-1} in row k (k >= 1)
    upper = bzf[1:nz] / (h * h)            # coefficient of q_{k+1} in row k (k <= nz-2)
    diag = -(bzf[:nz] + bzf[1:]) / (h * h) + bcell * mu
    ab = np.zeros((3, nz))
    ab[0, 1:] = upper
    ab[1, :] = diag
    ab[2, :-1] = lower
    q = scipy.linalg.solve_banded((1, 1), ab, np.asarray(g, dtype=np.float64))
    xc = (np.arange(nx) + 0.5) * h
    yc = (np.arange(ny) + 0.5) * h
    cx = np.cos(np.pi * mx * xc)
    cy = np.cos(np.pi * my * yc)
    mode = cy[:, None] * cx[None, :]
    rhs = np.asarray(g)[:, None, None] * mode[None, :, :]
    p = q[:, None, None] * mode[None, :, :]
    return rhs, p


def closed_form(n):
    """b = -3 pi^2 cos(pi x)cos(pi y)cos(pi z) at cell centres, beta = 1.

    Returns (b, p_discrete, p_continuous): the exact discrete solution is
    c(h) cos cos cos with c(h) = ((pi h/2)/sin(pi h/2))^2.
    """
    h = 1.0 / n
    xc = (np.arange(n) + 0.5) * h
    c = np.cos(np.pi * xc)
    mode = c[:, None, None] * c[None, :, None] * c[None, None, :]
    b = -3.0 * np.pi ** 2 * mode
    ch = ((np.pi * h / 2.0) / np.sin(np.pi * h / 2.0)) ** 2
    return b, ch * mode, mode


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
