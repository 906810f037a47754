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
  at constant coefficient 1;
* ``MatrixMultigrid``: the multigrid cycle composed from explicit level matrices
  (operator, restriction, prolongation), sequential point Gauss-Seidel over the
  two colours and a dense bordered coarsest solve (tiny grids).
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


# ---------------------------------------------------------------------------
# A multilevel cycle assembled from matrices (pins the oracle's V-cycle)
# ---------------------------------------------------------------------------
#
# Every piece below is a matrix or a loop written from its definition; nothing
# is taken from the oracle:
#   * operator of level l:      A_l = -G^T B_l G / h_l^2            (dense_operator)
#   * coarse coefficients:      coarse face = mean of the 4 fine faces that tile it
#   * restriction R:            coarse cell = mean of its 8 children (matrix of 1/8)
#   * prolongation P:           tensor product of the 1-D cell-centred linear
#                               interpolation (3/4 parent, 1/4 the parent's
#                               neighbour on the fine cell's side; at a wall the
#                               parent stands in for the missing neighbour)
#   * smoother:                 sequential point Gauss-Seidel with unit relaxation
#                               over the cells of one colour, (i+j+k) mod 2
#   * coarsest grid:            dense bordered solve [[A, 1], [1^T, 0]]
# and the cycle composes them: `pre` sweeps of (red, black), residual, restrict,
# recurse from zero, prolongate and add, `post` sweeps of (black, red).

def coarse_faces_from_definition(beta):
    """Coarse face coefficients: each coarse face is the arithmetic mean of the
    four fine faces lying in it; wall faces are zero."""
    bx, by, bz = beta
    nz, ny, nx1 = bx.shape
    nx = nx1 - 1
    cx, cy, cz = nx // 2, ny // 2, nz // 2
    fx = bx[:, :, 0:nx + 1:2]                         # fine x-faces on coarse x-face planes
    cbx = fx.reshape(cz, 2, cy, 2, cx + 1).mean(axis=(1, 3))
    fy = by[:, 0:ny + 1:2, :]
    cby = fy.reshape(cz, 2, cy + 1, cx, 2).mean(axis=(1, 4))
    fz = bz[0:nz + 1:2, :, :]
    cbz = fz.reshape(cz + 1, cy, 2, cx, 2).mean(axis=(2, 4))
    cbx[:, :, 0] = cbx[:, :, cx] = 0.0
    cby[:, 0, :] = cby[:, cy, :] = 0.0
    cbz[0] = cbz[cz] = 0.0
    return cbx, cby, cbz


def restriction_matrix(dims):
    """R (coarse cells x fine cells): 1/8 at each of a coarse cell's 8 children."""
    nx, ny, nz = dims
    R = np.zeros((nx * ny * nz // 8, nx * ny * nz))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                parent = ((k // 2) * (ny // 2) + j // 2) * (nx // 2) + i // 2
                R[parent, (k * ny + j) * nx + i] = 0.125
    return R


def linear_interp_1d(nf):
    """1-D cell-centred interpolation (nf x nf/2): fine cell i lies in parent
    I = i // 2, a quarter cell towards neighbour I - 1 (i even) or I + 1 (i odd)."""
    nc = nf // 2
    P = np.zeros((nf, nc))
    for i in range(nf):
        parent = i // 2
        nb = parent - 1 if i % 2 == 0 else parent + 1
        if nb < 0 or nb >= nc:
            nb = parent                     # wall: the parent replaces the missing neighbour
        P[i, parent] += 0.75
        P[i, nb] += 0.25
    return P


def prolongation_matrix(dims):
    """P (fine cells x coarse cells) = Pz (x) Py (x) Px for x-fastest ordering."""
    nx, ny, nz = dims
    return np.kron(linear_interp_1d(nz), np.kron(linear_interp_1d(ny), linear_interp_1d(nx)))


def colour_of_cells(dims):
    nx, ny, nz = dims
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((i + j + k) % 2).ravel()


def gauss_seidel_colour(A, b, x, colour_mask):
    """Sequential point Gauss-Seidel over the cells of one colour, in index
    order: x_i = (b_i - sum_{j != i} A_ij x_j) / A_ii, each update seen by the next."""
    for i in np.flatnonzero(colour_mask):
        row = A[i]
        x[i] = (b[i] - (row @ x - row[i] * x[i])) / row[i]
    return x


def bordered_solve(A, r):
    n = A.shape[0]
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = A
    M[:n, n] = 1.0
    M[n, :n] = 1.0
    return np.linalg.solve(M, np.concatenate([r, [0.0]]))[:n]


class MatrixMultigrid:
    """Level matrices for the cycle above; `coarse_max` as in the solver: halve
    every dimension while any exceeds it."""

    def __init__(self, beta, h, coarse_max=4):
        self.A, self.R, self.P, self.colour = [], [], [], []
        bx = beta[0]
        nz, ny, nx1 = bx.shape
        dims = (nx1 - 1, ny, nz)
        while True:
            self.A.append(dense_operator(beta, h))
            self.colour.append(colour_of_cells(dims))
            if max(dims) <= coarse_max:
                break
            self.R.append(restriction_matrix(dims))
            self.P.append(prolongation_matrix(dims))
            beta = coarse_faces_from_definition(beta)
            dims = tuple(d // 2 for d in dims)
            h = 2.0 * h

    def cycle(self, level, b, x, pre, post, post_order=(1, 0)):
        A = self.A[level]
        if level == len(self.A) - 1:
            return bordered_solve(A, b)
        red = self.colour[level] == 0
        black = ~red
        for _ in range(pre):
            gauss_seidel_colour(A, b, x, red)
            gauss_seidel_colour(A, b, x, black)
        r = b - A @ x
        e = self.cycle(level + 1, self.R[level] @ r, np.zeros(self.R[level].shape[0]), pre, post, post_order)
        x += self.P[level] @ e
        masks = {0: red, 1: black}
        for _ in range(post):
            gauss_seidel_colour(A, b, x, masks[post_order[0]])
            gauss_seidel_colour(A, b, x, masks[post_order[1]])
        return x

    def cycles(self, rhs, x0, count, pre=2, post=2, post_order=(1, 0)):
        """`count` cycles on L x = rhs - mean(rhs) from x0 (mean of x kept)."""
        b = rhs.ravel() - rhs.mean()
        x = np.array(x0, dtype=np.float64).ravel().copy()
        for _ in range(count):
            x = self.cycle(0, b, x, pre, post, post_order)
        return x.reshape(rhs.shape)
