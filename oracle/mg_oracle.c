/*
 * Plain FP64 CPU oracle for the variable-density pressure-Poisson solve
 *
 *     div( (1/rho) grad p ) = div(u*) / dt        (homogeneous Neumann walls)
 *
 * solved by a geometric-multigrid V-cycle with red-black Gauss-Seidel.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU library
 * is checked against.  Nothing in the product path may link, load or call it;
 * it shares no code, header, table or helper with the GPU library.  It is
 * written as plain loops over cells in the order the method defines, with no
 * blocking or fusion, and favours obviousness over speed.  The only
 * concession to speed is an OpenMP "parallel for" over z-layers in loops whose
 * iterations are independent (within one colour of a red-black half-sweep no
 * cell reads another cell of its own colour, so the result equals the
 * sequential loop bit for bit).
 *
 * What the paper fixes and what is read into it:
 *  - cell density is the volume-weighted sum over phases
 *    (Sec. 2, eq. "property_calculation"): rho = sum_i rho_i f_i, with the gas
 *    fraction 1 - f_drop - f_film clamped at zero;
 *  - the discretisation is a finite-volume one on Cartesian meshes (Sec. 2);
 *    it is read as the cell-centred 7-point operator on the unit cube with
 *    uniform spacing h, face coefficient beta_f = 1/rho_face where rho_face is
 *    the arithmetic mean of the two cell densities, i.e. beta_f is the
 *    harmonic mean of 1/rho_L and 1/rho_R;
 *  - the paper names a multigrid solver with "switch levels" (Sec. 4.3.2) and
 *    gives no further detail.  The multigrid is read as: 2 pre (red, black)
 *    and 2 post (black, red) Gauss-Seidel sweeps with unit relaxation,
 *    residual restriction by averaging the 8 children, cell-centred trilinear
 *    prolongation (weights 3/4, 1/4 per axis, edge value reused at walls),
 *    coarse face coefficients as the mean of the 4 coincident fine faces, and
 *    an exact dense solve of the bordered system [[L,1],[1^T,0]] on the
 *    coarsest grid (every dimension <= coarse_max).
 *
 * Layouts (x fastest):
 *   cell arrays   [nz][ny][nx]
 *   beta_x, g_x   [nz][ny][nx+1]  entry i = face between cells i-1 and i
 *   beta_y, g_y   [nz][ny+1][nx]
 *   beta_z, g_z   [nz+1][ny][nx]
 * Wall faces (i = 0 or nx, etc.) carry no flux: their entries are never read
 * by the operator and are written as 0.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -2
#define OR_ENOCONV -4
#define OR_ENONFINITE -5

#define CELL(i, j, k) (((long)(k) * ny + (j)) * nx + (i))
#define FX(i, j, k) (((long)(k) * ny + (j)) * (nx + 1) + (i))
#define FY(i, j, k) (((long)(k) * (ny + 1) + (j)) * nx + (i))
#define FZ(i, j, k) (((long)(k) * ny + (j)) * nx + (i))

void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * Inputs of the solve: density, face coefficients, right-hand side
 * ------------------------------------------------------------------------- */

/* rho = rho_drop f_drop + rho_film f_film + rho_gas f_gas, f_gas = max(0, 1 - f_drop - f_film)
 * (Sec. 2, eq. "property_calculation") */
void or_density(const double *f_drop, const double *f_film, long n,
                double rho_drop, double rho_film, double rho_gas, double *rho)
{
    long c;
    for (c = 0; c < n; c++) {
        double fg = 1.0 - f_drop[c] - f_film[c];
        if (fg < 0.0) fg = 0.0;
        rho[c] = rho_drop * f_drop[c] + rho_film * f_film[c] + rho_gas * fg;
    }
}

/* beta_f = 2 / (rho_L + rho_R) on interior faces, 0 on wall faces */
void or_face_coeffs(const double *rho, int nx, int ny, int nz,
                    double *bx, double *by, double *bz)
{
    int i, j, k;
    for (k = 0; k < nz; k++)
        for (j = 0; j < ny; j++)
            for (i = 0; i <= nx; i++)
                bx[FX(i, j, k)] = (i == 0 || i == nx) ? 0.0
                    : 2.0 / (rho[CELL(i - 1, j, k)] + rho[CELL(i, j, k)]);
    for (k = 0; k < nz; k++)
        for (j = 0; j <= ny; j++)
            for (i = 0; i < nx; i++)
                by[FY(i, j, k)] = (j == 0 || j == ny) ? 0.0
                    : 2.0 / (rho[CELL(i, j - 1, k)] + rho[CELL(i, j, k)]);
    for (k = 0; k <= nz; k++)
        for (j = 0; j < ny; j++)
            for (i = 0; i < nx; i++)
                bz[FZ(i, j, k)] = (k == 0 || k == nz) ? 0.0
                    : 2.0 / (rho[CELL(i, j, k - 1)] + rho[CELL(i, j, k)]);
}

/* b = div_h(u, v, w) / dt, the discrete divergence of the MAC face velocities */
void or_divergence(const double *u, const double *v, const double *w,
                   int nx, int ny, int nz, double h, double dt, double *b)
{
    int i, j, k;
    for (k = 0; k < nz; k++)
        for (j = 0; j < ny; j++)
            for (i = 0; i < nx; i++) {
                double d = (u[FX(i + 1, j, k)] - u[FX(i, j, k)])
                         + (v[FY(i, j + 1, k)] - v[FY(i, j, k)])
                         + (w[FZ(i, j, k + 1)] - w[FZ(i, j, k)]);
                b[CELL(i, j, k)] = d / h / dt;
            }
}

/* u <- u - dt * beta_f * (p_R - p_L) / h on interior faces (the projection) */
void or_velocity_correct(const double *bx, const double *by, const double *bz,
                         int nx, int ny, int nz, double h, double dt, const double *p,
                         double *u, double *v, double *w)
{
    int i, j, k;
    for (k = 0; k < nz; k++)
        for (j = 0; j < ny; j++)
            for (i = 1; i < nx; i++)
                u[FX(i, j, k)] -= dt * bx[FX(i, j, k)] * (p[CELL(i, j, k)] - p[CELL(i - 1, j, k)]) / h;
    for (k = 0; k < nz; k++)
        for (j = 1; j < ny; j++)
            for (i = 0; i < nx; i++)
                v[FY(i, j, k)] -= dt * by[FY(i, j, k)] * (p[CELL(i, j, k)] - p[CELL(i, j - 1, k)]) / h;
    for (k = 1; k < nz; k++)
        for (j = 0; j < ny; j++)
            for (i = 0; i < nx; i++)
                w[FZ(i, j, k)] -= dt * bz[FZ(i, j, k)] * (p[CELL(i, j, k)] - p[CELL(i, j, k - 1)]) / h;
}

/* Gradient of a loss with respect to the cell density, given its gradient g_f
 * with respect to the face coefficients beta_f = 2/(rho_L + rho_R) (face
 * layouts):  d beta_f / d rho_L = d beta_f / d rho_R = -2 / (rho_L + rho_R)^2.
 * Every interior face adds its share to both of its cells; wall entries of
 * g are ignored. */
void or_density_grad(const double *rho, int nx, int ny, int nz,
                     const double *gx, const double *gy, const double *gz, double *grho)
{
    long n = (long)nx * ny * nz, c;
    int i, j, k;
    for (c = 0; c < n; c++)
        grho[c] = 0.0;
    for (k = 0; k < nz; k++)
        for (j = 0; j < ny; j++)
            for (i = 1; i < nx; i++) {
                double s = rho[CELL(i - 1, j, k)] + rho[CELL(i, j, k)];
                double d = gx[FX(i, j, k)] * (-2.0 / (s * s));
                grho[CELL(i - 1, j, k)] += d;
                grho[CELL(i, j, k)] += d;
            }
    for (k = 0; k < nz; k++)
        for (j = 1; j < ny; j++)
            for (i = 0; i < nx; i++) {
                double s = rho[CELL(i, j - 1, k)] + rho[CELL(i, j, k)];
                double d = gy[FY(i, j, k)] * (-2.0 / (s * s));
                grho[CELL(i, j - 1, k)] += d;
                grho[CELL(i, j, k)] += d;
            }
    for (k = 1; k < nz; k++)
        for (j = 0; j < ny; j++)
            for (i = 0; i < nx; i++) {
                double s = rho[CELL(i, j, k - 1)] + rho[CELL(i, j, k)];
                double d = gz[FZ(i, j, k)] * (-2.0 / (s * s));
                grho[CELL(i, j, k - 1)] += d;
                grho[CELL(i, j, k)] += d;
            }
}

/* Gradient of a loss with respect to the VOF fractions, given its gradient
 * g_f with respect to the face coefficients (face layouts).  Chain rule
 * through the mixture density (Sec. 2, eq. "property_calculation", with the
 * gas fraction max(0, 1 - f_drop - f_film)) and or_density_grad:
 *   d rho / d f_drop = rho_drop - rho_gas (rho_drop where the gas fraction
 *   is clamped, i.e. 1 - f_drop - f_film < 0), likewise for f_film. */
int or_vof_grad(const double *f_drop, const double *f_film, int nx, int ny, int nz,
                double rho_drop, double rho_film, double rho_gas,
                const double *gx, const double *gy, const double *gz,
                double *g_drop, double *g_film)
{
    long n = (long)nx * ny * nz, c;
    double *rho = malloc(sizeof(double) * n), *grho = malloc(sizeof(double) * n);
    if (!rho || !grho) {
        free(rho);
        free(grho);
        return OR_ENOMEM;
    }
    or_density(f_drop, f_film, n, rho_drop, rho_film, rho_gas, rho);
    or_density_grad(rho, nx, ny, nz, gx, gy, gz, grho);
    for (c = 0; c < n; c++) {
        double gas = (1.0 - f_drop[c] - f_film[c] < 0.0) ? 0.0 : rho_gas;
        g_drop[c] = grho[c] * (rho_drop - gas);
        g_film[c] = grho[c] * (rho_film - gas);
    }
    free(rho);
    free(grho);
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * The operator and its pieces
 * ------------------------------------------------------------------------- */

/* Sum over the faces of cell (i,j,k) that have a neighbour:
 *   *diag = sum beta_f,  *off = sum beta_f x_neighbour */
static void stencil_sums(const double *bx, const double *by, const double *bz,
                         int nx, int ny, int nz, const double *x, int i, int j, int k,
                         double *diag, double *off)
{
    double d = 0.0, o = 0.0, bf;
    if (i > 0)      { bf = bx[FX(i, j, k)];     d += bf; o += bf * x[CELL(i - 1, j, k)]; }
    if (i < nx - 1) { bf = bx[FX(i + 1, j, k)]; d += bf; o += bf * x[CELL(i + 1, j, k)]; }
    if (j > 0)      { bf = by[FY(i, j, k)];     d += bf; o += bf * x[CELL(i, j - 1, k)]; }
    if (j < ny - 1) { bf = by[FY(i, j + 1, k)]; d += bf; o += bf * x[CELL(i, j + 1, k)]; }
    if (k > 0)      { bf = bz[FZ(i, j, k)];     d += bf; o += bf * x[CELL(i, j, k - 1)]; }
    if (k < nz - 1) { bf = bz[FZ(i, j, k + 1)]; d += bf; o += bf * x[CELL(i, j, k + 1)]; }
    *diag = d;
    *off = o;
}

/* y = L x,  (L x)_c = sum_f beta_f (x_nb - x_c) / h^2 */
void or_apply(const double *bx, const double *by, const double *bz,
              int nx, int ny, int nz, double h, const double *x, double *y)
{
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++) {
        int i, j;
        for (j = 0; j < ny; j++)
            for (i = 0; i < nx; i++) {
                double d, o;
                stencil_sums(bx, by, bz, nx, ny, nz, x, i, j, k, &d, &o);
                y[CELL(i, j, k)] = (o - d * x[CELL(i, j, k)]) / (h * h);
            }
    }
}

/* r = b - L p */
void or_residual(const double *bx, const double *by, const double *bz,
                 int nx, int ny, int nz, double h, const double *b, const double *p, double *r)
{
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++) {
        int i, j;
        for (j = 0; j < ny; j++)
            for (i = 0; i < nx; i++) {
                double d, o;
                stencil_sums(bx, by, bz, nx, ny, nz, p, i, j, k, &d, &o);
                r[CELL(i, j, k)] = b[CELL(i, j, k)] - (o - d * p[CELL(i, j, k)]) / (h * h);
            }
    }
}

/* One Gauss-Seidel half-sweep (unit relaxation) over the cells of one colour,
 * colour = (i + j + k) mod 2 (0 = red, 1 = black):
 *     p_c <- (sum_f beta_f p_nb - h^2 b_c) / sum_f beta_f
 * which makes the residual of every cell of that colour zero.  A cell with no
 * coupled face (sum beta = 0) is left unchanged. */
void or_rbgs_half(const double *bx, const double *by, const double *bz,
                  int nx, int ny, int nz, double h, const double *b, double *p, int colour)
{
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++) {
        int i, j;
        for (j = 0; j < ny; j++)
            for (i = 0; i < nx; i++) {
                double d, o;
                if (((i + j + k) & 1) != colour) continue;
                stencil_sums(bx, by, bz, nx, ny, nz, p, i, j, k, &d, &o);
                if (d > 0.0)
                    p[CELL(i, j, k)] = (o - h * h * b[CELL(i, j, k)]) / d;
            }
    }
}

/* Restriction: coarse cell = average of its 8 children (fine dims nx, ny, nz, all even) */
void or_restrict(const double *r, int nx, int ny, int nz, double *rc)
{
    int K, cx = nx / 2, cy = ny / 2, cz = nz / 2;
#pragma omp parallel for schedule(static)
    for (K = 0; K < cz; K++) {
        int I, J;
        for (J = 0; J < cy; J++)
            for (I = 0; I < cx; I++) {
                double s = 0.0;
                int a, b, c;
                for (c = 0; c < 2; c++)
                    for (b = 0; b < 2; b++)
                        for (a = 0; a < 2; a++)
                            s += r[CELL(2 * I + a, 2 * J + b, 2 * K + c)];
                rc[((long)K * cy + J) * cx + I] = s / 8.0;
            }
    }
}

/* 1-D cell-centred linear interpolation stencil: fine cell f of a fine axis
 * with 2*nc cells takes 3/4 of its parent and 1/4 of the parent's neighbour on
 * its side; at a wall the neighbour is the parent itself. */
static void interp_1d(int f, int nc, int *c0, int *c1)
{
    int parent = f / 2;
    int side = (f % 2 == 0) ? parent - 1 : parent + 1;
    if (side < 0) side = 0;
    if (side > nc - 1) side = nc - 1;
    *c0 = parent;
    *c1 = side;
}

/* p += P e  (trilinear cell-centred prolongation of the coarse correction e;
 * fine dims nx, ny, nz) */
void or_prolong_add(const double *e, int nx, int ny, int nz, double *p)
{
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    int k;
    const double wgt[2] = {0.75, 0.25};
#pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++) {
        int i, j;
        for (j = 0; j < ny; j++)
            for (i = 0; i < nx; i++) {
                int xi[2], yj[2], zk[2], a, b, c;
                double s = 0.0;
                interp_1d(i, cx, &xi[0], &xi[1]);
                interp_1d(j, cy, &yj[0], &yj[1]);
                interp_1d(k, cz, &zk[0], &zk[1]);
                for (c = 0; c < 2; c++)
                    for (b = 0; b < 2; b++)
                        for (a = 0; a < 2; a++)
                            s += wgt[a] * wgt[b] * wgt[c]
                               * e[((long)zk[c] * cy + yj[b]) * cx + xi[a]];
                p[CELL(i, j, k)] += s;
            }
    }
}

/* Coarse face coefficients: each coarse face is the mean of the 4 fine faces
 * that tile it; wall faces stay 0.  Input fine dims nx, ny, nz (all even);
 * outputs use the coarse face layouts. */
void or_coarsen_faces(const double *bx, const double *by, const double *bz,
                      int nx, int ny, int nz, double *cbx, double *cby, double *cbz)
{
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    int I, J, K;
    for (K = 0; K < cz; K++)
        for (J = 0; J < cy; J++)
            for (I = 0; I <= cx; I++) {
                double s = 0.0;
                if (I > 0 && I < cx)
                    s = (bx[FX(2 * I, 2 * J, 2 * K)] + bx[FX(2 * I, 2 * J + 1, 2 * K)]
                       + bx[FX(2 * I, 2 * J, 2 * K + 1)] + bx[FX(2 * I, 2 * J + 1, 2 * K + 1)]) / 4.0;
                cbx[((long)K * cy + J) * (cx + 1) + I] = s;
            }
    for (K = 0; K < cz; K++)
        for (J = 0; J <= cy; J++)
            for (I = 0; I < cx; I++) {
                double s = 0.0;
                if (J > 0 && J < cy)
                    s = (by[FY(2 * I, 2 * J, 2 * K)] + by[FY(2 * I + 1, 2 * J, 2 * K)]
                       + by[FY(2 * I, 2 * J, 2 * K + 1)] + by[FY(2 * I + 1, 2 * J, 2 * K + 1)]) / 4.0;
                cby[((long)K * (cy + 1) + J) * cx + I] = s;
            }
    for (K = 0; K <= cz; K++)
        for (J = 0; J < cy; J++)
            for (I = 0; I < cx; I++) {
                double s = 0.0;
                if (K > 0 && K < cz)
                    s = (bz[FZ(2 * I, 2 * J, 2 * K)] + bz[FZ(2 * I + 1, 2 * J, 2 * K)]
                       + bz[FZ(2 * I, 2 * J + 1, 2 * K)] + bz[FZ(2 * I + 1, 2 * J + 1, 2 * K)]) / 4.0;
                cbz[((long)K * cy + J) * cx + I] = s;
            }
}

/* Exact coarse solve: the zero-mean e with L e = r - mean(r), found from the
 * bordered system  [[L, 1], [1^T, 0]] [e; mu] = [r; 0]  by Gaussian elimination
 * with partial pivoting.  n = nx*ny*nz unknowns plus one. */
int or_coarse_solve(const double *bx, const double *by, const double *bz,
                    int nx, int ny, int nz, double h, const double *r, double *e)
{
    int n = nx * ny * nz, m = n + 1;
    double *M = (double *)calloc((size_t)m * m, sizeof(double));
    double *rhs = (double *)calloc((size_t)m, sizeof(double));
    int i, j, k, col, row;
    if (!M || !rhs) { free(M); free(rhs); return OR_ENOMEM; }
    for (k = 0; k < nz; k++)
        for (j = 0; j < ny; j++)
            for (i = 0; i < nx; i++) {
                long c = CELL(i, j, k);
                double bf, h2 = h * h;
                if (i > 0)      { bf = bx[FX(i, j, k)];     M[c * m + CELL(i - 1, j, k)] += bf / h2; M[c * m + c] -= bf / h2; }
                if (i < nx - 1) { bf = bx[FX(i + 1, j, k)]; M[c * m + CELL(i + 1, j, k)] += bf / h2; M[c * m + c] -= bf / h2; }
                if (j > 0)      { bf = by[FY(i, j, k)];     M[c * m + CELL(i, j - 1, k)] += bf / h2; M[c * m + c] -= bf / h2; }
                if (j < ny - 1) { bf = by[FY(i, j + 1, k)]; M[c * m + CELL(i, j + 1, k)] += bf / h2; M[c * m + c] -= bf / h2; }
                if (k > 0)      { bf = bz[FZ(i, j, k)];     M[c * m + CELL(i, j, k - 1)] += bf / h2; M[c * m + c] -= bf / h2; }
                if (k < nz - 1) { bf = bz[FZ(i, j, k + 1)]; M[c * m + CELL(i, j, k + 1)] += bf / h2; M[c * m + c] -= bf / h2; }
                M[c * m + n] = 1.0;
                M[(long)n * m + c] = 1.0;
                rhs[c] = r[c];
            }
    rhs[n] = 0.0;
    /* forward elimination with partial pivoting */
    for (col = 0; col < m; col++) {
        int piv = col;
        double best = fabs(M[(long)col * m + col]);
        for (row = col + 1; row < m; row++)
            if (fabs(M[(long)row * m + col]) > best) { best = fabs(M[(long)row * m + col]); piv = row; }
        if (best == 0.0) { free(M); free(rhs); return OR_EINVAL; }
        if (piv != col) {
            int t;
            for (t = 0; t < m; t++) {
                double s = M[(long)col * m + t];
                M[(long)col * m + t] = M[(long)piv * m + t];
                M[(long)piv * m + t] = s;
            }
            { double s = rhs[col]; rhs[col] = rhs[piv]; rhs[piv] = s; }
        }
        for (row = col + 1; row < m; row++) {
            double f = M[(long)row * m + col] / M[(long)col * m + col];
            int t;
            if (f == 0.0) continue;
            for (t = col; t < m; t++) M[(long)row * m + t] -= f * M[(long)col * m + t];
            rhs[row] -= f * rhs[col];
        }
    }
    /* back substitution */
    for (row = m - 1; row >= 0; row--) {
        double s = rhs[row];
        int t;
        for (t = row + 1; t < m; t++) s -= M[(long)row * m + t] * rhs[t];
        rhs[row] = s / M[(long)row * m + row];
    }
    for (i = 0; i < n; i++) e[i] = rhs[i];
    free(M);
    free(rhs);
    return OR_OK;
}

/* g_f = (lambda_R - lambda_L)(p_R - p_L) / h^2 on interior faces, 0 on walls:
 * the derivative of a loss sum(w p) with respect to beta_f when lambda is the
 * zero-mean solution of L lambda = w - mean(w). */
void or_face_grad(const double *lam, const double *p, int nx, int ny, int nz, double h,
                  double *gx, double *gy, double *gz)
{
    int i, j, k;
    double h2 = h * h;
    for (k = 0; k < nz; k++)
        for (j = 0; j < ny; j++)
            for (i = 0; i <= nx; i++)
                gx[FX(i, j, k)] = (i == 0 || i == nx) ? 0.0
                    : (lam[CELL(i, j, k)] - lam[CELL(i - 1, j, k)])
                    * (p[CELL(i, j, k)] - p[CELL(i - 1, j, k)]) / h2;
    for (k = 0; k < nz; k++)
        for (j = 0; j <= ny; j++)
            for (i = 0; i < nx; i++)
                gy[FY(i, j, k)] = (j == 0 || j == ny) ? 0.0
                    : (lam[CELL(i, j, k)] - lam[CELL(i, j - 1, k)])
                    * (p[CELL(i, j, k)] - p[CELL(i, j - 1, k)]) / h2;
    for (k = 0; k <= nz; k++)
        for (j = 0; j < ny; j++)
            for (i = 0; i < nx; i++)
                gz[FZ(i, j, k)] = (k == 0 || k == nz) ? 0.0
                    : (lam[CELL(i, j, k)] - lam[CELL(i, j, k - 1)])
                    * (p[CELL(i, j, k)] - p[CELL(i, j, k - 1)]) / h2;
}

/* ---------------------------------------------------------------------------
 * Multigrid V-cycle and solve loop
 * ------------------------------------------------------------------------- */

#define OR_MAX_LEVELS 24

typedef struct {
    int nx, ny, nz;
    double h;
    double *bx, *by, *bz;   /* face coefficients, public face layouts */
    double *x, *b, *r;      /* iterate, right-hand side, residual */
} or_level;

typedef struct {
    int nlev;
    or_level lev[OR_MAX_LEVELS];
} or_hier;

static long ncell(const or_level *L) { return (long)L->nx * L->ny * L->nz; }

/* Number of levels: halve every dimension while any exceeds coarse_max;
 * every halving needs all dimensions even.  Returns 0 when impossible. */
int or_num_levels(int nx, int ny, int nz, int coarse_max)
{
    int n = 1;
    if (nx < 1 || ny < 1 || nz < 1 || coarse_max < 1) return 0;
    while (nx > coarse_max || ny > coarse_max || nz > coarse_max) {
        if ((nx & 1) || (ny & 1) || (nz & 1)) return 0;
        nx /= 2; ny /= 2; nz /= 2;
        n++;
        if (n > OR_MAX_LEVELS) return 0;
    }
    return n;
}

static void free_hier(or_hier *H)
{
    int l;
    for (l = 0; l < H->nlev; l++) {
        or_level *L = &H->lev[l];
        free(L->bx); free(L->by); free(L->bz);
        free(L->x); free(L->b); free(L->r);
    }
    H->nlev = 0;
}

static int build_hier(or_hier *H, const double *bx, const double *by, const double *bz,
                      int nx, int ny, int nz, double h, int coarse_max)
{
    int l, nlev = or_num_levels(nx, ny, nz, coarse_max);
    memset(H, 0, sizeof(*H));
    if (nlev == 0) return OR_EINVAL;
    for (l = 0; l < nlev; l++) {
        or_level *L = &H->lev[l];
        long n;
        L->nx = nx; L->ny = ny; L->nz = nz; L->h = h;
        n = (long)nx * ny * nz;
        L->bx = (double *)calloc((size_t)nz * ny * (nx + 1), sizeof(double));
        L->by = (double *)calloc((size_t)nz * (ny + 1) * nx, sizeof(double));
        L->bz = (double *)calloc((size_t)(nz + 1) * ny * nx, sizeof(double));
        L->x = (double *)calloc((size_t)n, sizeof(double));
        L->b = (double *)calloc((size_t)n, sizeof(double));
        L->r = (double *)calloc((size_t)n, sizeof(double));
        H->nlev = l + 1;
        if (!L->bx || !L->by || !L->bz || !L->x || !L->b || !L->r) { free_hier(H); return OR_ENOMEM; }
        if (l == 0) {
            memcpy(L->bx, bx, sizeof(double) * (size_t)nz * ny * (nx + 1));
            memcpy(L->by, by, sizeof(double) * (size_t)nz * (ny + 1) * nx);
            memcpy(L->bz, bz, sizeof(double) * (size_t)(nz + 1) * ny * nx);
        } else {
            or_level *F = &H->lev[l - 1];
            or_coarsen_faces(F->bx, F->by, F->bz, F->nx, F->ny, F->nz, L->bx, L->by, L->bz);
        }
        nx /= 2; ny /= 2; nz /= 2; h *= 2.0;
    }
    return OR_OK;
}

static int vcycle(or_hier *H, int l, int pre, int post)
{
    or_level *L = &H->lev[l];
    int s;
    if (l == H->nlev - 1)
        return or_coarse_solve(L->bx, L->by, L->bz, L->nx, L->ny, L->nz, L->h, L->b, L->x);
    for (s = 0; s < pre; s++) {
        or_rbgs_half(L->bx, L->by, L->bz, L->nx, L->ny, L->nz, L->h, L->b, L->x, 0);
        or_rbgs_half(L->bx, L->by, L->bz, L->nx, L->ny, L->nz, L->h, L->b, L->x, 1);
    }
    or_residual(L->bx, L->by, L->bz, L->nx, L->ny, L->nz, L->h, L->b, L->x, L->r);
    {
        or_level *C = &H->lev[l + 1];
        int st;
        or_restrict(L->r, L->nx, L->ny, L->nz, C->b);
        memset(C->x, 0, sizeof(double) * (size_t)ncell(C));
        st = vcycle(H, l + 1, pre, post);
        if (st != OR_OK) return st;
        or_prolong_add(C->x, L->nx, L->ny, L->nz, L->x);
    }
    for (s = 0; s < post; s++) {
        or_rbgs_half(L->bx, L->by, L->bz, L->nx, L->ny, L->nz, L->h, L->b, L->x, 1);
        or_rbgs_half(L->bx, L->by, L->bz, L->nx, L->ny, L->nz, L->h, L->b, L->x, 0);
    }
    return OR_OK;
}

static double norm2(const double *x, long n)
{
    double s = 0.0;
    long c;
    for (c = 0; c < n; c++) s += x[c] * x[c];
    return sqrt(s);
}

static double mean(const double *x, long n)
{
    double s = 0.0;
    long c;
    for (c = 0; c < n; c++) s += x[c];
    return s / (double)n;
}

/* Solve L p = rhs - mean(rhs) for the zero-mean p.
 *   p          in: initial guess; out: zero-mean solution (last iterate on failure)
 *   tol        stop at the first cycle with ||r|| <= tol ||b - mean b||
 *   hist       (nullable) relative residual before cycle 1 and after each
 *              cycle: max_cycles + 1 entries
 *   cycles     (nullable) number of V-cycles run
 *   rel_res    (nullable) final relative residual
 *   rhs_mean   (nullable) mean removed from rhs
 * Returns OR_OK, OR_EINVAL, OR_ENOMEM, OR_ENOCONV or OR_ENONFINITE. */
int or_solve(const double *bx, const double *by, const double *bz, int nx, int ny, int nz,
             double h, const double *rhs, double *p, double tol, int max_cycles,
             int pre, int post, int coarse_max,
             double *hist, int *cycles, double *rel_res, double *rhs_mean)
{
    or_hier H;
    long n = (long)nx * ny * nz, c;
    int st, cyc = 0;
    double mu, bnorm, rr;
    if (tol <= 0.0 || max_cycles < 0 || pre < 0 || post < 0) return OR_EINVAL;
    st = build_hier(&H, bx, by, bz, nx, ny, nz, h, coarse_max);
    if (st != OR_OK) return st;
    or_level *F = &H.lev[0];
    mu = mean(rhs, n);
    for (c = 0; c < n; c++) F->b[c] = rhs[c] - mu;
    if (rhs_mean) *rhs_mean = mu;
    for (c = 0; c < n; c++) F->x[c] = p[c];
    bnorm = norm2(F->b, n);
    if (!isfinite(bnorm)) { free_hier(&H); return OR_ENONFINITE; }
    if (bnorm == 0.0) {
        for (c = 0; c < n; c++) p[c] = 0.0;
        if (hist) hist[0] = 0.0;
        if (cycles) *cycles = 0;
        if (rel_res) *rel_res = 0.0;
        free_hier(&H);
        return OR_OK;
    }
    or_residual(F->bx, F->by, F->bz, nx, ny, nz, h, F->b, F->x, F->r);
    rr = norm2(F->r, n) / bnorm;
    if (hist) hist[0] = rr;
    st = OR_ENOCONV;
    if (rr <= tol) st = OR_OK;
    while (st == OR_ENOCONV && cyc < max_cycles) {
        int vs = vcycle(&H, 0, pre, post);
        if (vs != OR_OK) { free_hier(&H); return vs; }
        cyc++;
        or_residual(F->bx, F->by, F->bz, nx, ny, nz, h, F->b, F->x, F->r);
        rr = norm2(F->r, n) / bnorm;
        if (hist) hist[cyc] = rr;
        if (!isfinite(rr)) { st = OR_ENONFINITE; break; }
        if (rr <= tol) st = OR_OK;
    }
    mu = mean(F->x, n);
    for (c = 0; c < n; c++) p[c] = F->x[c] - mu;
    if (cycles) *cycles = cyc;
    if (rel_res) *rel_res = rr;
    free_hier(&H);
    return st;
}

static double dot(const double *x, const double *y, long n)
{
    double s = 0.0;
    long c;
    for (c = 0; c < n; c++) s += x[c] * y[c];
    return s;
}

/* Flexible conjugate gradients with one V-cycle (from a zero guess) as the
 * preconditioner B; the variant keeps one previous search direction (Notay's
 * flexible CG truncated to one direction), which stays valid when B is not
 * exactly symmetric (the V-cycle's restriction is not a multiple of the
 * prolongation's transpose).  With r = b - L x, per iteration:
 *   z = B r
 *   d = z - ((z, q_prev) / (d_prev, q_prev)) d_prev     (d = z at the start)
 *   q = L d,  alpha = (d, r) / (d, q),  x += alpha d,  r -= alpha q
 * The system is the negative semi-definite L p = b - mean(b); the signs of
 * L and B cancel in alpha and in the direction update.  Stops at the first
 * iteration with ||r|| <= tol ||b - mean b|| (r is the updated residual).
 * Arguments and results as or_solve, with iterations in place of cycles. */
int or_fcg_solve(const double *bx, const double *by, const double *bz, int nx, int ny, int nz,
                 double h, const double *rhs, double *p, double tol, int max_iters,
                 int pre, int post, int coarse_max,
                 double *hist, int *iters, double *rel_res, double *rhs_mean)
{
    or_hier H;
    long n = (long)nx * ny * nz, c;
    int st, it = 0, have_prev = 0;
    double mu, bnorm, rr, dq_prev = 0.0;
    double *b, *x, *r, *z, *d, *q;
    if (tol <= 0.0 || max_iters < 0 || pre < 0 || post < 0) return OR_EINVAL;
    st = build_hier(&H, bx, by, bz, nx, ny, nz, h, coarse_max);
    if (st != OR_OK) return st;
    or_level *F = &H.lev[0];
    b = malloc(sizeof(double) * 6 * (size_t)n);
    if (!b) { free_hier(&H); return OR_ENOMEM; }
    x = b + n; r = x + n; z = r + n; d = z + n; q = d + n;
    mu = mean(rhs, n);
    for (c = 0; c < n; c++) { b[c] = rhs[c] - mu; x[c] = p[c]; }
    if (rhs_mean) *rhs_mean = mu;
    bnorm = norm2(b, n);
    if (!isfinite(bnorm)) { free(b); free_hier(&H); return OR_ENONFINITE; }
    if (bnorm == 0.0) {
        for (c = 0; c < n; c++) p[c] = 0.0;
        if (hist) hist[0] = 0.0;
        if (iters) *iters = 0;
        if (rel_res) *rel_res = 0.0;
        free(b);
        free_hier(&H);
        return OR_OK;
    }
    or_residual(F->bx, F->by, F->bz, nx, ny, nz, h, b, x, r);
    rr = norm2(r, n) / bnorm;
    if (hist) hist[0] = rr;
    st = rr <= tol ? OR_OK : OR_ENOCONV;
    while (st == OR_ENOCONV && it < max_iters) {
        double alpha, dqv;
        int vs;
        /* z = B r: one V-cycle on L z = r from z = 0 */
        memcpy(F->b, r, sizeof(double) * (size_t)n);
        memset(F->x, 0, sizeof(double) * (size_t)n);
        vs = vcycle(&H, 0, pre, post);
        if (vs != OR_OK) { st = vs; break; }
        memcpy(z, F->x, sizeof(double) * (size_t)n);
        if (have_prev) {
            double gamma = dot(z, q, n) / dq_prev;
            for (c = 0; c < n; c++) d[c] = z[c] - gamma * d[c];
        } else {
            memcpy(d, z, sizeof(double) * (size_t)n);
        }
        or_apply(F->bx, F->by, F->bz, nx, ny, nz, h, d, q);
        dqv = dot(d, q, n);
        alpha = dot(d, r, n) / dqv;
        for (c = 0; c < n; c++) {
            x[c] += alpha * d[c];
            r[c] -= alpha * q[c];
        }
        dq_prev = dqv;
        have_prev = 1;
        it++;
        rr = norm2(r, n) / bnorm;
        if (hist) hist[it] = rr;
        if (!isfinite(rr)) { st = OR_ENONFINITE; break; }
        if (rr <= tol) st = OR_OK;
    }
    mu = mean(x, n);
    for (c = 0; c < n; c++) p[c] = x[c] - mu;
    if (iters) *iters = it;
    if (rel_res) *rel_res = rr;
    free(b);
    free_hier(&H);
    return st;
}

/* Run exactly `cycles` V-cycles from the guess p on the projected rhs without a
 * stopping test and without removing the mean of p (used for lock-step
 * comparison of single cycles). */
int or_vcycles(const double *bx, const double *by, const double *bz, int nx, int ny, int nz,
               double h, const double *rhs, double *p, int cycles, int pre, int post, int coarse_max)
{
    or_hier H;
    long n = (long)nx * ny * nz, c;
    int st, cyc;
    double mu;
    st = build_hier(&H, bx, by, bz, nx, ny, nz, h, coarse_max);
    if (st != OR_OK) return st;
    or_level *F = &H.lev[0];
    mu = mean(rhs, n);
    for (c = 0; c < n; c++) { F->b[c] = rhs[c] - mu; F->x[c] = p[c]; }
    for (cyc = 0; cyc < cycles; cyc++) {
        st = vcycle(&H, 0, pre, post);
        if (st != OR_OK) break;
    }
    for (c = 0; c < n; c++) p[c] = F->x[c];
    free_hier(&H);
    return st;
}
