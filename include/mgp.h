/*
 * mgp.h -- C ABI of the MI355X (gfx950) multigrid solver for the
 * variable-density pressure-Poisson equation of a volume-of-fluid
 * incompressible flow solver:
 *
 *     div( beta grad p ) = div(u*) / dt,    beta = 1/rho,   on the unit cube,
 *     homogeneous Neumann (closed) walls.
 *
 * The paper's governing equations are the incompressible Navier-Stokes
 * equations (Sec. 2, eqs. "ns_mass" and "mom_mass"); enforcing div u = 0 on
 * the pressure-corrected velocity gives the equation above.  Cell density is
 * the volume-weighted sum over phases (Sec. 2, eq. "property_calculation").
 * The paper solves it with a multigrid method whose "switch levels" it names
 * as a scaling factor (Sec. 4.3.2, strong and weak scaling) without further
 * detail; the discretisation (cell-centred finite volumes, 7-point stencil)
 * follows from its finite-volume Cartesian-mesh description (Sec. 2).
 *
 * Discretisation.  N_x x N_y x N_z cells of spacing h, cell (i,j,k) centred at
 * ((i+1/2)h, (j+1/2)h, (k+1/2)h).  The operator is
 *     (L p)_c = sum over the faces f of cell c with a neighbour n of
 *               beta_f (p_n - p_c) / h^2 .
 * L is symmetric, negative semi-definite, and its null space is the constants:
 * every solve returns the zero-mean solution of L p = rhs - mean(rhs).
 *
 * Memory layouts.  Every array is contiguous, x fastest, double precision:
 *     cell arrays (rhs, p, g, lambda, b, f_*)   [nz][ny][nx]
 *     x-face arrays (beta_x, g_x, u)           [nz][ny][nx+1]
 *     y-face arrays (beta_y, g_y, v)           [nz][ny+1][nx]
 *     z-face arrays (beta_z, g_z, w)           [nz+1][ny][nx]
 * Entry i of an x-face array is the face between cells i-1 and i; entries 0
 * and nx are walls.  Wall entries of beta are ignored (no flux crosses a
 * wall); wall entries of every face array the library writes are 0.
 *
 * Pointers.  Unless a comment says "host", every pointer argument is a
 * DEVICE pointer into memory the caller owns (e.g. a torch CUDA tensor); the
 * library never frees caller memory.  All work is enqueued on the HIP stream
 * given to mg_setup (or to the context-free calls); a NULL stream is the
 * default stream.  Calls return after their last result is complete only where
 * stated (the solves read one convergence norm per cycle and therefore
 * synchronise the stream).
 *
 * Errors.  Every int-returning call returns a status code (MG_OK on success);
 * no C++ exception and no abort crosses this interface.  mg_last_error()
 * returns a NUL-terminated description of the last failure on a context.
 *
 * Threading.  A context may be used by one host thread at a time.  Calls on
 * different contexts are independent.
 */
#ifndef MGP_H
#define MGP_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_ctx mg_ctx; /* opaque: owns the level hierarchy and all scratch */

/* status codes */
enum {
    MG_OK = 0,
    MG_EINVAL = -1,     /* bad argument: NULL pointer, dims, h, tol, options, beta <= 0 or non-finite */
    MG_ENOMEM = -2,     /* device or pinned-host allocation failed */
    MG_EHIP = -3,       /* a HIP runtime call failed; text in mg_last_error */
    MG_ENOCONV = -4,    /* max_cycles reached, or residual grew 1e3 x above its best */
    MG_ENONFINITE = -5  /* NaN or Inf in the right-hand side or a residual norm */
};

enum { MG_BC_NEUMANN = 0 };                       /* the only boundary condition */
enum { MG_PREC_FP64 = 0, MG_PREC_MIXED = 1 };     /* V-cycle arithmetic */

/* option flags (mg_opts.flags) */
enum {
    MG_FLAG_ZERO_GUESS = 1,  /* mg_solve/mg_solve_adjoint ignore the initial contents of p
                                (lambda) and start from zero */
    MG_FLAG_TIMING = 2,      /* time every launch of the finest-grid kernels with HIP events
                                and report the totals in mg_stats */
    MG_FLAG_FCG = 4,         /* solve by flexible conjugate gradients with one V-cycle (of
                                the context's precision) as the preconditioner, one previous
                                direction kept; mg_stats.cycles then counts iterations.
                                Costs three more FP64 cell arrays.  The plain V-cycle
                                iteration (flag clear) is the method of the paper's solver;
                                this is a Krylov acceleration of it. */
    MG_FLAG_LEVEL_LAUNCHES = 8  /* run every step of a V-cycle as its own launch.  By default
                                (1) the levels of at most 4096 cells that no tiled kernel
                                serves (16^3 and below; every level of grids that small) run
                                in one single-workgroup launch, (2) in MG_PREC_MIXED the
                                first two-sweep launch of a post-smoothing adds the
                                prolongated coarse correction itself (no separate
                                prolongation pass), and (3) in MG_PREC_MIXED with pre = 2,
                                the pre-smoothing launch of a level also forms the
                                residual of its result and restricts it to the next level
                                (no separate residual + restriction pass).  All three
                                compute every value as the separate launches do: identical
                                results, fewer launches and HBM passes.  For comparison and
                                testing. */
};

/*
 * Solver options.  mg_setup(..., opts = NULL) uses
 *   {pre = 2, post = 2, max_cycles = 100, coarse_max = 4, precision = MG_PREC_FP64, flags = 0}.
 * pre, post      Gauss-Seidel sweeps before / after the coarse correction
 *                (pre sweeps visit red then black, post sweeps black then red;
 *                red = cells with i+j+k even).  0..8.
 * max_cycles     V-cycles (FP64) or outer defect-correction iterations (MIXED), 1..MG_HIST_MAX-1.
 * coarse_max     coarsening stops once every dimension is <= coarse_max (1..4);
 *                the coarsest grid (<= 64 cells) is solved exactly.
 * precision      MG_PREC_FP64: FP64 V-cycles.  MG_PREC_MIXED: FP32 V-cycles inside an FP64
 *                defect-correction loop (update, residual and norms in FP64).
 */
typedef struct {
    int pre, post, max_cycles, coarse_max, precision, flags;
} mg_opts;

#define MG_HIST_MAX 256
#define MG_MAX_LEVELS 16

/* kernel classes timed under MG_FLAG_TIMING */
enum {
    MG_K_SWEEP = 0,      /* red-black Gauss-Seidel sweep kernel (one sweep per launch) */
    MG_K_RESTRICT = 1,   /* fused residual + restriction */
    MG_K_PROLONG = 2,    /* fused prolongation + correction */
    MG_K_OUTER = 3,      /* FP64 update + residual + cast (mixed) */
    MG_K_NORM = 4,       /* residual norm */
    MG_K_SWEEP2 = 5,     /* two red-black sweeps per launch (FP32 smoothing pairs) */
    MG_K_SWEEP2R = 6,    /* FP32 pre-smoothing pair from a zero iterate that also writes the
                            restricted residual (one launch for both; see MG_FLAG_LEVEL_LAUNCHES) */
    MG_K_COUNT = 7
};

typedef struct {
    int cycles;                 /* V-cycles (FP64) or outer iterations (MIXED) run */
    int status;                 /* same as the return value */
    double rel_res;             /* ||rhs - mean - L p|| / ||rhs - mean|| at exit */
    double rhs_mean_removed;    /* mean(rhs) */
    double setup_ms;            /* wall time of mg_setup */
    double solve_ms;            /* wall time of this solve (host clock, stream synchronised) */
    double hist[MG_HIST_MAX];   /* rel_res before cycle 1 (hist[0]) and after each cycle */
    /* MG_FLAG_TIMING only: per kernel class, launches of the class's tiled
     * kernel (one kernel per class and precision) on every level ... */
    double kernel_ms[MG_K_COUNT];        /* summed HIP-event durations */
    long long kernel_launches[MG_K_COUNT];
    double kernel_bytes[MG_K_COUNT];     /* summed algorithmic HBM bytes of those launches */
    /* ... and the same totals for the finest grid alone */
    double kernel_ms_finest[MG_K_COUNT];
    long long kernel_launches_finest[MG_K_COUNT];
    double kernel_bytes_finest[MG_K_COUNT];
} mg_stats;

/*
 * mg_setup -- build the level hierarchy for one set of face coefficients.
 *   out        host: receives the new context (NULL on failure).
 *   beta_x/y/z face coefficients 1/rho_face in the face layouts above (device).
 *              Interior entries must be finite and > 0.  They are copied: later
 *              changes to the caller's arrays have no effect on this context.
 *   dims       host int[3] = {nx, ny, nz}.  Repeatedly halving every dimension
 *              while any exceeds coarse_max must keep all dimensions integral
 *              (e.g. 2^m, 3*2^m), else MG_EINVAL.
 *   h          grid spacing (> 0).
 *   bc         MG_BC_NEUMANN.
 *   opts       host, nullable.
 *   hip_stream hipStream_t (as void*), nullable.
 * Allocates every buffer any later call on the context needs, once; later
 * calls allocate nothing.  Coarse coefficients (the mean of the four fine
 * faces that tile a coarse face) and the exact coarse-grid inverse are built
 * on the GPU.  Synchronises the stream before returning.
 */
int mg_setup(mg_ctx **out, const double *beta_x, const double *beta_y, const double *beta_z,
             const int dims[3], double h, int bc, const mg_opts *opts, void *hip_stream);

/*
 * mg_setup_density -- mg_setup for coefficients defined by a cell density:
 * beta_f = 2/(rho_L + rho_R) on interior faces and 0 on walls, the face value
 * of the variable density of the projection equation (Sec. 2, with the
 * density of eq. "property_calculation" from mg_density_from_vof).
 *   rho  device [nz][ny][nx]; every entry finite and > 0, else MG_EINVAL.
 *        Copied into the context (one more cell array of device memory).
 * Other arguments, the level hierarchy and the results are those of mg_setup
 * given the faces mg_faces_from_density(rho) writes, bit for bit.  The
 * difference is bandwidth: the finest-grid FP64 residual passes (the
 * mixed-precision outer update, the FP64 restriction and residual norm, the
 * flexible-CG operator application) form each coefficient from rho as they
 * go, reading 8 bytes per cell where the three face arrays take 24.
 */
int mg_setup_density(mg_ctx **out, const double *rho, const int dims[3], double h, int bc,
                     const mg_opts *opts, void *hip_stream);

/*
 * mg_update_density -- new cell density for a context made by mg_setup_density
 * (same rules; MG_EINVAL for any other context).  mg_update on such a context
 * switches it to the face arrays given, and mg_update_density back.
 */
int mg_update_density(mg_ctx *c, const double *rho);

/*
 * mg_update -- replace the face coefficients of an existing context (same dims,
 * layouts and rules as mg_setup) and rebuild the coarse levels and the coarse
 * inverse, without allocating: the per-time-step call of a flow solver whose
 * density field moves.  On MG_EINVAL (a bad coefficient) the context keeps the
 * new, rejected coefficients and must be updated again before the next solve.
 * Synchronises the stream.
 */
int mg_update(mg_ctx *c, const double *beta_x, const double *beta_y, const double *beta_z);

/*
 * mg_set_timing_classes -- which kernel classes a context set up with
 * MG_FLAG_TIMING times from now on: bit k of mask selects class MG_K_k (all
 * after setup).  Each timed launch carries start/end events, which costs the
 * GPU a few microseconds before the kernel, so a caller timing one class can
 * leave the others untimed.  MG_EINVAL without MG_FLAG_TIMING or for bits at or
 * beyond MG_K_COUNT.
 */
int mg_set_timing_classes(mg_ctx *c, unsigned mask);

/*
 * mg_solve -- p = zero-mean solution of L p = rhs - mean(rhs): the pressure
 * projection that makes the corrected velocity meet the continuity equation
 * (Sec. 2, eqs. "ns_mass" and "mom_mass"), by multigrid V-cycles (the solver
 * whose "switch levels" Sec. 4.3.2 names; the paper gives no further detail,
 * so the cycle is this library's reading: red-black Gauss-Seidel, pre sweeps
 * red then black, post sweeps black then red, restriction by the mean of the
 * 8 children, trilinear prolongation, coarse faces as the mean of the 4 fine
 * faces they cover, the coarsest grid solved exactly).  The rhs is projected
 * to zero mean because L annihilates constants; the stopping test is checked
 * after every cycle (MG_PREC_MIXED: after every FP64 defect-correction step
 * around one FP32 V-cycle).
 *   rhs   device [nz][ny][nx]; not modified.
 *   p     device [nz][ny][nx], 16-byte aligned; in: initial guess (unless
 *         MG_FLAG_ZERO_GUESS), out: solution.
 *   tol   stop at the first cycle with ||r||_2 <= tol ||rhs - mean(rhs)||_2 (> 0).
 *   st    host, nullable: statistics.
 * Returns MG_OK, MG_ENOCONV (p holds the last iterate, mean removed),
 * MG_ENONFINITE, MG_EINVAL or MG_EHIP.  Synchronises the stream.
 * rhs and p must not alias.
 */
int mg_solve(mg_ctx *c, const double *rhs, double *p, double tol, mg_stats *st);

/*
 * mg_solve_adjoint -- lambda = zero-mean solution of L lambda = g - mean(g).
 * L is symmetric, so the adjoint of the solve of mg_solve (Sec. 2) is the same
 * solve; g is dLoss/dp and lambda = dLoss/drhs.
 * Same arguments, flags and return codes as mg_solve.
 */
int mg_solve_adjoint(mg_ctx *c, const double *g, double *lambda, double tol, mg_stats *st);

/*
 * mg_face_grad -- derivative of a loss through the solve with respect to each
 * face coefficient: g_f = (lambda_R - lambda_L)(p_R - p_L) / h^2 on interior
 * faces, 0 on walls (the chain rule through the operator of mg_solve, whose
 * face coefficient is the 1/rho of Sec. 2: with Loss = sum w p and
 * L lambda = w, dLoss/dbeta_f = +(delta lambda)(delta p)/h^2 across the face).
 * lambda from mg_solve_adjoint, p from mg_solve (device, cell layout);
 * g_x/g_y/g_z device, face layouts.  One fused pass.  MG_EINVAL on NULL
 * arguments or a context holding rejected coefficients.
 */
int mg_face_grad(mg_ctx *c, const double *lambda, const double *p,
                 double *g_x, double *g_y, double *g_z);

/* mg_apply -- y = L x on the finest grid, L the cell-centred finite-volume
 * operator defined at the top of this file (the discretisation of Sec. 2's
 * variable-density pressure equation); device cell arrays that must not alias. */
int mg_apply(mg_ctx *c, const double *x, double *y);

/* mg_destroy -- free the context (NULL is ignored). */
void mg_destroy(mg_ctx *c);

/* mg_last_error -- text of the last failure on c (never NULL; "" if none).
 * mg_last_error(NULL) gives the reason the calling thread's last mg_setup failed. */
const char *mg_last_error(const mg_ctx *c);

/*
 * mg_solve_noalloc -- mg_setup followed by mg_solve, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): no device, pinned or host-heap allocation, no event, no
 * allocating library routine.  The level hierarchy, copies and reduction
 * buffers live in one static device buffer of MG_NOALLOC_SCRATCH_BYTES per GPU
 * (held from the first call on that GPU until the process ends); the context
 * lives on the caller's stack for the duration of the call.
 *   beta_x/y/z, dims, h, bc, opts   as for mg_setup (MG_FLAG_TIMING: MG_EINVAL).
 *   rhs, p, tol, st                 as for mg_solve.
 *   hip_stream                      as for mg_setup.
 * A grid whose hierarchy (with these options) does not fit the buffer gets
 * MG_EINVAL and a text stating the bytes it needs (e.g. 64^3 fits in every
 * mode, 128^3 does not).  Results equal those of mg_setup + mg_solve on the same
 * arguments bit for bit; the mixed-precision loop cannot overlap its next
 * pre-smoothing with the host's wait for a norm, so it may run a little slower.
 * The buffer keeps the last call's contents; every value a call reads is
 * written by that call first.  Calls that overlap on one GPU (from two host
 * threads, or on two streams) race on the buffer: serialise them.  Returns
 * after the stream has finished the call's work.  mg_last_error(NULL) gives
 * the reason of the calling thread's last failure.
 */
#define MG_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int mg_solve_noalloc(const double *beta_x, const double *beta_y, const double *beta_z, const int dims[3],
                     double h, int bc, const mg_opts *opts, const double *rhs, double *p, double tol,
                     mg_stats *st, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Inputs of the solve, from the flow state (no context)
 * ------------------------------------------------------------------------- */

/*
 * mg_faces_from_vof -- face coefficients from the VOF fractions of two liquid
 * phases: rho = rho_drop f_drop + rho_film f_film + rho_gas max(0, 1 - f_drop - f_film)
 * per cell (Sec. 2, eq. "property_calculation"), then beta_f = 2/(rho_L + rho_R)
 * (= harmonic mean of 1/rho) on interior faces and 0 on walls.
 *   f_drop, f_film  device cell arrays; beta_x/y/z device face arrays (written).
 *   dims            host int[3].  Densities must be > 0.
 */
int mg_faces_from_vof(const double *f_drop, const double *f_film, const int dims[3],
                      double rho_drop, double rho_film, double rho_gas,
                      double *beta_x, double *beta_y, double *beta_z, void *hip_stream);

/*
 * mg_density_from_vof -- rho = rho_drop f_drop + rho_film f_film
 * + rho_gas max(0, 1 - f_drop - f_film) per cell (Sec. 2, eq.
 * "property_calculation"), each product rounded as written (no fused
 * multiply-add), so that mg_faces_from_density of the result equals
 * mg_faces_from_vof bit for bit.  f_drop, f_film, rho: device cell arrays.
 */
int mg_density_from_vof(const double *f_drop, const double *f_film, const int dims[3],
                        double rho_drop, double rho_film, double rho_gas, double *rho, void *hip_stream);

/*
 * mg_faces_from_density -- beta_f = 2/(rho_L + rho_R) on interior faces, 0 on
 * walls (public face layouts, device), from a device cell density.  The
 * density is not validated here (mg_setup_density does that); MG_EINVAL on
 * NULL pointers or non-positive dims.
 */
int mg_faces_from_density(const double *rho, const int dims[3], double *beta_x, double *beta_y,
                          double *beta_z, void *hip_stream);

/*
 * mg_density_grad -- gradient of a loss with respect to the cell density, given
 * its gradient with respect to the face coefficients (e.g. from mg_face_grad):
 * the chain rule through mg_faces_from_density,
 *   d beta_f / d rho_L = d beta_f / d rho_R = -2 / (rho_L + rho_R)^2,
 * summed over each cell's interior faces (each product rounded as written).
 *   rho, g_rho      device cell arrays (g_rho written).
 *   g_x, g_y, g_z   device face arrays (public layouts); wall entries ignored.
 *   dims host int[3].  MG_EINVAL on bad arguments.
 */
int mg_density_grad(const double *rho, const int dims[3], const double *g_x, const double *g_y,
                    const double *g_z, double *g_rho, void *hip_stream);

/*
 * mg_divergence -- b = div_h(u, v, w) / dt for MAC face velocities
 * (u: x-face layout, v: y-face layout, w: z-face layout; b: cell layout).
 */
int mg_divergence(const double *u, const double *v, const double *w, const int dims[3],
                  double h, double dt, double *b, void *hip_stream);

/*
 * mg_vof_grad -- gradient of a loss with respect to the VOF fractions, given
 * its gradient with respect to the face coefficients (e.g. from
 * mg_face_grad): the chain rule through mg_faces_from_vof,
 *   d beta_f / d rho_L = d beta_f / d rho_R = -2 / (rho_L + rho_R)^2,
 *   d rho / d f_drop = rho_drop - rho_gas, d rho / d f_film = rho_film - rho_gas
 * (rho_gas dropped in cells whose gas fraction is clamped, 1 - f_drop - f_film < 0).
 *   f_drop, f_film   device cell arrays (the forward's inputs).
 *   g_x, g_y, g_z    device face arrays (public layouts); wall entries ignored.
 *   g_drop, g_film   device cell arrays (written).
 *   dims host int[3]; densities > 0.  MG_EINVAL on bad arguments.
 */
int mg_vof_grad(const double *f_drop, const double *f_film, const int dims[3],
                double rho_drop, double rho_film, double rho_gas,
                const double *g_x, const double *g_y, const double *g_z,
                double *g_drop, double *g_film, void *hip_stream);

/*
 * mg_velocity_correct -- the projection after the solve: the pressure-gradient
 * term of the momentum equation applied over one step so that the velocity
 * meets the continuity equation (Sec. 2).  On every interior face
 *   u_f <- u_f - dt beta_f (p_R - p_L) / h
 * with beta_f = 1/rho_face, the coefficients the solve used; wall faces are
 * left untouched.  Then div_h u_new = div_h u - dt L p = dt (b - L p) for
 * b = div_h u / dt: divergence-free to the solve's residual.
 *   beta_x/y/z  device face arrays (public layouts), read only.
 *   p           device cell array.
 *   u, v, w     device face arrays, updated in place.
 *   dims host int[3]; h > 0, dt > 0.  MG_EINVAL on bad arguments.
 */
int mg_velocity_correct(const double *beta_x, const double *beta_y, const double *beta_z, const double *p,
                        const int dims[3], double h, double dt, double *u, double *v, double *w,
                        void *hip_stream);

/* ---------------------------------------------------------------------------
 * Single-kernel entry points on one level of a context, for verification.
 * Level 0 is the finest grid; mg_level_info gives each level's dims and h.
 * `precision` selects the FP64 or FP32 instance of the kernel; FP32 instances
 * read and write these FP64 arrays through FP32 copies held by the context
 * (available on MG_PREC_MIXED contexts only).
 * ------------------------------------------------------------------------- */

/* number of levels of a plan (host only, no GPU): 0 when dims are invalid */
int mg_plan_levels(const int dims[3], int coarse_max);

/* dims (host int[3]) and spacing (host double) of a level */
int mg_level_info(const mg_ctx *c, int level, int dims[3], double *h);

/* copy a level's face coefficients out in the public face layouts (device) */
int mg_level_faces(mg_ctx *c, int level, double *beta_x, double *beta_y, double *beta_z);

/* nsweeps full red-black Gauss-Seidel sweeps on level `level`:
 * order 0 = (red, black) per sweep, 1 = (black, red).  p in/out.
 * Sweeps run as in a V-cycle: in FP32 on grids at least 64 x 16 cells in
 * (x, y), pairs of sweeps go through the two-sweeps-per-pass kernel. */
int mg_smooth(mg_ctx *c, int level, int precision, const double *b, double *p,
              int nsweeps, int order);

/* b_coarse = restriction (mean of 8 children) of (b - L p) on level -> level+1 */
int mg_residual_restrict(mg_ctx *c, int level, int precision, const double *b, const double *p,
                         double *b_coarse);

/* The pre-smoothing of a V-cycle on `level` followed by the restriction of its
 * residual (the steps of the cycle before the coarse-grid correction): p
 * (written) = the opts.pre sweeps of order 0 from p = 0; b_coarse (written,
 * level+1 layout) = mean of the 8 children of b - L p.  In FP32 with pre = 2
 * this is the single launch a V-cycle uses on grids at least 64 x 16 cells in
 * (x, y) with even extents (unless MG_FLAG_LEVEL_LAUNCHES); the results equal
 * those of mg_smooth from p = 0 followed by mg_residual_restrict bit for bit. */
int mg_presmooth_restrict(mg_ctx *c, int level, int precision, const double *b, double *p,
                          double *b_coarse);

/* p += trilinear prolongation of e_coarse (level+1 -> level) */
int mg_prolong_correct(mg_ctx *c, int level, int precision, const double *e_coarse, double *p);

/* e = exact zero-mean solution of L e = r - mean(r) on the coarsest level */
int mg_coarse_solve(mg_ctx *c, const double *r, double *e);

/* ||b - L p||_2^2 on the finest level (host double out) */
int mg_residual_norm2(mg_ctx *c, const double *b, const double *p, double *norm2);

#ifdef __cplusplus
}
#endif

#endif /* MGP_H */
