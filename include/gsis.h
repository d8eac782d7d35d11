/*
 * gsis.h - C ABI of the MI355X (gfx950) GSIS / DVM library (libgsis.so).
 *
 * The library solves, to a steady state, the polyatomic radiative kinetic model of
 * the paper (Sec. 2.1: three reduced distributions for translational, rotational and
 * vibrational energy, gray radiation with one absorption coefficient) on an
 * unstructured finite-volume mesh with a discrete velocity set and a discrete ordinate
 * set.  Each outer iteration is one kinetic step (Sec. 6, Eq. delta_micro) and, for
 * GSIS, a solve of the macroscopic synthetic equations with high-order terms taken from
 * the kinetic moments (Sec. 2.2, Eqs. macroscopic_equation and getHoTs) followed by the
 * synchronisation of the distributions (Sec. 3).
 *
 * Conventions
 *  - All functions return int32_t: GSIS_OK (0) on success, a negative GSIS_E_* code on
 *    error, a positive GSIS_W_* code for a warning (results valid).  gsis_last_error()
 *    gives a message for the last failing call on that handle.
 *  - Host inputs are plain double / int64 arrays owned by the caller and copied during
 *    the call; the caller may free them on return.  Host outputs go to caller-owned
 *    buffers of the documented size.  Device state is owned by the handle and freed by
 *    gsis_destroy().
 *  - Velocity dimension equals the mesh dimension D (1, 2 or 3).  Below three dimensions
 *    the reduced model is used: per velocity node four distributions G = int f0, R = int f1,
 *    V = int f2, H = int |xi_perp|^2 f0 (velocity components normal to the simulated
 *    line/plane integrated out); in 3D the three distributions f0, f1, f2.
 *    Distribution arrays are laid out [nc][ND][nv] with ND = 4 (D < 3) or 3 (D = 3), in
 *    the order G, R, V[, H]; intensity arrays [nc][no].
 *  - One handle per host thread; distinct handles are independent.  All device work of a
 *    handle is issued on its stream (default: the null stream, see gsis_set_stream).
 */
#ifndef GSIS_H
#define GSIS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GSIS_OK = 0,
    GSIS_E_ARG = -1,      /* invalid argument or size */
    GSIS_E_OOM = -2,      /* device allocation failed */
    GSIS_E_DEVICE = -3,   /* HIP runtime error or no device */
    GSIS_E_STATE = -4,    /* call order violated (e.g. solve before mesh) */
    GSIS_E_DIVERGED = -5, /* NaN / non-positive density or temperature */
    GSIS_W_NOT_CONVERGED = 1 /* max_outer reached before tol */
};

enum { GSIS_BC_WALL = 0, GSIS_BC_FARFIELD = 1 };
enum { GSIS_CIS = 0, GSIS_GSIS = 1 };
enum { GSIS_FP64 = 0, GSIS_FP32 = 1 };
enum { GSIS_INIT_FIELDS = 0, GSIS_INIT_FREESTREAM = 1 };
/* Point relaxation of the first-order implicit kinetic operator (Sec. 6, Eq. delta_micro).  JACOBI:
 * kin_sweeps Jacobi sweeps (order-independent).  SGS: kin_sweeps symmetric Gauss-Seidel sweeps, the paper's
 * forward and backward sweep, taken colour by colour over a greedy distance-1 colouring of the cells (cells
 * in index order, each takes the smallest colour none of its face neighbours holds); the forward pass visits
 * the colours in ascending order, the backward pass in descending order.  One SGS sweep runs in place and
 * needs no increment buffer (the smallest memory footprint: f, its gradients and one residual buffer). */
enum { GSIS_SWEEP_JACOBI = 0, GSIS_SWEEP_SGS = 1 };

typedef struct gsis_s gsis_t;

/* Boundary condition of one boundary tag.  WALL: diffuse, fully accommodating wall at
 * temperature T moving with tangential velocity u (black for radiation; re-emission density
 * from zero net mass flux).  FARFIELD: equilibrium state (rho, u, T) on incoming velocities and
 * ordinates (radiation at B_R(T)). */
typedef struct {
    int32_t kind;
    double rho, T, u[3];
} gsis_bc;

/* Gas constants (Sec. 2.1): rotational / vibrational degrees of freedom, collision numbers, viscosity
 * index omega, Schmidt number of the Mason matrix A, normalised Stefan-Boltzmann constant sigma_R, and the
 * characteristic vibrational temperature Tv_ref (units of the reference temperature).  Tv_ref > 0 makes
 * the vibrational degrees of freedom temperature dependent, d_v(T) = 2 (Tv_ref / T) / (exp(Tv_ref / T) - 1):
 * the vibrational energy e_v = d_v(T_v) T_v / 2 everywhere (moments, reference distributions, equilibria,
 * boundary states, synthetic equations) and T_tv, T the roots of the energy balances of Sec. 2.1; d_v then
 * only sets the Mason matrix A and the synthetic equations' conductivities.  Tv_ref = 0: constant d_v. */
typedef struct {
    double d_r, d_v, Z_r, Z_v, omega, Sc, sigma_R;
    double Tv_ref;
} gsis_gas;

/* Flow parameters: Kn_gas enters tau = sqrt(2/pi) T_t^(omega-1) Kn_gas / rho; k_eff = 1/Kn_photon
 * (optical thickness per reference length; 0 switches absorption and emission off, and the radiation
 * energy then keeps its kinetic value in the synthetic solve, whose e_R row would be singular). */
typedef struct {
    double Kn_gas, k_eff;
} gsis_flow;

/* Iteration options.  Defaults (gsis_default_opts): GSIS, FP32, tol 1e-6, max_outer 1000,
 * n_precond 10, cfl_meso 1e5, cfl_v 5, kin_sweeps 8, kin_omega 1, limiter_K 10, second_order 1,
 * cfl_macro 1e3, inner_tol 1e-7, max_inner 100, n_sweeps 2, first_order_iters 0, sweep JACOBI, kin_fused 0, conservative 0. */
typedef struct {
    int32_t scheme;       /* GSIS_CIS or GSIS_GSIS */
    int32_t precision;    /* GSIS_FP64 or GSIS_FP32: storage and arithmetic of f and I */
    double tol;           /* convergence threshold on epsilon (Sec. 7) */
    int32_t max_outer;    /* outer iteration limit */
    int32_t n_precond;    /* CIS iterations before GSIS starts */
    double cfl_meso;      /* pseudo time step CFL of the kinetic equations (Sec. 6) */
    double cfl_v;         /* per-velocity pseudo time step CFL of the Jacobi point relaxation */
    int32_t kin_sweeps;   /* Jacobi sweeps of the first-order implicit kinetic operator */
    double kin_omega;     /* relaxation of the kinetic increment */
    double limiter_K;     /* Venkatakrishnan constant: eps^2 = (K h)^3 M^2, h = V^(1/D), M the largest |value| of the
                             limited variable over the cell and its face neighbours */
    int32_t second_order; /* limited second-order reconstruction of f and I */
    double cfl_macro;     /* pseudo time step CFL of the synthetic equations */
    double inner_tol;     /* relative drop of the macro residual that ends the inner solve */
    int32_t max_inner;    /* inner iteration limit */
    int32_t n_sweeps;     /* Jacobi sweeps of the macro implicit operator */
    int32_t first_order_iters; /* gsis_solve: the first this many outer iterations use first-order
                                  reconstruction (start-up of strongly non-equilibrium flows); 0 = none */
    int32_t sweep;        /* GSIS_SWEEP_JACOBI or GSIS_SWEEP_SGS (kin_sweeps counts the sweeps of either) */
    int32_t kin_fused;    /* 0: a gradient pass stores the limited gradients of f (nc x distributions x dim x
                             nv values) and the residual reads them; 1: the residual kernel recomputes the
                             gradients it needs (its cell's and its face neighbours', from the second ring of
                             f), so no gradient field is stored: dim x less memory for the kinetic buffers,
                             ~5x the gradient arithmetic.  Same arithmetic per velocity either way; velocity
                             counts not divisible by 16 bytes / element size always take the stored pass. */
    int32_t conservative; /* 1: discrete-conservative reference distributions: per cell and reference temperature
                             X, G gains a multiple e (psi . a) of e = rho f0^eq(T_X), psi = (1, c, c^2/2), whose
                             discrete moments restore (rho, 0, (D/2) rho T_X), and R, V, H scalar multiples of e
                             restoring their densities, so that the relaxation conserves mass, momentum and
                             energy on any velocity grid (a reduction over the velocities per cell and
                             iteration); 0 (default): the reference distributions as printed */
} gsis_opts;

typedef struct {
    int32_t iters;        /* outer iterations done */
    int32_t status;       /* return code of gsis_solve */
    double eps_final;     /* last epsilon */
    double t_total_s;     /* wall time of the solve (device-synchronised) */
    double t_kinetic_s;   /* time in the kinetic steps */
    double t_macro_s;     /* time in the macro solves */
    double t_other_s;     /* moments, synchronisation, residual */
    int64_t inner_total;  /* macro inner iterations summed over the solve */
} gsis_report;

/* Handle lifetime (infrastructure; no passage of the paper).  device: HIP device ordinal.  The destroy call
 * releases all device memory.  gsis_default_opts fills the defaults listed with gsis_opts (Sec. 6 and 7
 * settings: CFL numbers, 100 inner iterations, 10 conventional iterations before GSIS, tolerance 1e-6). */
int32_t gsis_create(int32_t device, gsis_t **out);
void gsis_destroy(gsis_t *h);
const char *gsis_last_error(gsis_t *h);
void gsis_default_opts(gsis_opts *o);

/* Use a caller-provided HIP stream (hipStream_t passed as void*), e.g. a torch stream handle
 * (infrastructure).  NULL selects the null stream.  The handle does not take ownership. */
int32_t gsis_set_stream(gsis_t *h, void *hip_stream);

/* Mesh (Sec. 6 finite-volume forms).  dim in {1,2,3}; vol[nc]; ctr[nc*dim] cell centroids;
 * face_cells[2*nf]: first cell of each face and the second cell, or -(1+tag) for a boundary
 * face with boundary tag `tag` (0 <= tag < nbc); face_n[nf*dim] unit normal from the first
 * to the second side; face_area[nf]; face_ctr[nf*dim].  Cells may have at most 2*dim faces.
 * Returns GSIS_E_ARG on inconsistent sizes, tags or a cell with too many faces. */
int32_t gsis_set_mesh(gsis_t *h, int32_t dim, int64_t nc, int64_t nf, const double *vol, const double *ctr,
                      const int64_t *face_cells, const double *face_n, const double *face_area,
                      const double *face_ctr, int32_t nbc, const gsis_bc *bcs);

/* Replace the state of boundary tag `tag` (0 <= tag < nbc of gsis_set_mesh) between iterations, e.g. to
 * raise a free-stream Mach number step by step from a converged state (continuation).  The kind must
 * stay the same (GSIS_E_ARG otherwise); the distributions are kept. */
int32_t gsis_set_boundary(gsis_t *h, int32_t tag, const gsis_bc *bc);

/* Discrete velocities xi[nv*dim] with quadrature weights w[nv] (int g dxi ~ sum w_k g(xi_k)): the discrete
 * velocity method of Sec. 6 (moments Eq. getmoment as weighted sums); any node set (tensor, spherical,
 * unstructured, Sec. 7.4).  GSIS_E_ARG for nv < 1 or null arrays. */
int32_t gsis_set_velocity_grid(gsis_t *h, int64_t nv, const double *xi, const double *w);

/* Discrete ordinates omega[no*3] (unit vectors) with weights w[no] summing to 4 pi (the angular
 * discretisation of the radiative transfer equation, Sec. 6); only the first dim components enter the
 * transport. */
int32_t gsis_set_ordinates(gsis_t *h, int64_t no, const double *omega, const double *w);

/* Gas constants and flow parameters of the kinetic model (Sec. 2.1, Eq. kinetic_equation and the relaxation
 * matrix A); GSIS_E_ARG for non-positive degrees of freedom or collision numbers, or a negative sigma_R,
 * Tv_ref, Kn or k_eff. */
int32_t gsis_set_gas(gsis_t *h, const gsis_gas *gas);
int32_t gsis_set_flow(gsis_t *h, const gsis_flow *flow);

/* Options; allocates the device state for the chosen precision (mesh, grids, gas and flow must be
 * set first, else GSIS_E_STATE).  Changing the precision discards the state: every call that reads the
 * state then returns GSIS_E_STATE until gsis_init_* or gsis_set_state initialises it again.  Other
 * changes (limiter constant, relaxation, counts) keep the state.
 * GSIS_E_ARG for an unknown scheme, precision or sweep, negative counts (sweeps, iteration limits,
 * n_precond, first_order_iters), second_order outside {0, 1}, negative tolerances, or a non-positive
 * limiter constant, relaxation factor or CFL number. */
int32_t gsis_set_opts(gsis_t *h, const gsis_opts *opts);

/* Equilibrium initial state from fields (the equilibrium of Sec. 3's synchronisation): rho[nc], u[nc*dim],
 * T[nc] (all modes and T_R equal T). */
int32_t gsis_init_equilibrium(gsis_t *h, const double *rho, const double *u, const double *T);

/* Multi-temperature equilibrium initial state (the f^eq of the synchronisation step, Sec. 3):
 * rho[nc], u[nc*dim], T_t[nc], T_r[nc], T_v[nc], T_R[nc] (radiation intensity sigma_R T_R^4 / pi on
 * every ordinate).  Used to start from predicted fields (learned warm start). */
int32_t gsis_init_fields(gsis_t *h, const double *rho, const double *u, const double *Tt, const double *Tr,
                         const double *Tv, const double *TR);

/* Full state in and out (double host arrays; f [nc][ND][nv], I [nc][no]): the reduced distributions of
 * Eq. reduced_distribution and the intensity I_R of Sec. 2.1, converted to and from the storage precision. */
int32_t gsis_set_state(gsis_t *h, const double *f, const double *I);
int32_t gsis_get_state(gsis_t *h, double *f, double *I);

/* The state rows of selected cells (double host arrays): f [n][ND][nv] and I [n][no] receive the reduced
 * distributions and intensities of cells[0 .. n) (cell indices of the mesh, in any order, repeats allowed),
 * the cell-averaged unknowns f_i of the discrete system of Sec. 6; either output may be null.  For checks and
 * probes of single cells of a state too large to copy whole.  GSIS_E_ARG for n < 0, null cells with n > 0,
 * or an index outside [0, nc); GSIS_E_STATE without an initialised state. */
int32_t gsis_get_state_cells(gsis_t *h, const int64_t *cells, int64_t n, double *f, double *I);

/* Checkpoint of the iteration state: f, I (in the storage precision, so a restore continues bit for bit)
 * and the residual history of the last gsis_solve, written to `path` (a binary file of the documented
 * layout, overwritten).  gsis_restore reads it into a handle set up with the same mesh, grids and
 * precision (GSIS_E_ARG otherwise, or for a missing, foreign or truncated file) and marks the state
 * initialised; the following iterations equal those the saved handle would have run.  GSIS_E_STATE before
 * gsis_set_opts (restore) or without an initialised state (checkpoint). */
int32_t gsis_checkpoint(gsis_t *h, const char *path);
int32_t gsis_restore(gsis_t *h, const char *path);

/* Outer iterations (Sec. 3).  gsis_iterate runs n iterations of the given scheme back to back (each
 * computes its residual; the host waits for the GPU once, after the last) and returns the last
 * epsilon in *eps, or a NaN of any iteration of the batch with GSIS_E_DIVERGED (the macro inner count
 * of the last iteration in *inner, may be NULL).
 * gsis_solve: n_precond CIS iterations, then opts.scheme until epsilon < tol or max_outer;
 * returns GSIS_OK, GSIS_W_NOT_CONVERGED or GSIS_E_DIVERGED. */
int32_t gsis_iterate(gsis_t *h, int32_t scheme, int32_t n, double *eps, int32_t *inner);
int32_t gsis_solve(gsis_t *h, gsis_report *rep);

/* Single stages, on the current state (for element-wise checks):
 *  kinetic step: f, I <- f + omega Delta (Eq. delta_micro with the Jacobi sweeps);
 *  macro solve: W[nc*(dim+5)] out = solution of the synthetic equations started from the moments
 *    of the current state, *inner = inner iterations;
 *  sync: f, I <- synchronised to the macro state W[nc*(dim+5)] (Sec. 3). */
int32_t gsis_kinetic_step(gsis_t *h);
int32_t gsis_macro_solve(gsis_t *h, double *W, int32_t *inner);
int32_t gsis_sync(gsis_t *h, const double *W);

/* Macroscopic fields of the current state (the moments of Eq. getmoment; T the total temperature of
 * Sec. 2.1; T_R from e_R = 4 sigma_R T_R^4), [nc][nfields] with nfields = 1 + D + 5 + 4 D + D(D+1)/2
 * in the order rho, u (D), T_t, T_r, T_v, T_R, T, q_t (D), q_r (D), q_v (D), q_R (D),
 * sigma (upper triangle, row by row). */
int32_t gsis_nfields(gsis_t *h);
int32_t gsis_get_fields(gsis_t *h, double *out);

/* Residual history of the last gsis_solve (epsilon of Sec. 7 per outer iteration): up to cap values into
 * buf, count in *n. */
int32_t gsis_get_residual_history(gsis_t *h, double *buf, int64_t cap, int64_t *n);

/* Surface quantities (the capsule's surface heat flux of Sec. 7.4) of the current state on boundary
 * faces, in face order (all nf faces; entries of
 * interior faces are 0): q_conv = gas energy flux into the boundary, q_rad = net radiative flux
 * through it, p_w = normal momentum flux. */
int32_t gsis_get_surface_flux(gsis_t *h, double *q_conv, double *q_rad, double *p_w);

/* Per-kernel timing with HIP events recorded on the handle's stream around each launch (measurement
 * infrastructure, no passage of the paper; off by default).
 * gsis_set_profiling(h, 1) clears and enables the counters for every kind; gsis_set_profiling(h,
 * GSIS_PROF_SELECT | (1 << kind) | ...) for the listed kinds only (fewer events in the timed stream);
 * 0 disables.  gsis_get_kernel_stats returns, for one kernel kind, the summed device time in ms, the
 * number of launches and the summed algorithmic bytes (each array the kernel must read or write, counted
 * once; 0 for kinds whose traffic is negligible). */
enum { GSIS_PROF_SELECT = 0x100 };
enum {
    GSIS_K_GRAD = 0,     /* limited gradients of the distributions */
    GSIS_K_RESIDUAL = 1, /* kinetic residual: fluxes, relaxation source, first increment */
    GSIS_K_SWEEP = 2,    /* Jacobi sweeps of the implicit kinetic operator (last one writes f) */
    GSIS_K_RAD = 3,      /* radiation kernels (gradients, residual, sweeps) */
    GSIS_K_MOMENTS = 4,  /* velocity-space moment reductions */
    GSIS_K_BOUNDARY = 5, /* wall re-emission densities and boundary flux moments */
    GSIS_K_SYNC = 6,     /* distribution synchronisation */
    GSIS_K_MACRO = 7     /* one synthetic-equation solve (all its kernels) */
};
int32_t gsis_set_profiling(gsis_t *h, int32_t on);
int32_t gsis_get_kernel_stats(gsis_t *h, int32_t kind, double *ms_total, int64_t *launches, double *bytes_total);

/* Counted work of the last gsis_solve / gsis_iterate calls (cell-velocity updates and algorithmic
 * HBM bytes of the kinetic steps), for throughput reporting (measurement infrastructure). */
int32_t gsis_get_counters(gsis_t *h, double *cellvel_updates, double *kinetic_bytes, double *kinetic_seconds);

#ifdef __cplusplus
}
#endif

#endif /* GSIS_H */
