/*
 * Plain FP64 CPU reference ("oracle") of the GSIS / DVM method for radiative
 * polyatomic gas flows.  TEST INFRASTRUCTURE ONLY: it is called by the tests,
 * by the package's smoke check and by the benchmark's CPU-baseline leg, never
 * by the product path.  It shares no code with the HIP library.
 *
 * Everything is written as the paper states it, in double precision, with no
 * blocking or fusion: loops over cells (OpenMP over cells only; every per-cell
 * result is computed in a fixed order, so results do not depend on the thread
 * count), then over discrete velocities / ordinates.
 *
 * Passages followed (paper section / equation):
 *   - kinetic model, reference distributions, equilibrium: Sec. 2.1,
 *     Eqs. (kinetic_equation), (reference_distribution), (equilibrium_distribution);
 *   - mode temperatures, pressures, moments: Sec. 2.1 and Eq. (getmoment);
 *   - tau, k_eff; heat-flux relaxation matrix A (Mason form) and the auxiliary
 *     heat fluxes q0, q1, q2: Sec. 2.1;
 *   - synthetic equations, NSF closure and HoTs: Sec. 2.2, Eqs. (macroscopic_equation),
 *     (NSF_constitutive), (NSF_thermal_conductivities), (split_constitutive), (getHoTs);
 *   - GSIS loop (kinetic step, macro solve with fixed HoTs, synchronisation,
 *     convergence test): Sec. 3;
 *   - finite-volume forms, implicit incremental schemes, upwind / Rusanov-type
 *     increments, limited second-order reconstruction, point relaxation,
 *     pseudo time step: Sec. 6, Eqs. (dis_micro), (deltaflux_micro);
 *   - convergence criterion: Sec. 7 (opening);
 *   - diagonal source Jacobian: Appendix A.
 *
 * Velocity space below three dimensions uses the reduced distributions
 * (velocity components normal to the simulated plane/line integrated out):
 * G = int f0, R = int f1, V = int f2, H = int |xi_perp|^2 f0, which is exact
 * integration of the paper's reference distributions (u and q have no
 * out-of-plane component).
 *
 * Where the paper is silent or garbled, the reading taken is marked
 * "reading:" at the place it applies.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

enum { BC_WALL = 0, BC_FARFIELD = 1 };

/* distribution slots per velocity node: G (f0), R (f1), V (f2), H (only below 3D) */
enum { DG = 0, DR = 1, DV = 2, DH = 3 };

typedef struct {
    double rho, u[3], Tt, Tr, Tv, er, ev, eR;
    double sig[3][3], qt[3], qr[3], qv[3], qR[3];
} mom_t;

typedef struct {
    double Ttr, Ttv, T, tau, q0[3], q1[3], q2[3], evR, B, cs, dt, dtR, radd;
    double ev_v, ev_tv; /* e_v(T_v), e_v(T_tv) */
    /* discrete-conservative corrections of the reference distributions (option `conservative`), per X in
     * (t, r, v): a0, aq, a[D] of G (times M_X: a0 + aq c^2 / (2 T_X) + a . c) and the scalars of R, V, H */
    int has_cons;
    double cons[3][8];
} der_t;

typedef struct orc_s {
    int D, ND;
    int64_t nc, nf;
    double *vol, *ctr, *fn, *fa, *fctr;
    int64_t *fc;
    int nbc;
    int *bck;
    double *bcrho, *bcT, *bcu;
    int64_t nv, no;
    double *xi, *w, *om, *wo;
    /* gas / flow */
    double dr, dv, Zr, Zv, omg, Sc, sigR, Kn, keff;
    double Tvref; /* characteristic vibrational temperature; <= 0: constant d_v */
    /* options */
    double cfl_meso, cfl_macro, limK, inner_tol, cfl_v, kin_omega;
    int kin_sweeps, diss_ref, macro_order2;
    int sweep; /* 0: Jacobi sweeps of the implicit kinetic operator; 1: colored symmetric Gauss-Seidel */
    double period;    /* > 0: the mesh is periodic along x with this length (test meshes of the Fourier analysis) */
    int rad_implicit; /* 1: the emission part of the gas-photon exchange joins the diagonal of f2 (default) */
    int conservative; /* 1: reference distributions corrected to conserve mass, momentum, energy on the grid */
    int max_inner, n_sweeps, second_order;
    /* derived constants */
    double A[3][3], Qm[3][3], K0[3][3];
    /* adjacency */
    int64_t *cptr, *cface;
    int *csign;
    int *color;   /* distance-1 colour of each cell (greedy, cells in index order) */
    int ncolor;
    int64_t *col_ptr, *col_cells; /* cells of colour q: col_cells[col_ptr[q] .. col_ptr[q+1]) */
    double *lsq; /* per slot: D coefficients (interior slots) */
    double *h;
    /* state */
    double *f, *I;
    /* boundary records (per face, valid on boundary faces) */
    double *bflux; /* NW per face: outward flux per unit area of (rho, rho u, e, e_r, e_v, e_R) */
    double *bsurf; /* 3 per face: q_conv, q_rad, p_w */
    double *rhow;  /* per face: wall re-emission density */
    int last_inner;
    int64_t safeguard_hits; /* cell updates the positivity / trust-region safeguard shortened (last solve) */
} orc_t;

static int NWof(int D) { return D + 5; }

/* Difference a - b of two coordinates along axis k.  On a mesh that is periodic along x (length o->period)
 * the nearest periodic image is taken, so that the face between the last and the first cell sees its two
 * cells at the distance they have across the period. */
static inline double gdiff(const struct orc_s *o, double a, double b, int k);

static inline double gdiff(const orc_t *o, double a, double b, int k)
{
    double d = a - b;
    if (k == 0 && o->period > 0) d -= o->period * floor(d / o->period + 0.5);
    return d;
}

/* ---------------------------------------------------------------- small linear algebra */
static int inv3(int n, const double *a, double *r)
{
    /* Gauss-Jordan with partial pivoting on an n x n matrix (n <= 3) */
    double m[3][6];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j) m[i][j] = (j < n) ? a[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int i = c + 1; i < n; ++i)
            if (fabs(m[i][c]) > fabs(m[p][c])) p = i;
        if (fabs(m[p][c]) < 1e-300) return -1;
        if (p != c)
            for (int j = 0; j < 2 * n; ++j) {
                double t = m[p][j];
                m[p][j] = m[c][j];
                m[c][j] = t;
            }
        double piv = m[c][c];
        for (int j = 0; j < 2 * n; ++j) m[c][j] /= piv;
        for (int i = 0; i < n; ++i)
            if (i != c) {
                double fct = m[i][c];
                for (int j = 0; j < 2 * n; ++j) m[i][j] -= fct * m[c][j];
            }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) r[i * n + j] = m[i][j + n];
    return 0;
}

/* ---------------------------------------------------------------- model constants */
/* A in the Mason approximation (Sec. 2.1), with constant d_v; q0..q2 coefficient
 * matrix (Sec. 2.1); K0 = A^{-1} diag(5, d_r, d_v) so that kappa_gas = (p_t tau / 2) K0. */
static void model_constants(orc_t *o)
{
    double dr = o->dr, dv = o->dv, Zr = o->Zr, Zv = o->Zv, Sc = o->Sc;
    double (*A)[3] = o->A;
    A[0][0] = 2.0 / 3.0 + 5.0 / 6.0 * (dr / ((3 + dr) * Zr) + dv / ((3 + dv) * Zv));
    A[0][1] = -5.0 / (2 * (3 + dr) * Zr);
    A[0][2] = -5.0 / (2 * (3 + dv) * Zv);
    A[1][0] = -dr / ((3 + dr) * Zr);
    A[1][1] = Sc + 3.0 / (2 * (3 + dr) * Zr);
    A[1][2] = 0.0;
    A[2][0] = -dv / ((3 + dv) * Zv);
    A[2][1] = 0.0;
    A[2][2] = Sc + 3.0 / (2 * (3 + dv) * Zv);
    double Zi = 1.0 / (1.0 / Zr + 1.0 / Zv);
    double (*Q)[3] = o->Qm;
    Q[0][0] = (2 - 3 * A[0][0]) * Zi + 1;
    Q[0][1] = -3 * A[0][1] * Zi;
    Q[0][2] = -3 * A[0][2] * Zi;
    Q[1][0] = -A[1][0] * Zi;
    Q[1][1] = 1 - A[1][1] * Zi;
    Q[1][2] = -A[1][2] * Zi;
    Q[2][0] = -A[2][0] * Zi;
    Q[2][1] = -A[2][1] * Zi;
    Q[2][2] = 1 - A[2][2] * Zi;
    double Ainv[9];
    inv3(3, &A[0][0], Ainv);
    double dg[3] = {5.0, dr, dv};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) o->K0[i][j] = Ainv[i * 3 + j] * dg[j];
}

/* ---------------------------------------------------------------- mesh adjacency, LSQ */
static void build_mesh(orc_t *o)
{
    int64_t nc = o->nc, nf = o->nf;
    int D = o->D;
    o->cptr = (int64_t *)calloc(nc + 1, sizeof(int64_t));
    for (int64_t f = 0; f < nf; ++f) {
        o->cptr[o->fc[2 * f] + 1]++;
        if (o->fc[2 * f + 1] >= 0) o->cptr[o->fc[2 * f + 1] + 1]++;
    }
    for (int64_t c = 0; c < nc; ++c) o->cptr[c + 1] += o->cptr[c];
    int64_t ns = o->cptr[nc];
    o->cface = (int64_t *)malloc(ns * sizeof(int64_t));
    o->csign = (int *)malloc(ns * sizeof(int));
    int64_t *fill = (int64_t *)calloc(nc, sizeof(int64_t));
    for (int64_t f = 0; f < nf; ++f) {
        int64_t L = o->fc[2 * f], R = o->fc[2 * f + 1];
        int64_t s = o->cptr[L] + fill[L]++;
        o->cface[s] = f;
        o->csign[s] = +1;
        if (R >= 0) {
            s = o->cptr[R] + fill[R]++;
            o->cface[s] = f;
            o->csign[s] = -1;
        }
    }
    free(fill);
    /* Distance-1 colouring for the ordered (Gauss-Seidel) point relaxation: cells visited in index order,
     * each takes the smallest colour none of its face neighbours already holds. */
    o->color = (int *)malloc(nc * sizeof(int));
    o->ncolor = 0;
    for (int64_t c = 0; c < nc; ++c) {
        int used[64] = {0};
        for (int64_t s = o->cptr[c]; s < o->cptr[c + 1]; ++s) {
            int64_t f = o->cface[s];
            int64_t j = (o->csign[s] > 0) ? o->fc[2 * f + 1] : o->fc[2 * f];
            if (j >= 0 && j < c) used[o->color[j]] = 1;
        }
        int q = 0;
        while (used[q]) ++q;
        o->color[c] = q;
        if (q + 1 > o->ncolor) o->ncolor = q + 1;
    }
    o->col_ptr = (int64_t *)calloc(o->ncolor + 1, sizeof(int64_t));
    o->col_cells = (int64_t *)malloc(nc * sizeof(int64_t));
    for (int64_t c = 0; c < nc; ++c) o->col_ptr[o->color[c] + 1]++;
    for (int q = 0; q < o->ncolor; ++q) o->col_ptr[q + 1] += o->col_ptr[q];
    {
        int64_t *pos = (int64_t *)malloc(o->ncolor * sizeof(int64_t));
        for (int q = 0; q < o->ncolor; ++q) pos[q] = o->col_ptr[q];
        for (int64_t c = 0; c < nc; ++c) o->col_cells[pos[o->color[c]]++] = c;
        free(pos);
    }
    o->h = (double *)malloc(nc * sizeof(double));
    o->lsq = (double *)calloc(ns * 3, sizeof(double));
    for (int64_t c = 0; c < nc; ++c) {
        o->h[c] = pow(o->vol[c], 1.0 / D);
        /* reading: weighted (1/|d|^2) least squares over face neighbours; a boundary face
         * contributes a ghost point at its centroid carrying the cell's own value. */
        double M[9] = {0};
        for (int64_t s = o->cptr[c]; s < o->cptr[c + 1]; ++s) {
            int64_t f = o->cface[s];
            int64_t j = (o->csign[s] > 0) ? o->fc[2 * f + 1] : o->fc[2 * f];
            double d[3] = {0, 0, 0}, d2 = 0;
            for (int a = 0; a < D; ++a) {
                d[a] = gdiff(o, j >= 0 ? o->ctr[j * D + a] : o->fctr[f * D + a], o->ctr[c * D + a], a);
                d2 += d[a] * d[a];
            }
            double wgt = 1.0 / d2;
            for (int a = 0; a < D; ++a)
                for (int b = 0; b < D; ++b) M[a * D + b] += wgt * d[a] * d[b];
        }
        double Mi[9];
        inv3(D, M, Mi);
        for (int64_t s = o->cptr[c]; s < o->cptr[c + 1]; ++s) {
            int64_t f = o->cface[s];
            int64_t j = (o->csign[s] > 0) ? o->fc[2 * f + 1] : o->fc[2 * f];
            double d[3] = {0, 0, 0}, d2 = 0;
            for (int a = 0; a < D; ++a) {
                d[a] = gdiff(o, j >= 0 ? o->ctr[j * D + a] : o->fctr[f * D + a], o->ctr[c * D + a], a);
                d2 += d[a] * d[a];
            }
            for (int a = 0; a < D; ++a) {
                double v = 0;
                for (int b = 0; b < D; ++b) v += Mi[a * D + b] * d[b];
                o->lsq[s * 3 + a] = v / d2;
            }
        }
    }
}

static inline int64_t other_cell(const orc_t *o, int64_t s)
{
    int64_t f = o->cface[s];
    return (o->csign[s] > 0) ? o->fc[2 * f + 1] : o->fc[2 * f];
}

/* least-squares gradient of a cell field a[c*stride + off] */
static void lsq_grad(const orc_t *o, const double *a, int64_t stride, int64_t off, int64_t c, double g[3])
{
    g[0] = g[1] = g[2] = 0;
    double ac = a[c * stride + off];
    for (int64_t s = o->cptr[c]; s < o->cptr[c + 1]; ++s) {
        int64_t j = other_cell(o, s);
        if (j < 0) continue;
        double da = a[j * stride + off] - ac;
        for (int k = 0; k < o->D; ++k) g[k] += o->lsq[s * 3 + k] * da;
    }
}

/* Venkatakrishnan limiter.  Reading: eps^2 = (K h)^3 M^2 with h = V^(1/D) and M the largest magnitude of
 * the limited variable over the cell and its face neighbours, so that the threshold follows the local size
 * of each variable (distributions at every velocity and intensities at every ordinate span many orders of
 * magnitude; an unscaled (K h)^3 leaves the small ones unlimited); phi per face capped at 1. */
static double venkat(const orc_t *o, const double *a, int64_t stride, int64_t off, int64_t c, const double g[3])
{
    double ac = a[c * stride + off], dmax = 0, dmin = 0, M = fabs(ac);
    for (int64_t s = o->cptr[c]; s < o->cptr[c + 1]; ++s) {
        int64_t j = other_cell(o, s);
        if (j < 0) continue;
        double aj = a[j * stride + off], da = aj - ac;
        if (da > dmax) dmax = da;
        if (da < dmin) dmin = da;
        if (fabs(aj) > M) M = fabs(aj);
    }
    double kh = o->limK * o->h[c];
    double eps2 = kh * kh * kh * M * M;
    double phi = 1.0;
    for (int64_t s = o->cptr[c]; s < o->cptr[c + 1]; ++s) {
        int64_t f = o->cface[s];
        double d2 = 0;
        for (int k = 0; k < o->D; ++k) d2 += g[k] * gdiff(o, o->fctr[f * o->D + k], o->ctr[c * o->D + k], k);
        double p = 1.0;
        if (d2 != 0.0) {
            double d1 = (d2 > 0) ? dmax : dmin;
            p = (d1 * d1 + eps2 + 2 * d1 * d2) / (d1 * d1 + 2 * d2 * d2 + d1 * d2 + eps2);
            if (p > 1.0) p = 1.0;
        }
        if (p < phi) phi = p;
    }
    return phi;
}

/* limited gradient phi * grad, or zero for first-order reconstruction */
static void limited_grad_o(const orc_t *o, int order2, const double *a, int64_t stride, int64_t off, int64_t c,
                           double gl[3]);
static void limited_grad(const orc_t *o, const double *a, int64_t stride, int64_t off, int64_t c, double gl[3])
{
    limited_grad_o(o, o->second_order, a, stride, off, c, gl);
}
static void limited_grad_o(const orc_t *o, int order2, const double *a, int64_t stride, int64_t off, int64_t c,
                           double gl[3])
{
    if (!order2) {
        gl[0] = gl[1] = gl[2] = 0;
        return;
    }
    double g[3];
    lsq_grad(o, a, stride, off, c, g);
    double phi = venkat(o, a, stride, off, c, g);
    for (int k = 0; k < 3; ++k) gl[k] = phi * g[k];
}

/* ---------------------------------------------------------------- vibrational energy (Sec. 2.1)
 * d_v(T) = 2 (T_ref / T) / (exp(T_ref / T) - 1) for a characteristic temperature T_ref > 0, so the energy per
 * unit mass e_v(T) = d_v(T) T / 2 = T_ref / (exp(T_ref / T) - 1), with inverse T = T_ref / ln(1 + T_ref / e_v)
 * and heat capacity c_v(T) = de_v/dT = x^2 / (4 sinh^2(x / 2)), x = T_ref / T.  Without T_ref the model's
 * constant d_v is used and every formula below reduces to its constant-d_v form. */
static double ev_of(const orc_t *o, double T) { return o->Tvref > 0 ? o->Tvref / expm1(o->Tvref / T) : 0.5 * o->dv * T; }

static double cv_of(const orc_t *o, double T)
{
    if (o->Tvref <= 0) return 0.5 * o->dv;
    double x = o->Tvref / T, sh = sinh(0.5 * x);
    return x * x / (4 * sh * sh);
}

/* rho e_v(T) */
static double rho_ev(const orc_t *o, double rho, double T) { return o->Tvref > 0 ? rho * ev_of(o, T) : 0.5 * o->dv * rho * T; }

/* T_v of the vibrational energy ev (per unit volume) of a gas of density rho */
static double Tv_of(const orc_t *o, double ev, double rho)
{
    return o->Tvref > 0 ? o->Tvref / log1p(o->Tvref * rho / ev) : 2 * ev / (o->dv * rho);
}

/* equilibrium temperature T of alpha T + e_v(T) = R (energy shared by modes of alpha = (3 + d)/2 constant
 * degrees of freedom and the vibrational mode): Newton from T = R / alpha, where alpha T + e_v(T) - R >= 0;
 * the left side is increasing and convex in T, so the iterates decrease monotonically to the root */
static double eq_temperature(const orc_t *o, double alpha, double R)
{
    double T = R / alpha;
    for (int it = 0; it < 100; ++it) {
        double dT = (alpha * T + ev_of(o, T) - R) / (alpha + cv_of(o, T));
        T -= dT;
        if (!(fabs(dT) > 1e-15 * T)) break;
    }
    return T;
}

/* T_tv (translational-vibrational equilibrium) and the total temperature T of Sec. 2.1 */
static double Ttv_of(const orc_t *o, double Tt, double Tv)
{
    if (o->Tvref <= 0) return (3 * Tt + o->dv * Tv) / (3 + o->dv);
    return eq_temperature(o, 1.5, 1.5 * Tt + ev_of(o, Tv));
}

static double Ttot_of(const orc_t *o, double Tt, double Tr, double Tv)
{
    if (o->Tvref <= 0) return (3 * Tt + o->dr * Tr + o->dv * Tv) / (3 + o->dr + o->dv);
    return eq_temperature(o, 0.5 * (3 + o->dr), 1.5 * Tt + 0.5 * o->dr * Tr + ev_of(o, Tv));
}

/* ---------------------------------------------------------------- moments (Eq. getmoment) */
static void cell_moments(const orc_t *o, const double *f, const double *I, int64_t c, mom_t *m)
{
    int D = o->D, ND = o->ND;
    int64_t nv = o->nv;
    memset(m, 0, sizeof(*m));
    const double *G = f + (c * ND + DG) * nv, *R = f + (c * ND + DR) * nv, *V = f + (c * ND + DV) * nv;
    const double *H = (ND == 4) ? f + (c * ND + DH) * nv : NULL;
    double rho = 0, mom[3] = {0, 0, 0};
    for (int64_t k = 0; k < nv; ++k) {
        rho += o->w[k] * G[k];
        for (int a = 0; a < D; ++a) mom[a] += o->w[k] * o->xi[k * D + a] * G[k];
    }
    m->rho = rho;
    for (int a = 0; a < D; ++a) m->u[a] = mom[a] / rho;
    double E = 0, er = 0, ev = 0;
    for (int64_t k = 0; k < nv; ++k) {
        double cc[3] = {0, 0, 0}, c2 = 0;
        for (int a = 0; a < D; ++a) {
            cc[a] = o->xi[k * D + a] - m->u[a];
            c2 += cc[a] * cc[a];
        }
        double h = H ? H[k] : 0.0;
        double wk = o->w[k];
        E += wk * (c2 * G[k] + h);
        er += wk * R[k];
        ev += wk * V[k];
        for (int a = 0; a < D; ++a) {
            for (int b = 0; b < D; ++b) m->sig[a][b] += wk * cc[a] * cc[b] * G[k];
            m->qt[a] += 0.5 * wk * cc[a] * (c2 * G[k] + h);
            m->qr[a] += wk * cc[a] * R[k];
            m->qv[a] += wk * cc[a] * V[k];
        }
    }
    m->Tt = E / (3 * rho);
    m->er = er;
    m->ev = ev;
    m->Tr = 2 * er / (o->dr * rho);
    m->Tv = Tv_of(o, ev, rho);
    for (int a = 0; a < D; ++a) m->sig[a][a] -= rho * m->Tt;
    double eR = 0;
    for (int64_t q = 0; q < o->no; ++q) {
        double Iq = I[c * o->no + q];
        eR += o->wo[q] * Iq;
        for (int a = 0; a < D; ++a) m->qR[a] += o->wo[q] * o->om[q * 3 + a] * Iq;
    }
    m->eR = eR;
}

static void ref_dists(const orc_t *o, const mom_t *m, const der_t *d, const double *xi, double Y[3][4]);
static double maxw(int D, double T, double c2);

/* solve the symmetric positive definite n x n system A x = b (Cholesky, row-major A); returns 0 when a pivot
 * falls below 1e-12 times its diagonal entry (the system is then left unsolved) */
static int spd_solve(int n, const double *A, const double *b, double *x)
{
    double L[8][8];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double v = A[i * n + j];
            for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(v > 1e-12 * A[i * n + i])) return 0;
                L[i][i] = sqrt(v);
            } else {
                L[i][j] = v / L[j][j];
            }
        }
    double y[8];
    for (int i = 0; i < n; ++i) {
        double v = b[i];
        for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
        y[i] = v / L[i][i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < n; ++k) v -= L[k][i] * x[k];
        x[i] = v / L[i][i];
    }
    return 1;
}

/* Discrete-conservative reference distributions (reading): on a discrete velocity grid the reference
 * distributions of Eq. (reference_distribution) do not carry exactly the moments the relaxation must
 * conserve.  For each X in (t, r, v), with M_X = rho f0^eq(T_X) and the polynomial basis psi = (1, c, c^2/2),
 * c = xi - u, the correction G += M_X (psi . a) is the one whose discrete moments make
 * sum w psi G = (rho, 0, (D/2) rho T_X) (the normal equations B a = target - sum w psi G with
 * B = sum w psi psi^T M_X); R, V and H get scalar multiples of M_X restoring their densities
 * (d_r/2) T_RX rho, e_v(T_VX) rho and (3 - D) T_X rho.  With the corrections the relaxation conserves mass,
 * momentum and energy to round-off on any grid; a system whose Cholesky pivot falls below 1e-12 of its
 * diagonal (a Maxwellian narrower than the grid resolves) is left uncorrected. */
static void conservative_corrections(const orc_t *o, const mom_t *m, der_t *d)
{
    int D = o->D, n = D + 2;
    double TX[3] = {m->Tt, d->Ttr, d->Ttv};
    double TRX[3] = {m->Tr, d->Ttr, m->Tr};
    double EVX[3] = {d->ev_v, d->ev_v, d->ev_tv};
    double TVX[3] = {m->Tv, m->Tv, d->Ttv};
    double B[3][25], mG[3][5], mR[3], mV[3], mH[3];
    for (int X = 0; X < 3; ++X) {
        for (int i = 0; i < 25; ++i) B[X][i] = 0;
        for (int i = 0; i < 5; ++i) mG[X][i] = 0;
        mR[X] = mV[X] = mH[X] = 0;
    }
    d->has_cons = 0;
    for (int64_t k = 0; k < o->nv; ++k) {
        const double *xi = o->xi + k * D;
        double Y[3][4], psi[5], c2 = 0;
        ref_dists(o, m, d, xi, Y);
        psi[0] = 1;
        for (int a = 0; a < D; ++a) {
            psi[1 + a] = xi[a] - m->u[a];
            c2 += psi[1 + a] * psi[1 + a];
        }
        psi[D + 1] = 0.5 * c2;
        double wk = o->w[k];
        for (int X = 0; X < 3; ++X) {
            double e = m->rho * maxw(D, TX[X], c2);
            for (int i = 0; i < n; ++i) {
                mG[X][i] += wk * psi[i] * Y[X][DG];
                for (int j = 0; j < n; ++j) B[X][i * n + j] += wk * psi[i] * psi[j] * e;
            }
            mR[X] += wk * Y[X][DR];
            mV[X] += wk * Y[X][DV];
            if (o->ND == 4) mH[X] += wk * Y[X][DH];
        }
    }
    for (int X = 0; X < 3; ++X) {
        double rhs[5] = {0, 0, 0, 0, 0}, a[5] = {0, 0, 0, 0, 0};
        for (int i = 0; i < n; ++i) rhs[i] = -mG[X][i];
        rhs[0] += m->rho;
        rhs[D + 1] += 0.5 * D * m->rho * TX[X];
        double *k = d->cons[X];
        for (int i = 0; i < 8; ++i) k[i] = 0;
        if (spd_solve(n, B[X], rhs, a)) {
            /* psi . a = a0 + a_E c^2/2 + a . c; stored as a0, a_E T_X (coefficient of c^2 / (2 T_X)), a */
            k[0] = a[0];
            k[1] = a[D + 1] * TX[X];
            for (int q = 0; q < D; ++q) k[2 + q] = a[1 + q];
        }
        double S = B[X][0];
        double evx = o->Tvref > 0 ? EVX[X] : 0.5 * o->dv * TVX[X];
        k[D + 2] = (0.5 * o->dr * TRX[X] * m->rho - mR[X]) / S;
        k[D + 3] = (evx * m->rho - mV[X]) / S;
        k[D + 4] = (o->ND == 4) ? ((3 - D) * TX[X] * m->rho - mH[X]) / S : 0.0;
    }
    d->has_cons = 1;
}

static void derived(const orc_t *o, const mom_t *m, int64_t c, der_t *d)
{
    double dr = o->dr;
    d->Ttr = (3 * m->Tt + dr * m->Tr) / (3 + dr);
    d->Ttv = Ttv_of(o, m->Tt, m->Tv);
    d->T = Ttot_of(o, m->Tt, m->Tr, m->Tv);
    d->ev_v = ev_of(o, m->Tv);
    d->ev_tv = ev_of(o, d->Ttv);
    d->tau = sqrt(2.0 / PI) * pow(m->Tt, o->omg - 1.0) * o->Kn / m->rho;
    for (int a = 0; a < 3; ++a) {
        d->q0[a] = o->Qm[0][0] * m->qt[a] + o->Qm[0][1] * m->qr[a] + o->Qm[0][2] * m->qv[a];
        d->q1[a] = o->Qm[1][0] * m->qt[a] + o->Qm[1][1] * m->qr[a] + o->Qm[1][2] * m->qv[a];
        d->q2[a] = o->Qm[2][0] * m->qt[a] + o->Qm[2][1] * m->qr[a] + o->Qm[2][2] * m->qv[a];
    }
    double Tv2 = m->Tv * m->Tv;
    d->evR = 4 * o->sigR * Tv2 * Tv2;
    /* reading: the emission part of the gas-photon exchange on f2 is treated point-implicitly in the
     * relaxation: its linearised rate d(k_eff e_vR)/d e_v = 4 k_eff e_vR / e_v joins the diagonal of f2.
     * This changes the iteration path only (the residual is unchanged) and keeps T_v positive where the
     * emission rate per unit vibrational energy is large (low density). */
    d->radd = o->rad_implicit ? 4 * o->keff * d->evR / m->ev : 0.0;
    if (o->rad_implicit && o->Tvref > 0) d->radd = 4 * o->keff * d->evR / (m->rho * m->Tv * cv_of(o, m->Tv));
    d->B = o->sigR * Tv2 * Tv2 / PI;
    d->cs = sqrt(5.0 / 3.0 * m->Tt);
    double un = 0;
    for (int a = 0; a < o->D; ++a) un += m->u[a] * m->u[a];
    /* reading: pseudo time step dt = CFL h / (|u| + c_s); photons move at unit speed */
    d->dt = o->cfl_meso * o->h[c] / (sqrt(un) + d->cs);
    d->dtR = o->cfl_meso * o->h[c];
    d->has_cons = 0;
    if (o->conservative) conservative_corrections(o, m, d);
}

/* normalised D-dimensional Maxwellian (reduced form of f0^eq) */
static double maxw(int D, double T, double c2)
{
    return pow(2 * PI * T, -0.5 * D) * exp(-c2 / (2 * T));
}

/* Reference distributions g_{l,X} for X in {t, r, v} at one velocity node (Eq. reference_distribution,
 * integrated over the velocity components outside the simulated space). Y[X][slot]. */
static void ref_dists(const orc_t *o, const mom_t *m, const der_t *d, const double *xi, double Y[3][4])
{
    int D = o->D;
    double cc[3] = {0, 0, 0}, c2 = 0;
    for (int a = 0; a < D; ++a) {
        cc[a] = xi[a] - m->u[a];
        c2 += cc[a] * cc[a];
    }
    double TX[3] = {m->Tt, d->Ttr, d->Ttv};
    const double *qX[3] = {m->qt, d->q0, d->q0};
    double TRX[3] = {m->Tr, d->Ttr, m->Tr};
    const double *qRX[3] = {m->qr, d->q1, d->q1};
    double TVX[3] = {m->Tv, m->Tv, d->Ttv};
    double EVX[3] = {d->ev_v, d->ev_v, d->ev_tv}; /* e_v(T_v), e_v(T_v), e_v(T_tv): d_v(T) T / 2 */
    const double *qVX[3] = {m->qv, d->q2, d->q2};
    for (int X = 0; X < 3; ++X) {
        double T = TX[X], p = m->rho * T;
        double M = maxw(D, T, c2);
        double qc = 0, qrc = 0, qvc = 0;
        for (int a = 0; a < D; ++a) {
            qc += qX[X][a] * cc[a];
            qrc += qRX[X][a] * cc[a];
            qvc += qVX[X][a] * cc[a];
        }
        double s = 2 * qc / (15 * T * p);
        double G = m->rho * M * (1 + s * (c2 / (2 * T) - 0.5 * (2 + D)));
        Y[X][DG] = G;
        Y[X][DR] = 0.5 * o->dr * TRX[X] * G + qrc / T * M;
        Y[X][DV] = (o->Tvref > 0 ? EVX[X] * G : 0.5 * o->dv * TVX[X] * G) + qvc / T * M;
        Y[X][DH] = (3 - D) * m->rho * T * M * (1 + s * (c2 / (2 * T) - 0.5 * D));
        if (d->has_cons) {
            const double *k = d->cons[X];
            double P = k[0] + k[1] * c2 / (2 * T);
            for (int a = 0; a < D; ++a) P += k[2 + a] * cc[a];
            double e = m->rho * M;
            Y[X][DG] += P * e;
            Y[X][DR] += k[D + 2] * e;
            Y[X][DV] += k[D + 3] * e;
            Y[X][DH] += k[D + 4] * e;
        }
    }
}

/* relaxation source J (Eq. kinetic_equation) for the ND slots at velocity k of cell c */
static void collision(const orc_t *o, const mom_t *m, const der_t *d, const double *fk /* ND values */,
                      const double *xi, double *J)
{
    double Y[3][4];
    ref_dists(o, m, d, xi, Y);
    double tau = d->tau;
    for (int s = 0; s < o->ND; ++s)
        J[s] = (Y[0][s] - fk[s]) / tau + (Y[1][s] - Y[0][s]) / (o->Zr * tau) + (Y[2][s] - Y[0][s]) / (o->Zv * tau);
    /* gas-photon exchange on f2: -(f0/rho) k_eff int (B_R(T_v) - I_R) dOmega, int B dOmega = 4 sigma_R T_v^4 */
    J[DV] -= fk[DG] / m->rho * o->keff * (d->evR - m->eR);
}

/* equilibrium boundary state (rho, u, T) values at velocity xi, all slots */
static void boundary_eq(const orc_t *o, double rho, const double *u, double T, const double *xi, double *Y)
{
    int D = o->D;
    double c2 = 0;
    for (int a = 0; a < D; ++a) c2 += (xi[a] - u[a]) * (xi[a] - u[a]);
    double G = rho * maxw(D, T, c2);
    Y[DG] = G;
    Y[DR] = 0.5 * o->dr * T * G;
    Y[DV] = o->Tvref > 0 ? ev_of(o, T) * G : 0.5 * o->dv * T * G;
    Y[DH] = (3 - D) * T * G;
}

/* ---------------------------------------------------------------- kinetic step */
typedef struct {
    mom_t *m;
    der_t *d;
    double *gl;  /* limited gradients of f: [nc*ND*nv][3] */
    double *glI; /* limited gradients of I: [nc*no][3] */
} kin_ws_t;

static void all_moments(const orc_t *o, const double *f, const double *I, mom_t *m)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < o->nc; ++c) cell_moments(o, f, I, c, &m[c]);
}

/* wall re-emission densities: zero net mass flux through each wall face (reading: diffuse walls) */
static void wall_densities(orc_t *o, const double *gl)
{
    int D = o->D, ND = o->ND;
    int64_t nv = o->nv;
    for (int64_t f = 0; f < o->nf; ++f) {
        int64_t R = o->fc[2 * f + 1];
        o->rhow[f] = 0;
        if (R >= 0) continue;
        int b = (int)(-R - 1);
        if (o->bck[b] != BC_WALL) continue;
        int64_t c = o->fc[2 * f];
        double out = 0, in = 0;
        for (int64_t k = 0; k < nv; ++k) {
            double xn = 0, dx = 0, c2 = 0;
            for (int a = 0; a < D; ++a) xn += o->xi[k * D + a] * o->fn[f * D + a];
            const double *g = gl + ((c * ND + DG) * nv + k) * 3;
            for (int a = 0; a < D; ++a) dx += g[a] * gdiff(o, o->fctr[f * D + a], o->ctr[c * D + a], a);
            for (int a = 0; a < D; ++a) c2 += (o->xi[k * D + a] - o->bcu[b * 3 + a]) * (o->xi[k * D + a] - o->bcu[b * 3 + a]);
            if (xn > 0)
                out += o->w[k] * xn * (o->f[(c * ND + DG) * nv + k] + dx);
            else
                in += o->w[k] * (-xn) * maxw(D, o->bcT[b], c2);
        }
        o->rhow[f] = out / in;
    }
}

/* boundary flux moments of the state f, I (outward from the interior cell, per unit area): the NW conserved
 * fluxes used by the macro solver's boundary faces, and the surface output (q_conv, q_rad, p_w) */
static void record_boundary(orc_t *o, const double *gl, const double *glI)
{
    int D = o->D, ND = o->ND;
    int64_t nv = o->nv, no = o->no;
    int NW = NWof(D);
    for (int64_t f = 0; f < o->nf; ++f) {
        int64_t R = o->fc[2 * f + 1];
        if (R >= 0) continue;
        int b = (int)(-R - 1);
        int64_t c = o->fc[2 * f];
        double *F = o->bflux + f * NW;
        for (int i = 0; i < NW; ++i) F[i] = 0;
        double qconv = 0, qrad = 0, pw = 0;
        for (int64_t k = 0; k < nv; ++k) {
            const double *xi = o->xi + k * D;
            double xn = 0, x2 = 0;
            for (int a = 0; a < D; ++a) {
                xn += xi[a] * o->fn[f * D + a];
                x2 += xi[a] * xi[a];
            }
            double fv[4];
            if (xn > 0) {
                for (int sl = 0; sl < ND; ++sl) {
                    const double *g = gl + ((c * ND + sl) * nv + k) * 3;
                    double dx = 0;
                    for (int a = 0; a < D; ++a) dx += g[a] * gdiff(o, o->fctr[f * D + a], o->ctr[c * D + a], a);
                    fv[sl] = o->f[(c * ND + sl) * nv + k] + dx;
                }
            } else {
                if (o->bck[b] == BC_WALL)
                    boundary_eq(o, o->rhow[f], o->bcu + b * 3, o->bcT[b], xi, fv);
                else
                    boundary_eq(o, o->bcrho[b], o->bcu + b * 3, o->bcT[b], xi, fv);
            }
            double hv = (ND == 4) ? fv[DH] : 0.0;
            double wk = o->w[k];
            double en = 0.5 * x2 * fv[DG] + 0.5 * hv + fv[DR] + fv[DV];
            F[0] += wk * xn * fv[DG];
            for (int a = 0; a < D; ++a) F[1 + a] += wk * xn * xi[a] * fv[DG];
            F[D + 1] += wk * xn * en;
            F[D + 2] += wk * xn * fv[DR];
            F[D + 3] += wk * xn * fv[DV];
            qconv += wk * xn * en;
            pw += wk * xn * xn * fv[DG];
        }
        for (int64_t q = 0; q < no; ++q) {
            const double *om = o->om + q * 3;
            double on = 0;
            for (int a = 0; a < D; ++a) on += om[a] * o->fn[f * D + a];
            double Iv;
            if (on > 0) {
                const double *g = glI + (c * no + q) * 3;
                double dx = 0;
                for (int a = 0; a < D; ++a) dx += g[a] * gdiff(o, o->fctr[f * D + a], o->ctr[c * D + a], a);
                Iv = o->I[c * no + q] + dx;
            } else {
                double Tb = o->bcT[b];
                Iv = o->sigR * Tb * Tb * Tb * Tb / PI;
            }
            qrad += o->wo[q] * on * Iv;
        }
        F[D + 4] = qrad;
        F[D + 1] += qrad;
        o->bsurf[f * 3 + 0] = qconv;
        o->bsurf[f * 3 + 1] = qrad;
        o->bsurf[f * 3 + 2] = pw;
    }
}

/* One kinetic step: f^{k+1/2} = f^k + Delta f with Delta f = r / d (point relaxation in Jacobi
 * form), Eqs. (delta_micro) and the d_i of Sec. 6; same for the radiative intensity. */
static void kinetic_step(orc_t *o, double *fout, double *Iout, double *racc /* optional residual out */)
{
    int D = o->D, ND = o->ND;
    int64_t nc = o->nc, nv = o->nv, no = o->no;
    mom_t *m = (mom_t *)malloc(nc * sizeof(mom_t));
    der_t *d = (der_t *)malloc(nc * sizeof(der_t));
    all_moments(o, o->f, o->I, m);
    for (int64_t c = 0; c < nc; ++c) derived(o, &m[c], c, &d[c]);
    double *gl = (double *)malloc((size_t)nc * ND * nv * 3 * sizeof(double));
    double *glI = (double *)malloc((size_t)nc * no * 3 * sizeof(double));
    double *dco = (double *)malloc((size_t)nc * nv * sizeof(double));
    double *dcoR = (double *)malloc((size_t)nc * no * sizeof(double));
    double *rr = (double *)malloc((size_t)nc * ND * nv * sizeof(double));
    double *rI = (double *)malloc((size_t)nc * no * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        for (int s = 0; s < ND; ++s)
            for (int64_t k = 0; k < nv; ++k)
                limited_grad(o, o->f, ND * nv, s * nv + k, c, gl + ((c * ND + s) * nv + k) * 3);
        for (int64_t q = 0; q < no; ++q) limited_grad(o, o->I, no, q, c, glI + (c * no + q) * 3);
    }
    wall_densities(o, gl);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        double V = o->vol[c];
        for (int64_t k = 0; k < nv; ++k) {
            const double *xi = o->xi + k * D;
            double flux[4] = {0, 0, 0, 0}, dsum = 0;
            for (int64_t s = o->cptr[c]; s < o->cptr[c + 1]; ++s) {
                int64_t f = o->cface[s];
                double n[3] = {0, 0, 0}, xn = 0;
                for (int a = 0; a < D; ++a) {
                    n[a] = o->csign[s] * o->fn[f * D + a];
                    xn += xi[a] * n[a];
                }
                double S = o->fa[f];
                double fv[4];
                if (xn > 0) {
                    for (int sl = 0; sl < ND; ++sl) {
                        const double *g = gl + ((c * ND + sl) * nv + k) * 3;
                        double dx = 0;
                        for (int a = 0; a < D; ++a) dx += g[a] * gdiff(o, o->fctr[f * D + a], o->ctr[c * D + a], a);
                        fv[sl] = o->f[(c * ND + sl) * nv + k] + dx;
                    }
                } else {
                    int64_t j = other_cell(o, s);
                    if (j >= 0) {
                        for (int sl = 0; sl < ND; ++sl) {
                            const double *g = gl + ((j * ND + sl) * nv + k) * 3;
                            double dx = 0;
                            for (int a = 0; a < D; ++a) dx += g[a] * gdiff(o, o->fctr[f * D + a], o->ctr[j * D + a], a);
                            fv[sl] = o->f[(j * ND + sl) * nv + k] + dx;
                        }
                    } else {
                        int b = (int)(-j - 1);
                        if (o->bck[b] == BC_WALL)
                            boundary_eq(o, o->rhow[f], o->bcu + b * 3, o->bcT[b], xi, fv);
                        else
                            boundary_eq(o, o->bcrho[b], o->bcu + b * 3, o->bcT[b], xi, fv);
                    }
                }
                for (int sl = 0; sl < ND; ++sl) flux[sl] += xn * fv[sl] * S;
                if (xn > 0) dsum += xn * S;
            }
            double fk[4], J[4];
            for (int sl = 0; sl < ND; ++sl) fk[sl] = o->f[(c * ND + sl) * nv + k];
            collision(o, &m[c], &d[c], fk, xi, J);
            /* reading: a per-velocity pseudo time step, 1/dt_v = (sum xi_n^+ S)/(V CFL_v), keeps the
             * Jacobi form of the point relaxation stable with the explicit second-order residual */
            double dcoef = 1.0 / d[c].dt + 1.0 / d[c].tau + dsum / V * (1.0 + 1.0 / o->cfl_v);
            dco[c * nv + k] = dcoef;
            for (int sl = 0; sl < ND; ++sl) {
                double r = J[sl] - flux[sl] / V;
                if (racc) racc[(c * ND + sl) * nv + k] = r;
                rr[(c * ND + sl) * nv + k] = r;
                fout[(c * ND + sl) * nv + k] = r / (dcoef + (sl == DV ? d[c].radd : 0.0));
            }
        }
        for (int64_t q = 0; q < no; ++q) {
            const double *om = o->om + q * 3;
            double flux = 0, dsum = 0;
            for (int64_t s = o->cptr[c]; s < o->cptr[c + 1]; ++s) {
                int64_t f = o->cface[s];
                double on = 0;
                for (int a = 0; a < D; ++a) on += om[a] * o->csign[s] * o->fn[f * D + a];
                double S = o->fa[f], Iv;
                if (on > 0) {
                    const double *g = glI + (c * no + q) * 3;
                    double dx = 0;
                    for (int a = 0; a < D; ++a) dx += g[a] * gdiff(o, o->fctr[f * D + a], o->ctr[c * D + a], a);
                    Iv = o->I[c * no + q] + dx;
                } else {
                    int64_t j = other_cell(o, s);
                    if (j >= 0) {
                        const double *g = glI + (j * no + q) * 3;
                        double dx = 0;
                        for (int a = 0; a < D; ++a) dx += g[a] * gdiff(o, o->fctr[f * D + a], o->ctr[j * D + a], a);
                        Iv = o->I[j * no + q] + dx;
                    } else {
                        int b = (int)(-j - 1);
                        double Tb = o->bcT[b];
                        /* reading: black walls and an equilibrium far field emit B_R(T_b) */
                        Iv = o->sigR * Tb * Tb * Tb * Tb / PI;
                    }
                }
                flux += on * Iv * S;
                if (on > 0) dsum += on * S;
            }
            double Ic = o->I[c * no + q];
            double r = o->keff * (d[c].B - Ic) - flux / V;
            double dcoef = 1.0 / d[c].dtR + o->keff + dsum / V * (1.0 + 1.0 / o->cfl_v);
            dcoR[c * no + q] = dcoef;
            rI[c * no + q] = r;
            Iout[c * no + q] = r / dcoef;
        }
    }
    /* Jacobi sweeps of the first-order implicit operator, Eq. (delta_micro) with the upwind increment
     * xi_n Delta f_ij = xi_n^+ Delta f_i + xi_n^- Delta f_j: Delta^s_i = (r_i - (1/V) sum xi_n^- S Delta^{s-1}_j) / d_i.
     * reading: boundary faces carry no increment; the update is f + omega Delta. */
    if (o->sweep == 1) {
        /* Symmetric Gauss-Seidel sweep of the same first-order implicit operator, the paper's forward and
         * backward point relaxation (Sec. 6), taken colour by colour (cells of one colour have no face in
         * common, so the order inside a colour does not matter).  With the lower part L (neighbours of a
         * smaller colour), the upper part U (a larger colour) and the diagonal d:
         *   forward, colours ascending:   Delta*_i = (r_i - (1/V) sum_{j in L} xi_n^- S Delta*_j) / d_i,
         *   backward, colours descending: Delta_i = Delta*_i - (1/(V d_i)) sum_{j in U} xi_n^- S Delta_j,
         * i.e. (D + L) D^-1 (D + U) Delta = r. */
        const int npass = 2 * (o->kin_sweeps > 0 ? o->kin_sweeps : 1);
        for (int ip = 0; ip < npass; ++ip) {
            const int pass = ip & 1, first = ip < 2;
            for (int qq = 0; qq < o->ncolor; ++qq) {
                const int q = pass == 0 ? qq : o->ncolor - 1 - qq;
#pragma omp parallel for schedule(static)
                for (int64_t ic = o->col_ptr[q]; ic < o->col_ptr[q + 1]; ++ic) {
                    const int64_t c = o->col_cells[ic];
                    double V = o->vol[c];
                    for (int64_t k = 0; k < nv; ++k) {
                        double acc[4] = {0, 0, 0, 0};
                        for (int64_t s = o->cptr[c]; s < o->cptr[c + 1]; ++s) {
                            int64_t f = o->cface[s];
                            int64_t j = other_cell(o, s);
                            if (j < 0) continue;
                            if (first && (pass == 0 ? !(o->color[j] < q) : !(o->color[j] > q))) continue;
                            double xn = 0;
                            for (int a = 0; a < D; ++a) xn += o->xi[k * D + a] * o->csign[s] * o->fn[f * D + a];
                            if (xn >= 0) continue;
                            for (int sl = 0; sl < ND; ++sl) acc[sl] += xn * o->fa[f] * fout[(j * ND + sl) * nv + k];
                        }
                        for (int sl = 0; sl < ND; ++sl) {
                            const double dg = dco[c * nv + k] + (sl == DV ? d[c].radd : 0.0);
                            double *x = &fout[(c * ND + sl) * nv + k];
                            if (pass == 0 || !first)
                                *x = (rr[(c * ND + sl) * nv + k] - acc[sl] / V) / dg;
                            else
                                *x -= acc[sl] / (V * dg);
                        }
                    }
                    for (int64_t qo = 0; qo < no; ++qo) {
                        double acc = 0;
                        for (int64_t s = o->cptr[c]; s < o->cptr[c + 1]; ++s) {
                            int64_t f = o->cface[s];
                            int64_t j = other_cell(o, s);
                            if (j < 0) continue;
                            if (first && (pass == 0 ? !(o->color[j] < q) : !(o->color[j] > q))) continue;
                            double on = 0;
                            for (int a = 0; a < D; ++a) on += o->om[qo * 3 + a] * o->csign[s] * o->fn[f * D + a];
                            if (on >= 0) continue;
                            acc += on * o->fa[f] * Iout[j * no + qo];
                        }
                        double *x = &Iout[c * no + qo];
                        if (pass == 0 || !first)
                            *x = (rI[c * no + qo] - acc / V) / dcoR[c * no + qo];
                        else
                            *x -= acc / (V * dcoR[c * no + qo]);
                    }
                }
            }
        }
    }
    double *tmp = (double *)malloc((size_t)nc * ND * nv * sizeof(double));
    double *tmpI = (double *)malloc((size_t)nc * no * sizeof(double));
    for (int sw = 0; sw < (o->sweep == 1 ? 0 : o->kin_sweeps); ++sw) {
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nc; ++c) {
            double V = o->vol[c];
            for (int64_t k = 0; k < nv; ++k) {
                double acc[4] = {0, 0, 0, 0};
                for (int64_t s = o->cptr[c]; s < o->cptr[c + 1]; ++s) {
                    int64_t f = o->cface[s];
                    int64_t j = other_cell(o, s);
                    if (j < 0) continue;
                    double xn = 0;
                    for (int a = 0; a < D; ++a) xn += o->xi[k * D + a] * o->csign[s] * o->fn[f * D + a];
                    if (xn >= 0) continue;
                    for (int sl = 0; sl < ND; ++sl) acc[sl] += xn * o->fa[f] * fout[(j * ND + sl) * nv + k];
                }
                for (int sl = 0; sl < ND; ++sl)
                    tmp[(c * ND + sl) * nv + k] = (rr[(c * ND + sl) * nv + k] - acc[sl] / V) /
                                                  (dco[c * nv + k] + (sl == DV ? d[c].radd : 0.0));
            }
            for (int64_t q = 0; q < no; ++q) {
                double acc = 0;
                for (int64_t s = o->cptr[c]; s < o->cptr[c + 1]; ++s) {
                    int64_t f = o->cface[s];
                    int64_t j = other_cell(o, s);
                    if (j < 0) continue;
                    double on = 0;
                    for (int a = 0; a < D; ++a) on += o->om[q * 3 + a] * o->csign[s] * o->fn[f * D + a];
                    if (on >= 0) continue;
                    acc += on * o->fa[f] * Iout[j * no + q];
                }
                tmpI[c * no + q] = (rI[c * no + q] - acc / V) / dcoR[c * no + q];
            }
        }
        memcpy(fout, tmp, (size_t)nc * ND * nv * sizeof(double));
        memcpy(Iout, tmpI, (size_t)nc * no * sizeof(double));
    }
    for (size_t i = 0; i < (size_t)nc * ND * nv; ++i) fout[i] = o->f[i] + o->kin_omega * fout[i];
    for (size_t i = 0; i < (size_t)nc * no; ++i) Iout[i] = o->I[i] + o->kin_omega * Iout[i];
    free(tmp);
    free(tmpI);
    free(dco);
    free(dcoR);
    free(rr);
    free(rI);
    free(gl);
    free(glI);
    free(m);
    free(d);
}

/* limited gradients of the current state at the cells next to boundary faces, then wall densities and
 * boundary records of the current state */
static void boundary_of_state(orc_t *o)
{
    int ND = o->ND;
    int64_t nc = o->nc, nv = o->nv, no = o->no;
    double *gl = (double *)calloc((size_t)nc * ND * nv * 3, sizeof(double));
    double *glI = (double *)calloc((size_t)nc * no * 3, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < o->nf; ++f) {
        if (o->fc[2 * f + 1] >= 0) continue;
        int64_t c = o->fc[2 * f];
        for (int sl = 0; sl < ND; ++sl)
            for (int64_t k = 0; k < nv; ++k)
                limited_grad(o, o->f, ND * nv, sl * nv + k, c, gl + ((c * ND + sl) * nv + k) * 3);
        for (int64_t q = 0; q < no; ++q) limited_grad(o, o->I, no, q, c, glI + (c * no + q) * 3);
    }
    wall_densities(o, gl);
    record_boundary(o, gl, glI);
    free(gl);
    free(glI);
}

/* ---------------------------------------------------------------- HoTs (Eqs. getHoTs / split_constitutive) */
#define NHOT 21 /* HoT_sigma (3x3 row-major), HoT_qt, HoT_qr, HoT_qv, HoT_qR (3 each) */

/* NSF stress and heat fluxes (Eqs. NSF_constitutive, NSF_thermal_conductivities) for viscosity mu and the
 * gradients g[field][axis] of (u_a (D), T_t, T_r, T_v, e_R), plus the given HoTs (hot = NULL: NSF only) */
static void constitutive(const orc_t *o, double mu, double g[8][3], const double *hot, double sig[3][3],
                         double q[4][3])
{
    int D = o->D;
    double kR = (o->keff > 0) ? 1.0 / (3 * o->keff) : 0.0;
    double div = 0;
    for (int a = 0; a < D; ++a) div += g[a][a];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) sig[a][b] = 0;
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
            /* g[b][a] = d u_b / d x_a */
            sig[a][b] = -mu * (g[b][a] + g[a][b] - (a == b ? 2.0 / 3.0 * div : 0.0));
            if (hot) sig[a][b] += hot[a * 3 + b];
        }
    for (int l = 0; l < 4; ++l)
        for (int a = 0; a < 3; ++a) q[l][a] = 0;
    for (int a = 0; a < D; ++a) {
        for (int l = 0; l < 3; ++l) {
            for (int m = 0; m < 3; ++m) q[l][a] -= 0.5 * mu * o->K0[l][m] * g[D + m][a];
            if (hot) q[l][a] += hot[9 + 3 * l + a];
        }
        q[3][a] = -kR * g[D + 3][a] + (hot ? hot[18 + a] : 0.0);
    }
}

static void kin_flux_moments(const mom_t *m, double *k)
{
    for (int i = 0; i < NHOT; ++i) k[i] = 0;
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) k[a * 3 + b] = m->sig[a][b];
        k[9 + a] = m->qt[a];
        k[12 + a] = m->qr[a];
        k[15 + a] = m->qv[a];
        k[18 + a] = m->qR[a];
    }
}

/* fields entering the constitutive relations, per cell: u_a (D), T_t, T_r, T_v, e_R */
static void grad_fields_of(const orc_t *o, const mom_t *m, double *fld)
{
    int D = o->D, nfld = D + 4;
    for (int64_t c = 0; c < o->nc; ++c) {
        for (int a = 0; a < D; ++a) fld[c * nfld + a] = m[c].u[a];
        fld[c * nfld + D] = m[c].Tt;
        fld[c * nfld + D + 1] = m[c].Tr;
        fld[c * nfld + D + 2] = m[c].Tv;
        fld[c * nfld + D + 3] = m[c].eR;
    }
}

/* Cell HoTs with the cell least-squares gradient (diagnostic output and the asymptotic tests). */
static void compute_hot(const orc_t *o, const mom_t *m, double *hot)
{
    int D = o->D, nfld = D + 4;
    int64_t nc = o->nc;
    double *fld = (double *)malloc(nc * nfld * sizeof(double));
    grad_fields_of(o, m, fld);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        double g[8][3], sig[3][3], q[4][3], k[NHOT];
        for (int i = 0; i < nfld; ++i) lsq_grad(o, fld, nfld, i, c, g[i]);
        double mu = sqrt(2.0 / PI) * o->Kn * pow(m[c].Tt, o->omg); /* mu = p_t tau */
        constitutive(o, mu, g, NULL, sig, q);
        kin_flux_moments(&m[c], k);
        double *hc = hot + c * NHOT;
        for (int i = 0; i < NHOT; ++i) hc[i] = 0;
        for (int a = 0; a < D; ++a) {
            for (int b = 0; b < D; ++b) hc[a * 3 + b] = k[a * 3 + b] - sig[a][b];
            for (int l = 0; l < 4; ++l) hc[9 + 3 * l + a] = k[9 + 3 * l + a] - q[l][a];
        }
    }
    free(fld);
}

/* Face gradient of each gradient field on an interior face: mean of the two cell least-squares gradients
 * with its component along the centroid line replaced by the centroid difference quotient. */
static void face_grads(const orc_t *o, const double *fld, const double *gf, int64_t c, int64_t j, double g[8][3])
{
    int D = o->D, nfld = D + 4;
    double dvec[3] = {0, 0, 0}, dl = 0;
    for (int a = 0; a < D; ++a) {
        dvec[a] = gdiff(o, o->ctr[j * D + a], o->ctr[c * D + a], a);
        dl += dvec[a] * dvec[a];
    }
    dl = sqrt(dl);
    for (int a = 0; a < D; ++a) dvec[a] /= dl;
    for (int i = 0; i < nfld; ++i) {
        double avg[3] = {0, 0, 0}, corr = 0;
        for (int a = 0; a < D; ++a) {
            avg[a] = 0.5 * (gf[(c * nfld + i) * 3 + a] + gf[(j * nfld + i) * 3 + a]);
            corr += avg[a] * dvec[a];
        }
        double jump = (fld[j * nfld + i] - fld[c * nfld + i]) / dl;
        for (int a = 0; a < 3; ++a) g[i][a] = (a < D) ? avg[a] + (jump - corr) * dvec[a] : 0.0;
    }
}

/* reading: HoTs of the macroscopic solve live on interior faces.  A face HoT is the mean of the two cells'
 * kinetic moments minus the NSF relation evaluated with the same face gradient operator the viscous flux
 * uses (so the two discretisations coincide when the macro state equals the kinetic moments). */
static void face_hot(const orc_t *o, const mom_t *m, double *hotf)
{
    int D = o->D, nfld = D + 4;
    int64_t nc = o->nc;
    double *fld = (double *)malloc(nc * nfld * sizeof(double));
    double *gf = (double *)malloc(nc * nfld * 3 * sizeof(double));
    grad_fields_of(o, m, fld);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c)
        for (int i = 0; i < nfld; ++i) lsq_grad(o, fld, nfld, i, c, gf + (c * nfld + i) * 3);
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < o->nf; ++f) {
        double *h = hotf + f * NHOT;
        for (int i = 0; i < NHOT; ++i) h[i] = 0;
        int64_t c = o->fc[2 * f], j = o->fc[2 * f + 1];
        if (j < 0) continue;
        double g[8][3], sig[3][3], q[4][3], kc[NHOT], kj[NHOT];
        face_grads(o, fld, gf, c, j, g);
        double mu = 0.5 * sqrt(2.0 / PI) * o->Kn * (pow(m[c].Tt, o->omg) + pow(m[j].Tt, o->omg));
        constitutive(o, mu, g, NULL, sig, q);
        kin_flux_moments(&m[c], kc);
        kin_flux_moments(&m[j], kj);
        for (int a = 0; a < D; ++a) {
            for (int b = 0; b < D; ++b) h[a * 3 + b] = 0.5 * (kc[a * 3 + b] + kj[a * 3 + b]) - sig[a][b];
            for (int l = 0; l < 4; ++l) h[9 + 3 * l + a] = 0.5 * (kc[9 + 3 * l + a] + kj[9 + 3 * l + a]) - q[l][a];
        }
    }
    free(fld);
    free(gf);
}

/* ---------------------------------------------------------------- macroscopic synthetic solver */
typedef struct {
    double rho, u[3], Tt, Tr, Tv, eR, mu, cs;
} prim_t;

static void prim_of(const orc_t *o, const double *W, prim_t *p)
{
    int D = o->D;
    p->rho = W[0];
    double ek = 0;
    for (int a = 0; a < 3; ++a) p->u[a] = 0;
    for (int a = 0; a < D; ++a) {
        p->u[a] = W[1 + a] / W[0];
        ek += 0.5 * W[0] * p->u[a] * p->u[a];
    }
    double e = W[D + 1], er = W[D + 2], ev = W[D + 3], eR = W[D + 4];
    p->Tt = 2.0 / (3.0 * W[0]) * (e - ek - er - ev - eR);
    p->Tr = 2.0 * er / (o->dr * W[0]);
    p->Tv = Tv_of(o, ev, W[0]);
    p->eR = eR;
    p->mu = sqrt(2.0 / PI) * o->Kn * pow(p->Tt, o->omg);
    p->cs = sqrt(5.0 / 3.0 * p->Tt);
}

/* Euler part of the flux projected on n (F_c . n of Sec. 6; zero for e_R) */
static void euler_flux(const orc_t *o, const double *W, const double *n, double *F)
{
    int D = o->D;
    prim_t p;
    prim_of(o, W, &p);
    double un = 0;
    for (int a = 0; a < D; ++a) un += p.u[a] * n[a];
    double pt = p.rho * p.Tt;
    F[0] = p.rho * un;
    for (int a = 0; a < D; ++a) F[1 + a] = W[1 + a] * un + pt * n[a];
    double egas = W[D + 1] - W[D + 4];
    F[D + 1] = un * (egas + pt);
    F[D + 2] = un * W[D + 2];
    F[D + 3] = un * W[D + 3];
    F[D + 4] = 0.0;
}

/* reading: Rusanov (local Lax-Friedrichs) numerical flux for the unnamed flux function; e_R carries no
 * convective flux and no numerical dissipation */
static void rusanov(const orc_t *o, const double *WL, const double *WR, const double *n, double *F)
{
    int D = o->D, NW = NWof(D);
    double FL[8], FR[8];
    euler_flux(o, WL, n, FL);
    euler_flux(o, WR, n, FR);
    prim_t pL, pR;
    prim_of(o, WL, &pL);
    prim_of(o, WR, &pR);
    double unL = 0, unR = 0;
    for (int a = 0; a < D; ++a) {
        unL += pL.u[a] * n[a];
        unR += pR.u[a] * n[a];
    }
    double lam = fmax(fabs(unL) + pL.cs, fabs(unR) + pR.cs);
    for (int i = 0; i < NW - 1; ++i) F[i] = 0.5 * (FL[i] + FR[i]) - 0.5 * lam * (WR[i] - WL[i]);
    F[NW - 1] = 0.0;
}

static void W_of_moments(const orc_t *o, const mom_t *m, double *W)
{
    int D = o->D;
    W[0] = m->rho;
    double ek = 0;
    for (int a = 0; a < D; ++a) {
        W[1 + a] = m->rho * m->u[a];
        ek += 0.5 * m->rho * m->u[a] * m->u[a];
    }
    double er = 0.5 * o->dr * m->rho * m->Tr, ev = rho_ev(o, m->rho, m->Tv);
    W[D + 1] = ek + 1.5 * m->rho * m->Tt + er + ev + m->eR;
    W[D + 2] = er;
    W[D + 3] = ev;
    W[D + 4] = m->eR;
}

static void W_of_state(const orc_t *o, double rho, const double *u, double T, double *W)
{
    int D = o->D;
    double ek = 0;
    W[0] = rho;
    for (int a = 0; a < D; ++a) {
        W[1 + a] = rho * u[a];
        ek += 0.5 * rho * u[a] * u[a];
    }
    W[D + 2] = 0.5 * o->dr * rho * T;
    W[D + 3] = rho_ev(o, rho, T);
    W[D + 4] = 4 * o->sigR * T * T * T * T;
    W[D + 1] = ek + 1.5 * rho * T + W[D + 2] + W[D + 3] + W[D + 4];
}

static int phys_ok(const orc_t *o, const double *W)
{
    prim_t p;
    if (!(W[0] > 0)) return 0;
    prim_of(o, W, &p);
    return p.Tt > 0 && W[o->D + 2] >= 0 && W[o->D + 3] >= 0;
}

/* viscous flux . n from a stress, heat fluxes and the face velocity (F_v of Sec. 6) */
static void viscous_flux(const orc_t *o, double sig[3][3], double q[4][3], const double *uf, const double *n,
                         double *F)
{
    int D = o->D;
    double sn[3] = {0, 0, 0}, work = 0, qall = 0, qrn = 0, qvn = 0, qRn = 0;
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) sn[a] += sig[a][b] * n[b];
    for (int a = 0; a < D; ++a) {
        work += sn[a] * uf[a];
        qall += (q[0][a] + q[1][a] + q[2][a] + q[3][a]) * n[a];
        qrn += q[1][a] * n[a];
        qvn += q[2][a] * n[a];
        qRn += q[3][a] * n[a];
    }
    F[0] = 0;
    for (int a = 0; a < D; ++a) F[1 + a] = sn[a];
    F[D + 1] = work + qall;
    F[D + 2] = qrn;
    F[D + 3] = qvn;
    F[D + 4] = qRn;
}

/* Boundary-face model flux of the synthetic equations (reading: the paper states no macroscopic boundary
 * condition).  The boundary flux used by the macro solver is
 *     F_b(W) = F_model(W) + [F_kinetic - F_model(W^{k+1/2})],
 * an NSF-type wall (or Rusanov far-field) flux of the current macro state plus the frozen difference
 * between the kinetic boundary flux of the kinetic step and the model at the start of the solve, which
 * mirrors the HoT construction.  Wall: impermeable, pressure p_t n, shear -mu (u_w - u)/delta, mode heat
 * fluxes from (T_w - T)/delta, radiation -kappa_R (4 sigma_R T_w^4 - e_R)/delta.  Far field: Rusanov flux
 * against the prescribed equilibrium state plus the same radiative term.  gdiag/gdiagR: spectral radii
 * for the implicit diagonal. */
static void bmodel_flux(const orc_t *o, int64_t f, const double *Wc, double *F, double *gdiag, double *gdiagR)
{
    int D = o->D, NW = NWof(D);
    int64_t c = o->fc[2 * f], R = o->fc[2 * f + 1];
    int b = (int)(-R - 1);
    prim_t p;
    prim_of(o, Wc, &p);
    const double *n = o->fn + f * D;
    double delta = 0;
    for (int a = 0; a < D; ++a) delta += n[a] * gdiff(o, o->fctr[f * D + a], o->ctr[c * D + a], a);
    delta = fabs(delta);
    double kR = (o->keff > 0) ? 1.0 / (3 * o->keff) : 0.0;
    double Tb = o->bcT[b];
    double eRb = 4 * o->sigR * Tb * Tb * Tb * Tb;
    double qRn = -kR * (eRb - p.eR) / delta;
    for (int i = 0; i < NW; ++i) F[i] = 0;
    double un = 0;
    for (int a = 0; a < D; ++a) un += p.u[a] * n[a];
    *gdiag = fabs(un) + p.cs + 2 * p.mu / (p.rho * delta);
    *gdiagR = 2 * kR / delta;
    if (o->bck[b] == BC_WALL) {
        const double *uw = o->bcu + b * 3;
        double pt = p.rho * p.Tt, work = 0;
        for (int a = 0; a < D; ++a) {
            double sn = -p.mu * (uw[a] - p.u[a]) / delta;
            F[1 + a] = pt * n[a] + sn;
            work += sn * uw[a];
        }
        double dT[3] = {(Tb - p.Tt) / delta, (Tb - p.Tr) / delta, (Tb - p.Tv) / delta};
        double qn[3];
        for (int l = 0; l < 3; ++l) {
            qn[l] = 0;
            for (int m = 0; m < 3; ++m) qn[l] -= 0.5 * p.mu * o->K0[l][m] * dT[m];
        }
        F[D + 1] = work + qn[0] + qn[1] + qn[2] + qRn;
        F[D + 2] = qn[1];
        F[D + 3] = qn[2];
        F[D + 4] = qRn;
    } else {
        double Wb[8];
        W_of_state(o, o->bcrho[b], o->bcu + b * 3, Tb, Wb);
        rusanov(o, Wc, Wb, n, F);
        F[D + 1] += qRn;
        F[D + 4] = qRn;
    }
}

/* Sources Q of the synthetic equations (Eq. macroscopic_equation): none for mass, momentum and total
 * energy; rotational (e_tr - e_r)/(Z_r tau), vibrational (e_tv - e_v)/(Z_v tau) - k_eff (e_vR - e_R) and
 * radiative k_eff (e_vR - e_R) with e_vR = 4 sigma_R T_v^4 and tau = mu / (rho T_t). */
static void macro_source(const orc_t *o, const prim_t *p, const double *Wc, double *Q)
{
    int D = o->D, NW = NWof(D);
    double rho = p->rho, Tt = p->Tt, Tr = p->Tr, Tv = p->Tv;
    double tau = p->mu / (rho * Tt);
    double Ttr = (3 * Tt + o->dr * Tr) / (3 + o->dr), Ttv = Ttv_of(o, Tt, Tv);
    double etr = 0.5 * o->dr * rho * Ttr, etv = rho_ev(o, rho, Ttv);
    double evR = 4 * o->sigR * Tv * Tv * Tv * Tv;
    double er = Wc[D + 2], ev = Wc[D + 3], eR = Wc[D + 4];
    for (int i = 0; i < NW; ++i) Q[i] = 0;
    Q[D + 2] = (etr - er) / (o->Zr * tau);
    Q[D + 3] = (etv - ev) / (o->Zv * tau) - o->keff * (evR - eR);
    Q[D + 4] = o->keff * (evR - eR);
}

/* residual of the synthetic equations, R_i = -(1/V) sum_faces F S + Q (Eq. delta_macro), for the state W,
 * face HoTs hotf and frozen boundary corrections bcorr; also returns the primitive states */
static void macro_residual(const orc_t *o, const double *hotf, const double *bcorr, const double *dref,
                           const double *W, prim_t *P, double *R)
{
    int D = o->D, NW = NWof(D), nfld = D + 4;
    int64_t nc = o->nc;
    double *fld = (double *)malloc(nc * nfld * sizeof(double));
    double *gl = (double *)malloc(nc * NW * 3 * sizeof(double));
    double *gf = (double *)malloc(nc * nfld * 3 * sizeof(double));
    for (int64_t c = 0; c < nc; ++c) {
        prim_of(o, W + c * NW, &P[c]);
        for (int a = 0; a < D; ++a) fld[c * nfld + a] = P[c].u[a];
        fld[c * nfld + D] = P[c].Tt;
        fld[c * nfld + D + 1] = P[c].Tr;
        fld[c * nfld + D + 2] = P[c].Tv;
        fld[c * nfld + D + 3] = P[c].eR;
    }
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        for (int i = 0; i < NW; ++i) limited_grad_o(o, o->macro_order2, W, NW, i, c, gl + (c * NW + i) * 3);
        for (int i = 0; i < nfld; ++i) lsq_grad(o, fld, nfld, i, c, gf + (c * nfld + i) * 3);
    }
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        double acc[8] = {0};
        for (int64_t s = o->cptr[c]; s < o->cptr[c + 1]; ++s) {
            int64_t f = o->cface[s];
            int64_t j = other_cell(o, s);
            double S = o->fa[f];
            double Ff[8] = {0};
            if (j < 0) {
                double g1, g2;
                bmodel_flux(o, f, W + c * NW, Ff, &g1, &g2);
                for (int i = 0; i < NW; ++i) Ff[i] += bcorr[f * NW + i];
            } else {
                double n[3] = {0, 0, 0};
                for (int a = 0; a < D; ++a) n[a] = o->csign[s] * o->fn[f * D + a];
                double WL[8] = {0}, WR[8] = {0};
                for (int i = 0; i < NW; ++i) {
                    double dl = 0, drr = 0;
                    for (int a = 0; a < D; ++a) {
                        dl += gl[(c * NW + i) * 3 + a] * gdiff(o, o->fctr[f * D + a], o->ctr[c * D + a], a);
                        drr += gl[(j * NW + i) * 3 + a] * gdiff(o, o->fctr[f * D + a], o->ctr[j * D + a], a);
                    }
                    WL[i] = W[c * NW + i] + dl;
                    WR[i] = W[j * NW + i] + drr;
                }
                if (!phys_ok(o, WL))
                    for (int i = 0; i < NW; ++i) WL[i] = W[c * NW + i];
                if (!phys_ok(o, WR))
                    for (int i = 0; i < NW; ++i) WR[i] = W[j * NW + i];
                rusanov(o, WL, WR, n, Ff);
                if (dref)
                    for (int i = 0; i < NW; ++i) Ff[i] += o->csign[s] * dref[f * NW + i];
                double g[8][3], sig[3][3], q[4][3], Fv[8], uf[3] = {0, 0, 0};
                face_grads(o, fld, gf, c, j, g);
                for (int a = 0; a < D; ++a) uf[a] = 0.5 * (P[c].u[a] + P[j].u[a]);
                constitutive(o, 0.5 * (P[c].mu + P[j].mu), g, hotf + f * NHOT, sig, q);
                viscous_flux(o, sig, q, uf, n, Fv);
                for (int i = 0; i < NW; ++i) Ff[i] += Fv[i];
            }
            for (int i = 0; i < NW; ++i) acc[i] += Ff[i] * S;
        }
        double Q[8];
        macro_source(o, &P[c], W + c * NW, Q);
        for (int i = 0; i < NW; ++i) R[c * NW + i] = -acc[i] / o->vol[c] + Q[i];
    }
    free(fld);
    free(gl);
    free(gf);
}

/* Numerical dissipation of the reference state on each interior face, 0.5 lam* (W*_R - W*_L) along fn.
 * reading: the Rusanov dissipation of the synthetic equations acts on the deviation from the state the solve
 * starts from (the kinetic moments), so that it vanishes when the two descriptions agree. */
static void dissipation_ref(const orc_t *o, const double *W0, double *dref)
{
    int D = o->D, NW = NWof(D);
    int64_t nc = o->nc;
    double *gl = (double *)malloc(nc * NW * 3 * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c)
        for (int i = 0; i < NW; ++i) limited_grad_o(o, o->macro_order2, W0, NW, i, c, gl + (c * NW + i) * 3);
    for (int64_t f = 0; f < o->nf; ++f) {
        int64_t c = o->fc[2 * f], j = o->fc[2 * f + 1];
        for (int i = 0; i < NW; ++i) dref[f * NW + i] = 0;
        if (j < 0) continue;
        const double *n = o->fn + f * D;
        double WL[8] = {0}, WR[8] = {0};
        for (int i = 0; i < NW; ++i) {
            double dl = 0, drr = 0;
            for (int a = 0; a < D; ++a) {
                dl += gl[(c * NW + i) * 3 + a] * gdiff(o, o->fctr[f * D + a], o->ctr[c * D + a], a);
                drr += gl[(j * NW + i) * 3 + a] * gdiff(o, o->fctr[f * D + a], o->ctr[j * D + a], a);
            }
            WL[i] = W0[c * NW + i] + dl;
            WR[i] = W0[j * NW + i] + drr;
        }
        if (!phys_ok(o, WL))
            for (int i = 0; i < NW; ++i) WL[i] = W0[c * NW + i];
        if (!phys_ok(o, WR))
            for (int i = 0; i < NW; ++i) WR[i] = W0[j * NW + i];
        prim_t pL, pR;
        prim_of(o, WL, &pL);
        prim_of(o, WR, &pR);
        double unL = 0, unR = 0;
        for (int a = 0; a < D; ++a) {
            unL += pL.u[a] * n[a];
            unR += pR.u[a] * n[a];
        }
        double lam = fmax(fabs(unL) + pL.cs, fabs(unR) + pR.cs);
        for (int i = 0; i < NW - 1; ++i) dref[f * NW + i] = 0.5 * lam * (WR[i] - WL[i]);
    }
    free(gl);
}

/* frozen boundary corrections F_kinetic - F_model(W0) */
static void boundary_corr(const orc_t *o, const double *W0, double *bcorr)
{
    int NW = NWof(o->D);
    for (int64_t f = 0; f < o->nf; ++f) {
        for (int i = 0; i < NW; ++i) bcorr[f * NW + i] = 0;
        if (o->fc[2 * f + 1] >= 0) continue;
        double Fm[8], g1, g2;
        bmodel_flux(o, f, W0 + o->fc[2 * f] * NW, Fm, &g1, &g2);
        for (int i = 0; i < NW; ++i) bcorr[f * NW + i] = o->bflux[f * NW + i] - Fm[i];
    }
}

/* Point solve of the implicit operator in the unknowns U = (rho, rho u, e_gas, e_r, e_v, e_R): diagonal
 * except for the gas-photon exchange k_eff (e_vR(T_v) - e_R), which couples e_gas, e_v and e_R and is
 * solved exactly per cell (reading: the printed diagonal Jacobian leaves this coupling lagged, which lets
 * e_gas and e_v respond inconsistently to strong emission).  With e' = d e_vR / d e_v:
 *   D_g dg = r_g - k e' dv + k dR,   D_v dv = r_v + k dR,   D_R dR = r_R + k e' dv.
 * Reading: with k_eff = 0 (absorption and emission off) the e_R row has neither a diffusion term nor a
 * source and is singular; e_R is then not a synthetic unknown (dR = 0), keeps its kinetic value, and the
 * synchronisation leaves I unchanged. */
static void local_solve(const orc_t *o, const prim_t *p, const double *rhs, const double *Dg, double *dU)
{
    int D = o->D, NW = NWof(D);
    for (int i = 0; i < NW; ++i) dU[i] = rhs[i] / Dg[i];
    const int ig = D + 1, iv = D + 3, iR = D + 4;
    const double k = o->keff;
    const double ep = o->Tvref > 0 ? 16.0 * o->sigR * p->Tv * p->Tv * p->Tv / (cv_of(o, p->Tv) * p->rho)
                                   : 32.0 * o->sigR * p->Tv * p->Tv * p->Tv / (o->dv * p->rho);
    const double dv = (rhs[iv] + k * rhs[iR] / Dg[iR]) / (Dg[iv] - k * k * ep / Dg[iR]);
    const double dR = (rhs[iR] + k * ep * dv) / Dg[iR];
    dU[iv] = dv;
    dU[iR] = (k > 0) ? dR : 0.0;
    dU[ig] = (rhs[ig] - k * ep * dv + k * dR) / Dg[ig];
}

/* W += alpha dU (the increment of e is dU_egas + dU_eR), alpha = 2^-m the largest factor (m <= 20) keeping
 * rho, T_t, e_r, e_v and e_R at least half their current values and within a factor two of their values Ws
 * at the start of the solve (the kinetic moments); no update when no such factor exists.
 * reading: a positivity and trust-region safeguard of the pseudo-time update.  The paper states none; it
 * never acts once the outer iteration is near its fixed point (the macro state then stays close to the
 * kinetic moments), but it keeps hypersonic start-ups (Ma 5 cylinder) from driving the synthetic solve to
 * vanishing temperatures in the expansion or to overflow. */
static int positive_update(const orc_t *o, double *W, const double *dU, const double *Ws)
{
    int D = o->D, NW = NWof(D);
    prim_t p0, ps;
    prim_of(o, W, &p0);
    prim_of(o, Ws, &ps);
    double a = 1.0;
    for (int m = 0; m <= 20; ++m, a *= 0.5) {
        double Wn[8];
        for (int i = 0; i < NW; ++i) Wn[i] = W[i] + a * dU[i];
        Wn[D + 1] += a * dU[D + 4];
        prim_t p1;
        prim_of(o, Wn, &p1);
        const double lo = 0.5, hi = 2.0;
        if (Wn[0] >= 0.5 * W[0] && p1.Tt >= 0.5 * p0.Tt && Wn[D + 2] >= 0.5 * W[D + 2] &&
            Wn[D + 3] >= 0.5 * W[D + 3] && Wn[D + 4] >= 0.5 * W[D + 4] && Wn[0] >= lo * Ws[0] &&
            p1.Tt >= lo * ps.Tt && Wn[D + 2] >= lo * Ws[D + 2] && Wn[D + 3] >= lo * Ws[D + 3] &&
            Wn[D + 4] >= lo * Ws[D + 4] && Wn[0] <= hi * Ws[0] && p1.Tt <= hi * ps.Tt &&
            Wn[D + 2] <= hi * Ws[D + 2] && Wn[D + 3] <= hi * Ws[D + 3] && Wn[D + 4] <= hi * Ws[D + 4]) {
            for (int i = 0; i < NW; ++i) W[i] = Wn[i];
            return m > 0;
        }
    }
    return 1;
}

/* 1 when every boundary face is a wall */
static int domain_closed(const orc_t *o)
{
    for (int64_t f = 0; f < o->nf; ++f) {
        int64_t R = o->fc[2 * f + 1];
        if (R < 0 && o->bck[-R - 1] != BC_WALL) return 0;
    }
    return 1;
}

/* reading: in a domain closed by walls the total mass is not fixed by the steady equations (kinetic or
 * synthetic), and neither the point-implicit macro update nor the point relaxation of the kinetic step
 * conserves it, so an unconstrained iteration would pick the mass of its converged state along the way.
 * The macro states W are rescaled to a target mass with u and the temperatures unchanged (every
 * component except e_R scales with the density; e contains e_R). */
static void rescale_mass(const orc_t *o, double *W, double mass_target)
{
    int D = o->D, NW = NWof(D);
    double m1 = 0;
    for (int64_t c = 0; c < o->nc; ++c) m1 += o->vol[c] * W[c * NW];
    double sc = mass_target / m1;
    for (int64_t c = 0; c < o->nc; ++c) {
        for (int i = 0; i < NW - 1; ++i) W[c * NW + i] *= sc;
        W[c * NW + D + 1] -= (sc - 1.0) * W[c * NW + D + 4];
    }
}

/* Solve the synthetic equations (Eq. macroscopic_equation; FV and implicit incremental forms of Sec. 6)
 * with the HoTs fixed, starting from W (in/out [nc*NW]) = W(M^{k+1/2}); m = M^{k+1/2}. */
static int macro_solve(orc_t *o, const mom_t *m, double mass_target, double *W)
{
    int D = o->D, NW = NWof(D);
    int64_t nc = o->nc;
    double *R = (double *)malloc(nc * NW * sizeof(double));
    double *Dg = (double *)malloc(nc * NW * sizeof(double));
    double *dW = (double *)malloc(nc * NW * sizeof(double));
    double *dW2 = (double *)malloc(nc * NW * sizeof(double));
    double *hotf = (double *)malloc((size_t)o->nf * NHOT * sizeof(double));
    double *bcorr = (double *)malloc((size_t)o->nf * NW * sizeof(double));
    prim_t *P = (prim_t *)malloc(nc * sizeof(prim_t));
    double *dref = o->diss_ref ? (double *)malloc((size_t)o->nf * NW * sizeof(double)) : NULL;
    double *W0 = (double *)malloc(nc * NW * sizeof(double));
    memcpy(W0, W, nc * NW * sizeof(double));
    face_hot(o, m, hotf);
    boundary_corr(o, W, bcorr);
    if (dref) dissipation_ref(o, W, dref);
    o->safeguard_hits = 0;
    double kR = (o->keff > 0) ? 1.0 / (3 * o->keff) : 0.0;
    double res0 = 0;
    int it;
    for (it = 0; it < o->max_inner; ++it) {
        macro_residual(o, hotf, bcorr, dref, W, P, R);
        double res = 0;
        for (int64_t c = 0; c < nc; ++c)
            for (int i = 0; i < NW; ++i) res += o->vol[c] * R[c * NW + i] * R[c * NW + i];
        res = sqrt(res);
        if (it == 0) res0 = res;
        if (res <= o->inner_tol * res0) break;
        /* diagonal D_i (Sec. 6 as printed: full sum of Gamma S / V) with the diagonal source Jacobian
         * (Appendix A); boundary faces add the model's spectral radius */
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nc; ++c) {
            double un = 0;
            for (int a = 0; a < D; ++a) un += P[c].u[a] * P[c].u[a];
            double dt = o->cfl_macro * o->h[c] / (sqrt(un) + P[c].cs);
            double gs = 0, gsR = 0;
            for (int64_t s = o->cptr[c]; s < o->cptr[c + 1]; ++s) {
                int64_t f = o->cface[s];
                int64_t j = other_cell(o, s);
                if (j < 0) {
                    double Fm[8], g1, g2;
                    bmodel_flux(o, f, W + c * NW, Fm, &g1, &g2);
                    gs += g1 * o->fa[f];
                    gsR += g2 * o->fa[f];
                    continue;
                }
                double n[3] = {0, 0, 0}, ufn = 0, nd = 0;
                for (int a = 0; a < D; ++a) {
                    n[a] = o->csign[s] * o->fn[f * D + a];
                    ufn += 0.5 * (P[c].u[a] + P[j].u[a]) * n[a];
                    nd += n[a] * gdiff(o, o->ctr[j * D + a], o->ctr[c * D + a], a);
                }
                nd = fabs(nd);
                double G = fabs(ufn) + 0.5 * (P[c].cs + P[j].cs) +
                           2 * 0.5 * (P[c].mu + P[j].mu) / (0.5 * (P[c].rho + P[j].rho) * nd);
                gs += G * o->fa[f];
                gsR += 2 * kR / nd * o->fa[f];
            }
            double rho = P[c].rho, Tt = P[c].Tt, Tr = P[c].Tr, Tv = P[c].Tv;
            double tau = P[c].mu / (rho * Tt);
            double Ttr = (3 * Tt + o->dr * Tr) / (3 + o->dr), Ttv = Ttv_of(o, Tt, Tv);
            double jr = -3.0 / ((3 + o->dr) * o->Zr * tau) + 2 * (o->omg - 1) * (Ttr - Tr) / (3 * o->Zr * tau * Tt);
            /* reading: the printed dQ6/de_v omits the emission term; its exact diagonal part is added */
            double jv = -3.0 / ((3 + o->dv) * o->Zv * tau) + 2 * (o->omg - 1) * (Ttv - Tv) / (3 * o->Zv * tau * Tt) -
                        o->keff * 16 * o->sigR * Tv * Tv * Tv * 2.0 / (o->dv * rho);
            /* variable d_v: the same diagonal with d_v replaced by the heat capacity 2 c_v (at T_tv in the
             * relaxation term, at T_v in the emission term) */
            if (o->Tvref > 0)
                jv = -3.0 / ((3 + 2 * cv_of(o, Ttv)) * o->Zv * tau) + 2 * (o->omg - 1) * (Ttv - Tv) / (3 * o->Zv * tau * Tt) -
                     o->keff * 16 * o->sigR * Tv * Tv * Tv / (cv_of(o, Tv) * rho);
            double jR = -o->keff;
            for (int i = 0; i < NW; ++i) Dg[c * NW + i] = 1.0 / dt + gs / o->vol[c];
            Dg[c * NW + D + 2] -= jr;
            Dg[c * NW + D + 3] -= jv;
            Dg[c * NW + D + 4] = 1.0 / dt + gsR / o->vol[c] - jR;
        }
        /* reading: the diagonal operator acts on the gas part of the total energy, e_gas = e - e_R, whose
         * residual is R_e - R_eR, and on e_R separately; the increment of e is their sum. */
        for (int64_t c = 0; c < nc; ++c) {
            R[c * NW + D + 1] -= R[c * NW + D + 4];
            local_solve(o, &P[c], R + c * NW, Dg + c * NW, dW + c * NW);
        }
        for (int sw = 0; sw < o->n_sweeps; ++sw) {
#pragma omp parallel for schedule(static)
            for (int64_t c = 0; c < nc; ++c) {
                double acc[8] = {0};
                for (int64_t s = o->cptr[c]; s < o->cptr[c + 1]; ++s) {
                    int64_t f = o->cface[s];
                    int64_t j = other_cell(o, s);
                    if (j < 0) continue;
                    double n[3] = {0, 0, 0}, ufn = 0, nd = 0;
                    for (int a = 0; a < D; ++a) {
                        n[a] = o->csign[s] * o->fn[f * D + a];
                        ufn += 0.5 * (P[c].u[a] + P[j].u[a]) * n[a];
                        nd += n[a] * gdiff(o, o->ctr[j * D + a], o->ctr[c * D + a], a);
                    }
                    nd = fabs(nd);
                    double G = fabs(ufn) + 0.5 * (P[c].cs + P[j].cs) +
                               2 * 0.5 * (P[c].mu + P[j].mu) / (0.5 * (P[c].rho + P[j].rho) * nd);
                    double GR = 2 * kR / nd;
                    double Wn[8], F1[8], F0[8];
                    for (int i = 0; i < NW; ++i) Wn[i] = W[j * NW + i] + dW[j * NW + i];
                    Wn[D + 1] += dW[j * NW + D + 4];
                    euler_flux(o, Wn, n, F1);
                    euler_flux(o, W + j * NW, n, F0);
                    for (int i = 0; i < NW - 1; ++i) acc[i] += (F1[i] - F0[i] - G * dW[j * NW + i]) * o->fa[f];
                    acc[NW - 1] += (-GR * dW[j * NW + NW - 1]) * o->fa[f];
                }
                double rhs[8];
                for (int i = 0; i < NW; ++i) rhs[i] = R[c * NW + i] - acc[i] / (2 * o->vol[c]);
                local_solve(o, &P[c], rhs, Dg + c * NW, dW2 + c * NW);
            }
            double *t = dW;
            dW = dW2;
            dW2 = t;
        }
        for (int64_t c = 0; c < nc; ++c) o->safeguard_hits += positive_update(o, W + c * NW, dW + c * NW, W0 + c * NW);
    }
    /* reading: in a domain closed by walls the solution is rescaled to the mass the outer iteration
     * started from (see rescale_mass) */
    if (domain_closed(o)) rescale_mass(o, W, mass_target);
    o->last_inner = it;
    free(W0);
    free(R);
    free(Dg);
    free(dW);
    free(dW2);
    free(hotf);
    free(bcorr);
    free(dref);
    free(P);
    return it;
}

/* multi-temperature equilibrium f^eq(M) (reading of the synchronisation step, Sec. 3) */
static void feq(const orc_t *o, double rho, const double *u, double Tt, double Tr, double Tv, const double *xi, double *Y)
{
    int D = o->D;
    double c2 = 0;
    for (int a = 0; a < D; ++a) c2 += (xi[a] - u[a]) * (xi[a] - u[a]);
    double G = rho * maxw(D, Tt, c2);
    Y[DG] = G;
    Y[DR] = 0.5 * o->dr * Tr * G;
    Y[DV] = o->Tvref > 0 ? ev_of(o, Tv) * G : 0.5 * o->dv * Tv * G;
    Y[DH] = (3 - D) * Tt * G;
}

static void sync_dist(orc_t *o, const mom_t *mh, const double *Wn)
{
    int D = o->D, ND = o->ND, NW = NWof(D);
    int64_t nv = o->nv, no = o->no;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < o->nc; ++c) {
        prim_t p;
        prim_of(o, Wn + c * NW, &p);
        for (int64_t k = 0; k < nv; ++k) {
            double Y1[4], Y0[4];
            feq(o, p.rho, p.u, p.Tt, p.Tr, p.Tv, o->xi + k * D, Y1);
            feq(o, mh[c].rho, mh[c].u, mh[c].Tt, mh[c].Tr, mh[c].Tv, o->xi + k * D, Y0);
            for (int s = 0; s < ND; ++s) o->f[(c * ND + s) * nv + k] += Y1[s] - Y0[s];
        }
        double dI = (p.eR - mh[c].eR) / (4 * PI);
        for (int64_t q = 0; q < no; ++q) o->I[c * no + q] += dI;
    }
}

/* convergence criterion (Sec. 7): max over (rho, u, T) of the volume-weighted relative L2 change.
 * reading: u uses all components in one norm with a denominator floor of ||1||_V (u may vanish). */
static double residual(const orc_t *o, const mom_t *mn, const mom_t *mo)
{
    int D = o->D;
    double num[3] = {0, 0, 0}, den[3] = {0, 0, 0}, vs = 0;
    for (int64_t c = 0; c < o->nc; ++c) {
        double V = o->vol[c];
        vs += V;
        num[0] += V * (mn[c].rho - mo[c].rho) * (mn[c].rho - mo[c].rho);
        den[0] += V * mo[c].rho * mo[c].rho;
        for (int a = 0; a < D; ++a) {
            num[1] += V * (mn[c].u[a] - mo[c].u[a]) * (mn[c].u[a] - mo[c].u[a]);
            den[1] += V * mo[c].u[a] * mo[c].u[a];
        }
        double Tn = Ttot_of(o, mn[c].Tt, mn[c].Tr, mn[c].Tv);
        double To = Ttot_of(o, mo[c].Tt, mo[c].Tr, mo[c].Tv);
        num[2] += V * (Tn - To) * (Tn - To);
        den[2] += V * To * To;
    }
    if (den[1] < vs) den[1] = vs;
    double e = 0;
    for (int i = 0; i < 3; ++i) {
        double r = sqrt(num[i]) / sqrt(den[i]);
        if (r != r) return r;
        if (r > e) e = r;
    }
    return e;
}

/* ================================================================ public API (ctypes) */
orc_t *orc_create(int D, int64_t nc, int64_t nf, const double *vol, const double *ctr, const int64_t *fc,
                  const double *fn, const double *fa, const double *fctr, int nbc, const int *bck,
                  const double *bcrho, const double *bcT, const double *bcu, int64_t nv, const double *xi,
                  const double *w, int64_t no, const double *om, const double *wo, const double *gas,
                  const double *flow, const double *opts)
{
    orc_t *o = (orc_t *)calloc(1, sizeof(orc_t));
    o->D = D;
    o->ND = (D == 3) ? 3 : 4;
    o->nc = nc;
    o->nf = nf;
#define CP(dst, src, n, T)                          \
    do {                                            \
        dst = (T *)malloc((size_t)(n) * sizeof(T)); \
        memcpy(dst, src, (size_t)(n) * sizeof(T));  \
    } while (0)
    CP(o->vol, vol, nc, double);
    CP(o->ctr, ctr, nc * D, double);
    CP(o->fc, fc, 2 * nf, int64_t);
    CP(o->fn, fn, nf * D, double);
    CP(o->fa, fa, nf, double);
    CP(o->fctr, fctr, nf * D, double);
    o->nbc = nbc;
    CP(o->bck, bck, nbc, int);
    CP(o->bcrho, bcrho, nbc, double);
    CP(o->bcT, bcT, nbc, double);
    CP(o->bcu, bcu, nbc * 3, double);
    o->nv = nv;
    o->no = no;
    CP(o->xi, xi, nv * D, double);
    CP(o->w, w, nv, double);
    CP(o->om, om, no * 3, double);
    CP(o->wo, wo, no, double);
#undef CP
    o->dr = gas[0];
    o->dv = gas[1];
    o->Zr = gas[2];
    o->Zv = gas[3];
    o->omg = gas[4];
    o->Sc = gas[5];
    o->sigR = gas[6];
    o->Tvref = gas[7];
    o->Kn = flow[0];
    o->keff = flow[1];
    o->cfl_meso = opts[0];
    o->cfl_macro = opts[1];
    o->limK = opts[2];
    o->inner_tol = opts[3];
    o->max_inner = (int)opts[4];
    o->n_sweeps = (int)opts[5];
    o->second_order = (int)opts[6];
    o->cfl_v = opts[7];
    o->kin_sweeps = (int)opts[8];
    o->kin_omega = opts[9];
    o->diss_ref = (int)opts[10];
    o->macro_order2 = (int)opts[11];
    o->sweep = (int)opts[12];
    o->period = opts[13];
    o->rad_implicit = (int)opts[14];
    o->conservative = (int)opts[15];
    model_constants(o);
    build_mesh(o);
    o->f = (double *)calloc((size_t)nc * o->ND * nv, sizeof(double));
    o->I = (double *)calloc((size_t)nc * no, sizeof(double));
    o->bflux = (double *)calloc((size_t)nf * NWof(D), sizeof(double));
    o->bsurf = (double *)calloc((size_t)nf * 3, sizeof(double));
    o->rhow = (double *)calloc((size_t)nf, sizeof(double));
    return o;
}

void orc_destroy(orc_t *o)
{
    if (!o) return;
    void *ptrs[] = {o->vol, o->ctr, o->fc, o->fn, o->fa, o->fctr, o->bck, o->bcrho, o->bcT, o->bcu, o->xi, o->w,
                    o->om, o->wo, o->cptr, o->cface, o->csign, o->color, o->col_ptr, o->col_cells, o->lsq, o->h, o->f, o->I, o->bflux, o->bsurf, o->rhow};
    for (size_t i = 0; i < sizeof(ptrs) / sizeof(ptrs[0]); ++i) free(ptrs[i]);
    free(o);
}

void orc_set_state(orc_t *o, const double *f, const double *I)
{
    memcpy(o->f, f, (size_t)o->nc * o->ND * o->nv * sizeof(double));
    memcpy(o->I, I, (size_t)o->nc * o->no * sizeof(double));
}

void orc_get_state(const orc_t *o, double *f, double *I)
{
    memcpy(f, o->f, (size_t)o->nc * o->ND * o->nv * sizeof(double));
    memcpy(I, o->I, (size_t)o->nc * o->no * sizeof(double));
}

/* equilibrium initial state with T_t = T_r = T_v = T_R = T per cell */
void orc_init_equilibrium(orc_t *o, const double *rho, const double *u, const double *T)
{
    int D = o->D;
    for (int64_t c = 0; c < o->nc; ++c) {
        double uu[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) uu[a] = u[c * D + a];
        for (int64_t k = 0; k < o->nv; ++k) {
            double Y[4];
            feq(o, rho[c], uu, T[c], T[c], T[c], o->xi + k * D, Y);
            for (int s = 0; s < o->ND; ++s) o->f[(c * o->ND + s) * o->nv + k] = Y[s];
        }
        for (int64_t q = 0; q < o->no; ++q) o->I[c * o->no + q] = o->sigR * pow(T[c], 4) / PI;
    }
}

int orc_nfields(int D) { return 1 + D + 5 + 4 * D + D * (D + 1) / 2; }

static void fields_of(const orc_t *o, const mom_t *m, double *out)
{
    int D = o->D;
    int p = 0;
    der_t d;
    out[p++] = m->rho;
    for (int a = 0; a < D; ++a) out[p++] = m->u[a];
    out[p++] = m->Tt;
    out[p++] = m->Tr;
    out[p++] = m->Tv;
    out[p++] = (o->sigR > 0) ? pow(m->eR / (4 * o->sigR), 0.25) : 0.0;
    d.T = Ttot_of(o, m->Tt, m->Tr, m->Tv);
    out[p++] = d.T;
    for (int a = 0; a < D; ++a) out[p++] = m->qt[a];
    for (int a = 0; a < D; ++a) out[p++] = m->qr[a];
    for (int a = 0; a < D; ++a) out[p++] = m->qv[a];
    for (int a = 0; a < D; ++a) out[p++] = m->qR[a];
    for (int a = 0; a < D; ++a)
        for (int b = a; b < D; ++b) out[p++] = m->sig[a][b];
}

/* macroscopic fields of the current state, [nc * nfields] */
void orc_fields(const orc_t *o, double *out)
{
    int nfl = orc_nfields(o->D);
    mom_t *m = (mom_t *)malloc(o->nc * sizeof(mom_t));
    all_moments(o, o->f, o->I, m);
    for (int64_t c = 0; c < o->nc; ++c) fields_of(o, &m[c], out + c * nfl);
    free(m);
}

/* relaxation source J for the current state, [nc*ND*nv] (tests of the collision operator) */
void orc_collision(const orc_t *o, double *J)
{
    int D = o->D, ND = o->ND;
    int64_t nv = o->nv;
    mom_t *m = (mom_t *)malloc(o->nc * sizeof(mom_t));
    all_moments(o, o->f, o->I, m);
    for (int64_t c = 0; c < o->nc; ++c) {
        der_t d;
        derived(o, &m[c], c, &d);
        for (int64_t k = 0; k < nv; ++k) {
            double fk[4], Jk[4];
            for (int s = 0; s < ND; ++s) fk[s] = o->f[(c * ND + s) * nv + k];
            collision(o, &m[c], &d, fk, o->xi + k * D, Jk);
            for (int s = 0; s < ND; ++s) J[(c * ND + s) * nv + k] = Jk[s];
        }
    }
    free(m);
}

/* radiative source k_eff (B(T_v) - I) for the current state, [nc*no] */
void orc_rad_source(const orc_t *o, double *JR)
{
    mom_t *m = (mom_t *)malloc(o->nc * sizeof(mom_t));
    all_moments(o, o->f, o->I, m);
    for (int64_t c = 0; c < o->nc; ++c) {
        der_t d;
        derived(o, &m[c], c, &d);
        for (int64_t q = 0; q < o->no; ++q) JR[c * o->no + q] = o->keff * (d.B - o->I[c * o->no + q]);
    }
    free(m);
}

/* one kinetic (CIS) step in place; optionally returns the kinetic residual r (before the update) */
void orc_kinetic_step(orc_t *o, double *r_out)
{
    size_t nf = (size_t)o->nc * o->ND * o->nv, ni = (size_t)o->nc * o->no;
    double *fn = (double *)malloc(nf * sizeof(double));
    double *In = (double *)malloc(ni * sizeof(double));
    kinetic_step(o, fn, In, r_out);
    memcpy(o->f, fn, nf * sizeof(double));
    memcpy(o->I, In, ni * sizeof(double));
    free(fn);
    free(In);
}

/* boundary records of the current state: per face NW flux moments and (q_conv, q_rad, p_w) */
void orc_boundary(orc_t *o, double *bflux, double *bsurf)
{
    boundary_of_state(o);
    if (bflux) memcpy(bflux, o->bflux, (size_t)o->nf * NWof(o->D) * sizeof(double));
    if (bsurf) memcpy(bsurf, o->bsurf, (size_t)o->nf * 3 * sizeof(double));
}

/* HoTs of the current state, [nc*21] */
void orc_hot(const orc_t *o, double *hot)
{
    mom_t *m = (mom_t *)malloc(o->nc * sizeof(mom_t));
    all_moments(o, o->f, o->I, m);
    compute_hot(o, m, hot);
    free(m);
}

/* macro solve from the moments of the current state (HoTs and boundary corrections from the current state
 * and the last kinetic step); W out [nc*NW]; returns the inner iteration count */
int orc_macro_solve(orc_t *o, double *W)
{
    mom_t *m = (mom_t *)malloc(o->nc * sizeof(mom_t));
    all_moments(o, o->f, o->I, m);
    int NW = NWof(o->D);
    for (int64_t c = 0; c < o->nc; ++c) W_of_moments(o, &m[c], W + c * NW);
    boundary_of_state(o);
    double mt = 0;
    for (int64_t c = 0; c < o->nc; ++c) mt += o->vol[c] * m[c].rho;
    int it = macro_solve(o, m, mt, W);
    free(m);
    return it;
}

/* residual of the synthetic equations for W, with HoTs and boundary corrections built from the current state */
void orc_macro_residual(orc_t *o, const double *W, double *R)
{
    int NW = NWof(o->D);
    int64_t nc = o->nc;
    mom_t *m = (mom_t *)malloc(nc * sizeof(mom_t));
    all_moments(o, o->f, o->I, m);
    double *W0 = (double *)malloc(nc * NW * sizeof(double));
    for (int64_t c = 0; c < nc; ++c) W_of_moments(o, &m[c], W0 + c * NW);
    double *hotf = (double *)malloc((size_t)o->nf * NHOT * sizeof(double));
    double *bcorr = (double *)malloc((size_t)o->nf * NW * sizeof(double));
    prim_t *P = (prim_t *)malloc(nc * sizeof(prim_t));
    double *dref = o->diss_ref ? (double *)malloc((size_t)o->nf * NW * sizeof(double)) : NULL;
    face_hot(o, m, hotf);
    boundary_of_state(o);
    boundary_corr(o, W0, bcorr);
    if (dref) dissipation_ref(o, W0, dref);
    macro_residual(o, hotf, bcorr, dref, W, P, R);
    free(dref);
    free(m);
    free(W0);
    free(hotf);
    free(bcorr);
    free(P);
}

/* face HoTs of the current state [nf*21] (zero on boundary faces) */
void orc_face_hot(orc_t *o, double *hotf)
{
    mom_t *m = (mom_t *)malloc(o->nc * sizeof(mom_t));
    all_moments(o, o->f, o->I, m);
    face_hot(o, m, hotf);
    free(m);
}

/* sources Q of the synthetic equations for the state W [nc*NW] -> Q [nc*NW] */
void orc_macro_sources(const orc_t *o, const double *W, double *Q)
{
    int NW = NWof(o->D);
    for (int64_t c = 0; c < o->nc; ++c) {
        prim_t p;
        prim_of(o, W + c * NW, &p);
        macro_source(o, &p, W + c * NW, Q + c * NW);
    }
}

/* W of the current state's moments [nc*NW] */
void orc_macro_state(orc_t *o, double *W)
{
    mom_t *m = (mom_t *)malloc(o->nc * sizeof(mom_t));
    all_moments(o, o->f, o->I, m);
    for (int64_t c = 0; c < o->nc; ++c) W_of_moments(o, &m[c], W + c * NWof(o->D));
    free(m);
}

/* synchronisation of the current state to the macro state W */
void orc_sync(orc_t *o, const double *W)
{
    mom_t *m = (mom_t *)malloc(o->nc * sizeof(mom_t));
    all_moments(o, o->f, o->I, m);
    sync_dist(o, m, W);
    free(m);
}

/* One outer iteration (Sec. 3). gsis = 0: CIS (kinetic step only); 1: full GSIS iteration.
 * Returns the residual epsilon between the moments after and before the iteration; inner = macro count. */
double orc_iterate(orc_t *o, int gsis, int *inner)
{
    int64_t nc = o->nc;
    mom_t *m0 = (mom_t *)malloc(nc * sizeof(mom_t));
    mom_t *m1 = (mom_t *)malloc(nc * sizeof(mom_t));
    all_moments(o, o->f, o->I, m0);
    orc_kinetic_step(o, NULL);
    if (inner) *inner = 0;
    if (!gsis && domain_closed(o)) {
        /* reading (closed domains, conventional iteration): the kinetic step does not conserve mass (point
         * relaxation); f^{k+1/2} is scaled uniformly by mass(f^k) / mass(f^{k+1/2}) (the radiation is not) */
        mom_t *mh = (mom_t *)malloc(nc * sizeof(mom_t));
        all_moments(o, o->f, o->I, mh);
        double mt = 0, mk = 0;
        for (int64_t c = 0; c < nc; ++c) {
            mt += o->vol[c] * m0[c].rho;
            mk += o->vol[c] * mh[c].rho;
        }
        const double sc = mt / mk;
        for (int64_t i = 0; i < nc * o->ND * o->nv; ++i) o->f[i] *= sc;
        free(mh);
    }
    if (gsis) {
        mom_t *mh = (mom_t *)malloc(nc * sizeof(mom_t));
        all_moments(o, o->f, o->I, mh);
        int NW = NWof(o->D);
        double *W = (double *)malloc(nc * NW * sizeof(double));
        for (int64_t c = 0; c < nc; ++c) W_of_moments(o, &mh[c], W + c * NW);
        boundary_of_state(o);
        double mt = 0;
        for (int64_t c = 0; c < nc; ++c) mt += o->vol[c] * m0[c].rho;
        int it = macro_solve(o, mh, mt, W);
        if (inner) *inner = it;
        sync_dist(o, mh, W);
        free(W);
        free(mh);
    }
    all_moments(o, o->f, o->I, m1);
    double e = residual(o, m1, m0);
    free(m0);
    free(m1);
    return e;
}

/* number of cell updates the safeguard of the last synthetic solve shortened or refused */
int64_t orc_safeguard_hits(const orc_t *o) { return o->safeguard_hits; }

/* Switch the face reconstruction between first (0) and second (1) order between iterations. */
void orc_set_second_order(orc_t *o, int so) { o->second_order = so; }

/* Solve: n_precond CIS iterations, then GSIS (or CIS only when gsis = 0) until eps < tol or max_outer.
 * hist receives eps per iteration (capacity max_outer). Returns the iteration count. */
int orc_solve(orc_t *o, int gsis, int n_precond, double tol, int max_outer, double *hist)
{
    int k;
    for (k = 0; k < max_outer; ++k) {
        double e = orc_iterate(o, gsis && k >= n_precond, NULL);
        if (hist) hist[k] = e;
        if (e != e) return -(k + 1);
        if (e < tol) return k + 1;
    }
    return k;
}
