// Synthetic-equation solver for gfx950 (Sec. 2.2 and Sec. 6 of the paper): FP64; set-up kernels run one
// thread per cell or face, the inner iteration one lane per (cell, face slot).
//
// Per inner iteration: primitive state and gradient fields, residual R_i = -(1/V) sum F S + Q with the
// Rusanov convective flux (its dissipation taken relative to the state the solve starts from), the NSF
// viscous flux from face gradients plus the fixed face HoTs, boundary model fluxes plus frozen kinetic
// corrections, the diagonal D_i with the diagonal source Jacobian (Appendix A), Jacobi sweeps of the
// implicit operator, and the update.  The stopping test (relative residual drop) is evaluated on the
// device; kernels of later iterations see the flag and return at once, so the host only polls it every
// few iterations.
#include "gsis_dev.h"
#include "gsis_kernels.h"

namespace gsis {

struct Prim {
    double rho, u[3], Tt, Tr, Tv, eR, mu, cs;
};

// density, velocity and translational temperature of a conserved state
struct PrimL {
    double rho, u[3], Tt;
};

template <int D>
__device__ __forceinline__ void prim_lite(const double *W, PrimL &q)
{
    q.rho = W[0];
    double ek = 0;
    q.u[0] = q.u[1] = q.u[2] = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        q.u[a] = W[1 + a] / W[0];
        ek += 0.5 * W[0] * q.u[a] * q.u[a];
    }
    q.Tt = 2.0 / (3.0 * W[0]) * (W[D + 1] - ek - W[D + 2] - W[D + 3] - W[D + 4]);
}

template <int D>
__device__ __forceinline__ void prim_of(const double *W, const Phys &p, Prim &q)
{
    PrimL l;
    prim_lite<D>(W, l);
    q.rho = l.rho;
    q.u[0] = l.u[0];
    q.u[1] = l.u[1];
    q.u[2] = l.u[2];
    q.Tt = l.Tt;
    q.Tr = 2.0 * W[D + 2] / (p.d_r * W[0]);
    q.Tv = vib_T(p, W[D + 3], W[0]);
    q.eR = W[D + 4];
    q.mu = sqrt(2.0 / kPi) * p.Kn * pow(q.Tt, p.omega);
    q.cs = sqrt(5.0 / 3.0 * q.Tt);
}

// primitive record of a cell: rho, u[D], Tt, Tr, Tv, eR, mu, cs, (pad)
template <int D>
__device__ __forceinline__ void prim_load(const double *Pc, PrimL &q)
{
    q.rho = Pc[0];
    q.u[0] = q.u[1] = q.u[2] = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) q.u[a] = Pc[1 + a];
    q.Tt = Pc[D + 1];
}

// Euler part of the synthetic-equation flux along n (the radiation energy is not convected)
template <int D>
__device__ __forceinline__ void euler_flux_q(const double *W, const PrimL &q, const double *n, double *F)
{
    double un = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) un += q.u[a] * n[a];
    const double pt = q.rho * q.Tt;
    F[0] = q.rho * un;
#pragma unroll
    for (int a = 0; a < D; ++a) F[1 + a] = W[1 + a] * un + pt * n[a];
    F[D + 1] = un * (W[D + 1] - W[D + 4] + pt);
    F[D + 2] = un * W[D + 2];
    F[D + 3] = un * W[D + 3];
    F[D + 4] = 0.0;
}

template <int D>
__device__ __forceinline__ void euler_flux(const double *W, const double *n, double *F)
{
    PrimL q;
    prim_lite<D>(W, q);
    euler_flux_q<D>(W, q, n, F);
}

// Rusanov flux from left/right conserved states, their primitives and sound speeds; exactly odd under
// the exchange of the two sides together with n -> -n
template <int D>
__device__ __forceinline__ double rusanov_q(const double *WL, const PrimL &qL, double csL, const double *WR,
                                            const PrimL &qR, double csR, const double *n, double *F)
{
    constexpr int NW = D + 5;
    double FL[NW], FR[NW];
    euler_flux_q<D>(WL, qL, n, FL);
    euler_flux_q<D>(WR, qR, n, FR);
    double unL = 0, unR = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        unL += qL.u[a] * n[a];
        unR += qR.u[a] * n[a];
    }
    const double lam = fmax(fabs(unL) + csL, fabs(unR) + csR);
#pragma unroll
    for (int i = 0; i < NW - 1; ++i) F[i] = 0.5 * (FL[i] + FR[i]) - 0.5 * lam * (WR[i] - WL[i]);
    F[NW - 1] = 0.0;
    return lam;
}

template <int D>
__device__ __forceinline__ void W_of_state(double rho, const double *u, double T, const Phys &p, double *W)
{
    double ek = 0;
    W[0] = rho;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        W[1 + a] = rho * u[a];
        ek += 0.5 * rho * u[a] * u[a];
    }
    W[D + 2] = 0.5 * p.d_r * rho * T;
    W[D + 3] = vib_rho_e(p, rho, T);
    W[D + 4] = 4 * p.sigma_R * T * T * T * T;
    W[D + 1] = ek + 1.5 * rho * T + W[D + 2] + W[D + 3] + W[D + 4];
}

// NSF stress and heat fluxes plus optional HoTs; g[i][a] gradients of (u[D], Tt, Tr, Tv, eR)
template <int D>
__device__ __forceinline__ void constitutive(double mu, const double g[][3], const double *hot, const Phys &p,
                                             double sig[3][3], double q[4][3])
{
    const double kR = (p.keff > 0) ? 1.0 / (3 * p.keff) : 0.0;
    double div = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) div += g[a][a];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
            sig[a][b] = -mu * (g[b][a] + g[a][b] - (a == b ? 2.0 / 3.0 * div : 0.0));
            if (hot) sig[a][b] += hot[a * 3 + b];
        }
#pragma unroll
    for (int a = 0; a < D; ++a) {
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            double v = 0;
#pragma unroll
            for (int mm = 0; mm < 3; ++mm) v -= 0.5 * mu * p.K0[l][mm] * g[D + mm][a];
            q[l][a] = v + (hot ? hot[9 + 3 * l + a] : 0.0);
        }
        q[3][a] = -kR * g[D + 3][a] + (hot ? hot[18 + a] : 0.0);
    }
}

template <int D>
__device__ __forceinline__ void viscous_flux(const double sig[3][3], const double q[4][3], const double *uf,
                                             const double *n, double *F)
{
    double sn[3] = {0, 0, 0}, work = 0, qall = 0, qrn = 0, qvn = 0, qRn = 0;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) sn[a] += sig[a][b] * n[b];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        work += sn[a] * uf[a];
        qall += (q[0][a] + q[1][a] + q[2][a] + q[3][a]) * n[a];
        qrn += q[1][a] * n[a];
        qvn += q[2][a] * n[a];
        qRn += q[3][a] * n[a];
    }
    F[0] = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) F[1 + a] = sn[a];
    F[D + 1] = work + qall;
    F[D + 2] = qrn;
    F[D + 3] = qvn;
    F[D + 4] = qRn;
}

// model flux of a boundary face for the cell state Wc (wall: impermeable NSF-type wall flux; far field:
// Rusanov against the prescribed state; both with radiative diffusion towards B_R(T_b)); g1/g2 spectral radii
// (q: the primitives of Wc, as prim_of gives them)
template <int D>
__device__ __forceinline__ void bmodel_flux_q(const MeshDev &m, int bfi, const double *Wc, const Prim &q,
                                              const Phys &p, double *F, double *g1, double *g2)
{
    constexpr int NW = D + 5;
    const BcDev bc = m.bf_bc[bfi];
    double n[D], delta = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        n[a] = m.bf_n[(int64_t)bfi * D + a];
        delta += n[a] * m.bf_dxc[(int64_t)bfi * D + a];
    }
    delta = fabs(delta);
    const double kR = (p.keff > 0) ? 1.0 / (3 * p.keff) : 0.0;
    const double Tb = bc.T;
    const double eRb = 4 * p.sigma_R * Tb * Tb * Tb * Tb;
    const double qRn = -kR * (eRb - q.eR) / delta;
#pragma unroll
    for (int i = 0; i < NW; ++i) F[i] = 0;
    double un = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) un += q.u[a] * n[a];
    *g1 = fabs(un) + q.cs + 2 * q.mu / (q.rho * delta);
    *g2 = 2 * kR / delta;
    if (bc.kind == 0) {
        const double pt = q.rho * q.Tt;
        double work = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double sn = -q.mu * (bc.u[a] - q.u[a]) / delta;
            F[1 + a] = pt * n[a] + sn;
            work += sn * bc.u[a];
        }
        const double dT[3] = {(Tb - q.Tt) / delta, (Tb - q.Tr) / delta, (Tb - q.Tv) / delta};
        double qn[3];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            qn[l] = 0;
#pragma unroll
            for (int mm = 0; mm < 3; ++mm) qn[l] -= 0.5 * q.mu * p.K0[l][mm] * dT[mm];
        }
        F[D + 1] = work + qn[0] + qn[1] + qn[2] + qRn;
        F[D + 2] = qn[1];
        F[D + 3] = qn[2];
        F[D + 4] = qRn;
    } else {
        double Wb[NW];
        W_of_state<D>(bc.rho, bc.u, Tb, p, Wb);
        PrimL qL, qR;
        qL.rho = q.rho;
        qL.u[0] = q.u[0];
        qL.u[1] = q.u[1];
        qL.u[2] = q.u[2];
        qL.Tt = q.Tt;
        prim_lite<D>(Wb, qR);
        rusanov_q<D>(Wc, qL, q.cs, Wb, qR, sqrt(5.0 / 3.0 * qR.Tt), n, F);
        F[D + 1] += qRn;
        F[D + 4] = qRn;
    }
}

template <int D>
__device__ __forceinline__ void bmodel_flux(const MeshDev &m, int bfi, const double *Wc, const Phys &p, double *F,
                                            double *g1, double *g2)
{
    Prim q;
    prim_of<D>(Wc, p, q);
    bmodel_flux_q<D>(m, bfi, Wc, q, p, F, g1, g2);
}

// point solve of the implicit operator in U = (rho, rho u, e_gas, e_r, e_v, e_R): diagonal except for the
// gas-photon exchange, solved exactly per cell (with e' = d e_vR / d e_v):
//   D_g dg = r_g - k e' dv + k dR,   D_v dv = r_v + k dR,   D_R dR = r_R + k e' dv
// With k = 0 (absorption and emission off) the e_R row is singular (no diffusion, no source): e_R is not
// a synthetic unknown there (dR = 0), so it keeps its kinetic value and the synchronisation leaves I alone.
template <int D>
__device__ __forceinline__ void local_solve(const double *rhs, const double *Dg, const double rho, const double Tv,
                                            const Phys &p, double *dU)
{
    constexpr int NW = D + 5, ig = D + 1, iv = D + 3, iR = D + 4;
#pragma unroll
    for (int i = 0; i < NW; ++i) dU[i] = rhs[i] / Dg[i];
    const double k = p.keff;
    const double ep = p.Tvref > 0 ? 16.0 * p.sigma_R * Tv * Tv * Tv / (vib_cv(p, Tv) * rho)
                                  : 32.0 * p.sigma_R * Tv * Tv * Tv / (p.d_v * rho);
    const double dv = (rhs[iv] + k * rhs[iR] / Dg[iR]) / (Dg[iv] - k * k * ep / Dg[iR]);
    const double dR = (rhs[iR] + k * ep * dv) / Dg[iR];
    dU[iv] = dv;
    dU[iR] = (k > 0) ? dR : 0.0;
    dU[ig] = (rhs[ig] - k * ep * dv + k * dR) / Dg[ig];
}

// W += a dU with a = 2^-m the largest factor (m <= 20) keeping rho, T_t, e_r, e_v, e_R at least half their
// current values and within a factor two of their values Ws at the start of the solve; no update if none
template <int D>
__device__ __forceinline__ void positive_update(double *W, const double *dU, const double *Ws)
{
    constexpr int NW = D + 5;
    PrimL p0, ps;
    prim_lite<D>(W, p0);
    prim_lite<D>(Ws, ps);
    double a = 1.0;
    for (int m = 0; m <= 20; ++m, a *= 0.5) {
        double Wn[NW];
#pragma unroll
        for (int i = 0; i < NW; ++i) Wn[i] = W[i] + a * dU[i];
        Wn[D + 1] += a * dU[D + 4];
        // the bounds on conserved components first: the temperature (divisions) only for a factor
        // that passes them
        bool ok = true;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = (i == 0) ? 0 : D + 1 + i;
            ok = ok && Wn[k] >= 0.5 * W[k] && Wn[k] >= 0.5 * Ws[k] && Wn[k] <= 2 * Ws[k];
        }
        if (!ok) continue;
        PrimL p1;
        prim_lite<D>(Wn, p1);
        if (p1.Tt >= 0.5 * p0.Tt && p1.Tt >= 0.5 * ps.Tt && p1.Tt <= 2 * ps.Tt) {
#pragma unroll
            for (int i = 0; i < NW; ++i) W[i] = Wn[i];
            return;
        }
    }
}

// The same update with the trial factors spread over the LS lanes of a cell's group (all of them call it
// with identical W, dU, Ws): round r tests m = LS r + s on lane s, and the lowest passing m of the first
// round with a pass is taken, which is the factor the serial halving above accepts.  T0 and Ts are the
// translational temperatures of W and Ws as prim_lite gives them (taken from the primitive records).
template <int D, int LS>
__device__ __forceinline__ void positive_update_lanes(double *W, const double *dU, const double *Ws, const double T0,
                                                      const double Ts, const int s, const int base)
{
    constexpr int NW = D + 5;
    PrimL p0, ps;
    p0.Tt = T0;
    ps.Tt = Ts;
    for (int r = 0; LS * r <= 20; ++r) {
        const int mm = LS * r + s;
        const double a = ldexp(1.0, -mm);
        double Wn[NW];
#pragma unroll
        for (int i = 0; i < NW; ++i) Wn[i] = W[i] + a * dU[i];
        Wn[D + 1] += a * dU[D + 4];
        bool ok = mm <= 20;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = (i == 0) ? 0 : D + 1 + i;
            ok = ok && Wn[k] >= 0.5 * W[k] && Wn[k] >= 0.5 * Ws[k] && Wn[k] <= 2 * Ws[k];
        }
        if (ok) {
            PrimL p1;
            prim_lite<D>(Wn, p1);
            ok = p1.Tt >= 0.5 * p0.Tt && p1.Tt >= 0.5 * ps.Tt && p1.Tt <= 2 * ps.Tt;
        }
        const unsigned grp = (unsigned)((__ballot(ok) >> base) & ((1ull << LS) - 1));
        if (grp) {
            const int sw = __builtin_ctz(grp);
#pragma unroll
            for (int i = 0; i < NW; ++i) W[i] = __shfl(Wn[i], base + sw, 64);
            return;
        }
    }
}

// ------------------------------------------------------------------ setup kernels
template <int D>
__global__ void k_W_from_mom(const double *__restrict__ mom, double *__restrict__ W, double *__restrict__ W0,
                             const int64_t nc, const Phys p)
{
    constexpr MomLayout L{D};
    constexpr int NW = D + 5;
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const double *M = mom + c * L.size();
    const double rho = M[L.rho()];
    double Wc[NW], ek = 0;
    Wc[0] = rho;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        Wc[1 + a] = rho * M[L.u() + a];
        ek += 0.5 * rho * M[L.u() + a] * M[L.u() + a];
    }
    const double er = 0.5 * p.d_r * rho * M[L.Tr()], ev = vib_rho_e(p, rho, M[L.Tv()]);
    Wc[D + 1] = ek + 1.5 * rho * M[L.Tt()] + er + ev + M[L.eR()];
    Wc[D + 2] = er;
    Wc[D + 3] = ev;
    Wc[D + 4] = M[L.eR()];
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        W[c * NW + i] = Wc[i];
        W0[c * NW + i] = Wc[i];
    }
}

// gradient fields (u[D], Tt, Tr, Tv, eR) from moments
template <int D>
__global__ void k_fld_from_mom(const double *__restrict__ mom, double *__restrict__ fld, double *__restrict__ P,
                               const int64_t nc, const Phys p)
{
    constexpr MomLayout L{D};
    constexpr int NF = D + 4;
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const double *M = mom + c * L.size();
#pragma unroll
    for (int a = 0; a < D; ++a) fld[c * NF + a] = M[L.u() + a];
    fld[c * NF + D] = M[L.Tt()];
    fld[c * NF + D + 1] = M[L.Tr()];
    fld[c * NF + D + 2] = M[L.Tv()];
    fld[c * NF + D + 3] = M[L.eR()];
    P[c] = sqrt(2.0 / kPi) * p.Kn * pow(M[L.Tt()], p.omega);  // mu
}

// unlimited least-squares gradient of the NF fields of cell c (zero-gradient ghosts on boundary faces)
template <int D, int NFM>
__device__ __forceinline__ void cell_grad(const double *__restrict__ fld, const MeshDev &m, const int64_t c,
                                          double g[][D])
{
    constexpr int NF = D + 4;
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int a = 0; a < D; ++a) g[i][a] = 0;
    const int nfc = m.nfc[c];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        const int j = (s < nfc) ? m.nbr[c * NFM + s] : -1;
        if (j < 0) continue;
        const double *gs = m.lsq + (c * NFM + s) * D;
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            const double df = fld[(int64_t)j * NF + i] - fld[c * NF + i];
#pragma unroll
            for (int a = 0; a < D; ++a) g[i][a] += gs[a] * df;
        }
    }
}

template <int D, int NFM>
__global__ void k_cell_grad(const double *__restrict__ fld, double *__restrict__ gfld, const MeshDev m)
{
    constexpr int NF = D + 4;
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= m.nc) return;
    double g[NF][D];
    cell_grad<D, NFM>(fld, m, c, g);
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int a = 0; a < D; ++a) gfld[(c * NF + i) * D + a] = g[i][a];
}

// adds the least-squares gradient of cell c (as cell_grad) to g, with the neighbour list of c given
// (nb[s] < 0: boundary or padded slot).  Branch-free, so that all loads are in flight together: a slot
// without a neighbour reads cell c itself, whose difference is exactly zero.
template <int D, int NFM>
__device__ __forceinline__ void cell_grad_add(const double *__restrict__ fld, const MeshDev &m, const int64_t c,
                                              const int *nb, double g[][D])
{
    constexpr int NF = D + 4;
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        const int64_t j = (nb[s] >= 0) ? (int64_t)nb[s] : c;
        const double *gs = m.lsq + (c * NFM + s) * D;
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            const double df = fld[(int64_t)j * NF + i] - fld[c * NF + i];
#pragma unroll
            for (int a = 0; a < D; ++a) g[i][a] += gs[a] * df;
        }
    }
}

// face gradient from the sum gs of the two cell gradients: their mean with the component along the
// centroid line replaced by the centroid difference quotient (fg: the face's geometry record, with the
// unit vector dh along d = x_j - x_c and 1 / |d|)
template <int D>
__device__ __forceinline__ void face_grad_sum(const double *fld, const double gs[][D], int64_t c, int64_t j,
                                              const double *fg, double g[][3])
{
    constexpr int NF = D + 4;
    double dh[D];
#pragma unroll
    for (int a = 0; a < D; ++a) dh[a] = fg[D + a];
    const double idl = fg[2 * D];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        double avg[D], corr = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            avg[a] = 0.5 * gs[i][a];
            corr += avg[a] * dh[a];
        }
        const double jump = (fld[j * NF + i] - fld[c * NF + i]) * idl;
#pragma unroll
        for (int a = 0; a < 3; ++a) g[i][a] = (a < D) ? avg[a] + (jump - corr) * dh[a] : 0.0;
    }
}

template <int D>
__device__ __forceinline__ void face_grad(const double *fld, const double *gfld, int64_t c, int64_t j,
                                          const double *fg, double g[][3])
{
    constexpr int NF = D + 4;
    double gs[NF][D];
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int a = 0; a < D; ++a) gs[i][a] = gfld[(c * NF + i) * D + a] + gfld[(j * NF + i) * D + a];
    face_grad_sum<D>(fld, gs, c, j, fg, g);
}

// Per-face constants of the synthetic flux, frozen for the whole solve (interior faces; zero rows on
// boundary faces): [0, NW) the reference dissipation 0.5 lam* (W0_R - W0_L) plus the HoT part of the
// viscous flux (HoT stress and heat fluxes along n), [NW, NW + D) the HoT stress along n alone, for the
// work term u_f . (sigma_HoT n).  The HoTs are the mean kinetic moments of the two cells minus the NSF
// relations with the face gradient (mu from the moments).
template <int D>
__global__ __launch_bounds__(256) void k_face_const(const double *__restrict__ mom, const double *__restrict__ fld,
                                                    const double *__restrict__ gfld, const double *__restrict__ mu,
                                                    const double *__restrict__ W0, double *__restrict__ fcon,
                                                    const MeshDev m, const Phys p)
{
    constexpr MomLayout L{D};
    constexpr int NW = D + 5, NC = NW + D;
    const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (f >= m.nf) return;
    double *h = fcon + f * NC;
    const int64_t c = m.f_L[f], j = m.f_R[f];
    if (j < 0) {
        for (int i = 0; i < NC; ++i) h[i] = 0;
        return;
    }
    double n[D];
#pragma unroll
    for (int a = 0; a < D; ++a) n[a] = m.fgeo[f * (2 * D + 2) + a];
    double g[D + 4][3], sig[3][3], q[4][3];
    face_grad<D>(fld, gfld, c, j, m.fgeo + f * (2 * D + 2), g);
    constitutive<D>(0.5 * (mu[c] + mu[j]), g, nullptr, p, sig, q);
    const double *Mc = mom + c * L.size(), *Mj = mom + j * L.size();
    double hs[D], hq[4] = {0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        hs[a] = 0;
#pragma unroll
        for (int b = 0; b < D; ++b)
            hs[a] += (0.5 * (Mc[L.sig() + a * D + b] + Mj[L.sig() + a * D + b]) - sig[a][b]) * n[b];
        hq[0] += (0.5 * (Mc[L.qt() + a] + Mj[L.qt() + a]) - q[0][a]) * n[a];
        hq[1] += (0.5 * (Mc[L.qr() + a] + Mj[L.qr() + a]) - q[1][a]) * n[a];
        hq[2] += (0.5 * (Mc[L.qv() + a] + Mj[L.qv() + a]) - q[2][a]) * n[a];
        hq[3] += (0.5 * (Mc[L.qR() + a] + Mj[L.qR() + a]) - q[3][a]) * n[a];
    }
    // reference dissipation (first-order face states of W0)
    const double *WL = W0 + c * NW, *WR = W0 + j * NW;
    Prim qL, qR;
    prim_of<D>(WL, p, qL);
    prim_of<D>(WR, p, qR);
    double unL = 0, unR = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        unL += qL.u[a] * n[a];
        unR += qR.u[a] * n[a];
    }
    const double lam = fmax(fabs(unL) + qL.cs, fabs(unR) + qR.cs);
    double F[NW];
#pragma unroll
    for (int i = 0; i < NW - 1; ++i) F[i] = 0.5 * lam * (WR[i] - WL[i]);
    F[NW - 1] = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) F[1 + a] += hs[a];
    F[D + 1] += hq[0] + hq[1] + hq[2] + hq[3];
    F[D + 2] += hq[1];
    F[D + 3] += hq[2];
    F[D + 4] += hq[3];
#pragma unroll
    for (int i = 0; i < NW; ++i) h[i] = F[i];
#pragma unroll
    for (int a = 0; a < D; ++a) h[NW + a] = hs[a];
}

// frozen boundary corrections: kinetic boundary flux minus the model flux at W0
template <int D>
__global__ void k_bcorr(const double *__restrict__ W0, const double *__restrict__ bflux, double *__restrict__ bcorr,
                        const MeshDev m, const Phys p)
{
    constexpr int NW = D + 5;
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= m.nbf) return;
    double F[NW], g1, g2;
    bmodel_flux<D>(m, (int)b, W0 + (int64_t)m.bf_cell[b] * NW, p, F, &g1, &g2);
#pragma unroll
    for (int i = 0; i < NW; ++i) bcorr[b * NW + i] = bflux[b * NW + i] - F[i];
}

// ------------------------------------------------------------------ inner-iteration kernels

// sum over the 64 lanes of the (single-wave) block in a fixed butterfly order; every lane gets lane 0's
// result (the lanes' own butterfly results may differ in the last bit)
__device__ __forceinline__ double wave_sum64(double v)
{
    static_assert(kMBlk == 64, "inner-iteration blocks are one wave");
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return __shfl(v, 0, 64);
}

// Stores of the inner-iteration kernels' outputs bypass the L2: the next kernel, a dependent launch,
// starts with the L2s of the other XCDs cold for these lines anyway, and lines left dirty would be
// written back when the kernel ends.
__device__ __forceinline__ void st_nt(double *p, double v) { __builtin_nontemporal_store(v, p); }

// primitive record and gradient fields of W
template <int D>
__device__ __forceinline__ void store_prim(const double *Wc, const Phys &p, double *pc, double *fc)
{
    Prim q;
    prim_of<D>(Wc, p, q);
    st_nt(pc, q.rho);
#pragma unroll
    for (int a = 0; a < D; ++a) st_nt(pc + 1 + a, q.u[a]);
    st_nt(pc + D + 1, q.Tt);
    st_nt(pc + D + 2, q.Tr);
    st_nt(pc + D + 3, q.Tv);
    st_nt(pc + D + 4, q.eR);
    st_nt(pc + D + 5, q.mu);
    st_nt(pc + D + 6, q.cs);
    st_nt(pc + D + 7, 0.0);
#pragma unroll
    for (int a = 0; a < D; ++a) st_nt(fc + a, q.u[a]);
    st_nt(fc + D, q.Tt);
    st_nt(fc + D + 1, q.Tr);
    st_nt(fc + D + 2, q.Tv);
    st_nt(fc + D + 3, q.eR);
}

template <int D>
__global__ void k_mprim(const double *__restrict__ W, double *__restrict__ P, double *__restrict__ fld,
                        double *__restrict__ Ts,
                        const int64_t nc, const Phys p)
{
    constexpr int NW = D + 5, NF = D + 4, NP = D + 8;
    const int64_t c = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    store_prim<D>(W + c * NW, p, P + c * NP, fld + c * NF);
    PrimL l;
    prim_lite<D>(W + c * NW, l);
    Ts[c] = l.Tt;
}

// ---- slot-parallel inner-iteration kernels: kSBlk threads per block, slot_lanes(NFM) = NFM consecutive lanes
// per cell, cells_per_wave(NFM) cells per wave, lane s of a cell's group handling its face slot s (padded
// slots hold nbr = INT32_MIN).  Packing the groups without power-of-two padding keeps the number of waves
// at or below the SIMD count for the largest 2D grids that fit the GPU at one wave per SIMD.  The per-face
// work runs on separate lanes; the cell's sums are gathered from its lanes in slot order with shuffles and
// the per-cell point solve runs on the group's first lane.

// Interior face fid in its own orientation (left cell cL -> right cell cR): Rusanov with the reference
// dissipation, NSF viscous flux with the face gradient plus the frozen face HoTs; spectral radii of the
// convective-viscous and radiative-diffusion operators for the diagonal.  Both sides of a face evaluate
// this same expression and the right side negates it, so the discrete flux is exactly odd.
template <int D, int NFM>
__device__ __forceinline__ void face_flux(const double *__restrict__ W, const double *__restrict__ P,
                                          const double *__restrict__ fld, const double *__restrict__ fcon,
                                          const MeshDev &m, const Phys &p,
                                          const int64_t fid, const int64_t cL, const int64_t cR,
                                          const int *nbL, const int *nbR, double *F, double *G, double *GR)
{
    constexpr int NW = D + 5, NP = D + 8, NF = D + 4;
    const double kR = (p.keff > 0) ? 1.0 / (3 * p.keff) : 0.0;
    const double *fg = m.fgeo + fid * (2 * D + 2);
    double n[D];
#pragma unroll
    for (int a = 0; a < D; ++a) n[a] = fg[a];
    const double ind = fg[2 * D + 1];
    const double *Pc = P + cL * NP, *Pj = P + cR * NP;
    PrimL qc, qj;
    prim_load<D>(Pc, qc);
    prim_load<D>(Pj, qj);
    double Fc[NW];
    rusanov_q<D>(W + cL * NW, qc, Pc[D + 6], W + cR * NW, qj, Pj[D + 6], n, Fc);
    const double *fc = fcon + fid * (NW + D);
#pragma unroll
    for (int i = 0; i < NW; ++i) Fc[i] += fc[i];
    double gsum[NF][D], g[NF][3], sig[3][3], q[4][3], Fv[NW], uf[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int a = 0; a < D; ++a) gsum[i][a] = 0;
    cell_grad_add<D, NFM>(fld, m, cL, nbL, gsum);
    cell_grad_add<D, NFM>(fld, m, cR, nbR, gsum);
    face_grad_sum<D>(fld, gsum, cL, cR, fg, g);
#pragma unroll
    for (int a = 0; a < D; ++a) uf[a] = 0.5 * (Pc[1 + a] + Pj[1 + a]);
    constitutive<D>(0.5 * (Pc[D + 5] + Pj[D + 5]), g, nullptr, p, sig, q);
    viscous_flux<D>(sig, q, uf, n, Fv);
    double wh = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) wh += fc[NW + a] * uf[a];
#pragma unroll
    for (int i = 0; i < NW; ++i) F[i] = Fc[i] + Fv[i];
    F[D + 1] += wh;
    double ufn = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) ufn += uf[a] * n[a];
    // 2 mu_f / (rho_f |n . d|) with face means of mu and rho
    *G = fabs(ufn) + 0.5 * (Pc[D + 6] + Pj[D + 6]) + 2 * (Pc[D + 5] + Pj[D + 5]) * ind / (Pc[0] + Pj[0]);
    *GR = 2 * kR * ind;
}

// Sum over the 64 partial sums per lane stride of the per-block residual sums, in a fixed order (every
// wave of every block forms the same value).  The loads are issued by the caller before its own work.
constexpr int kPartRegs = 8;
__device__ __forceinline__ void part_load(const double *__restrict__ part, const int nb, double pr[kPartRegs],
                                          double *rest)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < kPartRegs; ++u) {
        const int b = lane + 64 * u;
        pr[u] = (b < nb) ? part[b] : 0.0;
    }
    // beyond the first 64 kPartRegs partials (large grids), eight independent running sums so that eight
    // loads are in flight per step instead of one
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b0 = lane + 64 * kPartRegs; b0 < nb; b0 += 64 * 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int b = b0 + 64 * u;
            a[u] += (b < nb) ? part[b] : 0.0;
        }
    }
    *rest = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// Stopping test of inner iteration `it` from the loaded partial sums; block 0 records the norms and raises
// the flag that later kernels test.
__device__ __forceinline__ bool inner_converged(const double pr[kPartRegs], const double rest, const int it,
                                                const double tol, double *__restrict__ scal, int *__restrict__ flags)
{
    double v = 0;
#pragma unroll
    for (int u = 0; u < kPartRegs; ++u) v += pr[u];
    v += rest;
    const double res = sqrt(wave_sum64(v));
    const double res0 = (it == 0) ? res : scal[0];
    const bool done = res <= tol * res0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (it == 0) scal[0] = res;
        scal[1] = res;
        if (done) {
            flags[0] = 1;
            flags[1] = it;
        }
    }
    return done;
}

// Interior-face fluxes of the synthetic equations for grids that do not fit the GPU in one round of k_mres:
// one lane per face evaluates face_flux once, in the face's own orientation (k_mres<SPLIT> then negates it
// on the right cell, exactly as the fused kernel does, so both paths give identical residuals), and
// stores the spectral radii into the slots of both cells.
template <int D, int NFM>
__global__ __launch_bounds__(256) void k_mface(const double *__restrict__ W, const double *__restrict__ P,
                                               const double *__restrict__ fld, const double *__restrict__ fcon,
                                               double *__restrict__ Ff, double *__restrict__ Gs,
                                               const int *__restrict__ flags, const MeshDev m, const Phys p)
{
    constexpr int NW = D + 5;
    if (flags[0]) return;
    const int64_t f = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (f >= m.nf) return;
    const int sl = m.fslot[2 * f], sr = m.fslot[2 * f + 1];
    if (sl < 0 || sr < 0) return;
    const int64_t cL = sl / NFM, cR = sr / NFM;
    int nbL[NFM], nbR[NFM];
#pragma unroll
    for (int q = 0; q < NFM; ++q) {
        nbL[q] = m.nbr[cL * NFM + q];
        nbR[q] = m.nbr[cR * NFM + q];
    }
    double F[NW], G, GR;
    face_flux<D, NFM>(W, P, fld, fcon, m, p, f, cL, cR, nbL, nbR, F, &G, &GR);
#pragma unroll
    for (int i = 0; i < NW; ++i) Ff[f * NW + i] = F[i];
    Gs[(int64_t)sl * 2] = G;
    Gs[(int64_t)sl * 2 + 1] = GR;
    Gs[(int64_t)sr * 2] = G;
    Gs[(int64_t)sr * 2 + 1] = GR;
}

// Residual of every cell: R_i = -(1/V) sum_f F S + Q (face fluxes of the cell's slots gathered in slot
// order, boundary model fluxes plus the frozen kinetic corrections), the diagonal D_i and the first
// increment of the U unknowns; per-slot spectral radii for the sweeps; per-block sums of the
// volume-weighted squared residual.
// PRE: the cell's point-solve data is loaded up front with the slot tables (one dependent-load level
// less; 22 more VGPRs, two waves per SIMD), else in the per-cell tail (three waves per SIMD, for grids
// that would not fit the GPU in one round at two).
template <int D, int NFM, bool PRE, bool SPLIT = false>
__global__ __launch_bounds__(kSBlk) void k_mres(
    const double *__restrict__ W, const double *__restrict__ P, const double *__restrict__ fld,
    const double *__restrict__ fcon, const double *__restrict__ bcorr,
    double *__restrict__ Gs, double *__restrict__ R, double *__restrict__ Dg, double *__restrict__ dU,
    double *__restrict__ part, const int *__restrict__ flags, const MeshDev m, const Phys p, const double cfl_macro,
    const double *__restrict__ Ff = nullptr)
{
    constexpr int NW = D + 5, NP = D + 8, MG = 2 * D + 2, LS = slot_lanes(NFM);
    __shared__ double sh[kSBlk / 64];
    const int done = flags[0];
    constexpr int CPW = cells_per_wave(NFM);
    const int t = threadIdx.x, lane = t & 63, grp = lane / LS, s = lane - grp * LS, base = grp * LS;
    const int64_t wv = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * (kSBlk / 64) + (t >> 6);
    const int64_t c = wv * CPW + grp;
    const bool cell = grp < CPW && c < m.nc;
    const bool slot = cell && s < NFM;
    // every index this lane needs is read here (one level of dependent loads): the slot, the cell's own
    // neighbour list and the neighbour's (for the two cell gradients), and the cell's point-solve data.
    // The loads are unconditional, from a clamped cell and slot (always in bounds), so that they issue
    // without branches; the values of lanes without a cell or slot are replaced afterwards.
    const int64_t cc = cell ? c : m.nc - 1;
    const int ss = (s < NFM) ? s : 0;
    const int jr = m.nbr[cc * NFM + ss];
    const int sfr = m.sfid[cc * NFM + ss];
    const double Slr = m.mgeo[(cc * NFM + ss) * MG + D];
    const int j = slot ? jr : INT32_MIN;
    const int sf = slot ? sfr : 0;
    const double Sl = slot ? Slr : 0.0;
    int nbc[NFM], nbj[NFM];
    if constexpr (!SPLIT) {
#pragma unroll
        for (int q = 0; q < NFM; ++q) {
            const int a = m.nbr[cc * NFM + q], b = m.nb2[(cc * NFM + ss) * NFM + q];
            nbc[q] = cell ? a : INT32_MIN;
            nbj[q] = slot ? b : INT32_MIN;
        }
    }
    double Wc[NW], Pc[D + 7], V = 1, hc = 1;
    if constexpr (PRE) {
#pragma unroll
        for (int i = 0; i < NW; ++i) Wc[i] = W[cc * NW + i];
#pragma unroll
        for (int i = 0; i < D + 7; ++i) Pc[i] = P[cc * NP + i];
        V = m.vol[cc];
        hc = m.h[cc];
    }
    if (done) return;
    double Fs[NW], S = 0, gS = 0, gRS = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) Fs[i] = 0;
    if (j != INT32_MIN) {
        S = Sl;
        if (j < 0) {
            const int bfi = -j - 1;
            double g1, g2;
            // the cell's primitives are its record in P (written from W by the same prim_of)
            double Pb[D + 7];
#pragma unroll
            for (int i = 0; i < D + 7; ++i) Pb[i] = PRE ? Pc[i] : P[c * NP + i];
            Prim q;
            q.rho = Pb[0];
            q.u[0] = q.u[1] = q.u[2] = 0;
#pragma unroll
            for (int a = 0; a < D; ++a) q.u[a] = Pb[1 + a];
            q.Tt = Pb[D + 1];
            q.Tr = Pb[D + 2];
            q.Tv = Pb[D + 3];
            q.eR = Pb[D + 4];
            q.mu = Pb[D + 5];
            q.cs = Pb[D + 6];
            bmodel_flux_q<D>(m, bfi, PRE ? Wc : W + c * NW, q, p, Fs, &g1, &g2);
#pragma unroll
            for (int i = 0; i < NW; ++i) Fs[i] += bcorr[(int64_t)bfi * NW + i];
            gS = g1 * S;
            gRS = g2 * S;
        } else {
            const bool left = sf >= 0;
            const int64_t fid = left ? sf : -(int64_t)sf - 1;
            double G, GR;
            if constexpr (SPLIT) {
                // the face's flux and spectral radii, evaluated once per face by k_mface
#pragma unroll
                for (int i = 0; i < NW; ++i) Fs[i] = Ff[fid * NW + i];
                G = Gs[(c * NFM + s) * 2];
                GR = Gs[(c * NFM + s) * 2 + 1];
            } else {
                face_flux<D, NFM>(W, P, fld, fcon, m, p, fid, left ? c : j, left ? j : c, left ? nbc : nbj,
                                  left ? nbj : nbc, Fs, &G, &GR);
            }
            if (!left) {
#pragma unroll
                for (int i = 0; i < NW; ++i) Fs[i] = -Fs[i];
            }
            if constexpr (!SPLIT) {
                st_nt(Gs + (c * NFM + s) * 2, G);
                st_nt(Gs + (c * NFM + s) * 2 + 1, GR);
            }
            gS = G * S;
            gRS = GR * S;
        }
    }
    // the cell's sums, slot by slot (every lane takes part in the shuffles)
    double acc[NW], gs = 0, gsR = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) acc[i] = 0;
#pragma unroll
    for (int q = 0; q < NFM; ++q) {
        const double Sq = __shfl(S, base + q, 64);
#pragma unroll
        for (int i = 0; i < NW; ++i) acc[i] += __shfl(Fs[i], base + q, 64) * Sq;
        gs += __shfl(gS, base + q, 64);
        gsR += __shfl(gRS, base + q, 64);
    }
    double contrib = 0;
    if (cell && s == 0) {
        if constexpr (!PRE) {
#pragma unroll
            for (int i = 0; i < NW; ++i) Wc[i] = W[c * NW + i];
#pragma unroll
            for (int i = 0; i < D + 7; ++i) Pc[i] = P[c * NP + i];
            V = m.vol[c];
            hc = m.h[c];
        }
        const double rho = Pc[0], Tt = Pc[D + 1], Tr = Pc[D + 2], Tv = Pc[D + 3];
        const double tau = Pc[D + 5] / (rho * Tt);
        const double Ttr = (3 * Tt + p.d_r * Tr) / (3 + p.d_r), Ttv = vib_Ttv(p, Tt, Tv);
        const double etr = 0.5 * p.d_r * rho * Ttr, etv = vib_rho_e(p, rho, Ttv);
        const double evR = 4 * p.sigma_R * Tv * Tv * Tv * Tv;
        const double er = Wc[D + 2], ev = Wc[D + 3], eR = Wc[D + 4];
        double Q[NW];
#pragma unroll
        for (int i = 0; i < NW; ++i) Q[i] = 0;
        Q[D + 2] = (etr - er) / (p.Z_r * tau);
        Q[D + 3] = (etv - ev) / (p.Z_v * tau) - p.keff * (evR - eR);
        Q[D + 4] = p.keff * (evR - eR);
        const double iV = 1.0 / V;
        double Rc[NW], rs = 0;
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            Rc[i] = Q[i] - acc[i] * iV;
            rs += Rc[i] * Rc[i];
        }
        contrib = V * rs;
        double un = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) un += Pc[1 + a] * Pc[1 + a];
        const double dt = cfl_macro * hc / (sqrt(un) + Pc[D + 6]);
        const double jr =
            -3.0 / ((3 + p.d_r) * p.Z_r * tau) + 2 * (p.omega - 1) * (Ttr - Tr) / (3 * p.Z_r * tau * Tt);
        // variable d_v: d_v replaced by the heat capacity 2 c_v (at T_tv in the relaxation term, at T_v in the
        // emission term)
        const double jv =
            p.Tvref > 0 ? -3.0 / ((3 + 2 * vib_cv(p, Ttv)) * p.Z_v * tau) +
                              2 * (p.omega - 1) * (Ttv - Tv) / (3 * p.Z_v * tau * Tt) -
                              p.keff * 16 * p.sigma_R * Tv * Tv * Tv / (vib_cv(p, Tv) * rho)
                        : -3.0 / ((3 + p.d_v) * p.Z_v * tau) + 2 * (p.omega - 1) * (Ttv - Tv) / (3 * p.Z_v * tau * Tt) -
                              p.keff * 16 * p.sigma_R * Tv * Tv * Tv * 2.0 / (p.d_v * rho);
        double Dc[NW];
#pragma unroll
        for (int i = 0; i < NW; ++i) Dc[i] = 1.0 / dt + gs * iV;
        Dc[D + 2] -= jr;
        Dc[D + 3] -= jv;
        Dc[D + 4] = 1.0 / dt + gsR * iV + p.keff;
        Rc[D + 1] -= Rc[D + 4];
        double d0[NW];
        local_solve<D>(Rc, Dc, rho, Tv, p, d0);
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            st_nt(R + c * NW + i, Rc[i]);
            st_nt(Dg + c * NW + i, Dc[i]);
            st_nt(dU + c * NW + i, d0[i]);
        }
    }
    const double ws = wave_sum64(contrib);
    if (lane == 0) sh[t >> 6] = ws;
    __syncthreads();
    if (t == 0) {
        double tot = 0;
#pragma unroll
        for (int w = 0; w < kSBlk / 64; ++w) tot += sh[w];
        part[blockIdx.x] = tot;
    }
}

// One Jacobi sweep of the implicit operator (off-diagonal flux increments of the neighbours' current
// increments, halved; each slot lane forms its neighbour's term).  The first sweep of an inner iteration
// takes the stopping decision before it stores anything; the last applies the safeguarded update and
// writes the next state and its primitives into the other buffer of the ping-pong.
template <int D, int NFM, bool FIRST, bool LAST>
__global__ __launch_bounds__(kSBlk) void k_msweep(
    const double *__restrict__ W, const double *__restrict__ P, const double *__restrict__ R,
    const double *__restrict__ Dg, const double *__restrict__ Gs, const double *__restrict__ dUin,
    double *__restrict__ dUout, double *__restrict__ Wn_out, double *__restrict__ Pn_out, double *__restrict__ fn_out,
    const double *__restrict__ W0, const double *__restrict__ Ts, const MeshDev m, const Phys p,
    const double *__restrict__ part, const int npart, const int it, const double tol, double *__restrict__ scal,
    int *__restrict__ flags)
{
    constexpr int NW = D + 5, NP = D + 8, NF = D + 4, MG = 2 * D + 2, LS = slot_lanes(NFM);
    const int done = flags[0];
    double pr[kPartRegs], rest = 0;
    if constexpr (FIRST) part_load(part, npart, pr, &rest);
    constexpr int CPW = cells_per_wave(NFM);
    const int t = threadIdx.x, lane = t & 63, grp = lane / LS, s = lane - grp * LS, base = grp * LS;
    const int64_t wv = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * (kSBlk / 64) + (t >> 6);
    const int64_t c = wv * CPW + grp;
    const bool cell = grp < CPW && c < m.nc;
    const bool slot = cell && s < NFM;
    const int j = slot ? m.nbr[c * NFM + s] : INT32_MIN;
    // the point-solve data of the cell is requested now, with the neighbour index, on the lanes that
    // solve (the last sweep solves on every lane of the cell, the others on its first lane)
    const bool solver = LAST ? cell : (cell && s == 0);
    double Rc[NW], Dc[NW], Wc[NW], Ws[NW], rho = 1, Tv = 1, vol = 1, T0 = 1, T0s = 1;
    if (solver) {
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            Rc[i] = R[c * NW + i];
            Dc[i] = Dg[c * NW + i];
        }
        rho = P[c * NP];
        Tv = P[c * NP + D + 3];
        vol = m.vol[c];
        if constexpr (LAST) {
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                Wc[i] = W[c * NW + i];
                Ws[i] = W0[c * NW + i];
            }
            T0 = P[c * NP + D + 1];
            T0s = Ts[c];
        }
    }
    if (done) return;
    double x[NW], S = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) x[i] = 0;
    if (j >= 0) {
        const double *mg = m.mgeo + (c * NFM + s) * MG;
        const double *n = mg;
        S = mg[D];
        const double G = Gs[(c * NFM + s) * 2], GR = Gs[(c * NFM + s) * 2 + 1];
        double Wn[NW], F1[NW], F0[NW];
        const double *Wj = W + (int64_t)j * NW;
        const double *dj = dUin + (int64_t)j * NW;
#pragma unroll
        for (int i = 0; i < NW; ++i) Wn[i] = Wj[i] + dj[i];
        Wn[D + 1] += dj[D + 4];
        PrimL qj;
        prim_load<D>(P + (int64_t)j * NP, qj);
        euler_flux<D>(Wn, n, F1);
        euler_flux_q<D>(Wj, qj, n, F0);
#pragma unroll
        for (int i = 0; i < NW - 1; ++i) x[i] = F1[i] - F0[i] - G * dj[i];
        x[NW - 1] = -GR * dj[NW - 1];
    }
    double acc[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) acc[i] = 0;
#pragma unroll
    for (int q = 0; q < NFM; ++q) {
        const double Sq = __shfl(S, base + q, 64);
#pragma unroll
        for (int i = 0; i < NW; ++i) acc[i] += __shfl(x[i], base + q, 64) * Sq;
    }
    if constexpr (FIRST) {
        if (inner_converged(pr, rest, it, tol, scal, flags)) return;
    }
    // the last sweep runs the point solve on every lane of the cell (identical results) so that the
    // safeguard's trial factors can be spread over them; the others on the cell's first lane
    if (!solver) return;
    const double ihV = 0.5 / vol;
    double rhs[NW], d1[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) rhs[i] = Rc[i] - acc[i] * ihV;
    local_solve<D>(rhs, Dc, rho, Tv, p, d1);
    if constexpr (!LAST) {
#pragma unroll
        for (int i = 0; i < NW; ++i) st_nt(dUout + c * NW + i, d1[i]);
    } else {
        positive_update_lanes<D, LS>(Wc, d1, Ws, T0, T0s, s, base);
        if (s != 0) return;
#pragma unroll
        for (int i = 0; i < NW; ++i) st_nt(Wn_out + c * NW + i, Wc[i]);
        store_prim<D>(Wc, p, Pn_out + c * NP, fn_out + c * NF);
    }
}

// update without sweeps (in place: the kernel reads only its own cell) and the new primitives
template <int D>
__global__ __launch_bounds__(kMBlk) void k_mupdate(double *__restrict__ W, const double *__restrict__ dU,
                                                   double *__restrict__ P, double *__restrict__ fld,
                                                   const double *__restrict__ W0, const int64_t nc,
                                                   const Phys p, const double *__restrict__ part, const int npart,
                                                   const int it, const double tol, double *__restrict__ scal,
                                                   int *__restrict__ flags)
{
    constexpr int NW = D + 5, NP = D + 8, NF = D + 4;
    if (flags[0]) return;
    double pr[kPartRegs], rest;
    part_load(part, npart, pr, &rest);
    if (inner_converged(pr, rest, it, tol, scal, flags)) return;
    const int64_t c = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    double Wc[NW], d[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        Wc[i] = W[c * NW + i];
        d[i] = dU[c * NW + i];
    }
    positive_update<D>(Wc, d, W0 + c * NW);
#pragma unroll
    for (int i = 0; i < NW; ++i) W[c * NW + i] = Wc[i];
    store_prim<D>(Wc, p, P + c * NP, fld + c * NF);
}

// out[c] = V_c * x[c * stride]
__global__ void k_mass_terms(const double *__restrict__ x, const int stride, const double *__restrict__ vol,
                             double *__restrict__ out, const int64_t nc)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    out[c] = vol[c] * x[c * stride];
}

template <int D>
__global__ void k_mass_scale(double *__restrict__ W, const double *__restrict__ msum, const double *__restrict__ target,
                             const int64_t nc)
{
    constexpr int NW = D + 5;
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const double sc = target[0] / msum[0];
    for (int i = 0; i < NW - 1; ++i) W[c * NW + i] *= sc;
    W[c * NW + D + 1] -= (sc - 1.0) * W[c * NW + D + 4];
}

// Deterministic sums of k <= 8 interleaved components over n rows (in[i * k + comp]): kSumBlocks blocks
// each reduce a contiguous row range (per thread in row order, then a fixed butterfly in each wave and
// the block's waves in order) into part[comp * kSumBlocks + block]; a single wave then adds the
// partials of each component with a fixed butterfly.  Same order every run, no atomics.
__global__ __launch_bounds__(256) void k_block_sum1(const double *__restrict__ in, const int64_t n, const int k,
                                                    double *__restrict__ part)
{
    __shared__ double sh[8][4];
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk, hi = (lo + chunk < n) ? lo + chunk : n;
    const int t = threadIdx.x, w = t >> 6;
    double v[8];
#pragma unroll
    for (int comp = 0; comp < 8; ++comp) v[comp] = 0;
    for (int64_t i = lo + t; i < hi; i += 256)
#pragma unroll
        for (int comp = 0; comp < 8; ++comp)
            if (comp < k) v[comp] += in[i * k + comp];
#pragma unroll
    for (int comp = 0; comp < 8; ++comp) {
        if (comp >= k) break;
        const double ws = wave_sum64(v[comp]);
        if ((t & 63) == 0) sh[comp][w] = ws;
    }
    __syncthreads();
    if (t < k) part[t * gridDim.x + blockIdx.x] = ((sh[t][0] + sh[t][1]) + sh[t][2]) + sh[t][3];
}

__global__ __launch_bounds__(64) void k_block_sum2(const double *__restrict__ part, const int nb, const int k,
                                                   double *__restrict__ out)
{
    const int lane = threadIdx.x;
    double v[8];
#pragma unroll
    for (int comp = 0; comp < 8; ++comp) {
        v[comp] = 0;
        if (comp < k)
            for (int b = lane; b < nb; b += 64) v[comp] += part[comp * nb + b];
    }
#pragma unroll
    for (int comp = 0; comp < 8; ++comp) {
        if (comp >= k) break;
        const double s = wave_sum64(v[comp]);
        if (lane == 0) out[comp] = s;
    }
}

void launch_block_sum(const double *in, int64_t n, int k, double *out, double *part, hipStream_t st)
{
    hipLaunchKernelGGL(k_block_sum1, dim3(kSumBlocks), dim3(256), 0, st, in, n, k, part);
    hipLaunchKernelGGL(k_block_sum2, dim3(1), dim3(64), 0, st, part, kSumBlocks, k, out);
}

// B.W scaled to the total mass of the moments mom_mass (u and temperatures unchanged; e_R not scaled)
template <int D>
void rescale_mass(MacroBufs &B, const MeshDev &m, const double *mom_mass, hipStream_t st)
{
    constexpr MomLayout L{D};
    const int64_t nc = m.nc;
    const dim3 gc((nc + 255) / 256), blk(256);
    hipLaunchKernelGGL(k_mass_terms, gc, blk, 0, st, mom_mass, L.size(), m.vol, B.resc, nc);
    launch_block_sum(B.resc, nc, 1, B.scal + 3, B.bpart, st);
    hipLaunchKernelGGL(k_mass_terms, gc, blk, 0, st, B.W, D + 5, m.vol, B.resc, nc);
    launch_block_sum(B.resc, nc, 1, B.scal + 2, B.bpart, st);
    hipLaunchKernelGGL(k_mass_scale<D>, gc, blk, 0, st, B.W, B.scal + 2, B.scal + 3, nc);
}

// ------------------------------------------------------------------ driver of one macro solve
// After the inner loop: the solution of an odd inner count sits in the second buffer of the ping-pong;
// it is copied into the first, so that the host needs no count (and no wait) to find it.
template <int D>
__global__ void k_mfinal(double *__restrict__ W, double *__restrict__ P, double *__restrict__ fld,
                         const double *__restrict__ W2, const double *__restrict__ P2,
                         const double *__restrict__ fld2, const int *__restrict__ flags, const int max_inner,
                         const int64_t nc)
{
    constexpr int NW = D + 5, NP = D + 8, NF = D + 4;
    const int count = flags[0] ? flags[1] : max_inner;
    if (!(count & 1)) return;
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    for (int i = 0; i < NW; ++i) W[c * NW + i] = W2[c * NW + i];
    for (int i = 0; i < NP; ++i) P[c * NP + i] = P2[c * NP + i];
    for (int i = 0; i < NF; ++i) fld[c * NF + i] = fld2[c * NF + i];
}

int macro_count(const MacroBufs &B, int max_inner, hipStream_t st)
{
    int hf[2] = {0, 0};
    (void)hipMemcpyAsync(hf, B.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
    return hf[0] ? hf[1] : max_inner;
}

template <int D, int NFM>
void macro_solve(MacroBufs &B, const MeshDev &m, const Phys &p, const MacroOpts &o, const double *mom,
                 const double *bflux, const double *mom_mass, hipStream_t st)
{
    const int64_t nc = m.nc;
    const dim3 gc((nc + 255) / 256), gf((m.nf + 255) / 256), gb((m.nbf + 255) / 256), blk(256);
    (void)hipMemsetAsync(B.flags, 0, 2 * sizeof(int), st);
    hipLaunchKernelGGL(k_W_from_mom<D>, gc, blk, 0, st, mom, B.W, B.W0, nc, p);
    // face HoTs from the kinetic moments (mu kept in P[0..nc))
    hipLaunchKernelGGL(k_fld_from_mom<D>, gc, blk, 0, st, mom, B.fld, B.P, nc, p);
    hipLaunchKernelGGL((k_cell_grad<D, NFM>), gc, blk, 0, st, B.fld, B.gfld, m);
    hipLaunchKernelGGL(k_face_const<D>, gf, blk, 0, st, mom, B.fld, B.gfld, B.P, B.W0, B.fcon, m, p);
    if (m.nbf > 0) hipLaunchKernelGGL(k_bcorr<D>, gb, blk, 0, st, B.W0, bflux, B.bcorr, m, p);
    const dim3 gci((nc + kMBlk - 1) / kMBlk), bi(kMBlk);
    const int npart = (int)macro_nparts(nc, NFM);
    const dim3 gsl(npart), bsl(kSBlk);
    // the residual kernel that preloads the cell's state (more registers) runs while all its blocks are
    // resident at once; above that the lean variant, which fits more blocks per compute unit
    int dev = 0, ncu = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mres<D, NFM, true>, kSBlk, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const bool one_round = (int64_t)npart <= (int64_t)ncu * per_cu;
    hipLaunchKernelGGL(k_mprim<D>, gci, bi, 0, st, B.W, B.P, B.fld, B.Ts, nc, p);
    // inner iteration `it` starts from the state in buffer `it % 2` when the sweeps ping-pong
    double *Wb[2] = {B.W, B.W2}, *Pb[2] = {B.P, B.P2}, *Fb[2] = {B.fld, B.fld2};
    const bool pingpong = o.n_sweeps > 0;
    // progress polls: every `poll` iterations the flags are copied to pinned host memory behind the
    // launches; the host then waits for the previous poll's copy, which keeps at least `poll` iterations
    // queued ahead of the GPU while bounding how far the host runs ahead of a converged solve
    const int poll = 16;
    int npoll = 0;
    for (int it = 0; it < o.max_inner; ++it) {
        const int cur = pingpong ? (it & 1) : 0, nxt = cur ^ 1;
        double *W = Wb[cur], *P = Pb[cur], *fld = Fb[cur];
        if (one_round) {
            hipLaunchKernelGGL((k_mres<D, NFM, true>), gsl, bsl, 0, st, W, P, fld, B.fcon, B.bcorr, B.Gs, B.R,
                               B.Dg, B.dU0, B.part, B.flags, m, p, o.cfl_macro, nullptr);
        } else {
            // more than one round: each interior face once (half the flux evaluations, fewer registers per
            // kernel), then the per-cell sums and point solves
            hipLaunchKernelGGL((k_mface<D, NFM>), dim3((unsigned)((m.nf + 255) / 256)), dim3(256), 0, st, W, P, fld,
                               B.fcon, B.Ff, B.Gs, B.flags, m, p);
            hipLaunchKernelGGL((k_mres<D, NFM, false, true>), gsl, bsl, 0, st, W, P, fld, B.fcon, B.bcorr, B.Gs,
                               B.R, B.Dg, B.dU0, B.part, B.flags, m, p, o.cfl_macro, B.Ff);
        }
        double *din = B.dU0, *dout = B.dU1;
        const int ns = o.n_sweeps;
        for (int s = 0; s < ns; ++s) {
            const bool first = (s == 0), last = (s + 1 == ns);
            auto kern = first ? (last ? k_msweep<D, NFM, true, true> : k_msweep<D, NFM, true, false>)
                              : (last ? k_msweep<D, NFM, false, true> : k_msweep<D, NFM, false, false>);
            hipLaunchKernelGGL(kern, gsl, bsl, 0, st, W, P, B.R, B.Dg, B.Gs, din, last ? nullptr : dout,
                               last ? Wb[nxt] : nullptr, last ? Pb[nxt] : nullptr, last ? Fb[nxt] : nullptr, B.W0,
                               B.Ts, m, p, B.part, npart, it, o.inner_tol, B.scal, B.flags);
            std::swap(din, dout);
        }
        if (!pingpong)
            hipLaunchKernelGGL(k_mupdate<D>, gci, bi, 0, st, W, B.dU0, P, fld, B.W0, nc, p, B.part, npart, it,
                               o.inner_tol, B.scal, B.flags);
        if ((it + 1) % poll == 0 && it + 1 < o.max_inner) {
            const int k = npoll & 1;
            (void)hipMemcpyAsync(B.hflags + 2 * k, B.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st);
            (void)hipEventRecord(B.pev[k], st);
            ++npoll;
            if (npoll >= 2) {
                (void)hipEventSynchronize(B.pev[k ^ 1]);
                if (B.hflags[2 * (k ^ 1)]) break;
            }
        }
    }
    if (pingpong)
        hipLaunchKernelGGL(k_mfinal<D>, gc, blk, 0, st, B.W, B.P, B.fld, B.W2, B.P2, B.fld2, B.flags, o.max_inner,
                           nc);
    // reading: closed domains keep the mass of mom_mass (the state the outer iteration started from)
    if (m.closed) rescale_mass<D>(B, m, mom_mass, st);
}

template <int D>
void launch_mass_ratio(MacroBufs &B, const MeshDev &m, const double *mom_num, const double *mom_den, hipStream_t st)
{
    constexpr MomLayout L{D};
    const int64_t nc = m.nc;
    const dim3 gc((nc + 255) / 256), blk(256);
    hipLaunchKernelGGL(k_mass_terms, gc, blk, 0, st, mom_num, L.size(), m.vol, B.resc, nc);
    launch_block_sum(B.resc, nc, 1, B.scal + 3, B.bpart, st);
    hipLaunchKernelGGL(k_mass_terms, gc, blk, 0, st, mom_den, L.size(), m.vol, B.resc, nc);
    launch_block_sum(B.resc, nc, 1, B.scal + 2, B.bpart, st);
}

// ------------------------------------------------------------------ sync parameters and residual epsilon
template <int D>
__global__ void k_sync_params(const double *__restrict__ mom, const double *__restrict__ W, double *__restrict__ sp,
                              const int64_t nc, const Phys p, const int from_W)
{
    constexpr MomLayout L{D};
    constexpr int NS = D + 5, NW = D + 5;
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const double *M = mom + c * L.size();
    double *s0 = sp + c * 2 * NS, *s1 = s0 + NS;
    s0[0] = M[L.rho()];
    for (int a = 0; a < D; ++a) s0[1 + a] = M[L.u() + a];
    s0[D + 1] = M[L.Tt()];
    s0[D + 2] = M[L.Tr()];
    s0[D + 3] = M[L.Tv()];
    s0[D + 4] = M[L.eR()];
    if (from_W) {
        Prim q;
        prim_of<D>(W + c * NW, p, q);
        s1[0] = q.rho;
        for (int a = 0; a < D; ++a) s1[1 + a] = q.u[a];
        s1[D + 1] = q.Tt;
        s1[D + 2] = q.Tr;
        s1[D + 3] = q.Tv;
        s1[D + 4] = q.eR;
    }
}

template <int D>
void launch_sync_params(const double *mom, const double *W, double *sp, int64_t nc, const Phys &p, int from_W,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_sync_params<D>, dim3((nc + 255) / 256), dim3(256), 0, st, mom, W, sp, nc, p, from_W);
}

template <int D>
__global__ void k_resid_terms(const double *__restrict__ m1, const double *__restrict__ m0,
                              const double *__restrict__ vol, double *__restrict__ out, const int64_t nc, const Phys p)
{
    constexpr MomLayout L{D};
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const double *A = m1 + c * L.size(), *B = m0 + c * L.size();
    const double V = vol[c];
    double *o = out + c * 8;
    o[0] = V * (A[L.rho()] - B[L.rho()]) * (A[L.rho()] - B[L.rho()]);
    o[1] = V * B[L.rho()] * B[L.rho()];
    double nu = 0, du = 0;
    for (int a = 0; a < D; ++a) {
        nu += (A[L.u() + a] - B[L.u() + a]) * (A[L.u() + a] - B[L.u() + a]);
        du += B[L.u() + a] * B[L.u() + a];
    }
    o[2] = V * nu;
    o[3] = V * du;
    const double Tn = vib_Ttot(p, A[L.Tt()], A[L.Tr()], A[L.Tv()]);
    const double To = vib_Ttot(p, B[L.Tt()], B[L.Tr()], B[L.Tv()]);
    o[4] = V * (Tn - To) * (Tn - To);
    o[5] = V * To * To;
    o[6] = V;
    // cells of the new state that are not a physical gas state (density or a mode temperature not positive,
    // or not finite): counted, so that the driver reports divergence instead of iterating on
    const bool ok = A[L.rho()] > 0 && A[L.Tt()] > 0 && A[L.Tr()] > 0 && A[L.Tv()] > 0 && Tn < 1e300;
    o[7] = ok ? 0.0 : 1.0;
}

template <int D>
void launch_residual(const double *mom1, const double *mom0, const double *vol, double *cellbuf, double *out7,
                     double *part, int64_t nc, const Phys &p, hipStream_t st)
{
    hipLaunchKernelGGL(k_resid_terms<D>, dim3((nc + 255) / 256), dim3(256), 0, st, mom1, mom0, vol, cellbuf, nc, p);
    launch_block_sum(cellbuf, nc, 8, out7, part, st);
}

#define GSIS_INST_M(D, NFM)                                                                                      \
    template void macro_solve<D, NFM>(MacroBufs &, const MeshDev &, const Phys &, const MacroOpts &,               \
                                      const double *, const double *, const double *, hipStream_t);
GSIS_INST_M(1, 2)
GSIS_INST_M(2, 3)
GSIS_INST_M(2, 4)
GSIS_INST_M(3, 4)
GSIS_INST_M(3, 6)
template void launch_mass_ratio<1>(MacroBufs &, const MeshDev &, const double *, const double *, hipStream_t);
template void launch_mass_ratio<2>(MacroBufs &, const MeshDev &, const double *, const double *, hipStream_t);
template void launch_mass_ratio<3>(MacroBufs &, const MeshDev &, const double *, const double *, hipStream_t);
template void launch_sync_params<1>(const double *, const double *, double *, int64_t, const Phys &, int, hipStream_t);
template void launch_sync_params<2>(const double *, const double *, double *, int64_t, const Phys &, int, hipStream_t);
template void launch_sync_params<3>(const double *, const double *, double *, int64_t, const Phys &, int, hipStream_t);
template void launch_residual<1>(const double *, const double *, const double *, double *, double *, double *,
                                 int64_t, const Phys &, hipStream_t);
template void launch_residual<2>(const double *, const double *, const double *, double *, double *, double *,
                                 int64_t, const Phys &, hipStream_t);
template void launch_residual<3>(const double *, const double *, const double *, double *, double *, double *,
                                 int64_t, const Phys &, hipStream_t);

}  // namespace gsis
