// Host driver and C ABI of libgsis.so (declarations and documentation in include/gsis.h).
//
// The handle owns every device buffer.  set_mesh builds the per-cell face-slot tables (least-squares
// coefficients, normals scaled by S/V, face offsets) once on the host in FP64; set_opts allocates the
// state for the chosen precision.  One outer iteration issues: moments of f^k (reused from the previous
// iteration), per-cell coefficients, the kinetic step (gradients, wall densities, residual, Jacobi sweeps),
// and for GSIS the moments of f^{k+1/2}, its boundary flux moments, the macro solve and the
// synchronisation; then the moments of f^{k+1} and epsilon (7 doubles copied back).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <type_traits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gsis.h"
#include "../../include/gsis_warmstart.h"
#include "gsis_dev.h"
#include "gsis_kernels.h"

using namespace gsis;

namespace {

struct HostMesh {
    int D = 0;
    int64_t nc = 0, nf = 0;
    std::vector<double> vol, ctr, fn, fa, fctr;
    std::vector<int64_t> fc;
    std::vector<gsis_bc> bcs;
};

template <typename T>
T *dalloc(size_t n, bool &ok)
{
    if (n == 0) n = 1;
    void *p = nullptr;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) {
        ok = false;
        return nullptr;
    }
    return (T *)p;
}

template <typename T>
void dfree(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

}  // namespace

// residual sums per outer iteration: 7 for epsilon, then the count of cells that are not a physical gas state
constexpr int kRed = 8;

struct gsis_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    HostMesh hm;
    MeshDev m;
    std::vector<int> bf_tag;     // boundary-condition tag of each boundary face (host copy)
    std::vector<BcDev> bf_bc;    // host copy of MeshDev::bf_bc
    bool have_mesh = false, have_vel = false, have_ord = false, have_gas = false, have_flow = false;
    bool have_opts = false, have_state = false;
    bool have_init = false;  // f and I hold an initialised state (set by init_fields / set_state)
    std::vector<int64_t> col_ptr;  // cells of colour q: m.col_cells[col_ptr[q] .. col_ptr[q + 1])
    int64_t nv = 0, no = 0;
    std::vector<double> xi, w, om, wo;  // om: D components per ordinate
    gsis_gas gas{};
    gsis_flow flow{};
    Phys phys{};
    gsis_opts opts{};
    int prec = -1;
    KinBufs<float> Bf;
    KinBufs<double> Bd;
    MacroBufs Mb;
    double *mom0 = nullptr, *mom1 = nullptr, *momh = nullptr, *sp = nullptr, *cellbuf = nullptr, *red = nullptr;
    bool mom0_valid = false;
    std::vector<double> hist;
    double cnt_updates = 0, cnt_bytes = 0, cnt_seconds = 0;
    int last_inner = 0;
    // outer-iteration timing with events (start, kinetic step done, GSIS part done), read when the host
    // next waits for the stream
    struct TRec {
        hipEvent_t a, b, c;
    };
    std::vector<TRec> tpend;
    std::vector<hipEvent_t> tpool;
    double *red_h = nullptr;  // pinned host memory: the kRed residual sums of each iteration of a batch
    int64_t red_cap = 0;      // capacity in iterations
    Prof prof;
};

static int32_t fail(gsis_t *h, int32_t code, const std::string &msg)
{
    if (h) h->err = msg;
    return code;
}

#define HIPCHECK(h, call)                                                                                 \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess) return fail((h), GSIS_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------ model constants (Sec. 2.1, 2.2)
static void compute_phys(gsis_t *h)
{
    Phys &p = h->phys;
    const gsis_gas &g = h->gas;
    p.d_r = g.d_r;
    p.d_v = g.d_v;
    p.Z_r = g.Z_r;
    p.Z_v = g.Z_v;
    p.omega = g.omega;
    p.Sc = g.Sc;
    p.sigma_R = g.sigma_R;
    p.Tvref = g.Tv_ref;
    p.Kn = h->flow.Kn_gas;
    p.keff = h->flow.k_eff;
    const double dr = g.d_r, dv = g.d_v, Zr = g.Z_r, Zv = g.Z_v, Sc = g.Sc;
    double A[3][3] = {{2.0 / 3.0 + 5.0 / 6.0 * (dr / ((3 + dr) * Zr) + dv / ((3 + dv) * Zv)), -5.0 / (2 * (3 + dr) * Zr),
                       -5.0 / (2 * (3 + dv) * Zv)},
                      {-dr / ((3 + dr) * Zr), Sc + 3.0 / (2 * (3 + dr) * Zr), 0.0},
                      {-dv / ((3 + dv) * Zv), 0.0, Sc + 3.0 / (2 * (3 + dv) * Zv)}};
    const double Zi = 1.0 / (1.0 / Zr + 1.0 / Zv);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            p.A[i][j] = A[i][j];
            p.Q[i][j] = (i == j ? 1.0 : 0.0) - A[i][j] * Zi * (i == 0 ? 3.0 : 1.0);
        }
    p.Q[0][0] += 2.0 * Zi;  // (2 - 3 A_tt) Z_int + 1
    // K0 = A^{-1} diag(5, d_r, d_v)
    const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                       A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    double inv[3][3];
    inv[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
    inv[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
    inv[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
    inv[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
    inv[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
    inv[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
    inv[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
    inv[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
    inv[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
    const double dg[3] = {5.0, dr, dv};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) p.K0[i][j] = inv[i][j] * dg[j];
}

// ------------------------------------------------------------------ mesh tables
static void free_mesh(MeshDev &m)
{
    dfree(m.nbr);
    dfree(m.nb2);
    dfree(m.sfid);
    dfree(m.geo);
    dfree(m.mgeo);
    dfree(m.lsq);
    dfree(m.vol);
    dfree(m.h);
    dfree(m.eps2);
    dfree(m.nfc);
    dfree(m.bf_face);
    dfree(m.bf_cell);
    dfree(m.bf_tag);
    dfree(m.bf_n);
    dfree(m.bf_dxc);
    dfree(m.bcells);
    dfree(m.bf_bidx);
    dfree(m.f_L);
    dfree(m.f_R);
    dfree(m.fslot);
    dfree(m.fgeo);
    dfree(m.bcs);
    dfree(m.bf_bc);
    dfree(m.color);
    dfree(m.col_cells);
}

template <typename T>
static bool upload(T *&dst, const std::vector<T> &src)
{
    bool ok = true;
    dst = dalloc<T>(src.size(), ok);
    if (!ok) return false;
    if (!src.empty() && hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return false;
    return true;
}

static int32_t build_mesh(gsis_t *h)
{
    HostMesh &hm = h->hm;
    const int D = hm.D;
    const int64_t nc = hm.nc, nf = hm.nf;
    std::vector<int> cnt(nc, 0);
    for (int64_t f = 0; f < nf; ++f) {
        cnt[hm.fc[2 * f]]++;
        if (hm.fc[2 * f + 1] >= 0) cnt[hm.fc[2 * f + 1]]++;
    }
    int maxf = 0;
    for (int64_t c = 0; c < nc; ++c) maxf = std::max(maxf, cnt[c]);
    int NFM;
    if (D == 1)
        NFM = 2;
    else if (D == 2)
        NFM = (maxf <= 3) ? 3 : 4;
    else
        NFM = (maxf <= 4) ? 4 : 6;
    if (maxf > NFM) return fail(h, GSIS_E_ARG, "a cell has more faces than supported (2*dim)");
    // slots
    std::vector<int> nbr(nc * NFM, INT32_MIN), nfc(nc, 0), fid(nc * NFM, -1), sgn(nc * NFM, 0);
    std::vector<int64_t> bfidx(nf, -1);
    int64_t nbf = 0;
    std::vector<int> bf_face, bf_cell, bf_tag;
    for (int64_t f = 0; f < nf; ++f)
        if (hm.fc[2 * f + 1] < 0) {
            bfidx[f] = nbf++;
            bf_face.push_back((int)f);
            bf_cell.push_back((int)hm.fc[2 * f]);
            bf_tag.push_back((int)(-hm.fc[2 * f + 1] - 1));
        }
    for (int64_t f = 0; f < nf; ++f) {
        const int64_t L = hm.fc[2 * f], R = hm.fc[2 * f + 1];
        int s = nfc[L]++;
        fid[L * NFM + s] = (int)f;
        sgn[L * NFM + s] = 1;
        nbr[L * NFM + s] = (R >= 0) ? (int)R : -(int)(1 + bfidx[f]);
        if (R >= 0) {
            s = nfc[R]++;
            fid[R * NFM + s] = (int)f;
            sgn[R * NFM + s] = -1;
            nbr[R * NFM + s] = (int)L;
        }
    }
    std::vector<double> geo(nc * NFM * 4 * D, 0.0), mgeo(nc * NFM * (2 * D + 2), 0.0), hh(nc), eps2(nc);
    const double K = (h->have_opts ? h->opts.limiter_K : 1.0);
    for (int64_t c = 0; c < nc; ++c) {
        hh[c] = std::pow(hm.vol[c], 1.0 / D);
        eps2[c] = std::pow(K * hh[c], 3);
        // least-squares normal matrix with 1/|d|^2 weights; boundary faces add a ghost at the face centroid
        double M[9] = {0};
        for (int s = 0; s < nfc[c]; ++s) {
            const int64_t f = fid[c * NFM + s];
            const int j = nbr[c * NFM + s];
            double d[3] = {0, 0, 0}, d2 = 0;
            for (int a = 0; a < D; ++a) {
                d[a] = (j >= 0 ? hm.ctr[(int64_t)j * D + a] : hm.fctr[f * D + a]) - hm.ctr[c * D + a];
                d2 += d[a] * d[a];
            }
            for (int a = 0; a < D; ++a)
                for (int b = 0; b < D; ++b) M[a * D + b] += d[a] * d[b] / d2;
        }
        double Mi[9] = {0};
        if (D == 1) {
            Mi[0] = 1.0 / M[0];
        } else if (D == 2) {
            const double det = M[0] * M[3] - M[1] * M[2];
            Mi[0] = M[3] / det;
            Mi[1] = -M[1] / det;
            Mi[2] = -M[2] / det;
            Mi[3] = M[0] / det;
        } else {
            const double det = M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                               M[2] * (M[3] * M[7] - M[4] * M[6]);
            Mi[0] = (M[4] * M[8] - M[5] * M[7]) / det;
            Mi[1] = (M[2] * M[7] - M[1] * M[8]) / det;
            Mi[2] = (M[1] * M[5] - M[2] * M[4]) / det;
            Mi[3] = (M[5] * M[6] - M[3] * M[8]) / det;
            Mi[4] = (M[0] * M[8] - M[2] * M[6]) / det;
            Mi[5] = (M[2] * M[3] - M[0] * M[5]) / det;
            Mi[6] = (M[3] * M[7] - M[4] * M[6]) / det;
            Mi[7] = (M[1] * M[6] - M[0] * M[7]) / det;
            Mi[8] = (M[0] * M[4] - M[1] * M[3]) / det;
        }
        for (int s = 0; s < nfc[c]; ++s) {
            const int64_t f = fid[c * NFM + s];
            const int j = nbr[c * NFM + s];
            const double sg = sgn[c * NFM + s];
            const double S = hm.fa[f], V = hm.vol[c];
            double *g = &geo[(c * NFM + s) * 4 * D];
            double *mg = &mgeo[(c * NFM + s) * (2 * D + 2)];
            double d[3] = {0, 0, 0}, d2 = 0;
            for (int a = 0; a < D; ++a) {
                d[a] = (j >= 0 ? hm.ctr[(int64_t)j * D + a] : hm.fctr[f * D + a]) - hm.ctr[c * D + a];
                d2 += d[a] * d[a];
            }
            for (int a = 0; a < D; ++a) {
                const double n = sg * hm.fn[f * D + a];
                g[a] = n * S / V;
                g[D + a] = hm.fctr[f * D + a] - hm.ctr[c * D + a];
                g[2 * D + a] = (j >= 0) ? hm.fctr[f * D + a] - hm.ctr[(int64_t)j * D + a] : 0.0;
                double l = 0;
                for (int b = 0; b < D; ++b) l += Mi[a * D + b] * d[b];
                g[3 * D + a] = (j >= 0) ? l / d2 : 0.0;
                mg[a] = n;
                mg[D + 1 + a] = d[a];
            }
            mg[D] = S;
            mg[2 * D + 1] = (double)f;
        }
    }
    std::vector<double> bf_n(nbf * D), bf_dxc(nbf * D);
    std::vector<int> bcells, bf_bidx(nbf);
    {
        std::vector<int> pos(nc, -1);
        for (int64_t b = 0; b < nbf; ++b) {
            const int64_t f = bf_face[b], c = bf_cell[b];
            for (int a = 0; a < D; ++a) {
                bf_n[b * D + a] = hm.fn[f * D + a];
                bf_dxc[b * D + a] = hm.fctr[f * D + a] - hm.ctr[c * D + a];
            }
            if (pos[c] < 0) {
                pos[c] = (int)bcells.size();
                bcells.push_back((int)c);
            }
            bf_bidx[b] = pos[c];
        }
    }
    std::vector<int> fL(nf), fR(nf);
    const int FG = 2 * D + 2;
    std::vector<double> fgeo(nf * FG, 0.0);
    for (int64_t f = 0; f < nf; ++f) {
        fL[f] = (int)hm.fc[2 * f];
        fR[f] = (int)hm.fc[2 * f + 1];
        double *g = &fgeo[f * FG];
        for (int a = 0; a < D; ++a) g[a] = hm.fn[f * D + a];
        if (fR[f] >= 0) {
            double d[3] = {0, 0, 0}, dl = 0, nd = 0;
            for (int a = 0; a < D; ++a) {
                d[a] = hm.ctr[(int64_t)fR[f] * D + a] - hm.ctr[(int64_t)fL[f] * D + a];
                dl += d[a] * d[a];
                nd += g[a] * d[a];
            }
            dl = std::sqrt(dl);
            for (int a = 0; a < D; ++a) g[D + a] = d[a] / dl;
            g[2 * D] = 1.0 / dl;
            g[2 * D + 1] = 1.0 / std::fabs(nd);
        }
    }
    std::vector<BcDev> bcs(hm.bcs.size());
    int closed = 1;
    for (size_t i = 0; i < hm.bcs.size(); ++i) {
        bcs[i].kind = hm.bcs[i].kind;
        bcs[i].rho = hm.bcs[i].rho;
        bcs[i].T = hm.bcs[i].T;
        for (int a = 0; a < 3; ++a) bcs[i].u[a] = hm.bcs[i].u[a];
        bcs[i].ev = vib_e(h->phys, hm.bcs[i].T);
    }
    for (int64_t b = 0; b < nbf; ++b)
        if (hm.bcs[bf_tag[b]].kind != GSIS_BC_WALL) closed = 0;
    std::vector<BcDev> bf_bc(nbf);
    for (int64_t b = 0; b < nbf; ++b) bf_bc[b] = bcs[bf_tag[b]];
    h->bf_tag = bf_tag;
    h->bf_bc = bf_bc;
    free_mesh(h->m);
    MeshDev &m = h->m;
    m.D = D;
    m.NFM = NFM;
    m.nc = nc;
    m.nf = nf;
    m.nbf = nbf;
    m.nbcells = (int64_t)bcells.size();
    m.nbc = (int)hm.bcs.size();
    m.closed = closed;
    std::vector<int> sfid(nc * NFM, 0);
    std::vector<int> fslot(2 * nf, -1);
    for (int64_t k = 0; k < nc * NFM; ++k)
        if (fid[k] >= 0) {
            sfid[k] = (sgn[k] > 0) ? fid[k] : -(1 + fid[k]);
            if (nbr[k] >= 0) fslot[2 * (int64_t)fid[k] + (sgn[k] > 0 ? 0 : 1)] = (int)k;
        }
    // per slot (c, s) with an interior neighbour j: the slots of j (neighbour lists two cells away)
    std::vector<int> nb2(nc * NFM * NFM, INT32_MIN);
    for (int64_t k = 0; k < nc * NFM; ++k)
        if (nbr[k] >= 0)
            for (int t = 0; t < NFM; ++t) nb2[k * NFM + t] = nbr[(int64_t)nbr[k] * NFM + t];
    // Distance-1 colouring for the colored Gauss-Seidel sweeps: cells visited in index order, each takes the
    // smallest colour none of its face neighbours already holds; then the cells grouped by colour (ascending
    // cell index inside a colour).
    std::vector<int> color(nc, 0), col_cells(nc);
    int ncolor = 0;
    for (int64_t c = 0; c < nc; ++c) {
        unsigned used = 0;
        for (int s = 0; s < nfc[c]; ++s) {
            const int j = nbr[c * NFM + s];
            if (j >= 0 && j < c) used |= 1u << color[j];
        }
        int q = 0;
        while (used & (1u << q)) ++q;
        color[c] = q;
        ncolor = std::max(ncolor, q + 1);
    }
    h->col_ptr.assign(ncolor + 1, 0);
    for (int64_t c = 0; c < nc; ++c) h->col_ptr[color[c] + 1]++;
    for (int q = 0; q < ncolor; ++q) h->col_ptr[q + 1] += h->col_ptr[q];
    {
        std::vector<int64_t> pos(h->col_ptr.begin(), h->col_ptr.end() - 1);
        for (int64_t c = 0; c < nc; ++c) col_cells[pos[color[c]]++] = (int)c;
    }
    std::vector<double> lsq(nc * NFM * D);
    for (int64_t k = 0; k < nc * NFM; ++k)
        for (int a = 0; a < D; ++a) lsq[k * D + a] = geo[k * 4 * D + 3 * D + a];
    bool ok = upload(m.nbr, nbr) && upload(m.nb2, nb2) && upload(m.sfid, sfid) && upload(m.geo, geo) &&
              upload(m.mgeo, mgeo) && upload(m.lsq, lsq) && upload(m.vol, hm.vol) &&
              upload(m.h, hh) && upload(m.eps2, eps2) && upload(m.nfc, nfc) && upload(m.bf_face, bf_face) &&
              upload(m.bf_cell, bf_cell) && upload(m.bf_tag, bf_tag) && upload(m.bf_n, bf_n) &&
              upload(m.bf_dxc, bf_dxc) && upload(m.bcells, bcells) && upload(m.bf_bidx, bf_bidx) &&
              upload(m.f_L, fL) && upload(m.f_R, fR) && upload(m.fslot, fslot) &&
              upload(m.fgeo, fgeo) && upload(m.bcs, bcs) && upload(m.bf_bc, bf_bc) && upload(m.color, color) &&
              upload(m.col_cells, col_cells);
    if (!ok) return fail(h, GSIS_E_OOM, "device allocation of mesh tables failed");
    return GSIS_OK;
}

// ------------------------------------------------------------------ state buffers
template <typename T>
static void free_kin(KinBufs<T> &B)
{
    dfree(B.f);
    dfree(B.f2);
    dfree(B.gf);
    dfree(B.gfb);
    dfree(B.r);
    dfree(B.dl0);
    dfree(B.dl1);
    dfree(B.I);
    dfree(B.I2);
    dfree(B.gI);
    dfree(B.rI);
    dfree(B.dI0);
    dfree(B.dI1);
    dfree(B.coef);
    dfree(B.ccons);
    dfree(B.xi);
    dfree(B.xiT);
    dfree(B.om);
    dfree(B.rhow);
    dfree(B.xi_d);
    dfree(B.w_d);
    dfree(B.om_d);
    dfree(B.wo_d);
    dfree(B.bflux);
    dfree(B.bsurf);
}

static void free_macro(MacroBufs &B)
{
    dfree(B.W);
    dfree(B.W0);
    dfree(B.P);
    dfree(B.fld);
    dfree(B.W2);
    dfree(B.P2);
    dfree(B.fld2);
    dfree(B.Gs);
    dfree(B.Ff);
    dfree(B.part);
    dfree(B.bpart);
    dfree(B.Ts);
    dfree(B.gfld);
    dfree(B.R);
    dfree(B.Dg);
    dfree(B.dU0);
    dfree(B.dU1);
    dfree(B.fcon);
    dfree(B.bcorr);
    dfree(B.resc);
    dfree(B.scal);
    dfree(B.flags);
    if (B.hflags) (void)hipHostFree(B.hflags);
    B.hflags = nullptr;
    for (auto &e : B.pev)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
}

static int ndist(int D) { return D == 3 ? 3 : 4; }
static int coef_sz(int D) { return D + 6 + 3 * (5 + 3 * D); }

// Distribution-sized buffers beyond f and r that the options need: the stored gradient field unless the
// residual recomputes the gradients (which it does for velocity counts that fill 16-byte vectors); Jacobi
// sweeps two increment buffers (the last sweep writes f in place), no sweeps a second f; colored Gauss-Seidel
// with one symmetric sweep none (it runs in place in r), with more sweeps one increment buffer.  Buffers the
// options no longer need are released, so that switching keeps the state.
struct KinPlan {
    bool gf, dl0, dl1, f2;
};
static KinPlan kin_plan(const gsis_opts &o, int64_t nv, size_t es)
{
    const bool gf = !(o.kin_fused && nv % (int64_t)(16 / es) == 0);
    if (o.sweep == GSIS_SWEEP_SGS) return {gf, o.kin_sweeps > 1, false, false};
    return {gf, o.kin_sweeps > 0, o.kin_sweeps > 0, o.kin_sweeps == 0};
}
template <typename T>
static bool plan_kin(gsis_t *h, KinBufs<T> &B)
{
    const int D = h->hm.D, ND = ndist(D);
    const size_t nc = h->hm.nc, nv = h->nv;
    const KinPlan pl = kin_plan(h->opts, (int64_t)nv, sizeof(T));
    bool ok = true;
    auto want = [&](T *&p, bool need, size_t rows = 1) {
        if (need && !p) p = dalloc<T>(nc * ND * nv * rows, ok);
        if (!need) dfree(p);
    };
    want(B.gf, pl.gf, (size_t)D);
    want(B.dl0, pl.dl0);
    want(B.dl1, pl.dl1);
    want(B.f2, pl.f2);
    return ok;
}

template <typename T>
static bool alloc_kin(gsis_t *h, KinBufs<T> &B)
{
    const int D = h->hm.D, ND = ndist(D);
    const size_t nc = h->hm.nc, nv = h->nv, no = h->no, nbf = h->m.nbf;
    bool ok = true;
    B.f = dalloc<T>(nc * ND * nv, ok);
    B.gfb = dalloc<T>((size_t)h->m.nbcells * ND * D * nv, ok);
    B.r = dalloc<T>(nc * ND * nv, ok);
    if (ok) ok = plan_kin(h, B);
    B.I = dalloc<T>(nc * no, ok);
    B.I2 = dalloc<T>(nc * no, ok);
    B.gI = dalloc<T>(nc * D * no, ok);
    B.rI = dalloc<T>(nc * no, ok);
    B.dI0 = dalloc<T>(nc * no, ok);
    B.dI1 = dalloc<T>(nc * no, ok);
    B.coef = dalloc<T>(nc * coef_sz(D), ok);
    B.ccons = dalloc<T>(nc * 3 * 8, ok);
    B.xi = dalloc<T>(nv * D, ok);
    B.xiT = dalloc<T>(nv * D, ok);
    B.om = dalloc<T>(no * D, ok);
    B.rhow = dalloc<T>(nbf, ok);
    B.xi_d = dalloc<double>(nv * D, ok);
    B.w_d = dalloc<double>(nv, ok);
    B.om_d = dalloc<double>(no * D, ok);
    B.wo_d = dalloc<double>(no, ok);
    B.bflux = dalloc<double>(nbf * (D + 5), ok);
    B.bsurf = dalloc<double>(nbf * 3, ok);
    if (!ok) return false;
    std::vector<T> xt(h->xi.begin(), h->xi.end()), ot(h->om.begin(), h->om.end());
    (void)hipMemcpy(B.xi, xt.data(), xt.size() * sizeof(T), hipMemcpyHostToDevice);
    std::vector<T> xtT(nv * D);
    for (size_t k = 0; k < nv; ++k)
        for (int a = 0; a < D; ++a) xtT[a * nv + k] = xt[k * D + a];
    (void)hipMemcpy(B.xiT, xtT.data(), xtT.size() * sizeof(T), hipMemcpyHostToDevice);
    (void)hipMemcpy(B.om, ot.data(), ot.size() * sizeof(T), hipMemcpyHostToDevice);
    (void)hipMemcpy(B.xi_d, h->xi.data(), h->xi.size() * sizeof(double), hipMemcpyHostToDevice);
    (void)hipMemcpy(B.w_d, h->w.data(), h->w.size() * sizeof(double), hipMemcpyHostToDevice);
    (void)hipMemcpy(B.om_d, h->om.data(), h->om.size() * sizeof(double), hipMemcpyHostToDevice);
    (void)hipMemcpy(B.wo_d, h->wo.data(), h->wo.size() * sizeof(double), hipMemcpyHostToDevice);
    (void)hipMemset(B.rhow, 0, std::max<size_t>(nbf, 1) * sizeof(T));
    (void)hipMemset(B.ccons, 0, nc * 3 * 8 * sizeof(T));
    (void)hipMemset(B.bflux, 0, std::max<size_t>(nbf * (D + 5), 1) * sizeof(double));
    (void)hipMemset(B.bsurf, 0, std::max<size_t>(nbf * 3, 1) * sizeof(double));
    return true;
}

static bool alloc_macro(gsis_t *h)
{
    const int D = h->hm.D, NW = D + 5;
    const size_t nc = h->hm.nc, nf = h->hm.nf, nbf = h->m.nbf;
    bool ok = true;
    MacroBufs &B = h->Mb;
    B.W = dalloc<double>(nc * NW, ok);
    B.W0 = dalloc<double>(nc * NW, ok);
    B.P = dalloc<double>(nc * (D + 8), ok);
    B.fld = dalloc<double>(nc * (D + 4), ok);
    B.W2 = dalloc<double>(nc * NW, ok);
    B.P2 = dalloc<double>(nc * (D + 8), ok);
    B.fld2 = dalloc<double>(nc * (D + 4), ok);
    B.Gs = dalloc<double>(nc * h->m.NFM * 2, ok);
    B.Ff = dalloc<double>(nf * NW, ok);
    B.part = dalloc<double>(macro_nparts(nc, h->m.NFM) + 1, ok);
    B.gfld = dalloc<double>(nc * (D + 4) * D, ok);
    B.R = dalloc<double>(nc * NW, ok);
    B.Dg = dalloc<double>(nc * NW, ok);
    B.dU0 = dalloc<double>(nc * NW, ok);
    B.dU1 = dalloc<double>(nc * NW, ok);
    B.fcon = dalloc<double>(nf * (NW + D), ok);
    B.bcorr = dalloc<double>(nbf * NW, ok);
    B.resc = dalloc<double>(nc * 7, ok);
    B.scal = dalloc<double>(16, ok);
    B.bpart = dalloc<double>(8 * kSumBlocks, ok);
    B.Ts = dalloc<double>(nc, ok);
    B.flags = dalloc<int>(4, ok);
    if (hipHostMalloc((void **)&B.hflags, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess) ok = false;
    for (auto &e : B.pev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) ok = false;
    const MomLayout L{D};
    h->mom0 = dalloc<double>(nc * L.size(), ok);
    h->mom1 = dalloc<double>(nc * L.size(), ok);
    h->momh = dalloc<double>(nc * L.size(), ok);
    h->sp = dalloc<double>(nc * 2 * (D + 5), ok);
    h->cellbuf = dalloc<double>(nc * kRed, ok);
    h->red = dalloc<double>(16, ok);
    if (ok) {
        (void)hipMemset(B.flags, 0, 4 * sizeof(int));
        (void)hipMemset(h->mom0, 0, nc * L.size() * sizeof(double));
        (void)hipMemset(h->mom1, 0, nc * L.size() * sizeof(double));
        (void)hipMemset(h->momh, 0, nc * L.size() * sizeof(double));
    }
    return ok;
}

static void free_state(gsis_t *h)
{
    free_kin(h->Bf);
    free_kin(h->Bd);
    free_macro(h->Mb);
    dfree(h->mom0);
    dfree(h->mom1);
    dfree(h->momh);
    dfree(h->sp);
    dfree(h->cellbuf);
    dfree(h->red);
    h->have_state = false;
    h->have_init = false;
    h->mom0_valid = false;
}

// ------------------------------------------------------------------ dispatch helpers
template <typename Fn>
static void dispatch_dn(int D, int NFM, Fn &&fn)
{
    if (D == 1) fn(std::integral_constant<int, 1>{}, std::integral_constant<int, 2>{});
    else if (D == 2 && NFM == 3) fn(std::integral_constant<int, 2>{}, std::integral_constant<int, 3>{});
    else if (D == 2) fn(std::integral_constant<int, 2>{}, std::integral_constant<int, 4>{});
    else if (NFM == 4) fn(std::integral_constant<int, 3>{}, std::integral_constant<int, 4>{});
    else fn(std::integral_constant<int, 3>{}, std::integral_constant<int, 6>{});
}

static KinOpts kopts(const gsis_t *h)
{
    KinOpts o;
    o.cfl_meso = h->opts.cfl_meso;
    o.cfl_v = h->opts.cfl_v;
    o.kin_omega = h->opts.kin_omega;
    o.limK = h->opts.limiter_K;
    o.kin_sweeps = h->opts.kin_sweeps;
    o.second_order = h->opts.second_order;
    o.sweep = h->opts.sweep;
    o.fused = h->opts.kin_fused;
    o.conservative = h->opts.conservative;
    o.col_ptr = h->col_ptr.data();
    o.ncolor = (int)h->col_ptr.size() - 1;
    return o;
}

static MacroOpts mopts(const gsis_t *h)
{
    MacroOpts o;
    o.cfl_macro = h->opts.cfl_macro;
    o.inner_tol = h->opts.inner_tol;
    o.max_inner = h->opts.max_inner;
    o.n_sweeps = h->opts.n_sweeps;
    return o;
}

// moments of the current state into dst (reference velocity from uref, may be null)
template <typename T>
static void moments_T(gsis_t *h, KinBufs<T> &B, const double *uref, double *dst)
{
    const int D = h->hm.D;
    h->prof.st = h->stream;
    const int ev = h->prof.begin(4, (double)h->hm.nc * (ndist(D) * h->nv + h->no) * sizeof(T));
    struct End {
        Prof &p;
        int e;
        ~End() { p.end(e); }
    } end_{h->prof, ev};
    if (D == 1) launch_moments<T, 1>(B, uref, dst, h->hm.nc, h->nv, h->no, h->phys, h->stream);
    else if (D == 2) launch_moments<T, 2>(B, uref, dst, h->hm.nc, h->nv, h->no, h->phys, h->stream);
    else launch_moments<T, 3>(B, uref, dst, h->hm.nc, h->nv, h->no, h->phys, h->stream);
}

template <typename T>
static void prologue_T(gsis_t *h, KinBufs<T> &B, const double *mom)
{
    const int D = h->hm.D;
    if (D == 1) launch_prologue<T, 1>(mom, B.coef, h->m.h, h->hm.nc, h->phys, h->opts.cfl_meso, h->stream);
    else if (D == 2) launch_prologue<T, 2>(mom, B.coef, h->m.h, h->hm.nc, h->phys, h->opts.cfl_meso, h->stream);
    else launch_prologue<T, 3>(mom, B.coef, h->m.h, h->hm.nc, h->phys, h->opts.cfl_meso, h->stream);
    if (h->opts.conservative) {
        const int64_t nc = h->hm.nc, nv = h->nv;
        if (D == 1) launch_cons_sums<T, 1>(mom, B.coef, B.xi, B.w_d, B.ccons, nc, nv, h->phys, h->stream);
        else if (D == 2) launch_cons_sums<T, 2>(mom, B.coef, B.xi, B.w_d, B.ccons, nc, nv, h->phys, h->stream);
        else launch_cons_sums<T, 3>(mom, B.coef, B.xi, B.w_d, B.ccons, nc, nv, h->phys, h->stream);
    }
}

template <typename T>
static void kinetic_T(gsis_t *h, KinBufs<T> &B)
{
    const KinOpts o = kopts(h);
    h->prof.st = h->stream;
    dispatch_dn(h->hm.D, h->m.NFM, [&](auto Dc, auto Nc) {
        launch_kinetic<T, decltype(Dc)::value, decltype(Nc)::value>(B, h->m, h->phys, o, h->nv, h->no, h->stream,
                                                                     &h->prof);
    });
}

template <typename T>
static void boundary_T(gsis_t *h, KinBufs<T> &B)
{
    h->prof.st = h->stream;
    const int ev = h->prof.begin(5, 0.0);
    struct End {
        Prof &p;
        int e;
        ~End() { p.end(e); }
    } end_{h->prof, ev};
    dispatch_dn(h->hm.D, h->m.NFM, [&](auto Dc, auto Nc) {
        launch_boundary_state<T, decltype(Dc)::value, decltype(Nc)::value>(B, h->m, h->phys, h->opts.second_order, h->nv,
                                                                            h->no, h->stream);
    });
}

template <typename T>
static void sync_T(gsis_t *h, KinBufs<T> &B, const double *sp, int init)
{
    const int D = h->hm.D;
    h->prof.st = h->stream;
    const int ev = h->prof.begin(6, 2.0 * (double)h->hm.nc * (ndist(D) * h->nv + h->no) * sizeof(T));
    struct End {
        Prof &p;
        int e;
        ~End() { p.end(e); }
    } end_{h->prof, ev};
    if (D == 1) launch_sync<T, 1>(B, sp, h->hm.nc, h->nv, h->no, h->phys, init, h->stream);
    else if (D == 2) launch_sync<T, 2>(B, sp, h->hm.nc, h->nv, h->no, h->phys, init, h->stream);
    else launch_sync<T, 3>(B, sp, h->hm.nc, h->nv, h->no, h->phys, init, h->stream);
}

static void sync_params(gsis_t *h, const double *mom, const double *W, int from_W)
{
    const int D = h->hm.D;
    if (D == 1) launch_sync_params<1>(mom, W, h->sp, h->hm.nc, h->phys, from_W, h->stream);
    else if (D == 2) launch_sync_params<2>(mom, W, h->sp, h->hm.nc, h->phys, from_W, h->stream);
    else launch_sync_params<3>(mom, W, h->sp, h->hm.nc, h->phys, from_W, h->stream);
}

static void macro_T(gsis_t *h, const double *mom, const double *bflux, const double *mom_mass)
{
    h->prof.st = h->stream;
    const int ev = h->prof.begin(7, 0.0);
    struct End {
        Prof &p;
        int e;
        ~End() { p.end(e); }
    } end_{h->prof, ev};
    const MacroOpts o = mopts(h);
    dispatch_dn(h->hm.D, h->m.NFM, [&](auto Dc, auto Nc) {
        macro_solve<decltype(Dc)::value, decltype(Nc)::value>(h->Mb, h->m, h->phys, o, mom, bflux, mom_mass,
                                                              h->stream);
    });
}

// pinned room for the residual sums of n iterations (called with no copy into it pending)
static bool reserve_red(gsis_t *h, int64_t n)
{
    if (n <= h->red_cap) return true;
    if (h->red_h) (void)hipHostFree(h->red_h);
    h->red_h = nullptr;
    h->red_cap = 0;
    if (hipHostMalloc((void **)&h->red_h, (size_t)n * kRed * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        h->red_h = nullptr;
        return false;
    }
    h->red_cap = n;
    return true;
}

// enqueues the residual sums of (m1 against m0) and their copy into slot `slot` of the pinned buffer
static void epsilon_launch(gsis_t *h, const double *m1, const double *m0, int64_t slot)
{
    const int D = h->hm.D;
    if (D == 1) launch_residual<1>(m1, m0, h->m.vol, h->cellbuf, h->red, h->Mb.bpart, h->hm.nc, h->phys, h->stream);
    else if (D == 2) launch_residual<2>(m1, m0, h->m.vol, h->cellbuf, h->red, h->Mb.bpart, h->hm.nc,
                                         h->phys, h->stream);
    else launch_residual<3>(m1, m0, h->m.vol, h->cellbuf, h->red, h->Mb.bpart, h->hm.nc, h->phys, h->stream);
    (void)hipMemcpyAsync(h->red_h + kRed * slot, h->red, kRed * sizeof(double), hipMemcpyDeviceToHost, h->stream);
}

// epsilon from the sums of one iteration
static double epsilon_value(const double *sums)
{
    double s[7];
    for (int i = 0; i < 7; ++i) s[i] = sums[i];
    if (s[3] < s[6]) s[3] = s[6];
    double e = 0;
    for (int i = 0; i < 3; ++i) {
        const double r = std::sqrt(s[2 * i]) / std::sqrt(s[2 * i + 1]);
        if (r != r) return r;
        if (r > e) e = r;
    }
    return e;
}

// algorithmic HBM bytes of one kinetic step for the work counters: f read and written once per
// distribution and velocity (plus the same for the intensity)
static double kinetic_alg_bytes(const gsis_t *h)
{
    const double es = (h->prec == GSIS_FP32) ? 4.0 : 8.0;
    return (double)h->hm.nc * (2.0 * ndist(h->hm.D) * h->nv + 2.0 * h->no) * es;
}

static hipEvent_t tget(gsis_t *h)
{
    if (!h->tpool.empty()) {
        hipEvent_t e = h->tpool.back();
        h->tpool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// adds the timed intervals of the pending outer iterations (the stream has been synchronised)
static void tflush(gsis_t *h, double *tk, double *tm)
{
    for (auto &r : h->tpend) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            if (tk) *tk += 1e-3 * ms;
            h->cnt_seconds += 1e-3 * ms;
        }
        if (r.c && tm && hipEventElapsedTime(&ms, r.b, r.c) == hipSuccess) *tm += 1e-3 * ms;
        h->tpool.push_back(r.a);
        h->tpool.push_back(r.b);
        if (r.c) h->tpool.push_back(r.c);
    }
    h->tpend.clear();
}

// One outer iteration on storage type T, its residual sums copied into slot `slot` of the pinned buffer.
// With wait the host waits for the stream (once) and the iteration's epsilon is returned; without, the
// iteration is only enqueued (0 is returned), so that a batch of iterations runs back to back.
template <typename T>
static double iterate_T(gsis_t *h, KinBufs<T> &B, bool gsis, int *inner, double *tk, double *tm, bool wait,
                        int64_t slot = 0)
{
    const double *uref = h->mom0_valid ? h->mom0 : nullptr;
    if (!h->mom0_valid) {
        moments_T(h, B, nullptr, h->mom1);
        std::swap(h->mom0, h->mom1);
        h->mom0_valid = true;
    }
    (void)uref;
    gsis_s::TRec r{tget(h), tget(h), gsis ? tget(h) : nullptr};
    (void)hipEventRecord(r.a, h->stream);
    prologue_T(h, B, h->mom0);
    kinetic_T(h, B);
    (void)hipEventRecord(r.b, h->stream);
    h->cnt_updates += (double)h->hm.nc * h->nv;
    h->cnt_bytes += kinetic_alg_bytes(h);
    if (inner) *inner = 0;
    if (!gsis && h->m.closed) {
        // reading (closed domains, conventional iteration): the point relaxation does not conserve mass;
        // f^{k+1/2} is scaled uniformly by mass(f^k) / mass(f^{k+1/2}) (the radiation is not)
        moments_T(h, B, h->mom0, h->momh);
        dispatch_dn(h->hm.D, h->m.NFM, [&](auto Dc, auto) {
            launch_mass_ratio<decltype(Dc)::value>(h->Mb, h->m, h->mom0, h->momh, h->stream);
        });
        launch_scale<T>(B.f, (int64_t)h->hm.nc * ndist(h->hm.D) * h->nv, h->Mb.scal + 3, h->Mb.scal + 2, h->stream);
    }
    if (gsis) {
        moments_T(h, B, h->mom0, h->momh);
        boundary_T(h, B);
        macro_T(h, h->momh, B.bflux, h->mom0);
        sync_params(h, h->momh, h->Mb.W, 1);
        sync_T(h, B, h->sp, 0);
        (void)hipEventRecord(r.c, h->stream);
    }
    moments_T(h, B, h->mom0, h->mom1);
    h->tpend.push_back(r);
    epsilon_launch(h, h->mom1, h->mom0, slot);
    double e = 0;
    if (wait) {
        (void)hipStreamSynchronize(h->stream);
        e = epsilon_value(h->red_h + kRed * slot);
        tflush(h, tk, tm);
        if (gsis && inner) *inner = macro_count(h->Mb, mopts(h).max_inner, h->stream);
        h->prof.collect();
    }
    std::swap(h->mom0, h->mom1);
    return e;
}

template <typename T>
static int32_t set_state_T(gsis_t *h, KinBufs<T> &B, const double *f, const double *I)
{
    const size_t nfv = (size_t)h->hm.nc * ndist(h->hm.D) * h->nv, ni = (size_t)h->hm.nc * h->no;
    std::vector<T> tf(f, f + nfv), ti(I, I + ni);
    HIPCHECK(h, hipMemcpy(B.f, tf.data(), nfv * sizeof(T), hipMemcpyHostToDevice));
    HIPCHECK(h, hipMemcpy(B.I, ti.data(), ni * sizeof(T), hipMemcpyHostToDevice));
    return GSIS_OK;
}

template <typename T>
static int32_t get_state_T(gsis_t *h, KinBufs<T> &B, double *f, double *I)
{
    const size_t nfv = (size_t)h->hm.nc * ndist(h->hm.D) * h->nv, ni = (size_t)h->hm.nc * h->no;
    std::vector<T> tf(nfv), ti(ni);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipMemcpy(tf.data(), B.f, nfv * sizeof(T), hipMemcpyDeviceToHost));
    HIPCHECK(h, hipMemcpy(ti.data(), B.I, ni * sizeof(T), hipMemcpyDeviceToHost));
    if (f) std::copy(tf.begin(), tf.end(), f);
    if (I) std::copy(ti.begin(), ti.end(), I);
    return GSIS_OK;
}

template <typename T>
static int32_t get_state_cells_T(gsis_t *h, KinBufs<T> &B, const int64_t *cells, int64_t n, double *f, double *I)
{
    const size_t row = (size_t)ndist(h->hm.D) * h->nv, no = (size_t)h->no;
    std::vector<T> tf(f ? row : 0), ti(I ? no : 0);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    for (int64_t k = 0; k < n; ++k) {
        const size_t c = (size_t)cells[k];
        if (f) {
            HIPCHECK(h, hipMemcpy(tf.data(), B.f + c * row, row * sizeof(T), hipMemcpyDeviceToHost));
            std::copy(tf.begin(), tf.end(), f + (size_t)k * row);
        }
        if (I && no) {
            HIPCHECK(h, hipMemcpy(ti.data(), B.I + c * no, no * sizeof(T), hipMemcpyDeviceToHost));
            std::copy(ti.begin(), ti.end(), I + (size_t)k * no);
        }
    }
    return GSIS_OK;
}

// ------------------------------------------------------------------ checkpoint / restore
// File layout (native byte order): 8-byte tag "GSISCKP1"; int32 D, ND, precision, reserved; int64 nc, nv,
// no, history length; f [nc][ND][nv] and I [nc][no] in the storage type of the precision; the residual
// history (doubles).
namespace {
struct CkptHead {
    char tag[8];
    int32_t D, ND, prec, pad;
    int64_t nc, nv, no, nhist;
};
}  // namespace

template <typename T>
static int32_t checkpoint_T(gsis_t *h, KinBufs<T> &B, FILE *fp, const CkptHead &hd)
{
    const size_t nfv = (size_t)hd.nc * hd.ND * hd.nv, ni = (size_t)hd.nc * hd.no;
    std::vector<T> buf(std::max(nfv, ni));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipMemcpy(buf.data(), B.f, nfv * sizeof(T), hipMemcpyDeviceToHost));
    if (fwrite(buf.data(), sizeof(T), nfv, fp) != nfv) return fail(h, GSIS_E_ARG, "gsis_checkpoint: write failed");
    HIPCHECK(h, hipMemcpy(buf.data(), B.I, ni * sizeof(T), hipMemcpyDeviceToHost));
    if (fwrite(buf.data(), sizeof(T), ni, fp) != ni) return fail(h, GSIS_E_ARG, "gsis_checkpoint: write failed");
    return GSIS_OK;
}

template <typename T>
static int32_t restore_T(gsis_t *h, KinBufs<T> &B, FILE *fp, const CkptHead &hd)
{
    const size_t nfv = (size_t)hd.nc * hd.ND * hd.nv, ni = (size_t)hd.nc * hd.no;
    std::vector<T> buf(std::max(nfv, ni));
    if (fread(buf.data(), sizeof(T), nfv, fp) != nfv) return fail(h, GSIS_E_ARG, "gsis_restore: truncated file");
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipMemcpy(B.f, buf.data(), nfv * sizeof(T), hipMemcpyHostToDevice));
    if (fread(buf.data(), sizeof(T), ni, fp) != ni) return fail(h, GSIS_E_ARG, "gsis_restore: truncated file");
    HIPCHECK(h, hipMemcpy(B.I, buf.data(), ni * sizeof(T), hipMemcpyHostToDevice));
    return GSIS_OK;
}

// ------------------------------------------------------------------ learned warm start (device side)
// sync parameters (second slot of sp) of the predicted fields: the network outputs y_n [nc][D + 5] are
// de-standardised (y = y_n y_scale + y_mean) and read as log rho, u (D), log T_t, log T_r, log T_v, log T_R;
// resc[c] = V rho (for the mass of the prediction)
template <int D>
__global__ void k_ws_fields(const float *__restrict__ Y, const double *__restrict__ ym, const double *__restrict__ ys,
                            double *__restrict__ sp, double *__restrict__ resc, const double *__restrict__ vol,
                            const int64_t nc, const double sigR)
{
    constexpr int NO = D + 5;
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    double y[NO];
    for (int j = 0; j < NO; ++j) y[j] = (double)Y[c * NO + j] * ys[j] + ym[j];
    double *s1 = sp + c * 2 * (D + 5) + (D + 5);
    s1[0] = exp(y[0]);
    for (int a = 0; a < D; ++a) s1[1 + a] = y[1 + a];
    s1[D + 1] = exp(y[D + 1]);
    s1[D + 2] = exp(y[D + 2]);
    s1[D + 3] = exp(y[D + 3]);
    const double TR = exp(y[D + 4]);
    s1[D + 4] = 4 * sigR * TR * TR * TR * TR;
    resc[c] = vol[c] * s1[0];
}

template <int D>
__global__ void k_ws_mass(double *__restrict__ sp, const double *__restrict__ num, const double *__restrict__ den,
                          const int64_t nc)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    sp[c * 2 * (D + 5) + (D + 5)] *= num[0] / den[0];
}

template <int D>
static int32_t init_warmstart_D(gsis_t *h, gsis_mlp_t *m, const gsis_ws_norm *norm, const double *x)
{
    const int64_t nc = h->hm.nc;
    int n_in = 0, n_out = 0;
    mlp_dims(m, &n_in, &n_out);
    if (n_out != D + 5 || norm->n_in != n_in || norm->n_out != n_out)
        return fail(h, GSIS_E_ARG, "gsis_init_warmstart: the network must map n_in features to D + 5 outputs");
    for (int j = 0; j < n_in; ++j)
        if (!(norm->x_scale[j] > 0)) return fail(h, GSIS_E_ARG, "gsis_init_warmstart: non-positive input scale");
    bool ok = true;
    double *xd = dalloc<double>((size_t)nc * n_in, ok), *nd = dalloc<double>(4 * 64, ok);
    struct Guard {
        double *&a, *&b;
        ~Guard()
        {
            dfree(a);
            dfree(b);
        }
    } guard{xd, nd};
    float *X = ok ? mlp_input_rows(m, nc) : nullptr;
    if (!ok || !X) return fail(h, GSIS_E_OOM, "gsis_init_warmstart: device allocation failed");
    hipStream_t st = h->stream;
    HIPCHECK(h, hipMemcpyAsync(xd, x, (size_t)nc * n_in * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHECK(h, hipMemcpyAsync(nd, norm->x_mean, 64 * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHECK(h, hipMemcpyAsync(nd + 64, norm->x_scale, 64 * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHECK(h, hipMemcpyAsync(nd + 128, norm->y_mean, 64 * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHECK(h, hipMemcpyAsync(nd + 192, norm->y_scale, 64 * sizeof(double), hipMemcpyHostToDevice, st));
    launch_standardize(xd, nd, nd + 64, X, nc, n_in, st);
    const float *Y = mlp_forward_rows(m, nc, st);
    const dim3 g((unsigned)((nc + 255) / 256)), b(256);
    const bool rescale = h->m.closed && h->have_init;
    if (rescale) {
        // closed domain: the prediction's density is scaled to the mass of the current state (Mb.scal[3])
        if (h->prec == GSIS_FP32) moments_T(h, h->Bf, nullptr, h->momh);
        else moments_T(h, h->Bd, nullptr, h->momh);
        launch_mass_ratio<D>(h->Mb, h->m, h->momh, h->momh, st);
    }
    hipLaunchKernelGGL((k_ws_fields<D>), g, b, 0, st, Y, nd + 128, nd + 192, h->sp, h->Mb.resc, h->m.vol, nc,
                       h->gas.sigma_R);
    if (rescale) {
        launch_block_sum(h->Mb.resc, nc, 1, h->Mb.scal + 2, h->Mb.bpart, st);
        hipLaunchKernelGGL((k_ws_mass<D>), g, b, 0, st, h->sp, h->Mb.scal + 3, h->Mb.scal + 2, nc);
    }
    if (h->prec == GSIS_FP32) sync_T(h, h->Bf, h->sp, 1);
    else sync_T(h, h->Bd, h->sp, 1);
    HIPCHECK(h, hipStreamSynchronize(st));
    HIPCHECK(h, hipGetLastError());
    h->mom0_valid = false;
    h->have_init = true;
    return GSIS_OK;
}

// ================================================================== C ABI
extern "C" {

void gsis_default_opts(gsis_opts *o)
{
    if (!o) return;
    o->scheme = GSIS_GSIS;
    o->precision = GSIS_FP32;
    o->tol = 1e-6;
    o->max_outer = 1000;
    o->n_precond = 10;
    o->cfl_meso = 1e5;
    o->cfl_v = 5.0;
    o->kin_sweeps = 8;
    o->kin_omega = 1.0;
    o->limiter_K = 10.0;
    o->second_order = 1;
    o->cfl_macro = 1e3;
    o->inner_tol = 1e-7;
    o->max_inner = 100;
    o->first_order_iters = 0;
    o->n_sweeps = 2;
    o->sweep = GSIS_SWEEP_JACOBI;
    o->kin_fused = 0;
    o->conservative = 0;
}

int32_t gsis_create(int32_t device, gsis_t **out)
{
    if (!out) return GSIS_E_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return GSIS_E_DEVICE;
    if (device < 0 || device >= n) return GSIS_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return GSIS_E_DEVICE;
    gsis_t *h = new gsis_t();
    h->device = device;
    gsis_default_opts(&h->opts);
    *out = h;
    return GSIS_OK;
}

void gsis_destroy(gsis_t *h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    h->prof.destroy();
    for (auto &r : h->tpend) {
        h->tpool.push_back(r.a);
        h->tpool.push_back(r.b);
        if (r.c) h->tpool.push_back(r.c);
    }
    for (auto &ev : h->tpool) (void)hipEventDestroy(ev);
    if (h->red_h) (void)hipHostFree(h->red_h);
    free_state(h);
    free_mesh(h->m);
    delete h;
}

const char *gsis_last_error(gsis_t *h) { return h ? h->err.c_str() : "null handle"; }

int32_t gsis_set_stream(gsis_t *h, void *s)
{
    if (!h) return GSIS_E_ARG;
    h->stream = (hipStream_t)s;
    return GSIS_OK;
}

int32_t gsis_set_mesh(gsis_t *h, int32_t dim, int64_t nc, int64_t nf, const double *vol, const double *ctr,
                      const int64_t *face_cells, const double *face_n, const double *face_area, const double *face_ctr,
                      int32_t nbc, const gsis_bc *bcs)
{
    if (!h) return GSIS_E_ARG;
    if (dim < 1 || dim > 3 || nc <= 0 || nf <= 0 || nc > INT32_MAX || nf > INT32_MAX || !vol || !ctr || !face_cells ||
        !face_n || !face_area || !face_ctr || nbc < 0 || (nbc > 0 && !bcs))
        return fail(h, GSIS_E_ARG, "gsis_set_mesh: invalid sizes or null arrays");
    for (int64_t f = 0; f < nf; ++f) {
        const int64_t L = face_cells[2 * f], R = face_cells[2 * f + 1];
        if (L < 0 || L >= nc || R >= nc || (R < 0 && -R - 1 >= nbc))
            return fail(h, GSIS_E_ARG, "gsis_set_mesh: face_cells out of range or unknown boundary tag");
        if (!(face_area[f] > 0)) return fail(h, GSIS_E_ARG, "gsis_set_mesh: non-positive face area");
    }
    for (int64_t c = 0; c < nc; ++c)
        if (!(vol[c] > 0)) return fail(h, GSIS_E_ARG, "gsis_set_mesh: non-positive cell volume");
    for (int b = 0; b < nbc; ++b)
        if (bcs[b].kind != GSIS_BC_WALL && bcs[b].kind != GSIS_BC_FARFIELD)
            return fail(h, GSIS_E_ARG, "gsis_set_mesh: unknown boundary kind");
    (void)hipSetDevice(h->device);
    free_state(h);
    HostMesh &hm = h->hm;
    hm.D = dim;
    hm.nc = nc;
    hm.nf = nf;
    hm.vol.assign(vol, vol + nc);
    hm.ctr.assign(ctr, ctr + nc * dim);
    hm.fc.assign(face_cells, face_cells + 2 * nf);
    hm.fn.assign(face_n, face_n + nf * dim);
    hm.fa.assign(face_area, face_area + nf);
    hm.fctr.assign(face_ctr, face_ctr + nf * dim);
    hm.bcs.assign(bcs, bcs + nbc);
    const int32_t rc = build_mesh(h);
    h->have_mesh = (rc == GSIS_OK);
    h->have_opts = false;
    return rc;
}

int32_t gsis_set_boundary(gsis_t *h, int32_t tag, const gsis_bc *bc)
{
    if (!h || !bc) return GSIS_E_ARG;
    if (!h->have_mesh) return fail(h, GSIS_E_STATE, "gsis_set_boundary: call gsis_set_mesh first");
    if (tag < 0 || tag >= (int32_t)h->hm.bcs.size() || bc->kind != h->hm.bcs[tag].kind || !(bc->T > 0) ||
        !(bc->rho > 0))
        return fail(h, GSIS_E_ARG, "gsis_set_boundary: bad tag, kind change or non-positive state");
    h->hm.bcs[tag] = *bc;
    if (h->m.bcs) {
        BcDev d;
        d.kind = bc->kind;
        d.rho = bc->rho;
        d.T = bc->T;
        for (int a = 0; a < 3; ++a) d.u[a] = bc->u[a];
        d.ev = vib_e(h->phys, bc->T);
        (void)hipSetDevice(h->device);
        HIPCHECK(h, hipStreamSynchronize(h->stream));
        HIPCHECK(h, hipMemcpy(h->m.bcs + tag, &d, sizeof(BcDev), hipMemcpyHostToDevice));
        for (size_t b = 0; b < h->bf_tag.size(); ++b)
            if (h->bf_tag[b] == tag) h->bf_bc[b] = d;
        if (!h->bf_bc.empty())
            HIPCHECK(h, hipMemcpy(h->m.bf_bc, h->bf_bc.data(), h->bf_bc.size() * sizeof(BcDev),
                                  hipMemcpyHostToDevice));
    }
    return GSIS_OK;
}

int32_t gsis_set_velocity_grid(gsis_t *h, int64_t nv, const double *xi, const double *w)
{
    if (!h) return GSIS_E_ARG;
    if (!h->have_mesh) return fail(h, GSIS_E_STATE, "gsis_set_velocity_grid: set the mesh first");
    if (nv <= 0 || !xi || !w) return fail(h, GSIS_E_ARG, "gsis_set_velocity_grid: invalid arguments");
    free_state(h);
    h->nv = nv;
    h->xi.assign(xi, xi + nv * h->hm.D);
    h->w.assign(w, w + nv);
    h->have_vel = true;
    h->have_opts = false;
    return GSIS_OK;
}

int32_t gsis_set_ordinates(gsis_t *h, int64_t no, const double *omega, const double *w)
{
    if (!h) return GSIS_E_ARG;
    if (!h->have_mesh) return fail(h, GSIS_E_STATE, "gsis_set_ordinates: set the mesh first");
    if (no <= 0 || !omega || !w) return fail(h, GSIS_E_ARG, "gsis_set_ordinates: invalid arguments");
    free_state(h);
    const int D = h->hm.D;
    h->no = no;
    h->om.resize(no * D);
    for (int64_t q = 0; q < no; ++q)
        for (int a = 0; a < D; ++a) h->om[q * D + a] = omega[q * 3 + a];
    h->wo.assign(w, w + no);
    h->have_ord = true;
    h->have_opts = false;
    return GSIS_OK;
}

int32_t gsis_set_gas(gsis_t *h, const gsis_gas *gas)
{
    if (!h || !gas) return GSIS_E_ARG;
    if (!(gas->d_r > 0 && gas->d_v > 0 && gas->Z_r > 0 && gas->Z_v > 0 && gas->sigma_R >= 0 && gas->Tv_ref >= 0))
        return fail(h, GSIS_E_ARG, "gsis_set_gas: invalid gas constants");
    h->gas = *gas;
    h->have_gas = true;
    if (h->have_flow) compute_phys(h);
    // boundary states carry e_v(T) of the gas: refresh them when the mesh tables exist already
    if (h->m.bcs && h->have_flow) {
        (void)hipSetDevice(h->device);
        HIPCHECK(h, hipStreamSynchronize(h->stream));
        std::vector<BcDev> bcs(h->hm.bcs.size());
        HIPCHECK(h, hipMemcpy(bcs.data(), h->m.bcs, bcs.size() * sizeof(BcDev), hipMemcpyDeviceToHost));
        for (auto &b : bcs) b.ev = vib_e(h->phys, b.T);
        for (auto &b : h->bf_bc) b.ev = vib_e(h->phys, b.T);
        HIPCHECK(h, hipMemcpy(h->m.bcs, bcs.data(), bcs.size() * sizeof(BcDev), hipMemcpyHostToDevice));
        if (!h->bf_bc.empty())
            HIPCHECK(h, hipMemcpy(h->m.bf_bc, h->bf_bc.data(), h->bf_bc.size() * sizeof(BcDev),
                                  hipMemcpyHostToDevice));
    }
    return GSIS_OK;
}

int32_t gsis_set_flow(gsis_t *h, const gsis_flow *flow)
{
    if (!h || !flow) return GSIS_E_ARG;
    if (!(flow->Kn_gas > 0 && flow->k_eff >= 0)) return fail(h, GSIS_E_ARG, "gsis_set_flow: invalid Kn or k_eff");
    h->flow = *flow;
    h->have_flow = true;
    if (h->have_gas) compute_phys(h);
    return GSIS_OK;
}

int32_t gsis_set_opts(gsis_t *h, const gsis_opts *o)
{
    if (!h || !o) return GSIS_E_ARG;
    if (!(h->have_mesh && h->have_vel && h->have_ord && h->have_gas && h->have_flow))
        return fail(h, GSIS_E_STATE, "gsis_set_opts: mesh, grids, gas and flow must be set first");
    if ((o->precision != GSIS_FP32 && o->precision != GSIS_FP64) || (o->scheme != GSIS_CIS && o->scheme != GSIS_GSIS) ||
        o->kin_sweeps < 0 || o->max_inner < 0 || o->max_outer < 0 || o->n_precond < 0 || o->n_sweeps < 0 ||
        o->first_order_iters < 0 || (o->second_order != 0 && o->second_order != 1) || !(o->tol >= 0) ||
        !(o->inner_tol >= 0) || !(o->limiter_K > 0) || !(o->kin_omega > 0) || !(o->cfl_v > 0) ||
        !(o->cfl_meso > 0) || !(o->cfl_macro > 0) || (o->sweep != GSIS_SWEEP_JACOBI && o->sweep != GSIS_SWEEP_SGS) ||
        (o->kin_fused != 0 && o->kin_fused != 1) || (o->conservative != 0 && o->conservative != 1))
        return fail(h, GSIS_E_ARG, "gsis_set_opts: invalid options");
    // the kinetic kernels index waves over (cell, 64-velocity chunk) pairs with 32-bit integers
    if (h->hm.nc * ((h->nv + 63) / 64 + 1) > (int64_t)(INT32_MAX / 8))
        return fail(h, GSIS_E_ARG, "gsis_set_opts: mesh x velocity grid too large for one device");
    (void)hipSetDevice(h->device);
    // a new precision reallocates the state (which must then be initialised again); other changes keep it
    const bool realloc = !h->have_state || o->precision != h->prec;
    const bool newK = !realloc && o->limiter_K != h->opts.limiter_K;
    h->opts = *o;
    h->have_opts = true;
    if (realloc) {
        free_state(h);
        int32_t rc = build_mesh(h);  // limiter epsilon depends on K
        if (rc != GSIS_OK) return rc;
        h->prec = o->precision;
        bool ok = (h->prec == GSIS_FP32) ? alloc_kin(h, h->Bf) : alloc_kin(h, h->Bd);
        ok = ok && alloc_macro(h);
        if (!ok) {
            free_state(h);
            return fail(h, GSIS_E_OOM, "gsis_set_opts: device allocation failed");
        }
        h->have_state = true;
        return GSIS_OK;
    }
    if (newK) {
        std::vector<double> eps2(h->hm.nc);
        for (int64_t c = 0; c < h->hm.nc; ++c)
            eps2[c] = std::pow(o->limiter_K * std::pow(h->hm.vol[c], 1.0 / h->hm.D), 3);
        HIPCHECK(h, hipStreamSynchronize(h->stream));
        HIPCHECK(h, hipMemcpy(h->m.eps2, eps2.data(), eps2.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    const bool ok = (h->prec == GSIS_FP32) ? plan_kin(h, h->Bf) : plan_kin(h, h->Bd);
    if (!ok) return fail(h, GSIS_E_OOM, "gsis_set_opts: device allocation of the relaxation buffers failed");
    return GSIS_OK;
}

int32_t gsis_init_fields(gsis_t *h, const double *rho, const double *u, const double *Tt, const double *Tr,
                         const double *Tv, const double *TR)
{
    if (!h || !rho || !u || !Tt || !Tr || !Tv || !TR) return GSIS_E_ARG;
    if (!h->have_state) return fail(h, GSIS_E_STATE, "gsis_init_fields: call gsis_set_opts first");
    const int D = h->hm.D;
    const int64_t nc = h->hm.nc;
    std::vector<double> sp(nc * 2 * (D + 5), 0.0);
    for (int64_t c = 0; c < nc; ++c) {
        if (!(rho[c] > 0 && Tt[c] > 0 && Tr[c] > 0 && Tv[c] > 0 && TR[c] > 0))
            return fail(h, GSIS_E_ARG, "gsis_init_fields: non-positive density or temperature");
        double *s1 = &sp[c * 2 * (D + 5) + (D + 5)];
        s1[0] = rho[c];
        for (int a = 0; a < D; ++a) s1[1 + a] = u[c * D + a];
        s1[D + 1] = Tt[c];
        s1[D + 2] = Tr[c];
        s1[D + 3] = Tv[c];
        s1[D + 4] = 4 * h->gas.sigma_R * std::pow(TR[c], 4);
    }
    (void)hipSetDevice(h->device);
    HIPCHECK(h, hipMemcpy(h->sp, sp.data(), sp.size() * sizeof(double), hipMemcpyHostToDevice));
    if (h->prec == GSIS_FP32) sync_T(h, h->Bf, h->sp, 1);
    else sync_T(h, h->Bd, h->sp, 1);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    h->mom0_valid = false;
    h->have_init = true;
    return GSIS_OK;
}

int32_t gsis_init_equilibrium(gsis_t *h, const double *rho, const double *u, const double *T)
{
    return gsis_init_fields(h, rho, u, T, T, T, T);
}

int32_t gsis_set_state(gsis_t *h, const double *f, const double *I)
{
    if (!h || !f || !I) return GSIS_E_ARG;
    if (!h->have_state) return fail(h, GSIS_E_STATE, "gsis_set_state: call gsis_set_opts first");
    (void)hipSetDevice(h->device);
    h->mom0_valid = false;
    const int32_t rc = (h->prec == GSIS_FP32) ? set_state_T(h, h->Bf, f, I) : set_state_T(h, h->Bd, f, I);
    if (rc == GSIS_OK) h->have_init = true;
    return rc;
}

int32_t gsis_get_state(gsis_t *h, double *f, double *I)
{
    if (!h) return GSIS_E_ARG;
    if (!h->have_state || !h->have_init) return fail(h, GSIS_E_STATE, "gsis_get_state: no initialised state");
    (void)hipSetDevice(h->device);
    return (h->prec == GSIS_FP32) ? get_state_T(h, h->Bf, f, I) : get_state_T(h, h->Bd, f, I);
}

int32_t gsis_get_state_cells(gsis_t *h, const int64_t *cells, int64_t n, double *f, double *I)
{
    if (!h) return GSIS_E_ARG;
    if (n < 0 || (n > 0 && !cells)) return fail(h, GSIS_E_ARG, "gsis_get_state_cells: bad cell list");
    for (int64_t k = 0; k < n; ++k)
        if (cells[k] < 0 || cells[k] >= h->hm.nc)
            return fail(h, GSIS_E_ARG, "gsis_get_state_cells: cell index out of range");
    if (!h->have_state || !h->have_init) return fail(h, GSIS_E_STATE, "gsis_get_state_cells: no initialised state");
    (void)hipSetDevice(h->device);
    return (h->prec == GSIS_FP32) ? get_state_cells_T(h, h->Bf, cells, n, f, I)
                                  : get_state_cells_T(h, h->Bd, cells, n, f, I);
}

static int32_t check_ready(gsis_t *h, const char *who)
{
    if (!h) return GSIS_E_ARG;
    if (!h->have_state || !h->have_init)
        return fail(h, GSIS_E_STATE, std::string(who) + ": call gsis_set_opts and initialise the state first");
    (void)hipSetDevice(h->device);
    return GSIS_OK;
}

int32_t gsis_checkpoint(gsis_t *h, const char *path)
{
    int32_t rc = check_ready(h, "gsis_checkpoint");
    if (rc) return rc;
    if (!path) return fail(h, GSIS_E_ARG, "gsis_checkpoint: null path");
    CkptHead hd{};
    memcpy(hd.tag, "GSISCKP1", 8);
    hd.D = h->hm.D;
    hd.ND = ndist(hd.D);
    hd.prec = h->prec;
    hd.nc = h->hm.nc;
    hd.nv = h->nv;
    hd.no = h->no;
    hd.nhist = (int64_t)h->hist.size();
    FILE *fp = fopen(path, "wb");
    if (!fp) return fail(h, GSIS_E_ARG, std::string("gsis_checkpoint: cannot open ") + path);
    rc = (fwrite(&hd, sizeof(hd), 1, fp) == 1) ? GSIS_OK : fail(h, GSIS_E_ARG, "gsis_checkpoint: write failed");
    if (rc == GSIS_OK) rc = (h->prec == GSIS_FP32) ? checkpoint_T(h, h->Bf, fp, hd) : checkpoint_T(h, h->Bd, fp, hd);
    if (rc == GSIS_OK && hd.nhist > 0 && fwrite(h->hist.data(), sizeof(double), hd.nhist, fp) != (size_t)hd.nhist)
        rc = fail(h, GSIS_E_ARG, "gsis_checkpoint: write failed");
    if (fclose(fp) != 0 && rc == GSIS_OK) rc = fail(h, GSIS_E_ARG, "gsis_checkpoint: close failed");
    return rc;
}

int32_t gsis_restore(gsis_t *h, const char *path)
{
    if (!h || !path) return GSIS_E_ARG;
    if (!h->have_state) return fail(h, GSIS_E_STATE, "gsis_restore: call gsis_set_opts first");
    (void)hipSetDevice(h->device);
    FILE *fp = fopen(path, "rb");
    if (!fp) return fail(h, GSIS_E_ARG, std::string("gsis_restore: cannot open ") + path);
    CkptHead hd{};
    int32_t rc = GSIS_OK;
    if (fread(&hd, sizeof(hd), 1, fp) != 1 || memcmp(hd.tag, "GSISCKP1", 8) != 0)
        rc = fail(h, GSIS_E_ARG, "gsis_restore: not a checkpoint file");
    else if (hd.D != h->hm.D || hd.nc != h->hm.nc || hd.nv != h->nv || hd.no != h->no || hd.prec != h->prec ||
             hd.nhist < 0)
        rc = fail(h, GSIS_E_ARG, "gsis_restore: mesh, grids or precision differ from the checkpoint");
    if (rc == GSIS_OK) rc = (h->prec == GSIS_FP32) ? restore_T(h, h->Bf, fp, hd) : restore_T(h, h->Bd, fp, hd);
    std::vector<double> hist(hd.nhist > 0 ? hd.nhist : 0);
    if (rc == GSIS_OK && hd.nhist > 0 && fread(hist.data(), sizeof(double), hd.nhist, fp) != (size_t)hd.nhist)
        rc = fail(h, GSIS_E_ARG, "gsis_restore: truncated file");
    fclose(fp);
    if (rc != GSIS_OK) return rc;
    h->hist = hist;
    h->mom0_valid = false;
    h->have_init = true;
    return GSIS_OK;
}

int32_t gsis_iterate(gsis_t *h, int32_t scheme, int32_t n, double *eps, int32_t *inner)
{
    int32_t rc = check_ready(h, "gsis_iterate");
    if (rc) return rc;
    if (n < 0 || (scheme != GSIS_CIS && scheme != GSIS_GSIS)) return fail(h, GSIS_E_ARG, "gsis_iterate: invalid args");
    double e = 0;
    int in = 0;
    // the batch runs back to back: every iteration computes its residual, only the last waits
    if (!reserve_red(h, n)) return fail(h, GSIS_E_OOM, "gsis_iterate: pinned host allocation failed");
    for (int k = 0; k < n; ++k) {
        const bool wait = (k + 1 == n);
        e = (h->prec == GSIS_FP32) ? iterate_T(h, h->Bf, scheme == GSIS_GSIS, &in, nullptr, nullptr, wait, k)
                                   : iterate_T(h, h->Bd, scheme == GSIS_GSIS, &in, nullptr, nullptr, wait, k);
    }
    for (int k = 0; k + 1 < n; ++k) {
        const double ek = epsilon_value(h->red_h + kRed * k);
        if (ek != ek) {
            e = ek;
            break;
        }
    }
    int64_t bad = 0, bad_it = -1;
    for (int k = 0; k < n && bad_it < 0; ++k)
        if (h->red_h[kRed * k + 7] > 0) bad = (int64_t)h->red_h[kRed * k + 7], bad_it = k;
    hipError_t herr = hipGetLastError();
    if (herr != hipSuccess) return fail(h, GSIS_E_DEVICE, std::string("gsis_iterate: ") + hipGetErrorString(herr));
    if (eps) *eps = e;
    if (inner) *inner = in;
    h->last_inner = in;
    if (bad > 0)
        return fail(h, GSIS_E_DIVERGED, "gsis_iterate: non-positive density or temperature in " + std::to_string(bad) +
                                            " cells after iteration " + std::to_string(bad_it + 1) + " of the batch");
    if (e != e) return fail(h, GSIS_E_DIVERGED, "gsis_iterate: NaN residual");
    return GSIS_OK;
}

int32_t gsis_solve(gsis_t *h, gsis_report *rep)
{
    int32_t rc = check_ready(h, "gsis_solve");
    if (rc) return rc;
    if (!reserve_red(h, 1)) return fail(h, GSIS_E_OOM, "gsis_solve: pinned host allocation failed");
    h->hist.clear();
    double tk = 0, tm = 0, e = 0;
    int64_t inner_total = 0;
    int k = 0;
    int32_t status = GSIS_W_NOT_CONVERGED;
    double emin = INFINITY;
    std::string why;
    auto t0 = std::chrono::steady_clock::now();
    const int32_t so_user = h->opts.second_order;
    for (k = 0; k < h->opts.max_outer; ++k) {
        const bool g = (h->opts.scheme == GSIS_GSIS) && k >= h->opts.n_precond;
        h->opts.second_order = (k < h->opts.first_order_iters) ? 0 : so_user;
        int in = 0;
        e = (h->prec == GSIS_FP32) ? iterate_T(h, h->Bf, g, &in, &tk, &tm, true)
                                   : iterate_T(h, h->Bd, g, &in, &tk, &tm, true);
        inner_total += in;
        h->hist.push_back(e);
        const double nbad = h->red_h[7];
        // divergence: NaN, a state that is no gas state, or a residual that has grown by 1e3 over the smallest
        // one of this solve and exceeds 1 (the relative change of the fields per iteration)
        if (e != e || nbad > 0 || (e > 1.0 && e > 1e3 * emin)) {
            status = GSIS_E_DIVERGED;
            why = (e != e) ? "NaN residual"
                           : (nbad > 0 ? "non-positive density or temperature in " + std::to_string((int64_t)nbad) + " cells"
                                       : "residual grew above 1e3 times its smallest value");
            ++k;
            break;
        }
        emin = std::min(emin, e);
        if (e < h->opts.tol) {
            status = GSIS_OK;
            ++k;
            break;
        }
    }
    h->opts.second_order = so_user;
    const double tt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    hipError_t herr = hipGetLastError();
    if (herr != hipSuccess) return fail(h, GSIS_E_DEVICE, std::string("gsis_solve: ") + hipGetErrorString(herr));
    if (rep) {
        rep->iters = k;
        rep->status = status;
        rep->eps_final = e;
        rep->t_total_s = tt;
        rep->t_kinetic_s = tk;
        rep->t_macro_s = tm;
        rep->t_other_s = tt - tk - tm;
        rep->inner_total = inner_total;
    }
    if (status == GSIS_E_DIVERGED)
        return fail(h, GSIS_E_DIVERGED, "gsis_solve: " + why + " at iteration " + std::to_string(k));
    return status;
}

int32_t gsis_kinetic_step(gsis_t *h)
{
    int32_t rc = check_ready(h, "gsis_kinetic_step");
    if (rc) return rc;
    auto run = [&](auto &B) {
        moments_T(h, B, nullptr, h->mom0);
        prologue_T(h, B, h->mom0);
        kinetic_T(h, B);
    };
    if (h->prec == GSIS_FP32) run(h->Bf);
    else run(h->Bd);
    h->mom0_valid = false;
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipGetLastError());
    return GSIS_OK;
}

int32_t gsis_macro_solve(gsis_t *h, double *W, int32_t *inner)
{
    int32_t rc = check_ready(h, "gsis_macro_solve");
    if (rc) return rc;
    int it = 0;
    auto run = [&](auto &B) {
        moments_T(h, B, nullptr, h->momh);
        boundary_T(h, B);
        macro_T(h, h->momh, B.bflux, h->momh);
    };
    if (h->prec == GSIS_FP32) run(h->Bf);
    else run(h->Bd);
    it = macro_count(h->Mb, mopts(h).max_inner, h->stream);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipGetLastError());
    if (W) HIPCHECK(h, hipMemcpy(W, h->Mb.W, (size_t)h->hm.nc * (h->hm.D + 5) * sizeof(double), hipMemcpyDeviceToHost));
    if (inner) *inner = it;
    return GSIS_OK;
}

int32_t gsis_sync(gsis_t *h, const double *W)
{
    int32_t rc = check_ready(h, "gsis_sync");
    if (rc) return rc;
    if (!W) return GSIS_E_ARG;
    HIPCHECK(h, hipMemcpy(h->Mb.W, W, (size_t)h->hm.nc * (h->hm.D + 5) * sizeof(double), hipMemcpyHostToDevice));
    auto run = [&](auto &B) {
        moments_T(h, B, nullptr, h->momh);
        sync_params(h, h->momh, h->Mb.W, 1);
        sync_T(h, B, h->sp, 0);
    };
    if (h->prec == GSIS_FP32) run(h->Bf);
    else run(h->Bd);
    h->mom0_valid = false;
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipGetLastError());
    return GSIS_OK;
}

int32_t gsis_nfields(gsis_t *h)
{
    if (!h || !h->have_mesh) return 0;
    const int D = h->hm.D;
    return 1 + D + 5 + 4 * D + D * (D + 1) / 2;
}

int32_t gsis_get_fields(gsis_t *h, double *out)
{
    int32_t rc = check_ready(h, "gsis_get_fields");
    if (rc) return rc;
    if (!out) return GSIS_E_ARG;
    const int D = h->hm.D;
    const MomLayout L{D};
    const int64_t nc = h->hm.nc;
    if (h->prec == GSIS_FP32) moments_T(h, h->Bf, nullptr, h->momh);
    else moments_T(h, h->Bd, nullptr, h->momh);
    std::vector<double> M(nc * L.size());
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipMemcpy(M.data(), h->momh, M.size() * sizeof(double), hipMemcpyDeviceToHost));
    const int nfl = gsis_nfields(h);
    const gsis_gas &g = h->gas;
    for (int64_t c = 0; c < nc; ++c) {
        const double *m = &M[c * L.size()];
        double *o = out + c * nfl;
        int p = 0;
        o[p++] = m[L.rho()];
        for (int a = 0; a < D; ++a) o[p++] = m[L.u() + a];
        o[p++] = m[L.Tt()];
        o[p++] = m[L.Tr()];
        o[p++] = m[L.Tv()];
        o[p++] = (g.sigma_R > 0) ? std::pow(m[L.eR()] / (4 * g.sigma_R), 0.25) : 0.0;
        o[p++] = vib_Ttot(h->phys, m[L.Tt()], m[L.Tr()], m[L.Tv()]);
        for (int a = 0; a < D; ++a) o[p++] = m[L.qt() + a];
        for (int a = 0; a < D; ++a) o[p++] = m[L.qr() + a];
        for (int a = 0; a < D; ++a) o[p++] = m[L.qv() + a];
        for (int a = 0; a < D; ++a) o[p++] = m[L.qR() + a];
        for (int a = 0; a < D; ++a)
            for (int b = a; b < D; ++b) o[p++] = m[L.sig() + a * D + b];
    }
    return GSIS_OK;
}

int32_t gsis_get_residual_history(gsis_t *h, double *buf, int64_t cap, int64_t *n)
{
    if (!h) return GSIS_E_ARG;
    const int64_t k = (int64_t)h->hist.size();
    if (n) *n = k;
    if (buf)
        for (int64_t i = 0; i < k && i < cap; ++i) buf[i] = h->hist[i];
    return GSIS_OK;
}

int32_t gsis_get_surface_flux(gsis_t *h, double *q_conv, double *q_rad, double *p_w)
{
    int32_t rc = check_ready(h, "gsis_get_surface_flux");
    if (rc) return rc;
    const int64_t nbf = h->m.nbf, nf = h->hm.nf;
    if (h->prec == GSIS_FP32) boundary_T(h, h->Bf);
    else boundary_T(h, h->Bd);
    std::vector<double> bs(nbf * 3);
    std::vector<int> bface(nbf);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    const double *src = (h->prec == GSIS_FP32) ? h->Bf.bsurf : h->Bd.bsurf;
    if (nbf > 0) {
        HIPCHECK(h, hipMemcpy(bs.data(), src, bs.size() * sizeof(double), hipMemcpyDeviceToHost));
        HIPCHECK(h, hipMemcpy(bface.data(), h->m.bf_face, nbf * sizeof(int), hipMemcpyDeviceToHost));
    }
    for (int64_t f = 0; f < nf; ++f) {
        if (q_conv) q_conv[f] = 0;
        if (q_rad) q_rad[f] = 0;
        if (p_w) p_w[f] = 0;
    }
    for (int64_t b = 0; b < nbf; ++b) {
        if (q_conv) q_conv[bface[b]] = bs[b * 3 + 0];
        if (q_rad) q_rad[bface[b]] = bs[b * 3 + 1];
        if (p_w) p_w[bface[b]] = bs[b * 3 + 2];
    }
    return GSIS_OK;
}

int32_t gsis_set_profiling(gsis_t *h, int32_t on)
{
    if (!h) return GSIS_E_ARG;
    h->prof.st = h->stream;
    h->prof.reset();
    h->prof.on = (on != 0);
    h->prof.mask = (on & GSIS_PROF_SELECT) ? (unsigned)(on & 0xff) : 0xffu;
    return GSIS_OK;
}

int32_t gsis_get_kernel_stats(gsis_t *h, int32_t kind, double *ms_total, int64_t *launches, double *bytes_total)
{
    if (!h || kind < 0 || kind >= Prof::kKinds) return GSIS_E_ARG;
    h->prof.collect();
    if (ms_total) *ms_total = h->prof.ms[kind];
    if (launches) *launches = h->prof.n[kind];
    if (bytes_total) *bytes_total = h->prof.bytes[kind];
    return GSIS_OK;
}

int32_t gsis_get_counters(gsis_t *h, double *cellvel_updates, double *kinetic_bytes, double *kinetic_seconds)
{
    if (!h) return GSIS_E_ARG;
    if (cellvel_updates) *cellvel_updates = h->cnt_updates;
    if (kinetic_bytes) *kinetic_bytes = h->cnt_bytes;
    if (kinetic_seconds) *kinetic_seconds = h->cnt_seconds;
    h->cnt_updates = h->cnt_bytes = h->cnt_seconds = 0;
    return GSIS_OK;
}


int32_t gsis_init_warmstart(gsis_t *h, gsis_mlp_t *m, const gsis_ws_norm *norm, const double *x)
{
    if (!h || !m || !norm || !x) return GSIS_E_ARG;
    if (!h->have_state) return fail(h, GSIS_E_STATE, "gsis_init_warmstart: call gsis_set_opts first");
    (void)hipSetDevice(h->device);
    if (h->hm.D == 1) return init_warmstart_D<1>(h, m, norm, x);
    if (h->hm.D == 2) return init_warmstart_D<2>(h, m, norm, x);
    return init_warmstart_D<3>(h, m, norm, x);
}

int32_t gsis_ws_targets(gsis_t *h, double *t)
{
    if (!h || !t) return GSIS_E_ARG;
    const int D = h->hm.D, nf = gsis_nfields(h);
    if (nf <= 0) return fail(h, GSIS_E_STATE, "gsis_ws_targets: no mesh");
    std::vector<double> F((size_t)h->hm.nc * nf);
    int32_t rc = gsis_get_fields(h, F.data());
    if (rc != GSIS_OK) return rc;
    for (int64_t c = 0; c < h->hm.nc; ++c) {
        const double *f = &F[c * nf];
        double *o = t + c * (D + 5);
        // fields: rho, u (D), T_t, T_r, T_v, T_R, ...
        if (!(f[0] > 0 && f[D + 1] > 0 && f[D + 2] > 0 && f[D + 3] > 0 && f[D + 4] > 0))
            return fail(h, GSIS_E_DIVERGED, "gsis_ws_targets: non-positive density or temperature");
        o[0] = std::log(f[0]);
        for (int a = 0; a < D; ++a) o[1 + a] = f[1 + a];
        for (int j = 0; j < 4; ++j) o[D + 1 + j] = std::log(f[D + 1 + j]);
    }
    return GSIS_OK;
}

}  // extern "C"
