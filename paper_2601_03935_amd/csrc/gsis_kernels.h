// Buffers and launcher declarations shared by the kernel files and the C ABI.
#pragma once

#include "gsis_dev.h"
#include "../../include/gsis_warmstart.h"

#include <vector>

namespace gsis {

// Device buffers of the kinetic state for storage type T (float or double).
template <typename T>
struct KinBufs {
    T *f = nullptr, *f2 = nullptr, *gf = nullptr, *r = nullptr, *dl0 = nullptr, *dl1 = nullptr;
    T *I = nullptr, *I2 = nullptr, *gI = nullptr, *rI = nullptr, *dI0 = nullptr, *dI1 = nullptr;
    T *coef = nullptr, *xi = nullptr, *om = nullptr, *rhow = nullptr;
    T *gfb = nullptr;  // limited gradients of the boundary cells only, row i for cell bcells[i]
    T *ccons = nullptr;  // per cell: discrete-conservative corrections of the reference distributions (3 x 8)
    T *xiT = nullptr;  // velocity components component-major: xiT[a * nv + k]
    double *xi_d = nullptr, *w_d = nullptr, *om_d = nullptr, *wo_d = nullptr;  // om: D components per ordinate
    double *bflux = nullptr, *bsurf = nullptr;
};

// Device buffers of the synthetic-equation solver (FP64).
struct MacroBufs {
    double *W = nullptr, *W0 = nullptr, *P = nullptr, *fld = nullptr, *gfld = nullptr;
    double *W2 = nullptr, *P2 = nullptr, *fld2 = nullptr;  // second state of the inner-iteration ping-pong
    double *R = nullptr, *Dg = nullptr, *dU0 = nullptr, *dU1 = nullptr;
    double *fcon = nullptr;   // per face: frozen flux constants (dissipation + HoTs), HoT stress along n
    double *bcorr = nullptr;  // per boundary face: kinetic minus model flux at the start of the solve
    double *Gs = nullptr;                     // per cell slot (interior faces): spectral radii G, G_R
    double *Ff = nullptr;                     // per face: its flux (face orientation), large-grid split path
    double *part = nullptr;                   // per-block partial sums of the residual norm
    double *resc = nullptr, *scal = nullptr;  // per-cell scratch, device scalars (res0, mass, ...)
    double *bpart = nullptr;                  // partial sums of launch_block_sum (8 * kSumBlocks)
    double *Ts = nullptr;                     // per cell: translational temperature of W0
    int *hflags = nullptr;                    // pinned host memory: two copies of flags[0..1] (progress polls)
    hipEvent_t pev[2] = {nullptr, nullptr};   // completion of those copies
    int *flags = nullptr;                     // [0] done, [1] inner count, [2] block arrival counter
};

// Optional per-kernel timing with HIP events on the launch stream.  Kinds (see gsis.h GSIS_K_*):
// 0 gradients of f, 1 residual, 2 Jacobi sweeps, 3 radiation kernels, 4 moments, 5 wall densities and
// boundary fluxes, 6 synchronisation, 7 macro solve.
struct Prof {
    static constexpr int kKinds = 8;
    bool on = false;
    unsigned mask = 0xffu;  // kinds timed while on
    hipStream_t st = nullptr;
    struct Rec {
        int kind;
        double bytes;
        hipEvent_t a, b;
    };
    std::vector<Rec> pend;
    std::vector<hipEvent_t> pool;
    double ms[kKinds] = {0}, bytes[kKinds] = {0};
    int64_t n[kKinds] = {0};
    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        (void)hipEventCreate(&e);
        return e;
    }
    // returns an index to pass to end(); -1 when profiling is off
    int begin(int kind, double by)
    {
        if (!on || !(mask & (1u << kind))) return -1;
        Rec r{kind, by, get(), get()};
        (void)hipEventRecord(r.a, st);
        pend.push_back(r);
        return (int)pend.size() - 1;
    }
    void end(int i)
    {
        if (i >= 0) (void)hipEventRecord(pend[i].b, st);
    }
    void collect()
    {
        if (pend.empty()) return;
        (void)hipStreamSynchronize(st);
        for (auto &r : pend) {
            float t = 0;
            (void)hipEventElapsedTime(&t, r.a, r.b);
            ms[r.kind] += t;
            bytes[r.kind] += r.bytes;
            n[r.kind] += 1;
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pend.clear();
    }
    void reset()
    {
        collect();
        for (int i = 0; i < kKinds; ++i) ms[i] = bytes[i] = 0, n[i] = 0;
    }
    void destroy()
    {
        collect();
        for (auto e : pool) (void)hipEventDestroy(e);
        pool.clear();
    }
};

constexpr int kMBlk = 64;   // threads per block of the per-cell macro kernels (one wave)
constexpr int kSBlk = 256;  // threads per block of the slot-parallel inner-iteration kernels
// lanes per cell in the slot-parallel kernels (one per face slot) and cells per wave (the last
// 64 mod NFM lanes of a wave idle: 21 triangles or 10 hexahedra per wave)
__host__ __device__ constexpr int slot_lanes(int nfm) { return nfm; }
__host__ __device__ constexpr int cells_per_wave(int nfm) { return kWave / nfm; }
// blocks of the slot-parallel kernels = number of per-block partial sums of the inner residual norm
inline int64_t macro_nparts(int64_t nc, int nfm)
{
    const int64_t waves = (nc + cells_per_wave(nfm) - 1) / cells_per_wave(nfm);
    return (waves + kSBlk / kWave - 1) / (kSBlk / kWave);
}

struct MacroOpts {
    double cfl_macro, inner_tol;
    int max_inner, n_sweeps;
};

template <typename T, int D, int NFM>
void launch_kinetic(KinBufs<T> &B, const MeshDev &m, const Phys &p, const KinOpts &o, int64_t nv, int64_t no,
                    hipStream_t st, Prof *pf);
template <typename T, int D, int NFM>
void launch_boundary_state(KinBufs<T> &B, const MeshDev &m, const Phys &p, int so, int64_t nv, int64_t no,
                           hipStream_t st);
template <typename T, int D>
void launch_moments(const KinBufs<T> &B, const double *uref, double *mom, int64_t nc, int64_t nv, int64_t no,
                    const Phys &p, hipStream_t st);
template <typename T, int D>
void launch_prologue(const double *mom, T *coef, const double *h, int64_t nc, const Phys &p, double cfl,
                     hipStream_t st);
// discrete-conservative corrections of the reference distributions from the moments and the coefficients
template <typename T, int D>
void launch_cons_sums(const double *mom, const T *coef, const T *xi, const double *w, T *ccons, int64_t nc,
                      int64_t nv, const Phys &p, hipStream_t st);
template <typename T, int D>
void launch_sync(KinBufs<T> &B, const double *sp, int64_t nc, int64_t nv, int64_t no, const Phys &p, int init,
                 hipStream_t st);

// synthetic-equation solve from the moments mom (M^{k+1/2}); bflux: boundary flux moments of the same state;
// mom_mass: moments whose total mass a closed domain keeps.  Launches only: the solution ends in Mb.W (P,
// fld) whatever the inner count, and the host waits on the stream only to throttle itself (never with an
// empty queue); macro_count gives the inner iteration count afterwards.
template <int D, int NFM>
void macro_solve(MacroBufs &Mb, const MeshDev &m, const Phys &p, const MacroOpts &o, const double *mom,
                 const double *bflux, const double *mom_mass, hipStream_t st);
// inner iteration count of the last solve on the stream (synchronises the stream)
int macro_count(const MacroBufs &Mb, int max_inner, hipStream_t st);
// total masses of two moment arrays: B.scal[3] = sum V rho(mom_num), B.scal[2] = sum V rho(mom_den)
template <int D>
void launch_mass_ratio(MacroBufs &B, const MeshDev &m, const double *mom_num, const double *mom_den, hipStream_t st);
// f[i] *= num[0] / den[0] for n values (device scalars)
template <typename T>
void launch_scale(T *f, int64_t n, const double *num, const double *den, hipStream_t st);
// per-cell sync parameters [rho, u[D], Tt, Tr, Tv, eR] of the moments (slot 0) and of W (slot 1)
template <int D>
void launch_sync_params(const double *mom, const double *W, double *sp, int64_t nc, const Phys &p, int from_W,
                        hipStream_t st);
// epsilon contributions per cell between two moment arrays: 8 values (num rho, den rho, num u, den u,
// num T, den T, V, 1 if the new state is not a physical gas state) and their deterministic sum
template <int D>
void launch_residual(const double *mom1, const double *mom0, const double *vol, double *cellbuf, double *out7,
                     double *part, int64_t nc, const Phys &p, hipStream_t st);
// deterministic sums of n rows of k interleaved values (k sums); part: k * kSumBlocks doubles of scratch
constexpr int kSumBlocks = 128;
void launch_block_sum(const double *in, int64_t n, int k, double *out, double *part, hipStream_t st);

// warm-start network internals used by the solver's warm-start initialisation (mlp.hip): device row
// buffer of n standardised inputs, the forward pass on stream st (returns the device outputs [n][n_out]),
// and the dimensions
float *mlp_input_rows(gsis_mlp_t *m, int64_t n);
const float *mlp_forward_rows(gsis_mlp_t *m, int64_t n, hipStream_t st);
void mlp_dims(const gsis_mlp_t *m, int *n_in, int *n_out);
// x_out[i][j] = (x[i][j] - mean[j]) / scale[j] for n rows of k values (device arrays, FP64 in, FP32 out)
void launch_standardize(const double *x, const double *mean, const double *scale, float *out, int64_t n, int k,
                        hipStream_t st);

}  // namespace gsis
