// Internal declarations of the GSIS / DVM library: device tables, kernel launchers.
// The C ABI lives in capi.hip; kernels in kinetic.hip (O(N_cells x N_velocities) work) and
// macro.hip (per-cell synthetic-equation solver).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace gsis {

constexpr double kPi = 3.14159265358979323846;
constexpr int kWave = 64;

// Workgroup b of nb is dispatched to XCD b % 8; remap so that XCD x walks the contiguous block range
// [x nb/8, (x+1) nb/8) (cells and faces are in locality order, so neighbours share that XCD's L2).
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb)
{
    const int64_t q = nb / 8, r = nb % 8;
    const int64_t x = b % 8, i = b / 8;
    return x * q + (x < r ? x : r) + i;
}

// Moment vector per cell (FP64), index helpers for dimension D:
//   rho, u[D], Tt, Tr, Tv, eR, er, ev, sig[D*D] (full), qt[D], qr[D], qv[D], qR[D]
struct MomLayout {
    int D;
    __host__ __device__ constexpr int rho() const { return 0; }
    __host__ __device__ constexpr int u() const { return 1; }
    __host__ __device__ constexpr int Tt() const { return 1 + D; }
    __host__ __device__ constexpr int Tr() const { return 2 + D; }
    __host__ __device__ constexpr int Tv() const { return 3 + D; }
    __host__ __device__ constexpr int eR() const { return 4 + D; }
    __host__ __device__ constexpr int er() const { return 5 + D; }
    __host__ __device__ constexpr int ev() const { return 6 + D; }
    __host__ __device__ constexpr int sig() const { return 7 + D; }
    __host__ __device__ constexpr int qt() const { return 7 + D + D * D; }
    __host__ __device__ constexpr int qr() const { return 7 + 2 * D + D * D; }
    __host__ __device__ constexpr int qv() const { return 7 + 3 * D + D * D; }
    __host__ __device__ constexpr int qR() const { return 7 + 4 * D + D * D; }
    __host__ __device__ constexpr int size() const { return 7 + 5 * D + D * D; }
};
constexpr int kMomMax = 7 + 5 * 3 + 9;

// Physical constants of one run (host struct passed by value to kernels).
struct Phys {
    double d_r, d_v, Z_r, Z_v, omega, Sc, sigma_R, Kn, keff;
    double Tvref;  // characteristic vibrational temperature; <= 0: constant d_v
    double A[3][3], Q[3][3], K0[3][3];
};

// Vibrational mode (Sec. 2.1).  With a characteristic temperature T_ref > 0 the degrees of freedom are
// d_v(T) = 2 (T_ref / T) / (exp(T_ref / T) - 1), so the energy per unit mass is e_v(T) = d_v(T) T / 2 =
// T_ref / (exp(T_ref / T) - 1), with inverse T = T_ref / ln(1 + T_ref / e_v) and heat capacity
// c_v = de_v / dT = x^2 / (4 sinh^2(x / 2)), x = T_ref / T.  T_ref <= 0 keeps the constant d_v (and the
// constant-d_v forms of every expression).
__host__ __device__ inline double vib_e(const Phys &p, double T)
{
    return p.Tvref > 0 ? p.Tvref / expm1(p.Tvref / T) : 0.5 * p.d_v * T;
}
__host__ __device__ inline double vib_rho_e(const Phys &p, double rho, double T)
{
    return p.Tvref > 0 ? rho * (p.Tvref / expm1(p.Tvref / T)) : 0.5 * p.d_v * rho * T;
}
__host__ __device__ inline double vib_cv(const Phys &p, double T)
{
    if (!(p.Tvref > 0)) return 0.5 * p.d_v;
    const double x = p.Tvref / T, sh = sinh(0.5 * x);
    return x * x / (4 * sh * sh);
}
// T_v of the vibrational energy rho_ev (per unit volume) of a gas of density rho
__host__ __device__ inline double vib_T(const Phys &p, double rho_ev, double rho)
{
    return p.Tvref > 0 ? p.Tvref / log1p(p.Tvref * rho / rho_ev) : 2.0 * rho_ev / (p.d_v * rho);
}
// root T of alpha T + e_v(T) = R: the left side increases and is convex in T, so Newton from T = R / alpha
// (where it is >= 0) descends monotonically to the root
__host__ __device__ inline double vib_eq_T(const Phys &p, double alpha, double R)
{
    double T = R / alpha;
    for (int it = 0; it < 100; ++it) {
        const double dT = (alpha * T + vib_e(p, T) - R) / (alpha + vib_cv(p, T));
        T -= dT;
        if (!(fabs(dT) > 1e-15 * T)) break;
    }
    return T;
}
// translational-vibrational equilibrium temperature T_tv and the total temperature T of Sec. 2.1
__host__ __device__ inline double vib_Ttv(const Phys &p, double Tt, double Tv)
{
    if (!(p.Tvref > 0)) return (3 * Tt + p.d_v * Tv) / (3 + p.d_v);
    return vib_eq_T(p, 1.5, 1.5 * Tt + vib_e(p, Tv));
}
__host__ __device__ inline double vib_Ttot(const Phys &p, double Tt, double Tr, double Tv)
{
    if (!(p.Tvref > 0)) return (3 * Tt + p.d_r * Tr + p.d_v * Tv) / (3 + p.d_r + p.d_v);
    return vib_eq_T(p, 0.5 * (3 + p.d_r), 1.5 * Tt + 0.5 * p.d_r * Tr + vib_e(p, Tv));
}

// Options used by kernels.
struct KinOpts {
    double cfl_meso, cfl_v, kin_omega, limK;
    int kin_sweeps, second_order;
    int sweep;               // 0: Jacobi sweeps; 1: colored symmetric Gauss-Seidel sweeps
    int fused;               // 1: limited gradients recomputed inside the residual kernel
    int conservative;        // 1: discrete-conservative corrections of the reference distributions
    const int64_t *col_ptr;  // host: cells of colour q are col_cells[col_ptr[q] .. col_ptr[q + 1])
    int ncolor;
};

// Boundary tag data on the device.
struct BcDev {
    int kind;
    double rho, T, u[3];
    double ev;  // vibrational energy per unit mass e_v(T) of the boundary state
};

// Mesh tables on the device (all FP64 geometry; int32 connectivity).
//   per cell-slot (nc * NFM slots): nbr (>= 0 neighbour cell, -(1+bf) boundary face, INT32_MIN unused),
//   geo[(slot)*4D]: nSV[D] = n_out S / V, dxc[D] = x_f - x_c, dxj[D] = x_f - x_j, lsq[D];
//   mgeo[(slot)*(2D+2)]: n_out[D], S, dvec[D] (x_j - x_c, or x_f - x_c on a boundary), face id (as double);
//   per cell: vol, h, eps2 (limiter), nfc (faces), fsign per slot (+1 / -1)
struct MeshDev {
    int D = 0, NFM = 0;
    int64_t nc = 0, nf = 0, nbf = 0;
    int *nbr = nullptr;
    int *nb2 = nullptr;   // per slot (c, s): the NFM slots of neighbour j = nbr(c, s) (INT32_MIN if none)
    int *sfid = nullptr;  // per slot: face id if the cell is the face's left cell, -(1 + face id) otherwise
    double *geo = nullptr;
    double *mgeo = nullptr;
    double *lsq = nullptr;  // per slot: the D least-squares gradient weights of geo, packed (cell gradients)
    double *vol = nullptr, *h = nullptr, *eps2 = nullptr;
    int *nfc = nullptr;
    // distance-1 colouring (greedy, cells in index order): colour per cell, and the cells sorted by colour
    int *color = nullptr, *col_cells = nullptr;
    // boundary faces
    int *bf_face = nullptr, *bf_cell = nullptr, *bf_tag = nullptr;
    double *bf_n = nullptr, *bf_dxc = nullptr;  // outward unit normal, x_f - x_c
    int *bcells = nullptr;                       // distinct cells next to boundary faces
    int64_t nbcells = 0;
    int *bf_bidx = nullptr;                      // per boundary face: position of its cell in bcells
    // interior faces (for face HoTs / reference dissipation)
    int *f_L = nullptr, *f_R = nullptr;  // R < 0 on boundary faces
    int *fslot = nullptr;  // per face: the slot (c NFM + s) of its left cell and of its right cell (-1 on boundary)
    // per face, 2D + 2 values: the unit normal n (L -> R), and on interior faces with d = x_R - x_L the unit
    // vector d / |d|, 1 / |d| and 1 / |n . d| (zeros on boundary faces)
    double *fgeo = nullptr;
    BcDev *bcs = nullptr;
    BcDev *bf_bc = nullptr;  // per boundary face: its condition (the tag's entry of bcs, expanded)
    int nbc = 0;
    int closed = 1;
};

}  // namespace gsis
